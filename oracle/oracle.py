"""ctypes wrapper of the plain FP64 CPU oracle (``cgb_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``.  The product path never imports it.

The oracle follows Janoschek, Toschi & Harting (arXiv:1005.2594): Sec. II
(D3Q19 BGK lattice Boltzmann, Eqs. 1-8; mid-link and moving bounce-back,
Eqs. 9-11; momentum exchange, Eq. 12; cover/uncover; solid links, Eqs. 13-14;
single occupancy) and Sec. III (Berne-Pechukas pair and wall potentials,
Eqs. 15-20).  See ``cgb_oracle.c`` for the reading taken where the paper is
silent.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liborc.so")
_SRC = os.path.join(_HERE, "cgb_oracle.c")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2 -ffp-contract=off, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class OrcParams(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("tau", C.c_double), ("rho0", C.c_double),
        ("wall_y", C.c_int32),
        ("wall_v_bot", C.c_double * 3), ("wall_v_top", C.c_double * 3),
        ("force_mode", C.c_int32), ("g", C.c_double * 3), ("f0", C.c_double),
        ("force_on_particles", C.c_int32),
        ("R_perp", C.c_double), ("R_par", C.c_double),
        ("sig_perp", C.c_double), ("sig_par", C.c_double), ("sig_w", C.c_double),
        ("eps", C.c_double), ("eps_w", C.c_double),
        ("r_cut", C.c_double), ("rho_p", C.c_double), ("le_u", C.c_double),
        ("force_zlo", C.c_int32), ("force_zhi", C.c_int32),
    ]


def make_params(d: dict) -> OrcParams:
    p = OrcParams()
    for name, ctype in OrcParams._fields_:
        if name not in d:
            continue
        v = d[name]
        if isinstance(v, (list, tuple, np.ndarray)):
            arr = getattr(p, name)
            for i, x in enumerate(v):
                arr[i] = float(x)
        else:
            setattr(p, name, v)
    return p


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        L = _lib
        dp = C.POINTER(C.c_double)
        L.orc_create.argtypes = [C.POINTER(OrcParams), C.c_void_p, C.POINTER(C.c_void_p)]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_last_error.argtypes = [C.c_void_p]
        L.orc_last_error.restype = C.c_char_p
        L.orc_set_particles.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p]
        L.orc_init_fluid.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_set_deviations.argtypes = [C.c_void_p, C.c_void_p]
        L.orc_step.argtypes = [C.c_void_p, C.c_int32]
        for f in ("orc_get_deviations", "orc_get_owner", "orc_get_link_mask"):
            getattr(L, f).argtypes = [C.c_void_p, C.c_void_p]
        L.orc_get_fields.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_get_particles.argtypes = [C.c_void_p] + [C.c_void_p] * 4
        L.orc_get_forces.argtypes = [C.c_void_p] + [C.c_void_p] * 4
        L.orc_get_pairs.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(C.c_int64)]
        L.orc_get_link_static.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_get_observables.argtypes = [C.c_void_p, C.c_void_p]
        L.orc_mass_props.argtypes = [C.c_void_p, C.c_void_p]
        L.orc_mixture_sums.argtypes = [C.c_void_p, C.c_void_p]
        L.orc_mixture_field.argtypes = [C.c_void_p, C.c_void_p]
        L.orc_d3q19.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_equilibrium.argtypes = [C.c_double, C.c_void_p, C.c_void_p]
        L.orc_bp_pair.argtypes = [C.POINTER(OrcParams)] + [C.c_void_p] * 7
        L.orc_bp_wall.argtypes = [C.POINTER(OrcParams)] + [C.c_void_p] * 5
        L.orc_axis.argtypes = [C.c_void_p, C.c_void_p]
        L.orc_rotate.argtypes = [C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_void_p]
        L.orc_inside.argtypes = [C.POINTER(OrcParams), C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int32]
        L.orc_le_flux.argtypes = [C.c_void_p]
        L.orc_le_flux.restype = C.c_double
        del dp
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code


class Oracle:
    """One simulation state of the FP64 oracle."""

    def __init__(self, params: dict, wall_mask=None):
        self.params = dict(params)
        self._p = make_params(params)
        self.nx, self.ny, self.nz = int(params["nx"]), int(params["ny"]), int(params["nz"])
        self.ns = self.nx * self.ny * self.nz
        h = C.c_void_p()
        wm = None
        if wall_mask is not None:
            wm = np.ascontiguousarray(wall_mask, dtype=np.uint8).reshape(-1)
        rc = lib().orc_create(C.byref(self._p), _ptr(wm), C.byref(h))
        if rc != 0:
            raise OracleError(rc, "create failed")
        self.h = h
        self.n = 0

    def close(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != 0:
            raise OracleError(rc, lib().orc_last_error(self.h).decode())

    def set_particles(self, X, q, V=None, L=None, fixed=None):
        X = _f64(X, (-1, 3)); q = _f64(q, (-1, 4))
        n = X.shape[0]
        V = _f64(V, (n, 3)); L = _f64(L, (n, 3))
        fx = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.uint8)
        self.n = n
        self._check(lib().orc_set_particles(self.h, n, _ptr(X), _ptr(q), _ptr(V), _ptr(L), _ptr(fx)))

    def init_fluid(self, rho=None, u=None):
        rho = _f64(rho, (-1,)); u = _f64(u, (-1, 3))
        self._check(lib().orc_init_fluid(self.h, _ptr(rho), _ptr(u)))

    def set_deviations(self, d):
        d = _f64(d, (19, self.ns))
        self._check(lib().orc_set_deviations(self.h, _ptr(d)))

    def step(self, n=1):
        self._check(lib().orc_step(self.h, int(n)))

    def deviations(self):
        d = np.empty((19, self.ns))
        lib().orc_get_deviations(self.h, _ptr(d))
        return d

    def fields(self):
        rho = np.empty(self.ns); u = np.empty((self.ns, 3))
        lib().orc_get_fields(self.h, _ptr(rho), _ptr(u))
        return rho, u

    def particles(self):
        n = self.n
        X = np.empty((n, 3)); q = np.empty((n, 4)); V = np.empty((n, 3)); L = np.empty((n, 3))
        lib().orc_get_particles(self.h, _ptr(X), _ptr(q), _ptr(V), _ptr(L))
        return X, q, V, L

    def forces(self):
        n = self.n
        a = [np.empty((n, 3)) for _ in range(4)]
        lib().orc_get_forces(self.h, *[_ptr(x) for x in a])
        return tuple(a)

    def owner(self):
        o = np.empty(self.ns, dtype=np.int32)
        lib().orc_get_owner(self.h, _ptr(o))
        return o

    def link_mask(self):
        m = np.empty(self.ns, dtype=np.uint32)
        lib().orc_get_link_mask(self.h, _ptr(m))
        return m

    def pairs(self):
        n = C.c_int64()
        lib().orc_get_pairs(self.h, None, 0, C.byref(n))
        ij = np.empty((max(n.value, 1), 2), dtype=np.int32)
        lib().orc_get_pairs(self.h, _ptr(ij), n.value, C.byref(n))
        return ij[: n.value]

    def link_static(self):
        A = np.empty((self.n, 3), dtype=np.int64); B = np.empty((self.n, 3), dtype=np.int64)
        lib().orc_get_link_static(self.h, _ptr(A), _ptr(B))
        return A, B

    def observables(self):
        o = np.empty(12)
        lib().orc_get_observables(self.h, _ptr(o))
        return {"mass": o[0], "fluid_momentum": o[1:4].copy(), "particle_momentum": o[4:7].copy(),
                "n_fluid": int(o[7]), "body_force_last": o[8:11].copy(), "step": int(o[11])}

    def le_flux(self):
        """Delta p_LE,z of the last step: z momentum carried across the
        Lees-Edwards seam in -x (Eq. 23)."""
        return float(lib().orc_le_flux(self.h))

    def mass_props(self):
        o = np.empty(3)
        lib().orc_mass_props(self.h, _ptr(o))
        return {"M": o[0], "I_par": o[1], "I_perp": o[2]}

    def mixture(self):
        """(A, ubar) after the last step: A = (2/N) sum u_z sin(2 pi y/ny), the
        sine amplitude of the plane-averaged mixture velocity, and ubar = the
        mean mixture z velocity, over the N non-wall nodes."""
        o = np.empty(3)
        lib().orc_mixture_sums(self.h, _ptr(o))
        return 2.0 * o[0] / o[2], o[1] / o[2]

    def mixture_field(self):
        """Mixture velocity (ns, 3) after the last step: fluid nodes the
        velocity of the last collision, cell nodes the rigid-body velocity
        the last bounce-back used, 0 at walls."""
        u = np.empty((self.ns, 3))
        lib().orc_mixture_field(self.h, _ptr(u))
        return u

    def track(self, nsteps):
        """Steps nsteps times, recording mixture() after every step: (nsteps, 2)."""
        out = np.empty((nsteps, 2))
        for t in range(nsteps):
            self.step(1)
            out[t] = self.mixture()
        return out


# ---- pure functions ----
def d3q19():
    c = np.empty((19, 3), dtype=np.int32); w = np.empty(19); opp = np.empty(19, dtype=np.int32)
    lib().orc_d3q19(_ptr(c), _ptr(w), _ptr(opp))
    return c, w, opp


def equilibrium(rho, u):
    u = _f64(u, (3,)); out = np.empty(19)
    lib().orc_equilibrium(float(rho), _ptr(u), _ptr(out))
    return out


def bp_pair(params: dict, rvec, oi, oj):
    p = make_params(params)
    rvec = _f64(rvec, (3,)); oi = _f64(oi, (3,)); oj = _f64(oj, (3,))
    U = np.zeros(1); Fi = np.empty(3); ti = np.empty(3); tj = np.empty(3)
    lib().orc_bp_pair(C.byref(p), _ptr(rvec), _ptr(oi), _ptr(oj), _ptr(U), _ptr(Fi), _ptr(ti), _ptr(tj))
    return U[0], Fi, ti, tj


def bp_wall(params: dict, rvec, o):
    p = make_params(params)
    rvec = _f64(rvec, (3,)); o = _f64(o, (3,))
    U = np.zeros(1); F = np.empty(3); t = np.empty(3)
    lib().orc_bp_wall(C.byref(p), _ptr(rvec), _ptr(o), _ptr(U), _ptr(F), _ptr(t))
    return U[0], F, t


def axis(q):
    q = _f64(q, (4,)); o = np.empty(3)
    lib().orc_axis(_ptr(q), _ptr(o))
    return o


def rotate(q, L, I_par, I_perp, dt):
    q = _f64(q, (4,)); L = _f64(L, (3,)); out = np.empty(4)
    lib().orc_rotate(_ptr(q), _ptr(L), float(I_par), float(I_perp), float(dt), _ptr(out))
    return out


def inside(params: dict, X, o, node):
    p = make_params(params)
    X = _f64(X, (3,)); o = _f64(o, (3,)); node = _f64(node, (3,))
    return bool(lib().orc_inside(C.byref(p), _ptr(X), _ptr(o), _ptr(node)))


def num_threads():
    return int(lib().orc_num_threads())


def set_num_threads(n):
    lib().orc_set_num_threads(int(n))


# ---- apparent viscosity estimators (body-force driven flows) ----
def mu_rel_kolmogorov(A, f0, rho0, ny, first):
    """Relative apparent viscosity from the mode amplitudes A_t of a
    Kolmogorov flow driven by f0 sin(k y), k = 2 pi / ny, at tau = 1.

    At tau = 1 one step maps the amplitude of a pure shear mode exactly as
    A_{t+1} = lam A_t + (1 + lam) f0 / (2 rho0), lam = (2 + cos k)/3 (the
    third-order terms of Eq. 5 and the Guo term contribute nothing odd in
    c_z for a pure shear flow); the decay per step (1 - lam) A_t =
    (1 - cos k)/3 A_t is the viscous term nu k^2 A at nu = 1/6.  Writing the
    mixture's decay as mu_rel times the plasma's gives, per step,
      mu_rel(t) = [f0 (5 + cos k)/(6 rho0) - (A_{t+1} - A_t)] / [A_t (1 - cos k)/3],
    identically 1 for the particle-free fluid.  Returned: the mean of
    mu_rel(t) over t = first .. len(A) - 2."""
    A = np.asarray(A, dtype=np.float64)
    k = 2.0 * np.pi / ny
    t = np.arange(first, len(A) - 1)
    mu = (f0 * (5.0 + np.cos(k)) / (6.0 * rho0) - (A[t + 1] - A[t])) / (A[t] * (1.0 - np.cos(k)) / 3.0)
    return float(np.mean(mu))


def mu_app_le(flux, first, prof_x, ny, nz, rho0, tau):
    """Relative apparent viscosity of the plane-Couette viscometer (Sec. IV,
    Eq. 23): mu_app = Delta p_LE,z / (l_y l_z gammadot), with Delta p_LE,z the
    mean of the recorded per-step momentum transfers flux[first:] and
    gammadot the slope of a linear fit of the plane-averaged velocity profile
    v_z(x) over the central half of the planes, x in [nx/4, 3 nx/4); divided
    by the plasma's dynamic viscosity rho0 nu, nu = (2 tau - 1)/6."""
    prof_x = np.asarray(prof_x, dtype=np.float64)
    nx = len(prof_x)
    xs = np.arange(nx // 4, 3 * nx // 4)
    gd = np.polyfit(xs.astype(np.float64), prof_x[xs], 1)[0]
    dp = float(np.mean(np.asarray(flux, dtype=np.float64)[first:]))
    return dp / (ny * nz * gd) / (rho0 * (2.0 * tau - 1.0) / 6.0)


def mu_rel_slit(ubar, g, tau, ny, first):
    """Relative apparent viscosity of a body-force driven slit between
    mid-link walls (wall nodes y = 0 and ny - 1, N_f = ny - 2 fluid planes):
    the mean over t = first .. end of the mixture's mean velocity ubar_t,
    compared with the plasma's discrete steady state.  That state is the
    parabola with the slip of mid-link bounce-back,
    u(y) = g/(2 nu) [N_f^2/4 + (16 L - 3)/12 - (y - (N_f + 1)/2)^2],
    L = (tau - 1/2)^2, whose mean over the fluid planes is
    g (N_f^2 + 8 L - 1) / (12 nu) (= g (N_f^2 + 1)/(12 nu) at tau = 1), so
    mu_rel = g (N_f^2 + 8 L - 1) / (12 nu <ubar>), nu = (2 tau - 1)/6."""
    u = float(np.mean(np.asarray(ubar, dtype=np.float64)[first:]))
    nf = ny - 2
    nu = (2.0 * tau - 1.0) / 6.0
    lam = (tau - 0.5) ** 2
    return g * (nf * nf + 8.0 * lam - 1.0) / (12.0 * nu * u)
