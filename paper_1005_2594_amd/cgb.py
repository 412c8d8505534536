"""ctypes binding of libcgb.so (``include/cgb.h``): argument marshalling only.

Every step of the method runs in the HIP kernels of the library; there is no
host fallback.  Importing this module on a machine without the built library
raises ``ImportError``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcgb.so")

P64, P32, PMX16, PMXBF16, PMX16S = 0, 1, 2, 3, 4
PRECISIONS = {"p64": P64, "p32": P32, "pmx16": PMX16, "pmxbf16": PMXBF16, "pmx16s": PMX16S}
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EUNSTABLE", -5: "ESTATE"}


class CgbParams(C.Structure):
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
        ("r_cut", C.c_double), ("rho_p", C.c_double),
        ("precision", C.c_int32), ("pmx_scale", C.c_double), ("le_u", C.c_double), ("mem_layout", C.c_int32),
        ("force_zlo", C.c_int32), ("force_zhi", C.c_int32), ("indexed", C.c_int32),
    ]


class CgbSizes(C.Structure):
    _fields_ = [("arena_bytes", C.c_int64), ("staging_bytes", C.c_int64),
                ("cell_cap", C.c_int32), ("track_cap", C.c_int32)]


class CgbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"cgb {ERRORS.get(code, code)}: {msg}")
        self.code = code


_lib = None
VP = C.c_void_p


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run python -m paper_1005_2594_amd.build")
    # PyTorch ships its own HIP runtime under the same soname: loading it
    # first makes the library bind to that one, so that device memory and
    # streams can pass between the two (two runtimes in one process do not
    # share the device)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    L.cgb_params_default.argtypes = [C.POINTER(CgbParams)]
    L.cgb_create.argtypes = [C.POINTER(CgbParams), VP, VP, C.POINTER(VP)]
    L.cgb_query_sizes.argtypes = [C.POINTER(CgbParams), VP, C.c_int32, C.c_int32, C.POINTER(CgbSizes)]
    L.cgb_create_in.argtypes = [C.POINTER(CgbParams), VP, VP, C.POINTER(CgbSizes), VP, VP, C.POINTER(VP)]
    L.cgb_destroy.argtypes = [VP]
    L.cgb_destroy.restype = None
    L.cgb_last_error.argtypes = [VP]
    L.cgb_last_error.restype = C.c_char_p
    L.cgb_device_bytes.argtypes = [VP]
    L.cgb_device_bytes.restype = C.c_int64
    L.cgb_set_particles.argtypes = [VP, C.c_int32, VP, VP, VP, VP, VP]
    L.cgb_init_fluid.argtypes = [VP, VP, VP]
    L.cgb_set_populations.argtypes = [VP, VP]
    L.cgb_step.argtypes = [VP, C.c_int32]
    L.cgb_sync.argtypes = [VP]
    L.cgb_get_populations.argtypes = [VP, VP]
    L.cgb_get_fields.argtypes = [VP, VP, VP]
    L.cgb_get_box.argtypes = [VP, VP, VP, VP, VP]
    L.cgb_capture.argtypes = [VP, C.c_int32]
    L.cgb_replay.argtypes = [VP, C.c_int32]
    L.cgb_get_mixture_box.argtypes = [VP, VP, VP, VP]
    L.cgb_get_particles.argtypes = [VP, VP, VP, VP, VP]
    L.cgb_get_forces.argtypes = [VP, VP, VP, VP, VP]
    L.cgb_get_owner.argtypes = [VP, VP]
    L.cgb_get_link_mask.argtypes = [VP, VP]
    L.cgb_get_pairs.argtypes = [VP, VP, C.c_int64, C.POINTER(C.c_int64)]
    L.cgb_get_observables.argtypes = [VP, VP]
    L.cgb_get_profile_z.argtypes = [VP, VP]
    L.cgb_get_profile.argtypes = [VP, C.c_int32, VP]
    L.cgb_get_le_flux.argtypes = [VP, VP, C.c_int32, C.POINTER(C.c_int32)]
    L.cgb_mu_app_le.argtypes = [VP, C.c_int32, C.c_int32, VP, C.c_int32, C.c_int32, C.c_int32, C.c_double,
                                C.c_double, C.POINTER(C.c_double)]
    L.cgb_profile.argtypes = [VP, C.c_int]
    L.cgb_set_concurrency.argtypes = [VP, C.c_int]
    L.cgb_kernel_times.argtypes = [VP, VP, VP, VP, C.c_int32, C.POINTER(C.c_int32)]
    L.cgb_save.argtypes = [VP, C.c_char_p]
    L.cgb_load.argtypes = [VP, C.c_char_p]
    L.cgb_set_tiles.argtypes = [VP, C.c_int32, C.c_int32, C.c_int32]
    L.cgb_get_tiles.argtypes = [VP, VP]
    L.cgb_time_lb.argtypes = [VP, C.c_int32, C.POINTER(C.c_double)]
    L.cgb_batch_create.argtypes = [C.c_int32, VP, C.POINTER(VP)]
    L.cgb_batch_destroy.argtypes = [VP]
    L.cgb_batch_destroy.restype = None
    L.cgb_batch_last_error.argtypes = [VP]
    L.cgb_batch_last_error.restype = C.c_char_p
    L.cgb_batch_channel.argtypes = [VP, C.c_int32, C.POINTER(VP)]
    L.cgb_batch_autotune.argtypes = [VP, C.c_int32, VP]
    L.cgb_batch_capture.argtypes = [VP, C.c_int32]
    L.cgb_batch_run.argtypes = [VP, C.c_int32]
    L.cgb_batch_sync.argtypes = [VP]
    L.cgb_batch_track.argtypes = [VP, C.c_int32]
    L.cgb_batch_mu_rel.argtypes = [VP, C.c_int32, VP]
    L.cgb_track.argtypes = [VP, C.c_int32]
    L.cgb_get_track.argtypes = [VP, VP, C.c_int32, C.POINTER(C.c_int32)]
    L.cgb_mu_rel_kolmogorov.argtypes = [VP, C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_int32, C.POINTER(C.c_double)]
    L.cgb_mu_rel_slit.argtypes = [VP, C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_int32, C.POINTER(C.c_double)]
    L.cgb_mu_rel.argtypes = [VP, C.c_int32, C.POINTER(C.c_double)]
    L.cgb_mlp_create.argtypes = [C.c_int32, C.POINTER(VP)]
    L.cgb_mlp_destroy.argtypes = [VP]
    L.cgb_mlp_destroy.restype = None
    L.cgb_mlp_last_error.argtypes = [VP]
    L.cgb_mlp_last_error.restype = C.c_char_p
    L.cgb_mlp_set_params.argtypes = [VP, VP]
    L.cgb_mlp_get_params.argtypes = [VP, VP]
    L.cgb_mlp_set_norm.argtypes = [VP, VP, VP, C.c_float, C.c_float]
    L.cgb_mlp_forward.argtypes = [VP, C.c_int64, VP, VP]
    L.cgb_mlp_grad.argtypes = [VP, C.c_int32, VP, VP, VP, VP, VP]
    L.cgb_mlp_train.argtypes = [VP, C.c_int32, VP, VP, C.c_int32, VP, C.c_float, VP]
    L.cgb_mlp_train_noalloc.argtypes = [VP, C.c_int32, VP, VP, C.c_int32, VP, C.c_float, VP]
    L.cgb_mlp_predict.argtypes = [VP, C.c_int64, VP, VP, VP]
    L.cgb_mlp_predict_device.argtypes = [VP, C.c_int64, VP, VP, VP, VP]
    _lib = L
    return L


def _ptr(a):
    return None if a is None else a.ctypes.data_as(VP)


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a.reshape(shape) if shape is not None else a


def make_params(d: dict, precision=None) -> CgbParams:
    p = CgbParams()
    lib().cgb_params_default(C.byref(p))
    for name, _ in CgbParams._fields_:
        if name not in d:
            continue
        v = d[name]
        if isinstance(v, (list, tuple, np.ndarray)):
            arr = getattr(p, name)
            for i, x in enumerate(v):
                arr[i] = float(x)
        else:
            setattr(p, name, v)
    if precision is not None:
        p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    return p


def query_sizes(params: dict, wall_mask=None, cell_cap=0, track_cap=0, precision=None) -> CgbSizes:
    """Device bytes a lattice needs on caller-provided memory (``cgb_query_sizes``)."""
    p = make_params(params, precision)
    wm = None if wall_mask is None else np.ascontiguousarray(wall_mask, dtype=np.uint8).reshape(-1)
    sz = CgbSizes()
    rc = lib().cgb_query_sizes(C.byref(p), _ptr(wm), int(cell_cap), int(track_cap), C.byref(sz))
    if rc != 0:
        raise CgbError(rc, "cgb_query_sizes failed")
    return sz


class Sim:
    """One lattice with its cells on the GPU (one ``cgb_sim`` handle).

    With ``cell_cap`` set, the handle's device memory is two PyTorch tensors
    sized by ``cgb_query_sizes`` (kept alive by this object) and passed to
    ``cgb_create_in``; otherwise the library allocates it."""

    def __init__(self, params: dict, wall_mask=None, precision=None, stream=None, _handle=None,
                 cell_cap=None, track_cap=0):
        self._p = make_params(params, precision)
        self.nx, self.ny, self.nz = self._p.nx, self._p.ny, self._p.nz
        self.ns = self.nx * self.ny * self.nz
        self.n = 0
        self._owned = _handle is None
        if _handle is not None:
            self.h = _handle
            return
        h = VP()
        wm = None if wall_mask is None else np.ascontiguousarray(wall_mask, dtype=np.uint8).reshape(-1)
        st = None if stream is None else VP(int(stream))
        if cell_cap is None:
            rc = lib().cgb_create(C.byref(self._p), _ptr(wm), st, C.byref(h))
        else:
            import torch
            sz = CgbSizes()
            rc = lib().cgb_query_sizes(C.byref(self._p), _ptr(wm), int(cell_cap), int(track_cap), C.byref(sz))
            if rc == 0:
                self._arena = torch.empty(int(sz.arena_bytes), dtype=torch.uint8, device="cuda")
                self._staging = torch.empty(int(sz.staging_bytes), dtype=torch.uint8, device="cuda")
                torch.cuda.synchronize()
                rc = lib().cgb_create_in(C.byref(self._p), _ptr(wm), st, C.byref(sz), VP(self._arena.data_ptr()),
                                         VP(self._staging.data_ptr()), C.byref(h))
        if rc != 0:
            raise CgbError(rc, "cgb_create failed")
        self.h = h

    # -- lifecycle
    def close(self):
        if getattr(self, "h", None):
            if self._owned:
                lib().cgb_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, rc):
        if rc != 0:
            raise CgbError(rc, lib().cgb_last_error(self.h).decode())

    @property
    def device_bytes(self):
        return int(lib().cgb_device_bytes(self.h))

    # -- set-up
    def set_particles(self, X, q, V=None, L=None, fixed=None):
        X = _f64(X, (-1, 3)); q = _f64(q, (-1, 4))
        n = X.shape[0]
        V = _f64(V, (n, 3)); L = _f64(L, (n, 3))
        fx = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.uint8)
        self._check(lib().cgb_set_particles(self.h, n, _ptr(X), _ptr(q), _ptr(V), _ptr(L), _ptr(fx)))
        self.n = n

    def init_fluid(self, rho=None, u=None):
        rho = _f64(rho, (-1,)); u = _f64(u, (-1, 3))
        self._check(lib().cgb_init_fluid(self.h, _ptr(rho), _ptr(u)))

    def set_populations(self, d):
        d = _f64(d, (19, self.ns))
        self._check(lib().cgb_set_populations(self.h, _ptr(d)))

    # -- stepping
    def step(self, n=1):
        self._check(lib().cgb_step(self.h, int(n)))

    def sync(self):
        self._check(lib().cgb_sync(self.h))

    # -- read-out
    def populations(self):
        d = np.empty((19, self.ns))
        self._check(lib().cgb_get_populations(self.h, _ptr(d)))
        return d

    def capture(self, steps=2):
        """Records `steps` (even) steps as a HIP graph (``cgb_capture``)."""
        self._check(lib().cgb_capture(self.h, int(steps)))

    def replay(self, nsteps):
        """Replays the captured steps (``cgb_replay``), asynchronous."""
        self._check(lib().cgb_replay(self.h, int(nsteps)))

    def box(self, lo, ext):
        """Populations (19, ext_z, ext_y, ext_x) and owners (ext_z, ext_y, ext_x)
        of the sub-box lo + [0, ext) (``cgb_get_box``)."""
        lo3 = np.ascontiguousarray(lo, dtype=np.int32)
        ex3 = np.ascontiguousarray(ext, dtype=np.int32)
        nb = int(np.prod(ex3.astype(np.int64)))
        d = np.empty((19, nb)); own = np.empty(nb, dtype=np.int32)
        self._check(lib().cgb_get_box(self.h, _ptr(lo3), _ptr(ex3), _ptr(d), _ptr(own)))
        shp = (int(ex3[2]), int(ex3[1]), int(ex3[0]))
        return d.reshape((19,) + shp), own.reshape(shp)

    def mixture_box(self, lo, ext):
        """Mixture velocity (ext_z, ext_y, ext_x, 3) of the sub-box lo + [0, ext)
        (``cgb_get_mixture_box``)."""
        lo3 = np.ascontiguousarray(lo, dtype=np.int32)
        ex3 = np.ascontiguousarray(ext, dtype=np.int32)
        nb = int(np.prod(ex3.astype(np.int64)))
        u = np.empty((nb, 3))
        self._check(lib().cgb_get_mixture_box(self.h, _ptr(lo3), _ptr(ex3), _ptr(u)))
        return u.reshape(int(ex3[2]), int(ex3[1]), int(ex3[0]), 3)

    def fields(self):
        rho = np.empty(self.ns); u = np.empty((self.ns, 3))
        self._check(lib().cgb_get_fields(self.h, _ptr(rho), _ptr(u)))
        return rho, u

    def particles(self):
        n = self.n
        X = np.empty((n, 3)); q = np.empty((n, 4)); V = np.empty((n, 3)); L = np.empty((n, 3))
        self._check(lib().cgb_get_particles(self.h, _ptr(X), _ptr(q), _ptr(V), _ptr(L)))
        return X, q, V, L

    def forces(self):
        a = [np.empty((self.n, 3)) for _ in range(4)]
        self._check(lib().cgb_get_forces(self.h, *[_ptr(x) for x in a]))
        return tuple(a)

    def owner(self):
        o = np.empty(self.ns, dtype=np.int32)
        self._check(lib().cgb_get_owner(self.h, _ptr(o)))
        return o

    def link_mask(self):
        m = np.empty(self.ns, dtype=np.uint32)
        self._check(lib().cgb_get_link_mask(self.h, _ptr(m)))
        return m

    def pairs(self):
        n = C.c_int64()
        self._check(lib().cgb_get_pairs(self.h, None, 0, C.byref(n)))
        ij = np.empty((max(n.value, 1), 2), dtype=np.int32)
        self._check(lib().cgb_get_pairs(self.h, _ptr(ij), n.value, C.byref(n)))
        return ij[: n.value]

    def observables(self):
        o = np.empty(13)
        self._check(lib().cgb_get_observables(self.h, _ptr(o)))
        return {"mass": o[0], "fluid_momentum": o[1:4].copy(), "particle_momentum": o[4:7].copy(),
                "n_fluid": int(o[7]), "body_force_last": o[8:11].copy(), "step": int(o[11]),
                "bad_step": int(o[12])}

    def profile_z(self):
        p = np.empty(self.ny)
        self._check(lib().cgb_get_profile_z(self.h, _ptr(p)))
        return p

    def plane_profile(self, axis):
        """Mean mixture z velocity per plane normal to axis (0: x, 1: y, 2: z)."""
        n = (self.nx, self.ny, self.nz)[axis]
        p = np.empty(n)
        self._check(lib().cgb_get_profile(self.h, int(axis), _ptr(p)))
        return p

    def le_flux(self):
        """Recorded Delta p_LE,z per step (viscometer lattices)."""
        n = C.c_int32()
        self._check(lib().cgb_get_le_flux(self.h, None, 0, C.byref(n)))
        out = np.empty(max(n.value, 1))
        self._check(lib().cgb_get_le_flux(self.h, _ptr(out), n.value, C.byref(n)))
        return out[: n.value]

    # -- launch shape of the fused LB kernel
    def set_tiles(self, bx, by, tz):
        self._check(lib().cgb_set_tiles(self.h, int(bx), int(by), int(tz)))

    def tiles(self):
        t = np.zeros(3, dtype=np.int32)
        self._check(lib().cgb_get_tiles(self.h, _ptr(t)))
        return tuple(int(x) for x in t)

    # -- mixture record and apparent viscosity
    def track(self, cap):
        """Record the mixture sums after each of the next cap steps."""
        self._check(lib().cgb_track(self.h, int(cap)))

    def get_track(self):
        """(n, 2): per recorded step (A, ubar)."""
        n = C.c_int32()
        self._check(lib().cgb_get_track(self.h, None, 0, C.byref(n)))
        out = np.empty((max(n.value, 1), 2))
        self._check(lib().cgb_get_track(self.h, _ptr(out), n.value, C.byref(n)))
        return out[: n.value]

    def mu_rel(self, first=0):
        mu = C.c_double()
        self._check(lib().cgb_mu_rel(self.h, int(first), C.byref(mu)))
        return mu.value

    def time_lb(self, reps=10):
        """Average milliseconds of the fused LB kernel on the current state."""
        ms = C.c_double()
        self._check(lib().cgb_time_lb(self.h, int(reps), C.byref(ms)))
        return ms.value

    # -- timing
    def set_concurrency(self, on=True):
        """Independent phases of a step on side streams (on) or all kernels in sequence."""
        self._check(lib().cgb_set_concurrency(self.h, 1 if on else 0))

    def profile(self, enable=True):
        self._check(lib().cgb_profile(self.h, 1 if enable else 0))

    def kernel_times(self):
        cap = 32
        names = C.create_string_buffer(64 * cap)
        ms = np.zeros(cap); cnt = np.zeros(cap, dtype=np.int64); n = C.c_int32()
        self._check(lib().cgb_kernel_times(self.h, names, _ptr(ms), _ptr(cnt), cap, C.byref(n)))
        out = {}
        for k in range(n.value):
            nm = names.raw[64 * k: 64 * (k + 1)].split(b"\0", 1)[0].decode()
            out[nm] = (float(ms[k]), int(cnt[k]))
        return out

    # -- checkpoint
    def save(self, path):
        self._check(lib().cgb_save(self.h, str(path).encode()))

    def load(self, path):
        self._check(lib().cgb_load(self.h, str(path).encode()))


class Batch:
    """Independent channels of uneven size advanced together by one replayed
    HIP graph (``cgb_batch``).  ``channels[c]`` is a :class:`Sim` view of
    channel c (owned by the batch) for set-up and read-out."""

    def __init__(self, params_list, precision=None):
        ps = [make_params(d, precision) for d in params_list]
        arr = (CgbParams * len(ps))(*ps)
        h = VP()
        rc = lib().cgb_batch_create(len(ps), C.cast(arr, VP), C.byref(h))
        if rc != 0:
            raise CgbError(rc, "cgb_batch_create failed")
        self.h = h
        self.channels = []
        for c, d in enumerate(params_list):
            sh = VP()
            self._check(lib().cgb_batch_channel(self.h, c, C.byref(sh)))
            self.channels.append(Sim(d, precision=precision, _handle=sh))

    def close(self):
        if getattr(self, "h", None):
            for s in self.channels:
                s.close()
            lib().cgb_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __len__(self):
        return len(self.channels)

    def _check(self, rc):
        if rc != 0:
            raise CgbError(rc, lib().cgb_batch_last_error(self.h).decode())

    def autotune(self, reps=10):
        t = np.zeros((len(self), 3), dtype=np.int32)
        self._check(lib().cgb_batch_autotune(self.h, int(reps), _ptr(t)))
        return t

    def capture(self, steps=2):
        self._check(lib().cgb_batch_capture(self.h, int(steps)))

    def run(self, nsteps):
        self._check(lib().cgb_batch_run(self.h, int(nsteps)))

    def sync(self):
        self._check(lib().cgb_batch_sync(self.h))

    def track(self, cap):
        self._check(lib().cgb_batch_track(self.h, int(cap)))

    def mu_rel(self, first=0):
        mu = np.empty(len(self))
        self._check(lib().cgb_batch_mu_rel(self.h, int(first), _ptr(mu)))
        return mu


def mu_rel_kolmogorov(A, f0, rho0, ny, first):
    A = np.ascontiguousarray(A, dtype=np.float64)
    mu = C.c_double()
    rc = lib().cgb_mu_rel_kolmogorov(_ptr(A), len(A), int(first), float(f0), float(rho0), int(ny), C.byref(mu))
    if rc:
        raise CgbError(rc, "cgb_mu_rel_kolmogorov")
    return mu.value


def mu_app_le(flux, first, prof_x, ny, nz, rho0, tau):
    f = np.ascontiguousarray(flux, dtype=np.float64)
    px = np.ascontiguousarray(prof_x, dtype=np.float64)
    mu = C.c_double()
    rc = lib().cgb_mu_app_le(_ptr(f), len(f), int(first), _ptr(px), len(px), int(ny), int(nz), float(rho0),
                             float(tau), C.byref(mu))
    if rc:
        raise CgbError(rc, "cgb_mu_app_le")
    return mu.value


def mu_rel_slit(ubar, g, tau, ny, first):
    u = np.ascontiguousarray(ubar, dtype=np.float64)
    mu = C.c_double()
    rc = lib().cgb_mu_rel_slit(_ptr(u), len(u), int(first), float(g), float(tau), int(ny), C.byref(mu))
    if rc:
        raise CgbError(rc, "cgb_mu_rel_slit")
    return mu.value


MLP_PARAMS = 4481
MLP_BATCH = 128


def _f32(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a.reshape(shape) if shape is not None else a


class Mlp:
    """Ensemble of closure networks on the device (``cgb_mlp``)."""

    def __init__(self, members=5):
        h = VP()
        rc = lib().cgb_mlp_create(int(members), C.byref(h))
        if rc != 0:
            raise CgbError(rc, "cgb_mlp_create failed")
        self.h = h
        self.members = int(members)

    def close(self):
        if getattr(self, "h", None):
            lib().cgb_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != 0:
            raise CgbError(rc, lib().cgb_mlp_last_error(self.h).decode())

    def set_params(self, p):
        p = _f32(p, (self.members, MLP_PARAMS))
        self._check(lib().cgb_mlp_set_params(self.h, _ptr(p)))

    def params(self):
        p = np.empty((self.members, MLP_PARAMS), dtype=np.float32)
        self._check(lib().cgb_mlp_get_params(self.h, _ptr(p)))
        return p

    def set_norm(self, in_mean, in_std, out_mean, out_std):
        m = _f32(in_mean, (3,)); s = _f32(in_std, (3,))
        self._check(lib().cgb_mlp_set_norm(self.h, _ptr(m), _ptr(s), float(out_mean), float(out_std)))

    def forward(self, xn):
        xn = _f32(xn, (-1, 3))
        y = np.empty((self.members, len(xn)), dtype=np.float32)
        self._check(lib().cgb_mlp_forward(self.h, len(xn), _ptr(xn), _ptr(y)))
        return y

    def grad(self, xn, tn, idx):
        xn = _f32(xn, (-1, 3)); tn = _f32(tn, (-1,))
        idx = np.ascontiguousarray(idx, dtype=np.int32).reshape(self.members, MLP_BATCH)
        g = np.empty((self.members, MLP_PARAMS), dtype=np.float32)
        loss = np.empty(self.members, dtype=np.float32)
        self._check(lib().cgb_mlp_grad(self.h, len(xn), _ptr(xn), _ptr(tn), _ptr(idx), _ptr(g), _ptr(loss)))
        return g, loss

    def train(self, x, mu, idx, lr):
        """idx: [members][steps][MLP_BATCH] sample indices; returns the batch losses."""
        x = _f32(x, (-1, 3)); mu = _f32(mu, (-1,))
        idx = np.ascontiguousarray(idx, dtype=np.int32)
        steps = idx.shape[1]
        loss = np.empty((self.members, steps), dtype=np.float32)
        self._check(lib().cgb_mlp_train(self.h, len(x), _ptr(x), _ptr(mu), steps, _ptr(idx), float(lr), _ptr(loss)))
        return loss

    def train_noalloc(self, x, mu, idx, lr):
        """As train(), through the entry point that allocates no device memory."""
        x = _f32(x, (-1, 3)); mu = _f32(mu, (-1,))
        idx = np.ascontiguousarray(idx, dtype=np.int32)
        steps = idx.shape[1]
        loss = np.empty((self.members, steps), dtype=np.float32)
        self._check(lib().cgb_mlp_train_noalloc(self.h, len(x), _ptr(x), _ptr(mu), steps, _ptr(idx), float(lr),
                                                _ptr(loss)))
        return loss

    def predict(self, x):
        x = _f32(x, (-1, 3))
        mean = np.empty(len(x), dtype=np.float32); spread = np.empty(len(x), dtype=np.float32)
        self._check(lib().cgb_mlp_predict(self.h, len(x), _ptr(x), _ptr(mean), _ptr(spread)))
        return mean, spread

    def predict_device(self, n, x_ptr, mean_ptr, spread_ptr, stream=None):
        st = None if stream is None else VP(int(stream))
        self._check(lib().cgb_mlp_predict_device(self.h, int(n), VP(int(x_ptr)), VP(int(mean_ptr)),
                                                 VP(int(spread_ptr)), st))
