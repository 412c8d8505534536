"""Workload definitions and seeded input generators.

Parameter values are the paper's (Janoschek, Toschi & Harting,
arXiv:1005.2594) converted to lattice units, or the workload's own:

* tau = 1, rho0 = 1 (Sec. IV: tau is always 1 and the density is 1 in
  lattice units).
* eps-bar = eps-bar_w = 0.05: 1.47e-15 J (Sec. IV) divided by the energy unit
  dm dx^2/dt^2 with dx = 2/3 um, dt = 6.80e-8 s, dm = 3.05e-16 kg.
* sigma = (12/11) R: the paper's ratio R_par/sigma_par = 11/12 (Sec. IV) with
  the same aspect ratio for the cell-fluid and the cell-cell shapes.
* sigma_w = 1/2 (Sec. III).
* cell mass density rho_p: the paper gives none.  With the explicit
  (leap-frog) coupling a flat (2.5, 1.0) cell at rho_p = rho0 is unstable:
  its broadside added mass (8/3 a^3 ~ 42) exceeds its mass (26).  The
  channel with 20 cells runs at rho_p = 2 (the smallest stable value tried,
  closest to "equal to the fluid"); dense random suspensions need
  rho_p >= 12 for 500 steps and more for 2000 steps in narrow channels
  (rho_p = 16 grows a gap mode among crowded cells within ~1000 steps in a
  47-wide channel at Ht = 0.41, in the oracle as on the device), so they
  use rho_p = 64.
* body force on cells: force_on_particles = 2, i.e. rho0 times the cell
  volume times f(Y) -- the force on the plasma the cell displaces -- so that
  the heavier inertial mass does not also make the cells driven harder than
  neutrally buoyant ones.

Random cells: positions uniform in the box, orientations uniform on SO(3)
(normalised 4-D Gaussian quaternions), fluid at rest.
"""
from __future__ import annotations

import math

import numpy as np

EPS_LU = 0.05          # 1.47e-15 J in lattice units
SIGMA_OVER_R = 12.0 / 11.0
RHO_P_DILUTE = 2.0
RHO_P_DENSE = 64.0


def params(nx, ny, nz, **kw) -> dict:
    """Base parameter dictionary (numbers only)."""
    R_perp = kw.pop("R_perp", 2.5)
    R_par = kw.pop("R_par", 1.0)
    p = dict(
        nx=int(nx), ny=int(ny), nz=int(nz), tau=1.0, rho0=1.0, wall_y=0,
        wall_v_bot=(0.0, 0.0, 0.0), wall_v_top=(0.0, 0.0, 0.0),
        force_mode=0, g=(0.0, 0.0, 0.0), f0=0.0, force_on_particles=1,
        R_perp=R_perp, R_par=R_par,
        sig_perp=SIGMA_OVER_R * R_perp, sig_par=SIGMA_OVER_R * R_par, sig_w=0.5,
        eps=EPS_LU, eps_w=EPS_LU, r_cut=1.5 * max(R_perp, R_par), rho_p=1.0,
    )
    p.update(kw)
    return p


def random_quaternions(rng: np.random.Generator, n: int) -> np.ndarray:
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def uniform_positions(rng, n, box, y_range=None) -> np.ndarray:
    X = rng.random((n, 3)) * np.asarray(box, dtype=np.float64)
    if y_range is not None:
        X[:, 1] = y_range[0] + rng.random(n) * (y_range[1] - y_range[0])
    return X


def rsa_positions(rng, n, box, min_dist, y_range=None, periodic_y=True, max_tries=100000):
    """Random sequential addition: uniform draws, rejected while a centre lies
    closer than ``min_dist`` (minimum image) to an accepted one."""
    box = np.asarray(box, dtype=np.float64)
    out = np.empty((0, 3))
    tries = 0
    while out.shape[0] < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("random sequential addition did not converge")
        x = uniform_positions(rng, 1, box, y_range)[0]
        if out.shape[0]:
            d = out - x
            for a in range(3):
                if a == 1 and not periodic_y:
                    continue
                d[:, a] -= box[a] * np.round(d[:, a] / box[a])
            if np.min(np.einsum("ij,ij->i", d, d)) < min_dist * min_dist:
                continue
        out = np.vstack([out, x])
    return out


def cell_count(hematocrit, n_sites, R_perp, R_par) -> int:
    """Number of cells whose nominal ellipsoid volume fills the given fraction."""
    v_cell = 4.0 / 3.0 * math.pi * R_perp * R_perp * R_par
    return int(round(hematocrit * n_sites / v_cell))


def channel_walls(nx, ny, nz) -> np.ndarray:
    m = np.zeros((nz, ny, nx), dtype=np.uint8)
    m[:, 0, :] = 1
    m[:, ny - 1, :] = 1
    return m.reshape(-1)


# ---------------------------------------------------------------- workloads
def config1(seed=1):
    """24x24x48 wall-bounded channel, 20 cells (2.5, 1.0), g = 1e-6 z, FP64,
    100 steps.  Non-overlapping placement: bounding spheres of radius
    sigma_perp kept apart, and clear of the wall planes by sigma_perp+sigma_w."""
    p = params(24, 24, 48, wall_y=1, force_mode=1, g=(0.0, 0.0, 1e-6), rho_p=RHO_P_DILUTE, force_on_particles=2)
    rng = np.random.default_rng(seed)
    clear = p["sig_perp"] + p["sig_w"]
    X = rsa_positions(rng, 20, (24, 24, 48), 2.0 * p["sig_perp"], y_range=(clear, 23.0 - clear),
                      periodic_y=False)
    q = random_quaternions(rng, 20)
    return dict(params=p, X=X, q=q, steps=100, precision="p64", name="channel 24x24x48, 20 cells")


def kolmogorov(n, seed, hematocrit=0.4, f0=1e-6, steps=500, precision="p32"):
    """n^3 periodic box, f_z = f0 sin(2 pi y / n), random overlapping cells."""
    p = params(n, n, n, force_mode=2, f0=f0, rho_p=RHO_P_DENSE, force_on_particles=2)
    N = cell_count(hematocrit, n ** 3, p["R_perp"], p["R_par"])
    rng = np.random.default_rng(seed)
    X = uniform_positions(rng, N, (n, n, n))
    q = random_quaternions(rng, N)
    return dict(params=p, X=X, q=q, steps=steps, precision=precision,
                name=f"kolmogorov {n}^3 Ht={hematocrit}")


def config2(seed=2, n=256):
    return kolmogorov(n, seed, precision="p32")


def config3(seed=2, n=256):
    return kolmogorov(n, seed, precision="pmx16")


def config3_companion(seed=3, n=64):
    return kolmogorov(n, seed, precision="pmx16")


def config4(seed=4, n_channels=64, w_range=(32, 96), lz_range=(64, 192)):
    """Uneven wall-bounded channels (W, W, Lz): W ~ U{32..96}, Lz ~ U{64..192},
    Ht ~ U[0.1, 0.5], g ~ logU[1e-7, 1e-5] (ranges inclusive; smaller ranges
    give the same recipe at test sizes)."""
    rng = np.random.default_rng(seed)
    chans = []
    for c in range(n_channels):
        W = int(rng.integers(w_range[0], w_range[1] + 1))
        Lz = int(rng.integers(lz_range[0], lz_range[1] + 1))
        Ht = float(rng.uniform(0.1, 0.5))
        g = float(10.0 ** rng.uniform(-7.0, -5.0))
        p = params(W, W, Lz, wall_y=1, force_mode=1, g=(0.0, 0.0, g), rho_p=RHO_P_DENSE, force_on_particles=2)
        n_fluid = W * (W - 2) * Lz
        N = cell_count(Ht, n_fluid, p["R_perp"], p["R_par"])
        clear = p["R_perp"]
        X = uniform_positions(rng, N, (W, W, Lz), y_range=(clear, W - 1 - clear))
        q = random_quaternions(rng, N)
        chans.append(dict(params=p, X=X, q=q, hematocrit=Ht, g=g, width=W, length=Lz))
    return chans


# The paper's largest system (Sec. IV): a quasi-homogeneous suspension of
# 1024^2 x 2048 sites and 4.1e6 cells.  Built as 16 x 16 x 32 copies of one
# periodic 64^3 tile of 500 cells (4,096,000 cells, Ht 0.05), so that a run of
# the whole lattice can be checked against a run of the tile: positions on a
# 2^-10 grid keep every copy's coordinates exact in FP64.
PAPER_SCALE = (1024, 1024, 2048)
PAPER_TILE = 64
PAPER_TILE_CELLS = 500


def paper_scale_tile(seed=5, f=1e-6):
    """The 64^3 periodic tile: 500 cells (2.5, 1.0) placed by random
    sequential addition with bounding spheres apart (no two cells share a
    node, so no occupancy conflict depends on the cells' indices), positions
    on a 2^-10 grid, uniform orientations, random translational and angular
    momenta, constant body force f z on plasma and cells."""
    n = PAPER_TILE
    p = params(n, n, n, force_mode=1, g=(0.0, 0.0, f), rho_p=RHO_P_DENSE, force_on_particles=2)
    rng = np.random.default_rng(seed)
    X = rsa_positions(rng, PAPER_TILE_CELLS, (n, n, n), 2.0 * p["R_perp"] + 0.01)
    X = np.floor(X * 1024.0) / 1024.0
    q = random_quaternions(rng, PAPER_TILE_CELLS)
    V = 2e-3 * rng.standard_normal((PAPER_TILE_CELLS, 3))
    L = 0.1 * rng.standard_normal((PAPER_TILE_CELLS, 3))
    return dict(params=p, X=X, q=q, V=V, L=L)


def tile_copies(tile, reps):
    """Cells of reps = (kx, ky, kz) copies of a periodic tile, copy-major
    (cell i of copy (a, b, c) at index i + N (a + kx (b + ky c))), and the
    parameters of the whole lattice."""
    n = tile["params"]["nx"]
    kx, ky, kz = reps
    c, b, a = np.meshgrid(np.arange(kz), np.arange(ky), np.arange(kx), indexing="ij")
    off = n * np.stack([a.ravel(), b.ravel(), c.ravel()], axis=1).astype(np.float64)
    X = (off[:, None, :] + tile["X"][None, :, :]).reshape(-1, 3)
    rep = lambda v: np.tile(v, (kx * ky * kz, 1))
    p = dict(tile["params"], nx=n * kx, ny=n * ky, nz=n * kz)
    return dict(params=p, X=X, q=rep(tile["q"]), V=rep(tile["V"]), L=rep(tile["L"]))


def paper_scale_suspension(seed=6, f0=1e-6):
    """The paper's largest system as a random suspension: 1024^2 x 2048
    periodic, 4.1e6 cells (2.5, 1.0) at uniform positions and orientations
    (overlaps allowed, Ht 0.05), f_z = f0 sin(2 pi y / ny)."""
    nx, ny, nz = PAPER_SCALE
    p = params(nx, ny, nz, force_mode=2, f0=f0, rho_p=RHO_P_DENSE, force_on_particles=2)
    rng = np.random.default_rng(seed)
    N = 4_100_000
    X = uniform_positions(rng, N, (nx, ny, nz))
    q = random_quaternions(rng, N)
    return dict(params=p, X=X, q=q, name=f"kolmogorov {nx}x{ny}x{nz}, {N} cells")


# ---------------------------------------------------------------- vessels
# Wall masks (1 = wall node) of the paper's vessel geometries (Sec. IV):
# a straight cylinder, and a bifurcation of cylindrical capillaries whose
# daughter branches rejoin before the periodic end, one of them with a
# stenosis.  Layout [z][y][x], axis along z, periodic in z.
def cylinder_mask(R, L):
    """Cylinder of radius R about the box axis, box (2 ceil(R) + 3)^2 x L."""
    n = 2 * int(math.ceil(R)) + 3
    c = (n - 1) / 2.0
    y, x = np.mgrid[0:n, 0:n]
    wall2d = ((x - c) ** 2 + (y - c) ** 2) >= R * R
    return np.broadcast_to(wall2d, (L, n, n)).astype(np.uint8).copy()


def bifurcation_mask(Rp, Rd, D, L, stenosis=None):
    """A parent tube of radius Rp along z splits into two daughter tubes of
    radius Rd whose axes move apart to x offsets -D and +D and back, so that
    the two branches rejoin before the periodic end.  Segments along z:
    parent [0, L/4), opening [L/4, 3L/8), branches [3L/8, 5L/8), closing
    [5L/8, 3L/4), parent [3L/4, L).  stenosis = (Rs, length): the +x branch
    narrows to radius Rs over `length` nodes at the middle of the branch
    segment.  The box is mirror symmetric in x (centre (nx - 1)/2)."""
    nx = 2 * int(math.ceil(D + Rd)) + 3
    ny = 2 * int(math.ceil(max(Rp, Rd))) + 3
    cx, cy = (nx - 1) / 2.0, (ny - 1) / 2.0
    y, x = np.mgrid[0:ny, 0:nx]
    m = np.ones((L, ny, nx), dtype=np.uint8)
    q = L / 8.0

    def tube(tx, r):
        return ((x - tx) ** 2 + (y - cy) ** 2) < r * r

    for z in range(L):
        if z < 2 * q or z >= 6 * q:
            fluid = tube(cx, Rp)
        else:
            if z < 3 * q:
                f = (z - 2 * q) / q
            elif z < 5 * q:
                f = 1.0
            else:
                f = (6 * q - 1 - z) / q
            f = min(max(f, 0.0), 1.0)
            r = Rp + (Rd - Rp) * f
            rp = r
            if stenosis is not None and abs(z - 4 * q) < stenosis[1] / 2.0:
                rp = stenosis[0]
            # the +x branch is the mirror image of a -x branch of radius rp,
            # so that equal branches give an exactly mirror-symmetric mask
            fluid = tube(cx - D * f, r) | tube(cx - D * f, rp)[:, ::-1]
        m[z][fluid] = 0
    return m


def vessel_cells(mask, n, R_perp, seed, clear=1.0, min_dist=None):
    """n cell centres placed by random sequential addition inside the non-wall
    region, every node within R_perp + clear of a centre being non-wall, and
    centres at least min_dist apart (default 2 R_perp + 0.01: no two cells
    share a node); positions on a 2^-10 grid; uniform orientations."""
    rng = np.random.default_rng(seed)
    L, ny, nx = mask.shape
    rr = R_perp + clear
    k = int(math.ceil(rr))
    off = np.array([(a, b, c) for a in range(-k, k + 1) for b in range(-k, k + 1) for c in range(-k, k + 1)
                    if a * a + b * b + c * c <= rr * rr + 1e-9])
    md = 2.0 * R_perp + 0.01 if min_dist is None else min_dist
    # large boxes: draw candidates among the vessel nodes
    cand = np.argwhere(mask == 0) if mask.size > 1_000_000 else None
    X = np.empty((n, 3))
    k_acc = 0
    tries = 0
    while k_acc < n:
        tries += 1
        if tries > 50 * n + 200000:
            raise RuntimeError("cell placement did not converge")
        p = np.floor(rng.random(3) * np.array([nx, ny, L]) * 1024.0) / 1024.0
        if cand is not None:
            # a random vessel node, jittered within its unit cell
            j = cand[rng.integers(len(cand))]
            p = np.floor((np.array([j[2], j[1], j[0]], dtype=np.float64) + rng.random(3) - 0.5) * 1024.0) / 1024.0
            p[2] %= L
        nodes = np.round(p).astype(int)[None, :] + off
        zz = nodes[:, 2] % L
        if (nodes[:, 0] < 0).any() or (nodes[:, 0] >= nx).any() or (nodes[:, 1] < 0).any() or (nodes[:, 1] >= ny).any():
            continue
        if mask[zz, nodes[:, 1], nodes[:, 0]].any():
            continue
        if k_acc:
            d = X[:k_acc] - p
            d[:, 2] -= L * np.round(d[:, 2] / L)
            if np.min(np.einsum("ij,ij->i", d, d)) < md * md:
                continue
        X[k_acc] = p
        k_acc += 1
    return X, random_quaternions(rng, n)


def vessel_params(mask, **kw):
    """Parameters of a lattice holding the mask (walls from the mask only)."""
    L, ny, nx = mask.shape
    return params(nx, ny, L, **kw)


def vessel_network(seed=7, Ht=0.1):
    """A bifurcation with a stenosis at a size that fills the GPU: parent
    radius 16, branch radius 12, branch axes 18 apart from the middle,
    stenosis radius 8 over 64 nodes, length 2048 (periodic), cells at
    hematocrit Ht of the vessel volume, body force on the fluid of the
    entrance region (the first 128 planes)."""
    m = bifurcation_mask(16, 12, 18, 2048, stenosis=(8.0, 64))
    p = vessel_params(m, force_mode=1, g=(0.0, 0.0, 2e-5), force_zlo=0, force_zhi=128, rho_p=RHO_P_DENSE,
                      force_on_particles=0)
    nc = int((1 - m).sum())
    N = cell_count(Ht, nc, p["R_perp"], p["R_par"])
    X, q = vessel_cells(m, N, p["R_perp"], seed, clear=0.0, min_dist=2.5)
    return dict(params=p, mask=m, X=X, q=q, name=f"bifurcation with stenosis {p['nx']}x{p['ny']}x{p['nz']}, "
                f"{nc} vessel nodes, {N} cells (overlaps allowed)")
