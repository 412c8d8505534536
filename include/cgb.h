/*
 * cgb.h -- C ABI of the MI355X (gfx950) implementation of the time step of the
 * coarse-grained blood model of Janoschek, Toschi & Harting, "A simplified
 * particulate model for coarse-grained hemodynamics simulations"
 * (arXiv:1005.2594): a D3Q19 BGK lattice-Boltzmann plasma (Sec. II, Eqs. 1-8)
 * coupled by mid-link / moving bounce-back (Eqs. 9-11) and momentum exchange
 * (Eq. 12) to rigid oblate ellipsoidal cells that interact through
 * Berne-Pechukas-scaled Hookean repulsions (Sec. III, Eqs. 15-20).
 *
 * Conventions
 *  - Every call returns an int status: CGB_OK (0) or a negative CGB_E* code;
 *    cgb_last_error() gives a message.  Nothing throws or aborts across the ABI.
 *  - Lattice units.  Site index = x + nx*(y + ny*z).
 *  - D3Q19 order (fixed): 0 rest; 1..6 = +x,-x,+y,-y,+z,-z; 7..18 = the face
 *    diagonals (+x+y),(-x-y),(+x-y),(-x+y),(+x+z),(-x-z),(+x-z),(-x+z),
 *    (+y+z),(-y-z),(+y-z),(-y+z).  Opposite directions are adjacent pairs.
 *  - Populations cross the ABI as FP64 deviations d_r = n*_r - w_r*rho0 of the
 *    post-collision populations, whatever the storage precision.
 *  - All pointer arguments of cgb_set_* / cgb_get_* are HOST pointers owned by
 *    the caller, with the sizes stated.  Device memory is owned by the handle
 *    (cgb_create) or provided by the caller (cgb_query_sizes, cgb_create_in).
 *  - cgb_step is asynchronous on the handle's stream; device-side failures
 *    (instability, overflow of a work list) surface at the next cgb_sync or
 *    cgb_get_* call.
 */
#ifndef CGB_H
#define CGB_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

#define CGB_OK 0
#define CGB_EINVAL (-1)    /* bad argument or unsupported size            */
#define CGB_ENOMEM (-2)    /* device or host allocation failed            */
#define CGB_EDEVICE (-3)   /* HIP runtime error                           */
#define CGB_EUNSTABLE (-4) /* non-finite state, |u| > 0.4 or |V_a| >= 0.5 */
#define CGB_ESTATE (-5)    /* call out of order (e.g. step before init)   */

/* storage precision of the populations */
#define CGB_P64 0      /* FP64 storage, FP64 collision                          */
#define CGB_P32 1      /* FP32 storage, FP32 collision                          */
#define CGB_PMX16 2    /* FP16 scaled deviations, FP32 collision                */
#define CGB_PMXBF16 3  /* BF16 scaled deviations, FP32 collision                */
#define CGB_PMX16S 4   /* FP16 deviations split per node, FP32 collision: the
                          node's density deviation D = rho - rho0 is stored once
                          (FP16, the density field every PMX mode keeps) and each
                          direction stores the FP16 residual d_r / w_r - D, so
                          d_r = w_r (D + residual).  The common part of the 19
                          deviations (the density fluctuation) no longer sets the
                          FP16 rounding of the velocity-carrying part; 2 bytes per
                          population as in CGB_PMX16                         */
/* In every precision the momentum exchange, the per-cell force/torque sums,
 * the pair forces and the rigid-body integrator run in FP64. */

typedef struct cgb_params {
    int32_t nx, ny, nz;
    double tau;           /* BGK relaxation time, Eq. 4; nu = (2 tau - 1)/6   */
    double rho0;          /* reference density rho-bar (Sec. II)              */
    int32_t wall_y;       /* 1: wall planes at y = 0 and y = ny-1             */
    double wall_v_bot[3]; /* velocity of the plane y = 0 (Eq. 10)             */
    double wall_v_top[3]; /* velocity of the plane y = ny-1 (Eq. 10)          */
    int32_t force_mode;   /* 0 none, 1 constant g, 2 f0 sin(2 pi y/ny) e_z    */
    double g[3];
    double f0;
    int32_t force_on_particles; /* 0: body force on the plasma only; 1: cells
                                   feel M f(Y) too; 2: cells feel rho0 V f(Y),
                                   V their volume (driven as the plasma they
                                   displace, whatever their inertial mass)   */
    double R_perp, R_par;       /* discretised ellipsoid half axes (Sec. II)  */
    double sig_perp, sig_par;   /* potential size parameters (Eq. 18)         */
    double sig_w;               /* wall sphere radius (Sec. III)              */
    double eps, eps_w;          /* potential strengths                        */
    double r_cut;               /* pair cut-off (hard truncation of Eq. 15)   */
    double rho_p;               /* cell mass density                          */
    int32_t precision;          /* CGB_P64 ... CGB_PMX16S                     */
    double pmx_scale;           /* PMX: stored value = d_r / w_r * pmx_scale
                                   (PMX16S: (d_r / w_r - D) * pmx_scale, and the
                                   density field D * pmx_scale); 0 selects 32768 */
    double le_u;                /* plane-Couette viscometer (Sec. IV): velocity
                                   offset U along z across the periodic seam of x
                                   (Lees-Edwards: the image beyond x = nx - 1
                                   moves at +U e_z, shifted by U t along z);
                                   cells are reflected at the sheared planes
                                   x = 0 and nx - 1.  0 = plain periodic x.
                                   Needs wall_y = 0 and a storage precision other
                                   than CGB_PMX16S (CGB_EINVAL otherwise)         */
    int32_t mem_layout;         /* 0: chosen by size; 1: the large-lattice layout
                                   at any size.  The large-lattice layout (used
                                   when a population array passes 4 GB, e.g. the
                                   paper's 1024^2 x 2048 system, Sec. IV) addresses
                                   the lattice with 64-bit offsets and keeps each
                                   cell node's momentum (Eq. 12) in the node's own
                                   unused population slots instead of a separate
                                   32-byte-per-site array; results are identical.
                                   It needs tau = 1, le_u = 0 and LB sweeps of 16
                                   nodes (cgb_set_tiles tz = 16; the default)      */
    int32_t force_zlo, force_zhi; /* force_mode 1 only: the constant body force
                                   acts on the nodes with force_zlo <= z <
                                   force_zhi (and on cells whose centre lies
                                   there), e.g. the entrance region of the
                                   bifurcation runs (Sec. IV); force_zhi <=
                                   force_zlo: everywhere                          */
    int32_t indexed;            /* 1: the indexed layout for sparse geometries
                                   (vessel networks, Sec. IV): populations,
                                   densities, link moments and node momenta are
                                   stored for the non-wall nodes only, reached
                                   through a per-site index map; owner, flags
                                   and claims stay per site.  Results are
                                   identical to the dense layout.  Needs tau = 1,
                                   le_u = 0, a lattice within the 32-bit layout
                                   and LB sweeps of 16 nodes (tz = 16)            */
} cgb_params;

typedef struct cgb_sim cgb_sim;

/* Fills *p with a 32^3 periodic box and the paper's parameters in lattice
 * units (tau = 1, rho0 = 1, eps = eps_w = 0.05, sigma_w = 1/2). */
int cgb_params_default(cgb_params* p);

/* Device memory a lattice needs when the caller provides it (for instance
 * PyTorch tensors; the library then allocates no device memory of its own). */
typedef struct cgb_sizes {
    int64_t arena_bytes;    /* every state array of the lattice and its cells   */
    int64_t staging_bytes;  /* FP64 staging of the host transfers (19 nsites x 8) */
    int32_t cell_cap;       /* cells the arena holds                            */
    int32_t track_cap;      /* steps cgb_track can record                       */
} cgb_sizes;
/* Fills *out for parameters p, walls wall_mask (as cgb_create), room for
 * cell_cap cells and a track record of track_cap steps.  CGB_EINVAL for
 * parameters cgb_create refuses. */
int cgb_query_sizes(const cgb_params* p, const uint8_t* wall_mask, int32_t cell_cap, int32_t track_cap,
                    cgb_sizes* out);

/* Creates a lattice.  wall_mask: nullable host array of nx*ny*nz bytes,
 * nonzero = wall node (added to the planes selected by wall_y).
 * stream: a hipStream_t to run on, or NULL to create a private stream.
 * All lattice nodes start as fluid at rest with rho0. */
int cgb_create(const cgb_params* p, const uint8_t* wall_mask, void* stream, cgb_sim** out);
/* As cgb_create, on device memory the caller owns: arena (256-byte aligned)
 * and staging (8-byte aligned) DEVICE pointers of at least the sizes that
 * cgb_query_sizes gives for the same p, wall_mask, sz->cell_cap and
 * sz->track_cap (*sz as it filled them).  Every device array of the handle is
 * a piece of these two buffers: no call on the handle allocates device
 * memory; cgb_set_particles / cgb_load refuse more than cell_cap cells and
 * cgb_track more than track_cap steps (CGB_EINVAL).  The buffers must outlive
 * the handle; their initial contents do not matter.  Results are identical
 * to a handle made by cgb_create. */
int cgb_create_in(const cgb_params* p, const uint8_t* wall_mask, void* stream, const cgb_sizes* sz, void* arena,
                  void* staging, cgb_sim** out);
void cgb_destroy(cgb_sim* s);
const char* cgb_last_error(const cgb_sim* s);
/* device bytes held by the handle */
int64_t cgb_device_bytes(const cgb_sim* s);

/* Cells (Sec. II): X n*3 centres, q n*4 unit quaternions (scalar first; the
 * symmetry axis is R(q) e_z), V n*3 and L n*3 (space-frame angular momentum)
 * at t-1/2 (nullable: zero), fixed n bytes (nullable; 1 = held at rest).
 * Rasterises the cells from scratch: overlaps go to the lowest index, newly
 * covered fluid is dropped, freed nodes get rest fluid at rho0. */
int cgb_set_particles(cgb_sim* s, int32_t n, const double* X, const double* q,
                      const double* V, const double* L, const uint8_t* fixed);

/* Fluid at equilibrium (Eq. 5) with density rho (nullable: rho0, nsites) and
 * velocity u (nullable: 0, nsites*3) on every non-wall node. */
int cgb_init_fluid(cgb_sim* s, const double* rho, const double* u);
/* Overwrites the stored post-collision deviations (19*nsites FP64), encoded
 * to the storage precision. */
int cgb_set_populations(cgb_sim* s, const double* d);

/* Advances nsteps time steps (asynchronous).  One step: cell axes and angular
 * velocities -> rasterisation with single occupancy -> cover/uncover with
 * momentum bookkeeping (Sec. II) -> fused pull stream + bounce-back with the
 * moving-boundary correction (Eqs. 9-11) + BGK collision with Guo forcing +
 * momentum exchange per cell (Eq. 12, solid links Eqs. 13-14 folded in
 * exactly) -> cell list -> pair and wall potentials (Eqs. 15-20) -> FP64
 * leap-frog with quaternion rotation. */
int cgb_step(cgb_sim* s, int32_t nsteps);
/* Captures `steps` (even, >= 2) time steps into a HIP graph on the handle's
 * stream, for cgb_replay: a replay launches the whole step sequence (its
 * side stream included) at once instead of one launch per kernel, which
 * removes the launch gaps of long runs.  Nothing is stepped.  The capture
 * holds while the handle's launches stay the same: cgb_set_particles,
 * cgb_set_tiles, cgb_set_concurrency, cgb_track, cgb_load or an odd number of
 * eager steps make cgb_replay refuse (CGB_ESTATE) until the next capture.
 * CGB_ESTATE while kernel timing (cgb_profile) is on: replays record none. */
int cgb_capture(cgb_sim* s, int32_t steps);
/* Replays the captured steps nsteps / steps times (nsteps a multiple of the
 * captured count); asynchronous like cgb_step, results identical to it. */
int cgb_replay(cgb_sim* s, int32_t nsteps);

/* Waits for the stream; returns CGB_EUNSTABLE if any step tripped the
 * instability check (the first such step is in cgb_get_observables out[12]). */
int cgb_sync(cgb_sim* s);

/* The populations and owners of the sub-box lo + [0, ext) of the lattice (no
 * wrap: lo + ext <= (nx, ny, nz)), for lattices too large for the
 * whole-lattice getters: d (nullable) receives 19 * nb FP64 deviations,
 * d[r * nb + k], 0 at non-fluid nodes; owner (nullable) nb owners (cell
 * index, -1 fluid, -2 wall); k = x' + ext[0] * (y' + ext[1] * z'),
 * nb = ext[0] * ext[1] * ext[2].  Host arrays; device staging of the box
 * only.  CGB_EINVAL for a box outside the lattice. */
int cgb_get_box(cgb_sim* s, const int32_t* lo, const int32_t* ext, double* d, int32_t* owner);

/* The mixture velocity on the sub-box lo + [0, ext) (bounds as cgb_get_box):
 * u[3 k + c] (host array of 3 * nb doubles).  Fluid nodes: the velocity of
 * the last collision, (sum n* c - g/2) / rho (Eq. 1 with the forcing);
 * cell nodes: the rigid-body velocity V + Omega x (s - X) of their cell as
 * the last bounce-back used it (Eq. 10); walls: 0.  Summed over a plane
 * normal to an axis it gives the volumetric flow rate through that plane
 * (Q of the vessel runs, Sec. IV), over part of a plane the flow rate of a
 * branch. */
int cgb_get_mixture_box(cgb_sim* s, const int32_t* lo, const int32_t* ext, double* u);

/* Read-out (synchronises first; returns the current state and CGB_OK even
 * after an instability, which cgb_sync reports).  Sizes: d 19*nsites; rho nsites; u nsites*3
 * (u = (sum n* c - g/2)/rho, zero on non-fluid nodes); X,V,L n*3; q n*4;
 * forces n*3 each (hydrodynamic incl. cover/uncover, and potential) of the
 * last step; owner nsites (-2 wall, -1 fluid, p >= 0 cell); link mask
 * nsites (bit r set: fluid node whose source x - c_r is not fluid). */
int cgb_get_populations(cgb_sim* s, double* d);
int cgb_get_fields(cgb_sim* s, double* rho, double* u);
int cgb_get_particles(cgb_sim* s, double* X, double* q, double* V, double* L);
int cgb_get_forces(cgb_sim* s, double* F_hyd, double* T_hyd, double* F_pot, double* T_pot);
int cgb_get_owner(cgb_sim* s, int32_t* owner);
int cgb_get_link_mask(cgb_sim* s, uint32_t* mask);
/* Pair set {i<j : |X_i - X_j|^2 < r_cut^2} (minimum image) at the current
 * positions, sorted.  ij holds up to cap pairs; *n receives the count. */
int cgb_get_pairs(cgb_sim* s, int32_t* ij, int64_t cap, int64_t* n);
/* out[0] fluid mass, out[1..3] sum over fluid of sum_r n*_r c_r,
 * out[4..6] cell momentum sum M V, out[7] fluid node count,
 * out[8..10] body force added to fluid + cells in the last step,
 * out[11] step counter, out[12] first unstable step or -1. */
int cgb_get_observables(cgb_sim* s, double* out /* 13 */);
/* mean over non-wall nodes of the z velocity of the mixture, per y plane
 * (fluid u_z, or the rigid velocity of the owning cell): prof[ny]. */
int cgb_get_profile_z(cgb_sim* s, double* prof);
/* the same along any axis (0: x, 1: y, 2: z): prof[n_axis] */
int cgb_get_profile(cgb_sim* s, int32_t axis, double* prof);

/* Kernel timing with HIP events on the handle's stream.  enable = 1 starts
 * recording, 0 stops.  cgb_kernel_times: for each of up to cap kernel names
 * (NUL-separated into names, 64 bytes each) total milliseconds and launches
 * since enabling; *n receives the number of entries. */
int cgb_profile(cgb_sim* s, int enable);
int cgb_kernel_times(cgb_sim* s, char* names, double* ms, int64_t* count, int32_t cap, int32_t* n);

/* Concurrency of the phases of a step (on by default for lattices with
 * cells): the cell list and the pair/wall potentials (Eqs. 15-20), which need
 * only the cells' positions and axes, run on a side stream of the handle
 * beside the lattice part (rasterisation, transitions, LB with the link
 * momenta of the cell nodes, per-cell momentum sums), joined before the
 * integrator; results are identical either way.  on = 0 runs every kernel on
 * the handle's stream in sequence (kernel timing of isolated launches).
 * Returns CGB_EINVAL for a null handle. */
int cgb_set_concurrency(cgb_sim* s, int on);

/* ---- Apparent viscosity (Sec. V defines it from the mean flow; for the
 * body-force driven flows here the mean flow is the mixture velocity).
 * cgb_track: after every following step, record on the device the sums over
 * the N non-wall nodes of the mixture z velocity u_z -- fluid nodes: the
 * velocity of the step's collision, (sum n* c_z - g_z/2)/rho; cell nodes: the
 * rigid-body velocity of their cell that the step's bounce-back used --
 * weighted by sin(2 pi y/ny) and by 1, for up to cap steps (cap = 0 stops).
 * Replaces any earlier record.
 * cgb_get_track: out[2k] = A_k = (2/N) sum u_z sin(2 pi y/ny) (the sine
 * amplitude of the plane-averaged profile), out[2k+1] = ubar_k = (1/N) sum
 * u_z, for k < min(cap, recorded); *n = steps recorded (at most the record's
 * capacity). */
int cgb_track(cgb_sim* s, int32_t cap);
int cgb_get_track(cgb_sim* s, double* out, int32_t cap, int32_t* n);
/* Estimators (host arithmetic on a recorded series).
 * Kolmogorov flow f0 sin(2 pi y/ny) e_z at tau = 1: one step maps a pure
 * shear mode exactly as A' = lam A + (1 + lam) f0/(2 rho0), lam = (2 + cos
 * k)/3, the decay (1 - cos k)/3 A being nu k^2 A at nu = 1/6, so
 *   mu_rel(t) = [f0 (5 + cos k)/(6 rho0) - (A_{t+1} - A_t)] / [A_t (1 - cos k)/3],
 * averaged over t = first .. n-2 (1 for the plasma).
 * Slit (walls y = 0, ny-1, constant g along z): the plasma's discrete steady
 * mean velocity is g (N_f^2 + 8 (tau - 1/2)^2 - 1)/(12 nu), N_f = ny - 2, nu =
 * (2 tau - 1)/6; mu_rel = that / mean(ubar[first .. n-1]).
 * cgb_mu_rel picks the estimator from the handle's driving (CGB_EINVAL for
 * any other, and for Kolmogorov driving at tau != 1, where the one-step map
 * above does not hold) and applies it to the handle's record. */
int cgb_mu_rel_kolmogorov(const double* A, int32_t n, int32_t first, double f0, double rho0, int32_t ny, double* mu);
int cgb_mu_rel_slit(const double* ubar, int32_t n, int32_t first, double g, double tau, int32_t ny, double* mu);
int cgb_mu_rel(cgb_sim* s, int32_t first, double* mu);
/* Plane-Couette viscometer (Sec. IV, Eq. 23): mu_app = Delta p_LE,z /
 * (l_y l_z gammadot).  cgb_track also records, with le_u != 0, Delta p_LE,z
 * of every step: the z momentum carried across the Lees-Edwards seam in -x,
 * the mean of its values in the frames of the two sides of the seam;
 * cgb_get_le_flux returns that record (out[k], k < min(cap, recorded);
 * *n = steps recorded up to the record's capacity).
 * cgb_mu_app_le: gammadot is the slope of the least-squares line through the
 * plane-averaged mixture velocity prof_x[nx] (cgb_get_profile, axis 0) over
 * the central half of the planes, x in [nx/4, 3 nx/4); Delta p_LE,z is the
 * mean of flux[first .. n-1]; *mu_rel = mu_app / (rho0 nu), nu =
 * (2 tau - 1)/6.  cgb_mu_rel uses it for a handle with le_u != 0, with the
 * handle's current profile. */
int cgb_get_le_flux(cgb_sim* s, double* out, int32_t cap, int32_t* n);
int cgb_mu_app_le(const double* flux, int32_t n, int32_t first, const double* prof_x, int32_t nx, int32_t ny,
                  int32_t nz, double rho0, double tau, double* mu_rel);

/* ---- Learned closure: ensemble of MLPs 3 -> 64 -> 64 -> 1 (SiLU) mapping
 * (hematocrit, log shear rate, width / R_perp) to the relative apparent
 * viscosity, trained and evaluated on the device.  A member has
 * CGB_MLP_PARAMS FP32 master parameters in the order W1[64][3], b1[64],
 * W2[64][64], b2[64], W3[64], b3; weights enter the arithmetic rounded to
 * bfloat16, the 64 x 64 layer and its backward products run on the matrix
 * cores with FP32 accumulation.  The network sees standardised inputs
 * (x - in_mean)/in_std and predicts the standardised (log mu - out_mean)/
 * out_std (cgb_mlp_set_norm; identity until set).  Host pointers unless
 * stated; every call is synchronous except cgb_mlp_predict_device. */
#define CGB_MLP_PARAMS 4481
#define CGB_MLP_BATCH 128   /* training batch of one step */
typedef struct cgb_mlp cgb_mlp;
/* members in [1, 6]; parameters start at zero (set them before use) */
int cgb_mlp_create(int32_t members, cgb_mlp** out);
void cgb_mlp_destroy(cgb_mlp* h);
const char* cgb_mlp_last_error(const cgb_mlp* h);
/* p: members * CGB_MLP_PARAMS; setting resets the optimiser state */
int cgb_mlp_set_params(cgb_mlp* h, const float* p);
int cgb_mlp_get_params(cgb_mlp* h, float* p);
int cgb_mlp_set_norm(cgb_mlp* h, const float* in_mean, const float* in_std, float out_mean, float out_std);
/* raw outputs for standardised inputs xn[n][3]: y[members][n] */
int cgb_mlp_forward(cgb_mlp* h, int64_t n, const float* xn, float* y);
/* gradient of the mean squared error over one batch: the samples
 * idx[members][CGB_MLP_BATCH] (member m uses its own row) of standardised
 * inputs xn[n][3] and targets tn[n]; grad[members][CGB_MLP_PARAMS],
 * loss[members] (nullable).  Parameters unchanged. */
int cgb_mlp_grad(cgb_mlp* h, int32_t n, const float* xn, const float* tn, const int32_t* idx, float* grad, float* loss);
/* `steps` Adam steps (beta 0.9, 0.999, eps 1e-8, rate lr) on physical samples
 * x[n][3], mu[n] > 0 (standardised on the device with the handle's norm);
 * step s of member m uses the samples idx[m][s][0 .. CGB_MLP_BATCH-1]
 * (the caller draws them); loss[members][steps] (nullable) receives each
 * step's batch loss. */
int cgb_mlp_train(cgb_mlp* h, int32_t n, const float* x, const float* mu, int32_t steps, const int32_t* idx, float lr,
                  float* loss);
/* cgb_mlp_train for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid it): the same
 * arguments (host pointers) and the same result bit for bit, but no device
 * memory is allocated or freed: the inputs, their standardised copies, the
 * indices and the losses are staged in a fixed device array of the library
 * (one per device, about 5 MB, held until the process ends).  Limits:
 * n <= 65536 samples and steps <= 1024 per call (CGB_EINVAL beyond).  Every
 * call on a device shares that device's array: calls that overlap on one
 * device race.  Synchronous. */
int cgb_mlp_train_noalloc(cgb_mlp* h, int32_t n, const float* x, const float* mu, int32_t steps,
                          const int32_t* idx, float lr, float* loss);
/* ensemble mean of mu and relative spread (sample standard deviation over
 * members / mean) for physical inputs x[n][3] */
int cgb_mlp_predict(cgb_mlp* h, int64_t n, const float* x, float* mean, float* spread);
/* the same on device buffers, asynchronous on `stream` (NULL: the handle's) */
int cgb_mlp_predict_device(cgb_mlp* h, int64_t n, const float* x, float* mean, float* spread, void* stream);

/* Checkpoint: stored populations (as stored), owner, cell state and the step
 * counter.  Resume is bit-identical to an uninterrupted run. */
int cgb_save(cgb_sim* s, const char* path);
int cgb_load(cgb_sim* s, const char* path);

/* Launch shape of the fused LB kernel: bx*by threads per block (a multiple
 * of 64, at most 256) covering a bx x by patch of an x-y plane, each thread
 * sweeping tz consecutive z nodes (tz in {4, 8, 16, 32}).  by = 0 (tau = 1
 * only): bx threads per block cover bx consecutive sites of the flattened
 * x-y plane (index x + nx*y), so every lane has a node whatever nx is; the
 * form for narrow lattices, whose rows a 2-D patch covers only in part.
 * The populations and forces do not depend on the shape; the mixture record
 * (cgb_track) depends on it through the summation order of its per-block
 * partials.  Errors: CGB_EINVAL for a shape outside these sets, by = 0 at
 * tau != 1, or tz != 16 in the large-lattice and indexed layouts.
 * cgb_get_tiles: t[3] = (bx, by, tz). */
int cgb_set_tiles(cgb_sim* s, int32_t bx, int32_t by, int32_t tz);
int cgb_get_tiles(cgb_sim* s, int32_t* t);
/* Average duration in milliseconds (HIP events on the handle's stream) of
 * the fused LB kernel over `reps` launches on the current state, after two
 * untimed launches.  The state, including the force read-out of the last
 * step, is unchanged.  Synchronous. */
int cgb_time_lb(cgb_sim* s, int32_t reps, double* ms_avg);

/* ---- Ensemble of independent channels (uneven sizes) advanced together.
 * Each channel is a full cgb_sim with its own stream and device memory,
 * created from ch[c] (host array of nch parameter sets, copied).  Set the
 * cells and the fluid of each channel through cgb_batch_channel() and the
 * single-lattice calls; do not destroy those handles (the batch owns them). */
typedef struct cgb_batch cgb_batch;
int cgb_batch_create(int32_t nch, const cgb_params* ch, cgb_batch** out);
void cgb_batch_destroy(cgb_batch* b);
const char* cgb_batch_last_error(const cgb_batch* b);
int cgb_batch_channel(cgb_batch* b, int32_t c, cgb_sim** sim);
/* Times the fused LB kernel over `reps` launches for a fixed set of tile
 * shapes on the first channel of each width class (nx < 48, < 80, >= 80) and
 * applies the fastest to the class.  The state is unchanged.  chosen:
 * nullable host array nch*3 receiving (bx, by, tz) per channel. */
int cgb_batch_autotune(cgb_batch* b, int32_t reps, int32_t* chosen);
/* Records `steps` (even, >= 2) time steps of every channel into one HIP graph
 * (fork/join over the channel streams).  Nothing is executed.  Every channel
 * must be initialised; cell sets and tiles must not change afterwards
 * without capturing again. */
int cgb_batch_capture(cgb_batch* b, int32_t steps);
/* Replays the graph nsteps / steps times on the batch's stream
 * (asynchronous; nsteps a multiple of the captured count).  The result is
 * identical to cgb_step(channel, nsteps) on each channel. */
int cgb_batch_run(cgb_batch* b, int32_t nsteps);
/* Waits for the replays and checks every channel (CGB_EUNSTABLE as cgb_sync). */
int cgb_batch_sync(cgb_batch* b);
/* cgb_track on every channel (drops a captured graph: capture afterwards so
 * that the replays record too). */
int cgb_batch_track(cgb_batch* b, int32_t cap);
/* mu[nch]: cgb_mu_rel of every channel. */
int cgb_batch_mu_rel(cgb_batch* b, int32_t first, double* mu);

#ifdef __cplusplus
}
#endif
#endif
