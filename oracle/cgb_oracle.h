/*
 * cgb_oracle.h -- plain FP64 CPU reference of the coupled lattice-Boltzmann /
 * rigid-ellipsoid time step of Janoschek, Toschi & Harting, "A simplified
 * particulate model for coarse-grained hemodynamics simulations"
 * (arXiv:1005.2594).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that tests, the smoke
 * check and the CPU-baseline leg of the benchmark can check the HIP path
 * against an obviously correct implementation.  It shares no source with
 * the HIP library and must never be called by the product path.
 *
 * Units are lattice units.  Site index = x + nx*(y + ny*z).
 * Populations are stored as deviations d_r = n*_r - w_r*rho0 (an exact change
 * of variables that keeps the FP64 arithmetic away from cancellation).
 */
#ifndef CGB_ORACLE_H
#define CGB_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_params {
    int32_t nx, ny, nz;
    double tau;          /* BGK relaxation time (Sec. II, Eq. 4)                 */
    double rho0;         /* initial/reference density rho-bar (Sec. II)          */
    int32_t wall_y;      /* 1: wall planes at y=0 and y=ny-1, y not periodic     */
    double wall_v_bot[3];/* velocity of the wall plane y=0   (Eq. 10 correction) */
    double wall_v_top[3];/* velocity of the wall plane y=ny-1                    */
    int32_t force_mode;  /* 0 none, 1 constant g, 2 f0*sin(2 pi y/ny) along z    */
    double g[3];
    double f0;
    int32_t force_on_particles; /* 1: body force also acts on cells, M*f(Y);
                                   2: rho0*V_cell*f(Y) (driven as the displaced
                                   plasma, whatever the inertial mass M)        */
    double R_perp, R_par;       /* half axes of the discretised ellipsoid (Sec. II) */
    double sig_perp, sig_par;   /* potential size parameters (Sec. III, Eq. 18)     */
    double sig_w;               /* wall sphere radius (Sec. III, 1/2)               */
    double eps, eps_w;          /* potential strengths eps-bar, eps-bar_w           */
    double r_cut;               /* pair cut-off (hard truncation of Eq. 15)         */
    double rho_p;               /* cell mass density                                */
    double le_u;                /* plane-Couette viscometer (Sec. IV): Lees-Edwards
                                   offset U of the z velocity across the periodic
                                   seam of x (the image beyond x = nx - 1 moves at
                                   +U e_z, shifted by U t); 0 = plain periodic x.
                                   Needs wall_y = 0.                               */
    int32_t force_zlo, force_zhi; /* force_mode 1 only: the constant body force acts
                                   on the nodes with force_zlo <= z < force_zhi (and
                                   on cells whose centre lies there), e.g. an
                                   entrance region (Sec. IV bifurcation runs);
                                   force_zhi <= force_zlo: everywhere             */
} orc_params;

typedef struct orc_sim orc_sim;

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_EUNSTABLE = -4, ORC_ESTATE = -5 };

int  orc_create(const orc_params* p, const uint8_t* wall_mask /* nullable, nsites */, orc_sim** out);
void orc_destroy(orc_sim* s);
const char* orc_last_error(const orc_sim* s);
int  orc_num_threads(void);
void orc_set_num_threads(int32_t n);  /* host threads of the OpenMP loops (n > 0) */

/* Particle state: X n*3, q n*4 (scalar first), V n*3 (t-1/2), L n*3 (space-frame
 * angular momentum at t-1/2), fixed n (1 = held at rest).  Rasterises the
 * cells (lowest index wins initial overlaps) without momentum bookkeeping:
 * newly covered fluid is dropped, freed nodes get rest fluid at rho0. */
int  orc_set_particles(orc_sim* s, int32_t n, const double* X, const double* q,
                       const double* V, const double* L, const uint8_t* fixed);
int  orc_init_fluid(orc_sim* s, const double* rho /*nullable*/, const double* u /*nullable, sites*3*/);
int  orc_set_deviations(orc_sim* s, const double* d /* 19*nsites */);
/* z momentum carried across the Lees-Edwards seam in -x during the last step
 * (Delta p_LE,z of Eq. 23); 0 when le_u = 0 */
double orc_le_flux(const orc_sim* s);
int  orc_step(orc_sim* s, int32_t nsteps);

int  orc_get_deviations(const orc_sim* s, double* d);
int  orc_get_fields(const orc_sim* s, double* rho, double* u);
int  orc_get_particles(const orc_sim* s, double* X, double* q, double* V, double* L);
int  orc_get_forces(const orc_sim* s, double* Fh, double* Th, double* Fp, double* Tp);
int  orc_get_owner(const orc_sim* s, int32_t* owner);
int  orc_get_link_mask(const orc_sim* s, uint32_t* mask);
int  orc_get_pairs(const orc_sim* s, int32_t* ij, int64_t cap, int64_t* n);
int  orc_get_link_static(const orc_sim* s, int64_t* A /* n*3 */, int64_t* B /* n*3 */);
/* out[0]=fluid mass, out[1..3]=sum over fluid of sum_r n*_r c_r,
 * out[4..6]=particle momentum sum M V, out[7]=number of fluid nodes,
 * out[8..10] = body force added to fluid+cells during the last step,
 * out[11]=step counter */
int  orc_get_observables(const orc_sim* s, double* out /* 12 */);
int  orc_mass_props(const orc_sim* s, double* out /* M, I_par, I_perp */);
/* sums over the non-wall nodes of the mixture z velocity after the last step
 * (fluid: velocity of the last collision; cell node: rigid-body velocity of
 * its cell as the last bounce-back used it): out[0] weighted by
 * sin(2 pi y/ny), out[1] unweighted, out[2] node count */
int  orc_mixture_sums(const orc_sim* s, double* out /* 3 */);
/* the same mixture velocity, all three components, at every site (0 at walls) */
int  orc_mixture_field(const orc_sim* s, double* u /* nsites*3 */);

/* Pure functions for pins */
void orc_d3q19(int32_t* c /* 19*3 */, double* w /* 19 */, int32_t* opp /* 19 */);
void orc_equilibrium(double rho, const double* u, double* neq /* 19 */);
void orc_bp_pair(const orc_params* p, const double* rvec, const double* oi, const double* oj,
                 double* U, double* Fi, double* ti, double* tj);
void orc_bp_wall(const orc_params* p, const double* rvec, const double* o,
                 double* U, double* Fi, double* ti);
void orc_axis(const double* q, double* o);
void orc_rotate(const double* q, const double* L, double Ipar, double Iperp, double dt, double* qout);
int  orc_inside(const orc_params* p, const double* X, const double* o, const double* node);

#ifdef __cplusplus
}
#endif
#endif
