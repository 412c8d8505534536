/*
 * cgb_oracle.c -- plain FP64 CPU reference of one time step of the coupled
 * lattice-Boltzmann plasma / rigid ellipsoidal cell model of Janoschek,
 * Toschi & Harting (arXiv:1005.2594).
 *
 * TEST INFRASTRUCTURE ONLY: used by tests, the smoke check and the benchmark's
 * CPU-baseline leg.  Shares no code with the HIP library.
 *
 * Every routine follows the paper's definitions in the order the paper gives
 * them; where the paper is silent the reading taken is named in the comment.
 * Built with -O2 -ffp-contract=off so that the geometric predicates (inside
 * test, pair distance) are evaluated exactly as written.
 *
 * Step order (the paper shares one time step between LB and MD, Sec. II):
 *   axis/omega -> rasterise -> cover/uncover -> momentum exchange + solid links
 *   -> stream/collide -> pair and wall potentials -> integrate.
 */
#include "cgb_oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* D3Q19 velocity set, Sec. II (19 discrete velocities, weights of Eq. 6):
 * rest, six axis directions, twelve face diagonals.  Opposite pairs are
 * adjacent: (1,2) (3,4) ... (17,18). */
static const int CV[19][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
/* 36 * weight: 1/3, 1/18, 1/36 (Eq. 6) */
static const int W36[19] = {12, 2, 2, 2, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1};
static double WR[19];
static int OPPR[19];
static void init_tables(void) {
    for (int r = 0; r < 19; r++) {
        WR[r] = (double)W36[r] / 36.0;
        OPPR[r] = (r == 0) ? 0 : ((r % 2) ? r + 1 : r - 1);
    }
}

#define NO_OWNER 0x7fffffff

struct orc_sim {
    orc_params P;
    int64_t ns;
    double* dA;          /* deviations of post-collision populations, [19][ns] */
    double* dB;
    int32_t* owner;      /* -2 wall, -1 fluid, p >= 0 particle */
    uint8_t* wall;
    int32_t* cover_min;  /* scratch for the occupancy rule */
    uint8_t* old_in;
    int32_t n;
    double *X, *q, *V, *L;
    uint8_t* fixed;
    double M, Ipar, Iperp;
    double *o, *Om;
    double *Xl, *Vl;     /* X(t) and V(t-1/2) of the last step: the kinematics its bounce-back used */
    double *Fh, *Th, *Fp, *Tp;
    int64_t *Aint, *Bint;
    int32_t* pairs;
    int64_t npairs, pcap;
    int32_t* sw;         /* surface wall nodes (site indices, ascending) */
    int64_t nsw;
    double body_last[3];
    double le_flux;      /* Delta p_LE,z of the last step (Sec. IV, Eq. 23) */
    int64_t step;
    char err[256];
};

static int fail(orc_sim* s, int code, const char* msg) {
    if (s) snprintf(s->err, sizeof s->err, "%s", msg);
    return code;
}

static inline int64_t sid(const orc_sim* s, int x, int y, int z) {
    return (int64_t)x + (int64_t)s->P.nx * ((int64_t)y + (int64_t)s->P.ny * z);
}
static inline int wrapi(int i, int n) { int m = i % n; return m < 0 ? m + n : m; }

/* minimum image of a displacement along a periodic axis of length Lb;
 * *k receives the number of box lengths added */
static inline double mimg(double d, double Lb, int* k) {
    *k = 0;
    if (d >= 0.5 * Lb) { d -= Lb; *k = -1; }
    else if (d < -0.5 * Lb) { d += Lb; *k = 1; }
    return d;
}
/* displacement node - X with the minimum image on periodic axes */
static void disp(const orc_sim* s, const double* node, const double* X, double* d, int* k) {
    const double Lb[3] = {s->P.nx, s->P.ny, s->P.nz};
    for (int a = 0; a < 3; a++) {
        double v = node[a] - X[a];
        if (a == 1 && s->P.wall_y) { d[a] = v; k[a] = 0; }
        else d[a] = mimg(v, Lb[a], &k[a]);
    }
}

/* ---- external force field (Sec. IV: body force on plasma and cells) ---- */
static void force_at(const orc_params* P, double y, double z, double* g) {
    g[0] = g[1] = g[2] = 0.0;
    /* a constant force may be confined to a slab of z (the entrance region
     * of the bifurcation runs, Sec. IV) */
    const int region = P->force_zhi > P->force_zlo;
    if (P->force_mode == 1 && (!region || (z >= P->force_zlo && z < P->force_zhi))) {
        g[0] = P->g[0]; g[1] = P->g[1]; g[2] = P->g[2];
    }
    else if (P->force_mode == 2) { g[2] = P->f0 * sin(2.0 * M_PI * y / (double)P->ny); }
}

/* ---- equilibrium, Eq. 5 with c_s^2 = 1/3, written as n^eq - w*rho0 ----
 * drho = rho - rho0 is passed separately: it is the deviation sum itself,
 * which forming rho - rho0 from the rounded rho would truncate to ulp(rho0) */
static void feq_dev2(double drho, double rho, const double* u, double* out) {
    double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int r = 0; r < 19; r++) {
        double cu = CV[r][0] * u[0] + CV[r][1] * u[1] + CV[r][2] * u[2];
        double poly = 3.0 * cu + 4.5 * cu * cu - 1.5 * usq + 4.5 * cu * cu * cu - 4.5 * usq * cu;
        out[r] = WR[r] * (drho + rho * poly);
    }
}
static void feq_dev(double rho0, double rho, const double* u, double* out) {
    feq_dev2(rho - rho0, rho, u, out);
}

void orc_equilibrium(double rho, const double* u, double* neq) {
    init_tables();
    double d[19];
    feq_dev(0.0, rho, u, d);
    for (int r = 0; r < 19; r++) neq[r] = d[r];
}

void orc_d3q19(int32_t* c, double* w, int32_t* opp) {
    init_tables();
    for (int r = 0; r < 19; r++) {
        for (int a = 0; a < 3; a++) c[3 * r + a] = CV[r][a];
        w[r] = WR[r];
        opp[r] = OPPR[r];
    }
}

/* BGK collision (Eqs. 1, 4) with the forcing term of Guo et al. (the paper
 * names no forcing scheme; this reading adds exactly g per node per step).
 * In: pulled deviations d (pre-collision), force density g.
 * Out: post-collision deviations. Returns |u|^2 for the stability check. */
static double collide(const orc_params* P, const double* d, const double* g, double* out) {
    double drho = 0.0, j[3] = {0, 0, 0};
    for (int r = 0; r < 19; r++) {
        drho += d[r];
        j[0] += d[r] * CV[r][0]; j[1] += d[r] * CV[r][1]; j[2] += d[r] * CV[r][2];
    }
    double rho = P->rho0 + drho;
    double u[3] = {(j[0] + 0.5 * g[0]) / rho, (j[1] + 0.5 * g[1]) / rho, (j[2] + 0.5 * g[2]) / rho};
    double eq[19];
    feq_dev2(drho, rho, u, eq);
    double pref = 1.0 - 0.5 / P->tau;
    for (int r = 0; r < 19; r++) {
        double cu = CV[r][0] * u[0] + CV[r][1] * u[1] + CV[r][2] * u[2];
        double cg = CV[r][0] * g[0] + CV[r][1] * g[1] + CV[r][2] * g[2];
        double cmug = (CV[r][0] - u[0]) * g[0] + (CV[r][1] - u[1]) * g[1] + (CV[r][2] - u[2]) * g[2];
        double Fr = pref * WR[r] * (3.0 * cmug + 9.0 * cu * cg);
        out[r] = d[r] - (d[r] - eq[r]) / P->tau + Fr;
    }
    return u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
}

/* ---- particle geometry ---- */
void orc_axis(const double* q, double* o) {
    /* symmetry axis o = R(q) e_z, q scalar first */
    o[0] = 2.0 * (q[1] * q[3] + q[0] * q[2]);
    o[1] = 2.0 * (q[2] * q[3] - q[0] * q[1]);
    o[2] = q[0] * q[0] - q[1] * q[1] - q[2] * q[2] + q[3] * q[3];
}

/* inside test of the discretised ellipsoid (Sec. II: half axes R_par along o,
 * R_perp across).  Node centres at integer coordinates; strict inequality. */
static int inside_d(const orc_sim* s, const double* d, const double* o) {
    double iRpar2 = 1.0 / (s->P.R_par * s->P.R_par);
    double iRperp2 = 1.0 / (s->P.R_perp * s->P.R_perp);
    double dp = d[0] * o[0] + d[1] * o[1] + d[2] * o[2];
    double dd = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double val = dp * dp * iRpar2 + (dd - dp * dp) * iRperp2;
    return val < 1.0;
}

int orc_inside(const orc_params* p, const double* X, const double* o, const double* node) {
    orc_sim tmp;
    memset(&tmp, 0, sizeof tmp);
    tmp.P = *p;
    double d[3]; int k[3];
    disp(&tmp, node, X, d, k);
    return inside_d(&tmp, d, o);
}

static void omega_of(const orc_sim* s, const double* o, const double* L, double* w) {
    /* space-frame angular velocity of a symmetric top: w = R I^-1 R^T L */
    double oL = o[0] * L[0] + o[1] * L[1] + o[2] * L[2];
    double k = 1.0 / s->Ipar - 1.0 / s->Iperp;
    for (int a = 0; a < 3; a++) w[a] = L[a] / s->Iperp + k * oL * o[a];
}

static inline void cross(const double* a, const double* b, double* c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* ---- lifecycle ---- */
static void* xcalloc(size_t n, size_t sz) { return calloc(n ? n : 1, sz); }

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
void orc_set_num_threads(int32_t n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

static void rebuild_surface_walls(orc_sim* s) {
    free(s->sw);
    int64_t cnt = 0;
    s->sw = (int32_t*)xcalloc((size_t)s->ns, sizeof(int32_t));
    for (int z = 0; z < s->P.nz; z++)
        for (int y = 0; y < s->P.ny; y++)
            for (int x = 0; x < s->P.nx; x++) {
                int64_t i = sid(s, x, y, z);
                if (!s->wall[i]) continue;
                int surf = 0;
                for (int r = 1; r < 19 && !surf; r++) {
                    int xn = wrapi(x + CV[r][0], s->P.nx), yn = y + CV[r][1], zn = wrapi(z + CV[r][2], s->P.nz);
                    if (s->P.wall_y) { if (yn < 0 || yn >= s->P.ny) continue; }
                    else yn = wrapi(yn, s->P.ny);
                    if (!s->wall[sid(s, xn, yn, zn)]) surf = 1;
                }
                if (surf) s->sw[cnt++] = (int32_t)i;
            }
    s->nsw = cnt;
}

int orc_create(const orc_params* p, const uint8_t* wall_mask, orc_sim** out) {
    init_tables();
    if (!p || !out) return ORC_EINVAL;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1 || p->tau <= 0.5 || p->rho0 <= 0) return ORC_EINVAL;
    if (p->le_u != 0.0 && (p->wall_y || p->nx < 2)) return ORC_EINVAL;
    if (p->wall_y && p->ny < 3) return ORC_EINVAL;
    orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
    if (!s) return ORC_ENOMEM;
    s->P = *p;
    s->ns = (int64_t)p->nx * p->ny * p->nz;
    s->dA = (double*)xcalloc((size_t)(19 * s->ns), sizeof(double));
    s->dB = (double*)xcalloc((size_t)(19 * s->ns), sizeof(double));
    s->owner = (int32_t*)xcalloc((size_t)s->ns, sizeof(int32_t));
    s->wall = (uint8_t*)xcalloc((size_t)s->ns, 1);
    s->cover_min = (int32_t*)xcalloc((size_t)s->ns, sizeof(int32_t));
    s->old_in = (uint8_t*)xcalloc((size_t)s->ns, 1);
    if (!s->dA || !s->dB || !s->owner || !s->wall || !s->cover_min || !s->old_in) { orc_destroy(s); return ORC_ENOMEM; }
    for (int64_t i = 0; i < s->ns; i++) {
        int y = (int)((i / p->nx) % p->ny);
        uint8_t w = wall_mask ? (wall_mask[i] != 0) : 0;
        if (p->wall_y && (y == 0 || y == p->ny - 1)) w = 1;
        s->wall[i] = w;
        s->owner[i] = w ? -2 : -1;
    }
    s->M = p->rho_p * (4.0 / 3.0) * M_PI * p->R_perp * p->R_perp * p->R_par;
    s->Ipar = 0.4 * s->M * p->R_perp * p->R_perp;
    s->Iperp = 0.2 * s->M * (p->R_perp * p->R_perp + p->R_par * p->R_par);
    rebuild_surface_walls(s);
    *out = s;
    return ORC_OK;
}

static void free_particles(orc_sim* s) {
    free(s->X); free(s->q); free(s->V); free(s->L); free(s->fixed);
    free(s->o); free(s->Om); free(s->Xl); free(s->Vl); free(s->Fh); free(s->Th); free(s->Fp); free(s->Tp);
    free(s->Aint); free(s->Bint); free(s->pairs);
    s->X = s->q = s->V = s->L = s->o = s->Om = s->Xl = s->Vl = s->Fh = s->Th = s->Fp = s->Tp = NULL;
    s->fixed = NULL; s->Aint = s->Bint = NULL; s->pairs = NULL;
    s->n = 0; s->npairs = 0; s->pcap = 0;
}

void orc_destroy(orc_sim* s) {
    if (!s) return;
    free(s->dA); free(s->dB); free(s->owner); free(s->wall); free(s->cover_min); free(s->old_in);
    free(s->sw);
    free_particles(s);
    free(s);
}

const char* orc_last_error(const orc_sim* s) { return s ? s->err : "null handle"; }

int orc_mass_props(const orc_sim* s, double* out) {
    out[0] = s->M; out[1] = s->Ipar; out[2] = s->Iperp;
    return ORC_OK;
}

/* bounding box of a cell: |x_a - X_a| < max(R_par, R_perp) for every inside node */
static void bbox(const orc_sim* s, const double* X, int* lo, int* hi) {
    double Rb = s->P.R_perp > s->P.R_par ? s->P.R_perp : s->P.R_par;
    for (int a = 0; a < 3; a++) { lo[a] = (int)floor(X[a] - Rb); hi[a] = (int)ceil(X[a] + Rb); }
}

/* Occupancy rule (Sec. II: one cell per node, the first cell to arrive keeps
 * it).  Reading: the current owner keeps a node while the node is still inside
 * it; a node claimed by several cells at once goes to the lowest index.
 * Fills cover_min / old_in; wall nodes are never covered. */
static void cover_scan(orc_sim* s) {
    for (int64_t i = 0; i < s->ns; i++) { s->cover_min[i] = NO_OWNER; s->old_in[i] = 0; }
    for (int p = 0; p < s->n; p++) {
        int lo[3], hi[3];
        bbox(s, &s->X[3 * p], lo, hi);
        for (int z = lo[2]; z <= hi[2]; z++)
            for (int y = lo[1]; y <= hi[1]; y++) {
                if (s->P.wall_y && (y < 0 || y >= s->P.ny)) continue;
                for (int x = lo[0]; x <= hi[0]; x++) {
                    double node[3] = {x, y, z}, d[3];
                    int k[3];
                    int xw = wrapi(x, s->P.nx), yw = wrapi(y, s->P.ny), zw = wrapi(z, s->P.nz);
                    double nodew[3] = {xw, yw, zw};
                    (void)node;
                    disp(s, nodew, &s->X[3 * p], d, k);
                    int64_t i = sid(s, xw, yw, zw);
                    if (s->wall[i]) continue;
                    if (inside_d(s, d, &s->o[3 * p])) {
                        if (p < s->cover_min[i]) s->cover_min[i] = p;
                        if (s->owner[i] == p) s->old_in[i] = 1;
                    }
                }
            }
    }
}

static void compute_axes(orc_sim* s) {
    for (int p = 0; p < s->n; p++) {
        orc_axis(&s->q[4 * p], &s->o[3 * p]);
        omega_of(s, &s->o[3 * p], &s->L[3 * p], &s->Om[3 * p]);
    }
}

int orc_set_particles(orc_sim* s, int32_t n, const double* X, const double* q,
                      const double* V, const double* L, const uint8_t* fixed) {
    if (!s || n < 0 || (n > 0 && (!X || !q))) return fail(s, ORC_EINVAL, "bad particle arguments");
    free_particles(s);
    s->n = n;
    s->X = (double*)xcalloc((size_t)3 * n, sizeof(double));
    s->q = (double*)xcalloc((size_t)4 * n, sizeof(double));
    s->V = (double*)xcalloc((size_t)3 * n, sizeof(double));
    s->L = (double*)xcalloc((size_t)3 * n, sizeof(double));
    s->fixed = (uint8_t*)xcalloc((size_t)n, 1);
    s->o = (double*)xcalloc((size_t)3 * n, sizeof(double));
    s->Om = (double*)xcalloc((size_t)3 * n, sizeof(double));
    s->Xl = (double*)xcalloc((size_t)3 * n, sizeof(double));
    s->Vl = (double*)xcalloc((size_t)3 * n, sizeof(double));
    s->Fh = (double*)xcalloc((size_t)3 * n, sizeof(double));
    s->Th = (double*)xcalloc((size_t)3 * n, sizeof(double));
    s->Fp = (double*)xcalloc((size_t)3 * n, sizeof(double));
    s->Tp = (double*)xcalloc((size_t)3 * n, sizeof(double));
    s->Aint = (int64_t*)xcalloc((size_t)3 * n, sizeof(int64_t));
    s->Bint = (int64_t*)xcalloc((size_t)3 * n, sizeof(int64_t));
    if (n > 0) {
        memcpy(s->X, X, sizeof(double) * 3 * n);
        memcpy(s->q, q, sizeof(double) * 4 * n);
        if (V) memcpy(s->V, V, sizeof(double) * 3 * n);
        if (L) memcpy(s->L, L, sizeof(double) * 3 * n);
        if (fixed) memcpy(s->fixed, fixed, (size_t)n);
    }
    compute_axes(s);
    memcpy(s->Xl, s->X, sizeof(double) * 3 * n);
    memcpy(s->Vl, s->V, sizeof(double) * 3 * n);
    /* fresh occupancy: lowest covering index; nodes freed by this call get
     * rest fluid at rho0 */
    cover_scan(s);
    for (int64_t i = 0; i < s->ns; i++) {
        if (s->wall[i]) continue;
        int32_t nw = (s->cover_min[i] != NO_OWNER) ? s->cover_min[i] : -1;
        if (s->owner[i] >= 0 && nw == -1)
            for (int r = 0; r < 19; r++) s->dA[r * s->ns + i] = 0.0;
        s->owner[i] = nw;
    }
    return ORC_OK;
}

int orc_init_fluid(orc_sim* s, const double* rho, const double* u) {
    if (!s) return ORC_EINVAL;
    for (int64_t i = 0; i < s->ns; i++) {
        double eq[19];
        double rr = rho ? rho[i] : s->P.rho0;
        double uu[3] = {0, 0, 0};
        if (u) { uu[0] = u[3 * i]; uu[1] = u[3 * i + 1]; uu[2] = u[3 * i + 2]; }
        feq_dev(s->P.rho0, rr, uu, eq);
        for (int r = 0; r < 19; r++) {
            s->dA[r * s->ns + i] = s->wall[i] ? 0.0 : eq[r];
            s->dB[r * s->ns + i] = 0.0;
        }
    }
    return ORC_OK;
}

int orc_set_deviations(orc_sim* s, const double* d) {
    if (!s || !d) return ORC_EINVAL;
    memcpy(s->dA, d, sizeof(double) * 19 * s->ns);
    return ORC_OK;
}

/* velocity of a moving wall node (only the two wall planes may move) */
static const double* wall_velocity(const orc_sim* s, int y) {
    static const double zero[3] = {0, 0, 0};
    if (!s->P.wall_y) return zero;
    if (y == 0) return s->P.wall_v_bot;
    if (y == s->P.ny - 1) return s->P.wall_v_top;
    return zero;
}

/* ---- plane-Couette viscometer (Sec. IV): Lees-Edwards seam in x ----
 * Reading: the image of the box beyond x = nx - 1 moves at +U e_z and is
 * shifted by Delta = U t along z (t: steps completed before this one); the
 * image below x = 0 moves at -U e_z, shifted by -Delta.  A population pulled
 * across the seam -- into x = 0 along c_x = +1, or into x = nx - 1 along
 * c_x = -1 -- comes from the image: its source is the node (nx - 1 or 0,
 * y - c_y) at z - c_z + Delta (resp. - Delta), linearly interpolated between
 * the two nodes that bracket that z, and it is carried into this box's frame
 * by the Galilean shift n^eq(rho_s, u_s -/+ U e_z) - n^eq(rho_s, u_s), with
 * rho_s, u_s the moments of the interpolated source populations.  Returns
 * the deviation to pull; *orig receives the population before the shift. */
static double le_pull(const orc_sim* s, const double* A, int r, int x, int y, int z, double* orig) {
    const orc_params* P = &s->P;
    const int nx = P->nx, ny = P->ny, nz = P->nz;
    const double delta = fmod(P->le_u * (double)s->step, (double)nz);
    const int from_below = (x == 0 && CV[r][0] == 1);
    const int xs = from_below ? nx - 1 : 0;
    const int ys = wrapi(y - CV[r][1], ny);
    double zf = (double)(z - CV[r][2]) + (from_below ? delta : -delta);
    zf = fmod(zf, (double)nz);
    if (zf < 0.0) zf += nz;
    const double zl = floor(zf);
    const double w = zf - zl;
    const int64_t i0 = sid(s, xs, ys, wrapi((int)zl, nz)), i1 = sid(s, xs, ys, wrapi((int)zl + 1, nz));
    double n[19], drho = 0.0, j[3] = {0, 0, 0};
    for (int q = 0; q < 19; q++) {
        n[q] = (1.0 - w) * A[q * s->ns + i0] + w * A[q * s->ns + i1];
        drho += n[q];
        for (int a = 0; a < 3; a++) j[a] += n[q] * CV[q][a];
    }
    const double rho = P->rho0 + drho;
    double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
    double e0[19], e1[19];
    feq_dev(P->rho0, rho, u, e0);
    u[2] += from_below ? -P->le_u : P->le_u;
    feq_dev(P->rho0, rho, u, e1);
    *orig = n[r];
    return n[r] + (e1[r] - e0[r]);
}

/* Correction term of Eq. 10 for the population arriving at fluid node x along
 * c_r from solid node x - c_r: C = 6 w_r rho(x) (c_r . v_b).  For a cell the
 * boundary velocity is taken at the link midpoint x - c_r/2 (reading: rigid
 * body velocity V + Omega x (x_b - X) at the latest half step). */
static double corr_term(const orc_sim* s, int r, int64_t xi, int x, int y, int z, int32_t o, double rho_x) {
    double vb[3];
    if (o >= 0) {
        double b[3] = {x - 0.5 * CV[r][0], y - 0.5 * CV[r][1], z - 0.5 * CV[r][2]};
        double d[3]; int k[3];
        disp(s, b, &s->X[3 * o], d, k);
        double wx[3];
        cross(&s->Om[3 * o], d, wx);
        for (int a = 0; a < 3; a++) vb[a] = s->V[3 * o + a] + wx[a];
    } else {
        int ys = y - CV[r][1];
        const double* vw = wall_velocity(s, ys);
        vb[0] = vw[0]; vb[1] = vw[1]; vb[2] = vw[2];
    }
    (void)xi;
    double cv = CV[r][0] * vb[0] + CV[r][1] * vb[1] + CV[r][2] * vb[2];
    return 6.0 * WR[r] * rho_x * cv;
}

static double rho_at(const orc_sim* s, const double* D, int64_t i) {
    double drho = 0.0;
    for (int r = 0; r < 19; r++) drho += D[r * s->ns + i];
    return s->P.rho0 + drho;
}

/* ---- cell list + pair set (cell edge >= cut-off, minimum image) ---- */
static int cmp_pair(const void* a, const void* b) {
    const int32_t* x = (const int32_t*)a; const int32_t* y = (const int32_t*)b;
    if (x[0] != y[0]) return x[0] < y[0] ? -1 : 1;
    if (x[1] != y[1]) return x[1] < y[1] ? -1 : 1;
    return 0;
}
static int cmp_int(const void* a, const void* b) {
    int x = *(const int*)a, y = *(const int*)b;
    return (x > y) - (x < y);
}

static void build_pairs(orc_sim* s) {
    const double Lb[3] = {s->P.nx, s->P.ny, s->P.nz};
    int nb[3]; double edge[3];
    for (int a = 0; a < 3; a++) {
        nb[a] = (int)floor(Lb[a] / s->P.r_cut);
        if (nb[a] < 1) nb[a] = 1;
        edge[a] = Lb[a] / nb[a];
    }
    int64_t nbin = (int64_t)nb[0] * nb[1] * nb[2];
    int* head = (int*)malloc(sizeof(int) * (size_t)nbin);
    int* next = (int*)malloc(sizeof(int) * (size_t)(s->n ? s->n : 1));
    int* pb = (int*)malloc(sizeof(int) * 3 * (size_t)(s->n ? s->n : 1));
    for (int64_t b = 0; b < nbin; b++) head[b] = -1;
    for (int p = s->n - 1; p >= 0; p--) {
        int c[3];
        for (int a = 0; a < 3; a++) {
            int ci = (int)floor(s->X[3 * p + a] / edge[a]);
            if (ci < 0) ci = 0;
            if (ci >= nb[a]) ci = nb[a] - 1;
            c[a] = ci; pb[3 * p + a] = ci;
        }
        int64_t b = c[0] + (int64_t)nb[0] * (c[1] + (int64_t)nb[1] * c[2]);
        next[p] = head[b]; head[b] = p;
    }
    s->npairs = 0;
    double rc2 = s->P.r_cut * s->P.r_cut;
    for (int i = 0; i < s->n; i++) {
        int bins[27], nbn = 0;
        for (int dz = -1; dz <= 1; dz++)
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    int c[3] = {pb[3 * i] + dx, pb[3 * i + 1] + dy, pb[3 * i + 2] + dz};
                    int ok = 1;
                    for (int a = 0; a < 3; a++) {
                        if (a == 1 && s->P.wall_y) { if (c[a] < 0 || c[a] >= nb[a]) ok = 0; }
                        else c[a] = wrapi(c[a], nb[a]);
                    }
                    if (!ok) continue;
                    int b = c[0] + nb[0] * (c[1] + nb[1] * c[2]);
                    int dup = 0;
                    for (int t = 0; t < nbn; t++) if (bins[t] == b) dup = 1;
                    if (!dup) bins[nbn++] = b;
                }
        qsort(bins, (size_t)nbn, sizeof(int), cmp_int);
        for (int t = 0; t < nbn; t++)
            for (int j = head[bins[t]]; j >= 0; j = next[j]) {
                if (j <= i) continue;
                double dd[3]; int k[3];
                disp(s, &s->X[3 * i], &s->X[3 * j], dd, k);
                double r2 = dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2];
                if (r2 < rc2) {
                    if (s->npairs >= s->pcap) {
                        s->pcap = s->pcap ? 2 * s->pcap : 1024;
                        s->pairs = (int32_t*)realloc(s->pairs, sizeof(int32_t) * 2 * (size_t)s->pcap);
                    }
                    s->pairs[2 * s->npairs] = i;
                    s->pairs[2 * s->npairs + 1] = j;
                    s->npairs++;
                }
            }
    }
    if (s->npairs > 1) qsort(s->pairs, (size_t)s->npairs, 2 * sizeof(int32_t), cmp_pair);
    free(head); free(next); free(pb);
}

/* ---- Berne-Pechukas pair potential, Eqs. 15-18 ----
 * U = eps (1 - r/sigma)^2 for r < sigma with eps from Eq. 16, sigma from Eq. 17,
 * sigma-bar = 2 sigma_perp and chi from Eq. 18.  rvec = X_i - X_j.
 * Forces are -grad_{X_i} U, torques -o x dU/do. */
void orc_bp_pair(const orc_params* P, const double* rvec, const double* oi, const double* oj,
                 double* U, double* Fi, double* ti, double* tj) {
    *U = 0.0;
    for (int a = 0; a < 3; a++) Fi[a] = ti[a] = tj[a] = 0.0;
    double r2 = rvec[0] * rvec[0] + rvec[1] * rvec[1] + rvec[2] * rvec[2];
    if (r2 == 0.0) return;
    double r = sqrt(r2);
    double rh[3] = {rvec[0] / r, rvec[1] / r, rvec[2] / r};
    double sp2 = P->sig_perp * P->sig_perp, sl2 = P->sig_par * P->sig_par;
    double chi = (sl2 - sp2) / (sl2 + sp2);
    double sbar = 2.0 * P->sig_perp;
    double a = rh[0] * oi[0] + rh[1] * oi[1] + rh[2] * oi[2];
    double b = rh[0] * oj[0] + rh[1] * oj[1] + rh[2] * oj[2];
    double g = oi[0] * oj[0] + oi[1] * oj[1] + oi[2] * oj[2];
    double Pp = 1.0 + chi * g, Qq = 1.0 - chi * g;
    double S = (a + b) * (a + b) / Pp + (a - b) * (a - b) / Qq;
    double sigma = sbar / sqrt(1.0 - 0.5 * chi * S);
    if (r >= sigma) return;
    double e1 = 1.0 - chi * chi * g * g;
    double eps = P->eps / sqrt(e1);
    double sr = 1.0 - r / sigma;
    *U = eps * sr * sr;
    double dUdr = -2.0 * eps * sr / sigma;                     /* at fixed sigma */
    double dUdsig = 2.0 * eps * sr * r / (sigma * sigma);
    double dsigdS = 0.25 * chi * sigma * sigma * sigma / (sbar * sbar);
    double K = dUdsig * dsigdS;
    double Sa = 2.0 * (a + b) / Pp + 2.0 * (a - b) / Qq;
    double Sb = 2.0 * (a + b) / Pp - 2.0 * (a - b) / Qq;
    double Sg = -chi * (a + b) * (a + b) / (Pp * Pp) + chi * (a - b) * (a - b) / (Qq * Qq);
    double epsg = P->eps * chi * chi * g / (e1 * sqrt(e1));   /* d eps / d g */
    for (int c = 0; c < 3; c++)
        Fi[c] = -(dUdr * rh[c] + K * (Sa * (oi[c] - a * rh[c]) + Sb * (oj[c] - b * rh[c])) / r);
    double gi[3], gj[3];
    for (int c = 0; c < 3; c++) {
        gi[c] = K * (Sa * rh[c] + Sg * oj[c]) + sr * sr * epsg * oj[c];
        gj[c] = K * (Sb * rh[c] + Sg * oi[c]) + sr * sr * epsg * oi[c];
    }
    cross(oi, gi, ti); cross(oj, gj, tj);
    for (int c = 0; c < 3; c++) { ti[c] = -ti[c]; tj[c] = -tj[c]; }
}

/* Cell-wall potential, Eqs. 19-20: a sphere of radius sigma_w on each surface
 * wall node, fixed strength eps_w.  rvec = X_i - x_wall. */
void orc_bp_wall(const orc_params* P, const double* rvec, const double* o,
                 double* U, double* Fi, double* ti) {
    *U = 0.0;
    for (int a = 0; a < 3; a++) Fi[a] = ti[a] = 0.0;
    double r2 = rvec[0] * rvec[0] + rvec[1] * rvec[1] + rvec[2] * rvec[2];
    if (r2 == 0.0) return;
    double r = sqrt(r2);
    double rh[3] = {rvec[0] / r, rvec[1] / r, rvec[2] / r};
    double sp2 = P->sig_perp * P->sig_perp, sl2 = P->sig_par * P->sig_par, sw2 = P->sig_w * P->sig_w;
    double sbw = sqrt(sp2 + sw2);
    double chiw = (sl2 - sp2) / (sl2 + sw2);
    double a = rh[0] * o[0] + rh[1] * o[1] + rh[2] * o[2];
    double den = 1.0 - chiw * a * a;
    if (den <= 0.0) return;
    double sigma = sbw / sqrt(den);
    if (r >= sigma) return;
    double sr = 1.0 - r / sigma;
    *U = P->eps_w * sr * sr;
    double dUdr = -2.0 * P->eps_w * sr / sigma;
    double dUdsig = 2.0 * P->eps_w * sr * r / (sigma * sigma);
    double dsigda = chiw * a * sigma * sigma * sigma / (sbw * sbw);
    double K = dUdsig * dsigda;
    for (int c = 0; c < 3; c++) Fi[c] = -(dUdr * rh[c] + K * (o[c] - a * rh[c]) / r);
    double kr[3] = {K * rh[0], K * rh[1], K * rh[2]};
    cross(o, kr, ti);
    for (int c = 0; c < 3; c++) ti[c] = -ti[c];
}

/* largest distance at which the wall potential can act */
static double wall_range(const orc_params* P) {
    double sp2 = P->sig_perp * P->sig_perp, sl2 = P->sig_par * P->sig_par, sw2 = P->sig_w * P->sig_w;
    double chiw = (sl2 - sp2) / (sl2 + sw2);
    double sbw = sqrt(sp2 + sw2);
    if (chiw <= 0.0) return sbw;
    if (chiw >= 1.0) return 1e300;
    return sbw / sqrt(1.0 - chiw);
}

/* ---- rigid body rotation (leap-frog on unit quaternions, Sec. II) ----
 * Reading: explicit midpoint.  Predict q~ by a half-step rotation with the
 * angular velocity from q(t) and L(t+1/2), then rotate q(t) by a full step
 * with the angular velocity evaluated at q~. */
static void qmul(const double* a, const double* b, double* c) {
    c[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    c[1] = a[0] * b[1] + b[0] * a[1] + a[2] * b[3] - a[3] * b[2];
    c[2] = a[0] * b[2] + b[0] * a[2] + a[3] * b[1] - a[1] * b[3];
    c[3] = a[0] * b[3] + b[0] * a[3] + a[1] * b[2] - a[2] * b[1];
}
static void qrot(const double* w, double h, double* dq) {
    double wn = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    if (wn == 0.0) { dq[0] = 1; dq[1] = dq[2] = dq[3] = 0; return; }
    double ang = 0.5 * wn * h;
    double sn = sin(ang) / wn;
    dq[0] = cos(ang); dq[1] = sn * w[0]; dq[2] = sn * w[1]; dq[3] = sn * w[2];
}
static void qnorm(double* q) {
    double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int a = 0; a < 4; a++) q[a] /= n;
}
static void omega_top(double Ipar, double Iperp, const double* o, const double* L, double* w) {
    double oL = o[0] * L[0] + o[1] * L[1] + o[2] * L[2];
    double k = 1.0 / Ipar - 1.0 / Iperp;
    for (int a = 0; a < 3; a++) w[a] = L[a] / Iperp + k * oL * o[a];
}
void orc_rotate(const double* q, const double* L, double Ipar, double Iperp, double dt, double* qout) {
    double o[3], w[3], dq[4], qh[4];
    orc_axis(q, o);
    omega_top(Ipar, Iperp, o, L, w);
    qrot(w, 0.5 * dt, dq);
    qmul(dq, q, qh);
    qnorm(qh);
    orc_axis(qh, o);
    omega_top(Ipar, Iperp, o, L, w);
    qrot(w, dt, dq);
    qmul(dq, q, qout);
    qnorm(qout);
}

/* ---- one time step ---- */
static int one_step(orc_sim* s) {
    const orc_params* P = &s->P;
    const int nx = P->nx, ny = P->ny, nz = P->nz;
    const int64_t ns = s->ns;
    double* A = s->dA;
    double* B = s->dB;
    const double c36 = 2.0 * P->rho0 / 36.0;

    /* 1. axes at X(t), q(t); angular velocity at t-1/2 */
    compute_axes(s);
    memcpy(s->Xl, s->X, sizeof(double) * 3 * s->n);
    memcpy(s->Vl, s->V, sizeof(double) * 3 * s->n);
    for (int a = 0; a < 3 * s->n; a++) { s->Fh[a] = s->Th[a] = s->Fp[a] = s->Tp[a] = 0.0; s->Aint[a] = s->Bint[a] = 0; }

    /* 2. rasterise and apply the occupancy rule */
    cover_scan(s);
    if (P->le_u != 0.0)
        for (int z = 0; z < nz; z++)
            for (int y = 0; y < ny; y++)
                if (s->cover_min[sid(s, 0, y, z)] != NO_OWNER || s->cover_min[sid(s, nx - 1, y, z)] != NO_OWNER)
                    return fail(s, ORC_EUNSTABLE, "a cell covers a node of a sheared plane");

    /* 3. cover / uncover in site order (Sec. II: deleted or created fluid
     *    momentum is balanced by a force on the cell; torque likewise) */
    for (int64_t i = 0; i < ns; i++) {
        if (s->wall[i]) continue;
        int32_t old = s->owner[i];
        int32_t nw = (old >= 0 && s->old_in[i]) ? old : (s->cover_min[i] != NO_OWNER ? s->cover_min[i] : -1);
        if (nw == old) continue;
        int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((int64_t)nx * ny));
        double node[3] = {x, y, z};
        if (old == -1 && nw >= 0) {
            double m[3] = {0, 0, 0};
            for (int r = 0; r < 19; r++)
                for (int a = 0; a < 3; a++) m[a] += A[r * ns + i] * CV[r][a];
            double d[3], t[3]; int k[3];
            disp(s, node, &s->X[3 * nw], d, k);
            cross(d, m, t);
            for (int a = 0; a < 3; a++) { s->Fh[3 * nw + a] += m[a]; s->Th[3 * nw + a] += t[a]; }
        } else if (old >= 0 && nw == -1) {
            double d[3], t[3], us[3], eq[19]; int k[3];
            disp(s, node, &s->X[3 * old], d, k);
            cross(&s->Om[3 * old], d, us);
            for (int a = 0; a < 3; a++) us[a] += s->V[3 * old + a];
            feq_dev(P->rho0, P->rho0, us, eq);
            double m[3] = {0, 0, 0};
            for (int r = 0; r < 19; r++) {
                A[r * ns + i] = eq[r];
                for (int a = 0; a < 3; a++) m[a] += eq[r] * CV[r][a];
            }
            cross(d, m, t);
            for (int a = 0; a < 3; a++) { s->Fh[3 * old + a] -= m[a]; s->Th[3 * old + a] -= t[a]; }
        }
        s->owner[i] = nw;
    }

    /* 4a. momentum exchange, Eq. 12: every population bounced at a cell
     *     transfers (2 n*_rbar + C) c_rbar.  With n* = w rho0 + d the constant
     *     part 2 w rho0 c_rbar is accumulated exactly in units of 2 rho0 / 36. */
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                int64_t i = sid(s, x, y, z);
                if (s->owner[i] != -1) continue;
                double rho_x = 0.0;
                int have = 0;
                for (int r = 1; r < 19; r++) {
                    int xs = wrapi(x - CV[r][0], nx), ys = wrapi(y - CV[r][1], ny), zs = wrapi(z - CV[r][2], nz);
                    int32_t o = s->owner[sid(s, xs, ys, zs)];
                    if (o < 0) continue;
                    if (!have) { rho_x = rho_at(s, A, i); have = 1; }
                    int rb = OPPR[r];
                    double C = corr_term(s, r, i, x, y, z, o, rho_x);
                    double dyn = 2.0 * A[rb * ns + i] + C;
                    double f[3] = {dyn * CV[rb][0], dyn * CV[rb][1], dyn * CV[rb][2]};
                    double node[3] = {x, y, z}, d[3], t[3]; int k[3];
                    disp(s, node, &s->X[3 * o], d, k);
                    cross(d, f, t);
                    for (int a = 0; a < 3; a++) { s->Fh[3 * o + a] += f[a]; s->Th[3 * o + a] += t[a]; }
                    int xu[3] = {x + k[0] * nx, y + k[1] * ny, z + k[2] * nz};
                    int64_t cs[3] = {W36[rb] * CV[rb][0], W36[rb] * CV[rb][1], W36[rb] * CV[rb][2]};
                    for (int a = 0; a < 3; a++) s->Aint[3 * o + a] += cs[a];
                    s->Bint[3 * o + 0] += (int64_t)xu[1] * cs[2] - (int64_t)xu[2] * cs[1];
                    s->Bint[3 * o + 1] += (int64_t)xu[2] * cs[0] - (int64_t)xu[0] * cs[2];
                    s->Bint[3 * o + 2] += (int64_t)xu[0] * cs[1] - (int64_t)xu[1] * cs[0];
                }
            }

    /* 4b. solid links, Eqs. 13-14: at each link from a cell node s to a node of
     *     another cell or a wall, the cell receives 2 n^eq(rho0, 0) c pointing
     *     from the foreign node into its own node.  Forces on walls are dropped. */
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                int64_t i = sid(s, x, y, z);
                int32_t p = s->owner[i];
                if (p < 0) continue;
                double node[3] = {x, y, z}, d[3]; int k[3];
                disp(s, node, &s->X[3 * p], d, k);
                int su[3] = {x + k[0] * nx, y + k[1] * ny, z + k[2] * nz};
                for (int r = 1; r < 19; r++) {
                    int xn = wrapi(x + CV[r][0], nx), yn = wrapi(y + CV[r][1], ny), zn = wrapi(z + CV[r][2], nz);
                    int32_t o = s->owner[sid(s, xn, yn, zn)];
                    if (!(o == -2 || (o >= 0 && o != p))) continue;
                    int rb = OPPR[r];
                    int64_t cs[3] = {W36[rb] * CV[rb][0], W36[rb] * CV[rb][1], W36[rb] * CV[rb][2]};
                    for (int a = 0; a < 3; a++) s->Aint[3 * p + a] += cs[a];
                    s->Bint[3 * p + 0] += (int64_t)su[1] * cs[2] - (int64_t)su[2] * cs[1];
                    s->Bint[3 * p + 1] += (int64_t)su[2] * cs[0] - (int64_t)su[0] * cs[2];
                    s->Bint[3 * p + 2] += (int64_t)su[0] * cs[1] - (int64_t)su[1] * cs[0];
                }
            }
    for (int p = 0; p < s->n; p++) {
        for (int a = 0; a < 3; a++) s->Fh[3 * p + a] += c36 * (double)s->Aint[3 * p + a];
        /* torque of the constant part about X_p: c36 * (B - X_p x A) */
        double XA[3], Ad[3] = {(double)s->Aint[3 * p], (double)s->Aint[3 * p + 1], (double)s->Aint[3 * p + 2]};
        cross(&s->X[3 * p], Ad, XA);
        for (int a = 0; a < 3; a++) s->Th[3 * p + a] += c36 * ((double)s->Bint[3 * p + a] - XA[a]);
    }

    /* 5. stream (pull) + bounce-back (Eqs. 2, 9, 11) + collide; with the
     *    viscometer's seam, pulls across it come from the sheared image, and
     *    the z momentum they carry across the seam is recorded */
    int unstable = 0;
    double bodyf[3] = {0, 0, 0};
    double le_flux = 0.0;
#pragma omp parallel for reduction(| : unstable) reduction(+ : bodyf[:3], le_flux) schedule(static)
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                int64_t i = sid(s, x, y, z);
                if (s->owner[i] != -1) {
                    for (int r = 0; r < 19; r++) B[r * ns + i] = 0.0;
                    continue;
                }
                double d[19], out[19], g[3];
                double rho_x = -1.0;
                for (int r = 0; r < 19; r++) {
                    if (P->le_u != 0.0 && ((x == 0 && CV[r][0] == 1) || (x == nx - 1 && CV[r][0] == -1))) {
                        /* Delta p_LE,z: the z momentum crossing in -x, the
                         * mean of its values in the frames of the two sides
                         * (before and after the Galilean shift) */
                        double orig;
                        d[r] = le_pull(s, A, r, x, y, z, &orig);
                        le_flux += -0.5 * CV[r][0] * CV[r][2] * (orig + d[r]);
                        continue;
                    }
                    int xs = wrapi(x - CV[r][0], nx), ys = wrapi(y - CV[r][1], ny), zs = wrapi(z - CV[r][2], nz);
                    int64_t j = sid(s, xs, ys, zs);
                    int32_t o = s->owner[j];
                    if (o == -1) { d[r] = A[r * ns + j]; continue; }
                    int rb = OPPR[r];
                    double C = 0.0;
                    const double* vw = wall_velocity(s, ys);
                    if (o >= 0 || vw[0] != 0.0 || vw[1] != 0.0 || vw[2] != 0.0) {
                        if (rho_x < 0.0) rho_x = rho_at(s, A, i);
                        C = corr_term(s, r, i, x, y, z, o, rho_x);
                    }
                    d[r] = A[rb * ns + i] + C;
                }
                force_at(P, (double)y, (double)z, g);
                double usq = collide(P, d, g, out);
                if (!(usq <= 0.16)) unstable = 1;
                for (int a = 0; a < 3; a++) bodyf[a] += g[a];
                for (int r = 0; r < 19; r++) B[r * ns + i] = out[r];
            }
    s->dA = B; s->dB = A;
    s->le_flux = le_flux;
    if (unstable) return fail(s, ORC_EUNSTABLE, "fluid velocity non-finite or |u| > 0.4");

    /* 6. pair and wall potentials (Sec. III) */
    build_pairs(s);
    for (int64_t t = 0; t < s->npairs; t++) {
        int i = s->pairs[2 * t], j = s->pairs[2 * t + 1];
        double rv[3]; int k[3];
        disp(s, &s->X[3 * i], &s->X[3 * j], rv, k);
        double U, Fi[3], ti[3], tj[3];
        orc_bp_pair(P, rv, &s->o[3 * i], &s->o[3 * j], &U, Fi, ti, tj);
        for (int a = 0; a < 3; a++) {
            s->Fp[3 * i + a] += Fi[a]; s->Fp[3 * j + a] -= Fi[a];
            s->Tp[3 * i + a] += ti[a]; s->Tp[3 * j + a] += tj[a];
        }
    }
    if (s->nsw > 0) {
        double wr = wall_range(P), wr2 = wr * wr;
        for (int p = 0; p < s->n; p++)
            for (int64_t t = 0; t < s->nsw; t++) {
                int64_t w = s->sw[t];
                double node[3] = {(double)(w % nx), (double)((w / nx) % ny), (double)(w / ((int64_t)nx * ny))};
                double nd[3], rv[3]; int k[3];
                disp(s, node, &s->X[3 * p], nd, k);
                for (int a = 0; a < 3; a++) rv[a] = -nd[a];
                double r2 = rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2];
                if (!(r2 < wr2)) continue;
                double U, F[3], tq[3];
                orc_bp_wall(P, rv, &s->o[3 * p], &U, F, tq);
                for (int a = 0; a < 3; a++) { s->Fp[3 * p + a] += F[a]; s->Tp[3 * p + a] += tq[a]; }
            }
    }

    /* 7. body force on cells and integration (leap-frog, Sec. II) */
    for (int p = 0; p < s->n; p++) {
        if (s->fixed[p]) {
            for (int a = 0; a < 3; a++) { s->V[3 * p + a] = 0.0; s->L[3 * p + a] = 0.0; }
            continue;
        }
        double gb[3] = {0, 0, 0};
        if (P->force_on_particles) force_at(P, s->X[3 * p + 1], s->X[3 * p + 2], gb);
        /* C14: the body force acts on the cells too; mode 2 gives them the
         * force on the plasma they displace (rho0 times their volume), so
         * that a cell made heavier for the stability of the explicit coupling
         * is still driven as a neutrally buoyant one */
        const double Md = P->force_on_particles == 2
                              ? P->rho0 * (4.0 / 3.0) * M_PI * P->R_perp * P->R_perp * P->R_par : s->M;
        for (int a = 0; a < 3; a++) {
            bodyf[a] += Md * gb[a];
            double F = s->Fh[3 * p + a] + s->Fp[3 * p + a] + Md * gb[a];
            s->V[3 * p + a] += F / s->M;
            s->L[3 * p + a] += s->Th[3 * p + a] + s->Tp[3 * p + a];
        }
        const double Lb[3] = {nx, ny, nz};
        for (int a = 0; a < 3; a++) {
            double v = s->V[3 * p + a];
            if (!(fabs(v) < 0.5)) unstable = 1;
            double xn = s->X[3 * p + a] + v;
            if (!(a == 1 && P->wall_y)) {
                if (xn >= Lb[a]) xn -= Lb[a];
                else if (xn < 0.0) xn += Lb[a];
            }
            s->X[3 * p + a] = xn;
        }
        /* viscometer (Sec. IV): a cell whose centre has come closer than
         * sigma_perp to one of the sheared side planes (reading: the node
         * planes x = 0 and x = nx - 1) while moving towards it has its
         * normal velocity negated */
        if (P->le_u != 0.0) {
            const double xc = s->X[3 * p];
            if ((xc < P->sig_perp && s->V[3 * p] < 0.0) || (nx - 1 - xc < P->sig_perp && s->V[3 * p] > 0.0))
                s->V[3 * p] = -s->V[3 * p];
        }
        double qn[4];
        orc_rotate(&s->q[4 * p], &s->L[3 * p], s->Ipar, s->Iperp, 1.0, qn);
        for (int a = 0; a < 4; a++) s->q[4 * p + a] = qn[a];
    }
    for (int a = 0; a < 3; a++) s->body_last[a] = bodyf[a];
    s->step++;
    if (unstable) return fail(s, ORC_EUNSTABLE, "cell velocity non-finite or >= 0.5");
    return ORC_OK;
}

int orc_step(orc_sim* s, int32_t nsteps) {
    if (!s || nsteps < 0) return ORC_EINVAL;
    for (int t = 0; t < nsteps; t++) {
        int rc = one_step(s);
        if (rc) return rc;
    }
    return ORC_OK;
}

/* ---- read-out ---- */

/* Mixture z velocity after the last step, summed over the non-wall nodes
 * (the observable behind the apparent-viscosity estimators; the paper
 * defines the apparent viscosity from the mean flow, Sec. V, and these sums
 * are that mean flow for body-force driving):
 *   fluid node: u_z = (sum n* c_z - g_z/2)/rho, the velocity of the last
 *               collision (the forcing adds exactly g to sum n* c);
 *   cell node:  the rigid-body velocity of its cell at the node, V + Omega x
 *               (x - X), with the X, V, Omega the last step's bounce-back used.
 * out[0] = sum u_z sin(2 pi y / ny), out[1] = sum u_z, out[2] = node count. */
int orc_mixture_sums(const orc_sim* s, double* out) {
    const orc_params* P = &s->P;
    double ssin = 0.0, sone = 0.0, cnt = 0.0;
    for (int64_t i = 0; i < s->ns; i++) {
        if (s->wall[i]) continue;
        int x = (int)(i % P->nx), y = (int)((i / P->nx) % P->ny), z = (int)(i / ((int64_t)P->nx * P->ny));
        double uz;
        int32_t o = s->owner[i];
        if (o == -1) {
            double drho = 0.0, jz = 0.0;
            for (int r = 0; r < 19; r++) {
                double v = s->dA[r * s->ns + i];
                drho += v;
                jz += v * CV[r][2];
            }
            double g[3];
            force_at(P, (double)y, (double)z, g);
            uz = (jz - 0.5 * g[2]) / (P->rho0 + drho);
        } else {
            double node[3] = {x, y, z}, d[3], w[3]; int k[3];
            disp(s, node, &s->Xl[3 * o], d, k);
            cross(&s->Om[3 * o], d, w);
            uz = s->Vl[3 * o + 2] + w[2];
        }
        ssin += uz * sin(2.0 * M_PI * y / P->ny);
        sone += uz;
        cnt += 1.0;
    }
    out[0] = ssin; out[1] = sone; out[2] = cnt;
    return ORC_OK;
}
int orc_mixture_field(const orc_sim* s, double* u) {
    const orc_params* P = &s->P;
    for (int64_t i = 0; i < s->ns; i++) {
        double* ui = u + 3 * i;
        ui[0] = ui[1] = ui[2] = 0.0;
        if (s->wall[i]) continue;
        int x = (int)(i % P->nx), y = (int)((i / P->nx) % P->ny), z = (int)(i / ((int64_t)P->nx * P->ny));
        int32_t o = s->owner[i];
        if (o == -1) {
            double drho = 0.0, j[3] = {0, 0, 0};
            for (int r = 0; r < 19; r++) {
                double v = s->dA[r * s->ns + i];
                drho += v;
                for (int a = 0; a < 3; a++) j[a] += v * CV[r][a];
            }
            double g[3];
            force_at(P, (double)y, (double)z, g);
            for (int a = 0; a < 3; a++) ui[a] = (j[a] - 0.5 * g[a]) / (P->rho0 + drho);
        } else {
            double node[3] = {x, y, z}, d[3], w[3]; int k[3];
            disp(s, node, &s->Xl[3 * o], d, k);
            cross(&s->Om[3 * o], d, w);
            for (int a = 0; a < 3; a++) ui[a] = s->Vl[3 * o + a] + w[a];
        }
    }
    return ORC_OK;
}

double orc_le_flux(const orc_sim* s) { return s->le_flux; }

int orc_get_deviations(const orc_sim* s, double* d) {
    memcpy(d, s->dA, sizeof(double) * 19 * s->ns);
    return ORC_OK;
}

/* rho = sum n*, u = (sum n* c - g/2)/rho: the velocity used in the last
 * collision (the forcing adds exactly g to sum n* c) */
int orc_get_fields(const orc_sim* s, double* rho, double* u) {
    for (int64_t i = 0; i < s->ns; i++) {
        if (s->owner[i] != -1) {
            if (rho) rho[i] = 0.0;
            if (u) u[3 * i] = u[3 * i + 1] = u[3 * i + 2] = 0.0;
            continue;
        }
        double drho = 0.0, j[3] = {0, 0, 0};
        for (int r = 0; r < 19; r++) {
            double v = s->dA[r * s->ns + i];
            drho += v;
            for (int a = 0; a < 3; a++) j[a] += v * CV[r][a];
        }
        double rr = s->P.rho0 + drho;
        double g[3];
        force_at(&s->P, (double)((i / s->P.nx) % s->P.ny), (double)(i / ((int64_t)s->P.nx * s->P.ny)), g);
        if (rho) rho[i] = rr;
        if (u) for (int a = 0; a < 3; a++) u[3 * i + a] = (j[a] - 0.5 * g[a]) / rr;
    }
    return ORC_OK;
}

int orc_get_particles(const orc_sim* s, double* X, double* q, double* V, double* L) {
    if (X) memcpy(X, s->X, sizeof(double) * 3 * s->n);
    if (q) memcpy(q, s->q, sizeof(double) * 4 * s->n);
    if (V) memcpy(V, s->V, sizeof(double) * 3 * s->n);
    if (L) memcpy(L, s->L, sizeof(double) * 3 * s->n);
    return ORC_OK;
}

int orc_get_forces(const orc_sim* s, double* Fh, double* Th, double* Fp, double* Tp) {
    if (Fh) memcpy(Fh, s->Fh, sizeof(double) * 3 * s->n);
    if (Th) memcpy(Th, s->Th, sizeof(double) * 3 * s->n);
    if (Fp) memcpy(Fp, s->Fp, sizeof(double) * 3 * s->n);
    if (Tp) memcpy(Tp, s->Tp, sizeof(double) * 3 * s->n);
    return ORC_OK;
}

int orc_get_owner(const orc_sim* s, int32_t* owner) {
    memcpy(owner, s->owner, sizeof(int32_t) * s->ns);
    return ORC_OK;
}

/* bit r set when the fluid node x has a non-fluid source node x - c_r */
int orc_get_link_mask(const orc_sim* s, uint32_t* mask) {
    const int nx = s->P.nx, ny = s->P.ny, nz = s->P.nz;
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                int64_t i = sid(s, x, y, z);
                uint32_t m = 0;
                if (s->owner[i] == -1)
                    for (int r = 1; r < 19; r++) {
                        int xs = wrapi(x - CV[r][0], nx), ys = wrapi(y - CV[r][1], ny), zs = wrapi(z - CV[r][2], nz);
                        if (s->owner[sid(s, xs, ys, zs)] != -1) m |= 1u << r;
                    }
                mask[i] = m;
            }
    return ORC_OK;
}

int orc_get_pairs(const orc_sim* s, int32_t* ij, int64_t cap, int64_t* n) {
    /* pair set at the current positions */
    orc_sim* w = (orc_sim*)s;
    build_pairs(w);
    *n = w->npairs;
    int64_t m = w->npairs < cap ? w->npairs : cap;
    if (ij && m > 0) memcpy(ij, w->pairs, sizeof(int32_t) * 2 * (size_t)m);
    return ORC_OK;
}

int orc_get_link_static(const orc_sim* s, int64_t* A, int64_t* B) {
    if (A) memcpy(A, s->Aint, sizeof(int64_t) * 3 * s->n);
    if (B) memcpy(B, s->Bint, sizeof(int64_t) * 3 * s->n);
    return ORC_OK;
}

int orc_get_observables(const orc_sim* s, double* out) {
    double mass = 0.0, mom[3] = {0, 0, 0}, pm[3] = {0, 0, 0};
    int64_t nf = 0;
    for (int64_t i = 0; i < s->ns; i++) {
        if (s->owner[i] != -1) continue;
        nf++;
        double drho = 0.0;
        for (int r = 0; r < 19; r++) {
            double v = s->dA[r * s->ns + i];
            drho += v;
            for (int a = 0; a < 3; a++) mom[a] += v * CV[r][a];
        }
        mass += s->P.rho0 + drho;
    }
    for (int p = 0; p < s->n; p++)
        if (!s->fixed[p]) for (int a = 0; a < 3; a++) pm[a] += s->M * s->V[3 * p + a];
    out[0] = mass;
    for (int a = 0; a < 3; a++) { out[1 + a] = mom[a]; out[4 + a] = pm[a]; out[8 + a] = s->body_last[a]; }
    out[7] = (double)nf;
    out[11] = (double)s->step;
    return ORC_OK;
}
