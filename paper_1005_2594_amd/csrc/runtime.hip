// runtime.hip -- host side of libcgb: the C ABI of include/cgb.h.
//
// Owns all device memory of a lattice, sequences the kernels of one time step
// on one HIP stream, and moves data across the ABI.  Populations live as two
// structure-of-arrays buffers [19][pstride] (x fastest within a plane) that
// swap roles every step; a density-deviation field travels with them because
// the moving-boundary correction (Eq. 10) needs the density of the fluid node
// at the time of the bounced populations.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "cgb_dev.h"
#include "sim.h"

using namespace cgb;

static const char* kKindNames[] = {"prep", "raster", "transitions", "lb", "mem_reduce", "cells", "potentials", "integrate", "track"};

#define FAIL(s, code, ...)                                  \
    do {                                                    \
        char _b[512];                                       \
        snprintf(_b, sizeof _b, __VA_ARGS__);               \
        (s)->err = _b;                                      \
        return code;                                        \
    } while (0)

#define HIPCHK(s, call)                                                               \
    do {                                                                              \
        hipError_t _e = (call);                                                       \
        if (_e != hipSuccess) FAIL(s, CGB_EDEVICE, "%s: %s", #call, hipGetErrorString(_e)); \
    } while (0)

// Device memory of a handle: its own allocations (MEM_OWN), 256-byte aligned
// pieces of a caller's arena (MEM_ARENA), or only counted (MEM_COUNT, the size
// query: the pointers are placeholders that nothing dereferences).
template <class T>
static hipError_t dalloc(cgb_sim* s, T** p, size_t bytes) {
    if (s->mem_mode != MEM_OWN) {
        const size_t b = bytes ? (bytes + 255) & ~(size_t)255 : 256;
        if (s->mem_mode == MEM_ARENA && s->arena_used + b > s->arena_bytes) return hipErrorOutOfMemory;
        *p = (T*)(s->mem_mode == MEM_ARENA ? s->arena + s->arena_used : (char*)nullptr + 4096 + s->arena_used);
        s->arena_used += b;
        s->dev_bytes += (int64_t)bytes;
        return hipSuccess;
    }
    void* v = nullptr;
    hipError_t e = hipMalloc(&v, bytes ? bytes : 8);
    if (e != hipSuccess) return e;
    s->allocs.push_back(v);
    s->dev_bytes += (int64_t)bytes;
    *p = (T*)v;
    return hipSuccess;
}

// frees an own allocation; pieces of an arena stay where they are
static void dfree(cgb_sim* s, void* p) {
    if (!p || s->mem_mode != MEM_OWN) return;
    auto it = std::find(s->allocs.begin(), s->allocs.end(), p);
    if (it != s->allocs.end()) s->allocs.erase(it);
    (void)hipFree(p);
}

// Bound on the lattice nodes strictly inside one ellipsoid with half axes
// (R_perp, R_perp, R_par): the unit cubes centred on those nodes are disjoint
// and lie within distance rho = sqrt(3)/2 of the ellipsoid, and that
// neighbourhood lies inside the ellipsoid with every half axis grown by t,
// t^2 + (a_min - rho) t - rho a_max = 0 (from |e + v|_A' <= |e|_A' + |v|_A'
// in the norm of the grown ellipsoid), so the count is below its volume.
static int inside_bound(double Rp, double Rl) {
    const double rho = 0.8660254037844386 + 1e-3;
    const double amin = std::min(Rp, Rl), amax = std::max(Rp, Rl);
    const double t = 0.5 * (-(amin - rho) + sqrt((amin - rho) * (amin - rho) + 4.0 * rho * amax));
    const double v = (4.0 / 3.0) * M_PI * (Rp + t) * (Rp + t) * (Rl + t);
    return (int)std::min(v + 1.0, 1e8);
}

static double wall_range(const cgb_params& P) {
    const double sp2 = P.sig_perp * P.sig_perp, sl2 = P.sig_par * P.sig_par, sw2 = P.sig_w * P.sig_w;
    const double chiw = (sl2 - sp2) / (sl2 + sw2);
    const double sbw = sqrt(sp2 + sw2);
    if (chiw <= 0.0) return sbw;
    if (chiw >= 1.0) return 1e30;
    return sbw / sqrt(1.0 - chiw);
}

// ---------------------------------------------------------------- profiling
static hipEvent_t take_event(cgb_sim* s) {
    if (!s->ev_pool.empty()) {
        hipEvent_t e = s->ev_pool.back();
        s->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

static void harvest(cgb_sim* s) {
    for (auto& r : s->recs) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.e0, r.e1) == hipSuccess) {
            s->ktime[r.kind] += ms;
            s->kcount[r.kind] += 1;
        }
        s->ev_pool.push_back(r.e0);
        s->ev_pool.push_back(r.e1);
    }
    s->recs.clear();
}

// launch(es) f bracketed by timing events on stream st (when profiling)
template <class F>
static hipError_t timed_on(cgb_sim* s, int kind, hipStream_t st, F&& f) {
    if (!s->prof) return f();
    if (s->recs.size() > 4096) {
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return e;
        harvest(s);
    }
    LaunchRec r{kind, take_event(s), take_event(s)};
    if (!r.e0 || !r.e1) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(r.e0, st);
    if (e != hipSuccess) return e;
    e = f();
    if (e != hipSuccess) return e;
    e = hipEventRecord(r.e1, st);
    s->recs.push_back(r);
    return e;
}
template <class F>
static hipError_t timed(cgb_sim* s, int kind, F&& f) { return timed_on(s, kind, s->st, f); }

// ---------------------------------------------------------------- helpers
static void bind_buffers(cgb_sim* s) {
    s->a.A = s->pop[s->cur];
    s->a.B = s->pop[1 - s->cur];
    s->a.rhoA = s->rho[s->cur];
    s->a.rhoB = s->rho[1 - s->cur];
    s->a.step = s->step;
}

static int ensure_tmp(cgb_sim* s, size_t bytes) {
    if (bytes <= s->tmp_bytes) return CGB_OK;
    if (s->mem_mode != MEM_OWN) FAIL(s, CGB_ENOMEM, "staging buffer of %zu bytes is smaller than %zu", s->tmp_bytes, bytes);
    dfree(s, s->tmp);
    s->tmp = nullptr;
    s->tmp_bytes = 0;
    HIPCHK(s, dalloc(s, &s->tmp, bytes));
    s->tmp_bytes = bytes;
    return CGB_OK;
}

static int check_status(cgb_sim* s) {
    int st = 0, bad = 0;
    HIPCHK(s, hipMemcpyAsync(&st, s->a.status, sizeof(int), hipMemcpyDeviceToHost, s->st));
    HIPCHK(s, hipMemcpyAsync(&bad, s->a.bad_step, sizeof(int), hipMemcpyDeviceToHost, s->st));
    HIPCHK(s, hipStreamSynchronize(s->st));
    if (st & ST_TRANS_OVERFLOW) FAIL(s, CGB_ENOMEM, "transition list overflow (capacity %d per segment)", s->a.trans_cap);
    if (st & ST_LIST_OVERFLOW) FAIL(s, CGB_ENOMEM, "covered-node list overflow (capacity %d per cell)", s->a.lcap);
    if (st & ST_LE_SEAM) FAIL(s, CGB_EUNSTABLE, "a cell covers a node of a sheared plane of the viscometer");
    if (st & ST_UNSTABLE) FAIL(s, CGB_EUNSTABLE, "unstable at step %d: non-finite state, |u| > 0.4 or |V| >= 0.5", bad);
    return CGB_OK;
}

// ---------------------------------------------------------------- ABI
extern "C" {

int cgb_params_default(cgb_params* p) {
    if (!p) return CGB_EINVAL;
    memset(p, 0, sizeof *p);
    p->nx = p->ny = p->nz = 32;
    p->tau = 1.0;
    p->rho0 = 1.0;
    p->R_perp = 2.5;
    p->R_par = 1.0;
    p->sig_perp = 2.5 * 12.0 / 11.0;
    p->sig_par = 1.0 * 12.0 / 11.0;
    p->sig_w = 0.5;
    p->eps = 0.05;
    p->eps_w = 0.05;
    p->r_cut = 3.75;
    p->rho_p = 1.0;
    p->force_on_particles = 1;
    p->precision = CGB_P32;
    p->pmx_scale = 32768.0;
    return CGB_OK;
}

const char* cgb_last_error(const cgb_sim* s) { return s ? s->err.c_str() : "null handle"; }
int64_t cgb_device_bytes(const cgb_sim* s) { return s ? s->dev_bytes : 0; }

static void drop_step_graph(cgb_sim* s);

void cgb_destroy(cgb_sim* s) {
    if (!s) return;
    if (s->st) (void)hipStreamSynchronize(s->st);
    drop_step_graph(s);
    if (s->st_pot) { (void)hipStreamSynchronize(s->st_pot); (void)hipStreamDestroy(s->st_pot); }
    for (hipEvent_t e : {s->ev_ras, s->ev_pot})
        if (e) (void)hipEventDestroy(e);
    for (auto& r : s->recs) { (void)hipEventDestroy(r.e0); (void)hipEventDestroy(r.e1); }
    for (auto e : s->ev_pool) (void)hipEventDestroy(e);
    for (void* p : s->allocs) (void)hipFree(p);
    if (s->own_stream && s->st) (void)hipStreamDestroy(s->st);
    delete s;
}

// LB launch shape
static void set_tiles(cgb_sim* s, LaunchCfg cfg) {
    DevArgs& a = s->a;
    s->lbcfg = cfg;
    a.tile[0] = cfg.bx; a.tile[1] = cfg.by; a.tile[2] = cfg.tz;
}

static LaunchCfg default_tiles(const DevArgs& a) {
    LaunchCfg c{a.nx >= 256 ? 256 : (a.nx >= 128 ? 128 : 64), a.nx >= 256 ? 1 : (a.nx >= 128 ? 2 : 4), 16};
    if (a.nx < 48) c = LaunchCfg{32, 8, 16};
    if (a.nx < 24) c = LaunchCfg{16, 16, 16};
    if (a.nz < 32 && !a.big && !a.cidx) c.tz = 8;  // the large-lattice and indexed layouts sweep 16 nodes
    return c;
}

// allocation only (the size query runs it too); init_particle_buffers clears
static int alloc_particles(cgb_sim* s, int ncap) {
    DevArgs& a = s->a;
    void* olds[] = {a.X, a.q, a.V, a.L, a.fixed, a.Xprev, a.Hprev, a.kin, a.kinf, a.crec, a.FTh, a.FTp, a.FTt,
                    a.clist, a.ccount, a.trans, a.pbin, a.bin_idx, a.rank, a.Xs, a.body_part};
    for (void* p : olds) dfree(s, p);
    const size_t n = (size_t)std::max(ncap, 1);
    HIPCHK(s, dalloc(s, &a.X, 3 * n * 8));
    HIPCHK(s, dalloc(s, &a.q, 4 * n * 8));
    HIPCHK(s, dalloc(s, &a.V, 3 * n * 8));
    HIPCHK(s, dalloc(s, &a.L, 3 * n * 8));
    HIPCHK(s, dalloc(s, &a.fixed, n));
    HIPCHK(s, dalloc(s, &a.Xprev, 3 * n * 8));
    HIPCHK(s, dalloc(s, &a.Hprev, 3 * n * 8));
    HIPCHK(s, dalloc(s, &a.kin, 12 * n * 8));
    HIPCHK(s, dalloc(s, &a.kinf, 12 * n * 4));
    HIPCHK(s, dalloc(s, &a.crec, n * sizeof(CellRec)));
    HIPCHK(s, dalloc(s, &a.FTh, 6 * n * 8));
    HIPCHK(s, dalloc(s, &a.FTp, 6 * n * 8));
    HIPCHK(s, dalloc(s, &a.FTt, 12 * n * 8));
    HIPCHK(s, dalloc(s, &a.clist, n * (size_t)a.lcap * 4));
    HIPCHK(s, dalloc(s, &a.ccount, n * 4));
    HIPCHK(s, dalloc(s, &a.pbin, n * 4));
    HIPCHK(s, dalloc(s, &a.bin_idx, n * 4));
    HIPCHK(s, dalloc(s, &a.rank, n * 4));
    HIPCHK(s, dalloc(s, &a.Xs, n * 4 * 8));
    HIPCHK(s, dalloc(s, &a.body_part, ((n + 255) / 256) * 3 * 8));
    long long cap = 96LL * (long long)n + 65536;
    if (cap > s->a.ns + 65536) cap = s->a.ns + 65536;
    a.trans_cap = (int)(cap / TSEG + 4096);  // per segment
    HIPCHK(s, dalloc(s, &a.trans, (size_t)a.trans_cap * TSEG * 3 * 4));
    s->ncap = ncap;
    return CGB_OK;
}

static int init_particle_buffers(cgb_sim* s) {
    DevArgs& a = s->a;
    const long long n = std::max(s->ncap, 1);
    HIPCHK(s, launch_fill_i32(a.ccount, n, 0, s->st));
    HIPCHK(s, launch_fill_f64(a.body_part, ((n + 255) / 256) * 3, 0.0, s->st));
    return CGB_OK;
}

// host-side state of a new handle that the device set-up uploads
struct HostInit {
    std::vector<int32_t> own;   // owner map: walls and fluid
    std::vector<int32_t> cidx;  // indexed layout: storage index of each site (-1 at walls)
    std::vector<double> ysin;   // sin(2 pi y / ny)
    std::vector<int> wstart, widx;  // surface wall nodes per cell-list bin
};

// The narrow layout addresses the population, density, flag and link-moment
// arrays with 32-bit byte offsets; lattices past that (or a request) take the
// large-lattice layout (64-bit lane addresses, node momenta in the nodes' own
// unused population slots)
static bool big_layout(const cgb_params* p) {
    if (p->mem_layout == 1) return true;
    const double esz = p->precision == CGB_P64 ? 8.0 : (p->precision == CGB_P32 ? 4.0 : 2.0);
    const double msz = p->precision == CGB_P64 ? 8.0 : 4.0;
    const double pst = (double)(((long long)p->nx * p->ny * p->nz + 255) / 256 * 256);
    return 19.0 * esz * pst >= 4294901760.0 || 4.0 * msz * pst >= 4294901760.0;
}

static bool params_ok(const cgb_params* p) {
    if (p->nx < 3 || p->ny < 3 || p->nz < 3 || !(p->tau > 0.5) || !(p->rho0 > 0) || p->precision < 0 ||
        p->force_on_particles < 0 || p->force_on_particles > 2 ||
        p->precision > CGB_PMX16S || !(p->R_perp > 0) || !(p->R_par > 0) || !(p->rho_p > 0) || !(p->r_cut > 0))
        return false;
    if (p->le_u != 0.0 && (p->wall_y || p->precision == CGB_PMX16S || !(fabs(p->le_u) < 0.5))) return false;
    // site indices are 32-bit (signed in the transition records)
    if ((long long)p->nx * p->ny * p->nz > (1ll << 31)) return false;
    if (p->mem_layout < 0 || p->mem_layout > 1) return false;
    // the large-lattice layout has the tau = 1 kernel only, without the viscometer
    if (big_layout(p) && (p->tau != 1.0 || p->le_u != 0.0)) return false;
    // so has the indexed layout, within the 32-bit layout
    if (p->indexed < 0 || p->indexed > 1) return false;
    if (p->indexed && (p->tau != 1.0 || p->le_u != 0.0 || big_layout(p))) return false;
    return true;
}

// parameters, constants and the host-side geometry (no device work)
static int setup_host(cgb_sim* s, const cgb_params* p, const uint8_t* wall_mask, HostInit& hi) {
    s->P = *p;
    if (s->P.pmx_scale == 0.0) s->P.pmx_scale = 32768.0;
    DevArgs& a = s->a;
    memset(&a, 0, sizeof a);
    a.nx = p->nx; a.ny = p->ny; a.nz = p->nz;
    a.ns = (long long)p->nx * p->ny * p->nz;
    a.pstride = (a.ns + 255) / 256 * 256;
    a.wall_y = p->wall_y;
    for (int c = 0; c < 3; c++) { a.wvb[c] = p->wall_v_bot[c]; a.wvt[c] = p->wall_v_top[c]; a.g[c] = p->g[c]; }
    a.moving_walls = p->wall_y && (p->wall_v_bot[0] != 0 || p->wall_v_bot[1] != 0 || p->wall_v_bot[2] != 0 ||
                                   p->wall_v_top[0] != 0 || p->wall_v_top[1] != 0 || p->wall_v_top[2] != 0);
    a.tau = p->tau; a.rho0 = p->rho0;
    a.force_mode = p->force_mode; a.f0 = p->f0; a.force_on_particles = p->force_on_particles;
    a.fregion = (p->force_mode == 1 && p->force_zhi > p->force_zlo) ? 1 : 0;
    a.fzlo = p->force_zlo; a.fzhi = p->force_zhi;
    a.le_u = p->le_u;
    a.big = big_layout(p) ? 1 : 0;
    a.precision = p->precision;
    a.pmx_scale = (float)s->P.pmx_scale;
    a.pmx_inv = (float)(1.0 / s->P.pmx_scale);
    a.M = p->rho_p * (4.0 / 3.0) * M_PI * p->R_perp * p->R_perp * p->R_par;
    a.Mdrive = p->force_on_particles == 2 ? p->rho0 * (4.0 / 3.0) * M_PI * p->R_perp * p->R_perp * p->R_par : a.M;
    a.Ipar = 0.4 * a.M * p->R_perp * p->R_perp;
    a.Iperp = 0.2 * a.M * (p->R_perp * p->R_perp + p->R_par * p->R_par);
    a.iRpar2 = 1.0 / (p->R_par * p->R_par);
    a.iRperp2 = 1.0 / (p->R_perp * p->R_perp);
    a.Rb = std::max(p->R_perp, p->R_par);
    a.lcap = inside_bound(p->R_perp, p->R_par);
    a.r_cut2 = p->r_cut * p->r_cut;
    const double wr = wall_range(*p);
    a.wall_range2 = wr * wr;
    a.sig_perp = p->sig_perp; a.sig_par = p->sig_par; a.sig_w = p->sig_w; a.eps = p->eps; a.eps_w = p->eps_w;
    s->esize = p->precision == CGB_P64 ? 8 : (p->precision == CGB_P32 ? 4 : 2);
    // owner map: walls from the mask and the wall planes
    hi.own.assign((size_t)a.ns, OWN_FLUID);
    s->n_nonwall = (double)a.ns;
    if (wall_mask || p->wall_y) {
        for (long long i = 0; i < a.ns; i++) {
            const int y = (int)((i / a.nx) % a.ny);
            bool w = wall_mask ? wall_mask[i] != 0 : false;
            if (p->wall_y && (y == 0 || y == a.ny - 1)) w = true;
            if (w) hi.own[(size_t)i] = OWN_WALL;
        }
        s->n_nonwall = 0;
        for (long long i = 0; i < a.ns; i++) s->n_nonwall += hi.own[(size_t)i] != OWN_WALL ? 1.0 : 0.0;
    }
    if (p->indexed) {
        // storage for the non-wall nodes only, in lattice order
        hi.cidx.assign((size_t)a.ns, -1);
        long long nc = 0;
        for (long long i = 0; i < a.ns; i++)
            if (hi.own[(size_t)i] != OWN_WALL) hi.cidx[(size_t)i] = (int32_t)nc++;
        a.pstride = (std::max(nc, 1ll) + 255) / 256 * 256;
        s->n_stored = nc;
    }
    // streamed outputs bypass the caches only where the populations outgrow
    // the 256 MB last-level cache (smaller lattices find last step's output
    // there)
    a.nt_out = 19.0 * (double)a.pstride * (double)s->esize > 256.0 * 1024 * 1024 ? 1 : 0;
    hi.ysin.resize((size_t)a.ny);
    for (int y = 0; y < a.ny; y++) hi.ysin[(size_t)y] = sin(2.0 * M_PI * y / (double)a.ny);
    // cell-list geometry: bin edge >= max(cut-off, wall potential range)
    const double Lb[3] = {(double)a.nx, (double)a.ny, (double)a.nz};
    const double emin = std::max(p->r_cut, wr);
    long long nbins = 1;
    for (int c = 0; c < 3; c++) {
        a.nb[c] = std::max(1, (int)floor(Lb[c] / emin));
        a.bedge[c] = Lb[c] / a.nb[c];
        nbins *= a.nb[c];
    }
    if (nbins > (1LL << 30)) FAIL(s, CGB_EINVAL, "too many cell-list bins");
    a.nbins = (int)nbins;
    // surface wall nodes (wall nodes with a non-wall neighbour), binned
    const bool any_wall = wall_mask || p->wall_y;
    std::vector<std::vector<int>> per(any_wall ? (size_t)nbins : 0);
    long long nsw = 0;
    for (long long i = 0; any_wall && i < a.ns; i++) {
        if (hi.own[(size_t)i] != OWN_WALL) continue;
        const int x = (int)(i % a.nx), y = (int)((i / a.nx) % a.ny), z = (int)(i / ((long long)a.nx * a.ny));
        bool surf = false;
        for (int r = 1; r < 19 && !surf; r++) {
            int yn = y + CY(r);
            if (p->wall_y) { if (yn < 0 || yn >= a.ny) continue; }
            else yn = wrap(yn, a.ny);
            const long long j = wrap(x + CX(r), a.nx) + (long long)a.nx * (yn + (long long)a.ny * wrap(z + CZ(r), a.nz));
            if (hi.own[(size_t)j] != OWN_WALL) surf = true;
        }
        if (!surf) continue;
        int bc[3] = {x, y, z};
        for (int c = 0; c < 3; c++) {
            int b = (int)floor(bc[c] / a.bedge[c]);
            bc[c] = std::min(std::max(b, 0), a.nb[c] - 1);
        }
        per[(size_t)(bc[0] + a.nb[0] * (bc[1] + (long long)a.nb[1] * bc[2]))].push_back((int)i);
        nsw++;
    }
    hi.wstart.assign((size_t)nbins + 1, 0);
    hi.widx.clear();
    hi.widx.reserve((size_t)nsw);
    for (long long b = 0; any_wall && b < nbins; b++) {
        hi.wstart[(size_t)b] = (int)hi.widx.size();
        for (int v : per[(size_t)b]) hi.widx.push_back(v);
    }
    hi.wstart[(size_t)nbins] = (int)hi.widx.size();
    a.nsw = (int)nsw;
    return CGB_OK;
}

// Every device buffer of the handle.  cell_cap < 0: own memory, the cell
// arrays grow with the cells; otherwise (arena, size query) the cell arrays,
// the pair buffer and the track record are sized once for cell_cap cells and
// track_cap steps, and the FP64 staging buffer is allocated too.
static int alloc_state(cgb_sim* s, int cell_cap, int track_cap) {
    DevArgs& a = s->a;
    const size_t popb = 19 * (size_t)a.pstride * s->esize;
    HIPCHK(s, dalloc(s, &s->pop[0], popb));
    HIPCHK(s, dalloc(s, &s->pop[1], popb));
    HIPCHK(s, dalloc(s, &s->rho[0], (size_t)a.pstride * s->esize));
    HIPCHK(s, dalloc(s, &s->rho[1], (size_t)a.pstride * s->esize));
    HIPCHK(s, dalloc(s, &a.owner, (size_t)a.ns * 4));
    const size_t msz = s->P.precision == CGB_P64 ? 8 : 4;
    if (s->P.tau == 1.0) HIPCHK(s, dalloc(s, &a.lmom, 4 * (size_t)a.pstride * msz));
    else HIPCHK(s, dalloc(s, &a.usol, 3 * (size_t)a.pstride * msz));
    HIPCHK(s, dalloc(s, &a.flags, (size_t)a.ns * 4));
    HIPCHK(s, dalloc(s, &a.cand, (size_t)a.ns * 4));
    if (!a.big) HIPCHK(s, dalloc(s, &a.fnode, 24 * (size_t)(s->P.indexed ? a.pstride : a.ns)));
    if (s->P.indexed) HIPCHK(s, dalloc(s, (int32_t**)&a.cidx, (size_t)a.ns * 4));
    HIPCHK(s, dalloc(s, &s->zero_buf, 256));
    a.zero = s->zero_buf;
    HIPCHK(s, dalloc(s, &a.ntrans, TSEG * 4));
    HIPCHK(s, dalloc(s, &a.status, 16));
    HIPCHK(s, dalloc(s, &a.bad_step, 16));
    HIPCHK(s, dalloc(s, &a.dstep, 16));
    HIPCHK(s, dalloc(s, &s->obs_partial, (size_t)s->obs_nblk * 8 * 8));
    HIPCHK(s, dalloc(s, &a.ysin, (size_t)a.ny * 8));
    {
        // partials of the mixture record: one per LB block (the tau = 1
        // kernel sums the record), at least the track pass's
        const LaunchCfg d = default_tiles(a);
        const long long nb = (long long)((a.nx + d.bx - 1) / d.bx) * ((a.ny + d.by - 1) / d.by) * ((a.nz + d.tz - 1) / d.tz);
        a.track_slots = (int)std::max<long long>(TRACK_BLOCKS, nb);
        HIPCHK(s, dalloc(s, &a.track_part, (size_t)a.track_slots * 2 * 8));
    }
    HIPCHK(s, dalloc(s, &a.track_n, 16));
    HIPCHK(s, dalloc(s, &a.bin_count, (size_t)a.nbins * 4));
    HIPCHK(s, dalloc(s, &a.bin_start, (size_t)(a.nbins + 1) * 4));
    HIPCHK(s, dalloc(s, &a.bin_fill, (size_t)a.nbins * 4));
    HIPCHK(s, dalloc(s, &a.scan_tmp, (size_t)((a.nbins + 4095) / 4096 + 1) * 4));
    HIPCHK(s, dalloc(s, &a.wall_start, (size_t)(a.nbins + 1) * 4));
    HIPCHK(s, dalloc(s, &a.wall_idx, (size_t)std::max(a.nsw, 1) * 4));
    if (a.le_u != 0.0) {
        HIPCHK(s, dalloc(s, &a.le_buf, 2 * 5 * (size_t)a.ny * a.nz * (s->P.precision == CGB_P64 ? 8 : 4)));
        HIPCHK(s, dalloc(s, &a.le_part, (size_t)le_blocks(a) * 8));
    }
    int rc = alloc_particles(s, std::max(cell_cap, 0));
    if (rc) return rc;
    if (cell_cap >= 0) {
        s->cell_cap = cell_cap;
        s->pair_cap = std::max(1024, 64 * cell_cap);
        HIPCHK(s, dalloc(s, &s->pair_cnt, 16));
        HIPCHK(s, dalloc(s, &s->pair_buf, (size_t)s->pair_cap * 2 * 4));
        s->track_max = std::max(track_cap, 0);
        HIPCHK(s, dalloc(s, &s->track_buf, 2 * (size_t)std::max(s->track_max, 1) * 8));
        if (a.le_u != 0.0) HIPCHK(s, dalloc(s, &s->le_rec_buf, (size_t)std::max(s->track_max, 1) * 8));
        s->arena_state = s->arena_used;
    }
    return CGB_OK;
}

// uploads and set-up kernels of a new handle (fluid at rest everywhere)
static int init_device(cgb_sim* s, const HostInit& hi) {
    DevArgs& a = s->a;
    const size_t msz = s->P.precision == CGB_P64 ? 8 : 4;
    if (a.lmom) HIPCHK(s, launch_fill_i32((int*)a.lmom, (long long)(4 * (size_t)a.pstride * msz / 4), 0, s->st));
    HIPCHK(s, hipMemcpyAsync(a.owner, hi.own.data(), (size_t)a.ns * 4, hipMemcpyHostToDevice, s->st));
    if (a.cidx)
        HIPCHK(s, hipMemcpyAsync(const_cast<int32_t*>(a.cidx), hi.cidx.data(), (size_t)a.ns * 4, hipMemcpyHostToDevice, s->st));
    if (a.usol) HIPCHK(s, launch_usol(a, s->st, true));
    HIPCHK(s, hipMemcpyAsync(a.ysin, hi.ysin.data(), (size_t)a.ny * 8, hipMemcpyHostToDevice, s->st));
    HIPCHK(s, hipMemcpyAsync(a.wall_start, hi.wstart.data(), hi.wstart.size() * 4, hipMemcpyHostToDevice, s->st));
    if (!hi.widx.empty())
        HIPCHK(s, hipMemcpyAsync(a.wall_idx, hi.widx.data(), hi.widx.size() * 4, hipMemcpyHostToDevice, s->st));
    HIPCHK(s, launch_fill_i32(a.cand, a.ns, NO_CAND, s->st));
    HIPCHK(s, launch_fill_i32((int*)s->zero_buf, 64, 0, s->st));
    HIPCHK(s, launch_fill_i32(a.status, 4, 0, s->st));
    HIPCHK(s, launch_fill_i32(a.bad_step, 4, 0x7fffffff, s->st));
    HIPCHK(s, launch_fill_i32(a.dstep, 1, -1, s->st));
    HIPCHK(s, launch_fill_i32(a.track_n, 4, 0, s->st));
    int rc = init_particle_buffers(s);
    if (rc) return rc;
    set_tiles(s, default_tiles(a));
    a.n = 0;
    bind_buffers(s);
    HIPCHK(s, launch_equilibrium_fill(a, nullptr, nullptr, s->st));
    HIPCHK(s, launch_flags_rebuild(a, s->st));
    if (a.lmom) HIPCHK(s, launch_lmom(a, s->st));
    HIPCHK(s, hipStreamSynchronize(s->st));  // the host vectors are temporaries
    s->fluid_ready = true;
    return CGB_OK;
}

static int make_stream(cgb_sim* s, void* stream) {
    if (stream) {
        s->st = (hipStream_t)stream;
    } else {
        HIPCHK(s, hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking));
        s->own_stream = true;
    }
    s->fork = true;  // side streams are created at the first step that uses them
    return CGB_OK;
}

int cgb_create(const cgb_params* p, const uint8_t* wall_mask, void* stream, cgb_sim** out) {
    if (!p || !out) return CGB_EINVAL;
    *out = nullptr;
    if (!params_ok(p)) return CGB_EINVAL;
    cgb_sim* s = new cgb_sim();
    HostInit hi;
    int rc = setup_host(s, p, wall_mask, hi);
    if (!rc) rc = make_stream(s, stream);
    if (!rc) rc = alloc_state(s, -1, 0);
    if (!rc) rc = init_device(s, hi);
    if (rc) {
        cgb_destroy(s);
        return rc;
    }
    *out = s;
    return CGB_OK;
}

int cgb_query_sizes(const cgb_params* p, const uint8_t* wall_mask, int32_t cell_cap, int32_t track_cap,
                    cgb_sizes* out) {
    if (!p || !out || cell_cap < 0 || track_cap < 0 || !params_ok(p)) return CGB_EINVAL;
    cgb_sim s;
    s.mem_mode = MEM_COUNT;
    HostInit hi;
    int rc = setup_host(&s, p, wall_mask, hi);
    if (!rc) rc = alloc_state(&s, cell_cap, track_cap);
    if (rc) return rc;
    out->arena_bytes = (int64_t)s.arena_used;
    // FP64 staging of the largest host transfer: 19 deviations per site
    out->staging_bytes = (int64_t)(19 * (size_t)s.a.ns * 8);
    out->cell_cap = cell_cap;
    out->track_cap = track_cap;
    return CGB_OK;
}

int cgb_create_in(const cgb_params* p, const uint8_t* wall_mask, void* stream, const cgb_sizes* sz, void* arena,
                  void* staging, cgb_sim** out) {
    if (!p || !sz || !arena || !staging || !out) return CGB_EINVAL;
    *out = nullptr;
    cgb_sizes want;
    int rc = cgb_query_sizes(p, wall_mask, sz->cell_cap, sz->track_cap, &want);
    if (rc) return rc;
    if (sz->arena_bytes < want.arena_bytes || sz->staging_bytes < want.staging_bytes) return CGB_EINVAL;
    if (((uintptr_t)arena & 255) != 0 || ((uintptr_t)staging & 7) != 0) return CGB_EINVAL;
    cgb_sim* s = new cgb_sim();
    s->mem_mode = MEM_ARENA;
    s->arena = (char*)arena;
    s->arena_bytes = (size_t)sz->arena_bytes;
    s->tmp = (double*)staging;
    s->tmp_bytes = (size_t)sz->staging_bytes;
    HostInit hi;
    rc = setup_host(s, p, wall_mask, hi);
    if (!rc) rc = make_stream(s, stream);
    if (!rc) rc = alloc_state(s, sz->cell_cap, sz->track_cap);
    if (!rc) rc = init_device(s, hi);
    if (rc) {
        cgb_destroy(s);
        return rc;
    }
    *out = s;
    return CGB_OK;
}

int cgb_set_particles(cgb_sim* s, int32_t n, const double* X, const double* q, const double* V, const double* L,
                      const uint8_t* fixed) {
    if (!s) return CGB_EINVAL;
    if (n < 0 || (n > 0 && (!X || !q))) FAIL(s, CGB_EINVAL, "bad particle arguments");
    DevArgs& a = s->a;
    if (n > 0) {
        const int span = 2 * (int)ceil(a.Rb) + 6;
        if (a.nx < span || a.nz < span || (!a.wall_y && a.ny < span))
            FAIL(s, CGB_EINVAL, "periodic box smaller than a cell's rasterisation box (%d nodes)", span);
        for (int i = 0; i < n; i++) {
            const double qn = q[4 * i] * q[4 * i] + q[4 * i + 1] * q[4 * i + 1] + q[4 * i + 2] * q[4 * i + 2] +
                              q[4 * i + 3] * q[4 * i + 3];
            if (!(fabs(qn - 1.0) < 1e-6)) FAIL(s, CGB_EINVAL, "quaternion %d is not a unit quaternion", i);
            for (int c = 0; c < 3; c++)
                if (!(X[3 * i + c] == X[3 * i + c])) FAIL(s, CGB_EINVAL, "position %d is not finite", i);
            if (a.wall_y && !(X[3 * i + 1] >= 0.0 && X[3 * i + 1] <= a.ny - 1)) FAIL(s, CGB_EINVAL, "cell %d outside the channel", i);
        }
    }
    HIPCHK(s, hipStreamSynchronize(s->st));
    if (n > s->ncap) {
        if (s->mem_mode != MEM_OWN) FAIL(s, CGB_EINVAL, "%d cells exceed the arena's %d", n, s->ncap);
        int rc = alloc_particles(s, n);
        if (!rc) rc = init_particle_buffers(s);
        if (rc) return rc;
    }
    a.n = n;
    // host copies, wrapped into the periodic box
    std::vector<double> Xw(3 * (size_t)std::max(n, 1), 0.0), zero(3 * (size_t)std::max(n, 1), 0.0);
    const double Lb[3] = {(double)a.nx, (double)a.ny, (double)a.nz};
    for (int i = 0; i < n; i++)
        for (int c = 0; c < 3; c++) {
            double v = X[3 * i + c];
            if (!(c == 1 && a.wall_y)) { v = fmod(v, Lb[c]); if (v < 0) v += Lb[c]; if (v >= Lb[c]) v -= Lb[c]; }
            Xw[3 * (size_t)i + c] = v;
        }
    std::vector<uint8_t> fx((size_t)std::max(n, 1), 0);
    if (fixed) for (int i = 0; i < n; i++) fx[(size_t)i] = fixed[i] ? 1 : 0;
    if (n > 0) {
        HIPCHK(s, hipMemcpyAsync(a.X, Xw.data(), 3 * (size_t)n * 8, hipMemcpyHostToDevice, s->st));
        HIPCHK(s, hipMemcpyAsync(a.Xprev, Xw.data(), 3 * (size_t)n * 8, hipMemcpyHostToDevice, s->st));
        HIPCHK(s, launch_fill_f64(a.Hprev, 3 * (long long)n, a.Rb + 1e-6, s->st));
        HIPCHK(s, hipMemcpyAsync(a.q, q, 4 * (size_t)n * 8, hipMemcpyHostToDevice, s->st));
        HIPCHK(s, hipMemcpyAsync(a.V, V ? V : zero.data(), 3 * (size_t)n * 8, hipMemcpyHostToDevice, s->st));
        HIPCHK(s, hipMemcpyAsync(a.L, L ? L : zero.data(), 3 * (size_t)n * 8, hipMemcpyHostToDevice, s->st));
        HIPCHK(s, hipMemcpyAsync(a.fixed, fx.data(), (size_t)n, hipMemcpyHostToDevice, s->st));
    }
    bind_buffers(s);
    HIPCHK(s, launch_clear_cells(a, s->st));
    HIPCHK(s, launch_prep(a, s->st));
    HIPCHK(s, launch_cells(a, s->st));  // the per-cell kernels walk the cells in cell-list order
    HIPCHK(s, launch_raster(a, s->st, true));
    HIPCHK(s, launch_transitions(a, s->st, false));
    HIPCHK(s, launch_flags_rebuild(a, s->st));
    HIPCHK(s, a.lmom ? launch_lmom(a, s->st) : launch_usol(a, s->st, true));
    HIPCHK(s, hipStreamSynchronize(s->st));
    return check_status(s);
}

int cgb_init_fluid(cgb_sim* s, const double* rho, const double* u) {
    if (!s) return CGB_EINVAL;
    DevArgs& a = s->a;
    const size_t nsb = (size_t)a.ns * 8;
    if (rho || u) {
        int rc = ensure_tmp(s, 4 * nsb);
        if (rc) return rc;
    }
    double* drho = nullptr;
    double* du = nullptr;
    if (rho) { drho = s->tmp; HIPCHK(s, hipMemcpyAsync(drho, rho, nsb, hipMemcpyHostToDevice, s->st)); }
    if (u) { du = s->tmp + a.ns; HIPCHK(s, hipMemcpyAsync(du, u, 3 * nsb, hipMemcpyHostToDevice, s->st)); }
    bind_buffers(s);
    HIPCHK(s, launch_equilibrium_fill(a, drho, du, s->st));
    // the split codec's link moments carry density parts: rebuild them for
    // the new state (every step rebuilds them before its LB as well)
    if (a.lmom && a.precision == CGB_PMX16S) HIPCHK(s, launch_lmom(a, s->st));
    HIPCHK(s, hipStreamSynchronize(s->st));
    s->fluid_ready = true;
    return CGB_OK;
}

int cgb_set_populations(cgb_sim* s, const double* d) {
    if (!s || !d) return CGB_EINVAL;
    DevArgs& a = s->a;
    const size_t bytes = 19 * (size_t)a.ns * 8;
    int rc = ensure_tmp(s, bytes);
    if (rc) return rc;
    HIPCHK(s, hipMemcpyAsync(s->tmp, d, bytes, hipMemcpyHostToDevice, s->st));
    bind_buffers(s);
    HIPCHK(s, launch_encode(a, s->tmp, s->st));
    if (a.lmom && a.precision == CGB_PMX16S) HIPCHK(s, launch_lmom(a, s->st));
    HIPCHK(s, hipStreamSynchronize(s->st));
    return CGB_OK;
}

// the side stream of the step and its two events (default priority)
static int make_side_stream(cgb_sim* s) {
    HIPCHK(s, hipStreamCreateWithFlags(&s->st_pot, hipStreamNonBlocking));
    for (hipEvent_t* e : {&s->ev_ras, &s->ev_pot}) HIPCHK(s, hipEventCreateWithFlags(e, hipEventDisableTiming));
    return CGB_OK;
}

static void drop_step_graph(cgb_sim* s) {
    if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    s->gexec = nullptr;
    s->graph = nullptr;
    s->graph_steps = 0;
}

int cgb_step(cgb_sim* s, int32_t nsteps) {
    if (!s || nsteps < 0) return CGB_EINVAL;
    if (!s->fluid_ready) FAIL(s, CGB_ESTATE, "fluid not initialised");
    DevArgs& a = s->a;
    for (int t = 0; t < nsteps; t++) {
        bind_buffers(s);
        // with cells, two streams: the cell list and the potentials need only
        // the positions and axes (after the rasterisation, whose record kernel
        // reads the previous cell list) and run beside the lattice part; the
        // integrator joins
        const bool fk = s->fork && a.n > 0;
        if (fk && !s->st_pot) {
            const int rc = make_side_stream(s);
            if (rc) return rc;
        }
        hipStream_t sp = fk ? s->st_pot : s->st;
        HIPCHK(s, timed(s, K_PREP, [&] { return launch_step_prep(a, s->st); }));
        HIPCHK(s, timed(s, K_RASTER, [&] { return launch_raster(a, s->st, false, false); }));
        if (fk) {
            HIPCHK(s, hipEventRecord(s->ev_ras, s->st));
            HIPCHK(s, hipStreamWaitEvent(sp, s->ev_ras, 0));
            HIPCHK(s, timed_on(s, K_CELLS, sp, [&] { return launch_cells(a, sp); }));
            HIPCHK(s, timed_on(s, K_POT, sp, [&] { return launch_potentials(a, sp); }));
            HIPCHK(s, hipEventRecord(s->ev_pot, sp));
        }
        HIPCHK(s, timed(s, K_TRANS, [&] {
            hipError_t e = launch_transitions(a, s->st, true);
            if (e == hipSuccess) e = a.lmom ? launch_lmom(a, s->st) : launch_usol(a, s->st, false);
            // the viscometer's seam: the populations pulled across it and Delta p_LE,z
            return e != hipSuccess ? e : launch_le(a, s->st);
        }));
        // the LB kernel also stores the link momenta of every cell node; the
        // per-cell pass sums them
        HIPCHK(s, timed(s, K_LB, [&] { return launch_lb(a, s->lbcfg, s->st); }));
        HIPCHK(s, timed(s, K_MEM, [&] { return launch_mem_reduce(a, s->st); }));
        if (a.track) HIPCHK(s, timed(s, K_TRACK, [&] { return launch_track(a, s->st); }));
        if (fk) {
            HIPCHK(s, hipStreamWaitEvent(s->st, s->ev_pot, 0));
        } else {
            HIPCHK(s, timed(s, K_CELLS, [&] { return launch_cells(a, s->st); }));
            HIPCHK(s, timed(s, K_POT, [&] { return launch_potentials(a, s->st); }));
        }
        HIPCHK(s, timed(s, K_INT, [&] { return launch_integrate(a, s->st); }));
        s->cur = 1 - s->cur;
        s->step++;
    }
    bind_buffers(s);
    return CGB_OK;
}

// Captures `steps` (even) steps into a HIP graph on the handle's stream; the
// state is left as it was.  A replay launches the whole sequence, side stream
// included, at once, instead of one launch per kernel.
int cgb_capture(cgb_sim* s, int32_t steps) {
    if (!s || steps < 2 || (steps & 1)) return CGB_EINVAL;
    if (!s->fluid_ready) FAIL(s, CGB_ESTATE, "fluid not initialised");
    if (s->prof) FAIL(s, CGB_ESTATE, "kernel timing is on: a captured sequence records none; turn it off first");
    drop_step_graph(s);
    HIPCHK(s, hipStreamSynchronize(s->st));
    if (s->fork && s->a.n > 0 && !s->st_pot) {
        const int rc = make_side_stream(s);
        if (rc) return rc;
    }
    const int cur = s->cur;
    const long long stp = s->step;
    HIPCHK(s, hipStreamBeginCapture(s->st, hipStreamCaptureModeRelaxed));
    const int rc = cgb_step(s, steps);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(s->st, &g);
    s->cur = cur;
    s->step = stp;
    bind_buffers(s);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e2 != hipSuccess) FAIL(s, CGB_EDEVICE, "end capture: %s", hipGetErrorString(e2));
    s->graph = g;
    HIPCHK(s, hipGraphInstantiate(&s->gexec, s->graph, nullptr, nullptr, 0));
    s->graph_steps = steps;
    memcpy(&s->cap_args, &s->a, sizeof(DevArgs));
    s->cap_cfg = s->lbcfg;
    s->cap_fork = s->fork;
    return CGB_OK;
}

// Replays the captured sequence nsteps / graph_steps times (asynchronous).
int cgb_replay(cgb_sim* s, int32_t nsteps) {
    if (!s || nsteps < 0) return CGB_EINVAL;
    if (!s->gexec) FAIL(s, CGB_ESTATE, "no captured steps");
    if (nsteps % s->graph_steps) FAIL(s, CGB_EINVAL, "steps must be a multiple of %d", s->graph_steps);
    if (!sim_same_args(s->a, s->cap_args) || s->lbcfg.bx != s->cap_cfg.bx || s->lbcfg.by != s->cap_cfg.by ||
        s->lbcfg.tz != s->cap_cfg.tz || s->fork != s->cap_fork)
        FAIL(s, CGB_ESTATE, "the handle changed since the capture (cells, tiles, record, concurrency, odd eager steps); capture again");
    for (int k = 0; k < nsteps / s->graph_steps; k++) HIPCHK(s, hipGraphLaunch(s->gexec, s->st));
    s->step += nsteps;
    return CGB_OK;
}

int cgb_sync(cgb_sim* s) {
    if (!s) return CGB_EINVAL;
    HIPCHK(s, hipStreamSynchronize(s->st));
    if (s->prof) harvest(s);
    return check_status(s);
}

int cgb_get_populations(cgb_sim* s, double* d) {
    if (!s || !d) return CGB_EINVAL;
    int rc = cgb_sync(s);
    if (rc && rc != CGB_EUNSTABLE) return rc;
    DevArgs& a = s->a;
    const size_t bytes = 19 * (size_t)a.ns * 8;
    int rc2 = ensure_tmp(s, bytes);
    if (rc2) return rc2;
    bind_buffers(s);
    HIPCHK(s, launch_decode(a, s->tmp, s->st));
    HIPCHK(s, hipMemcpyAsync(d, s->tmp, bytes, hipMemcpyDeviceToHost, s->st));
    HIPCHK(s, hipStreamSynchronize(s->st));
    return CGB_OK;
}

int cgb_get_box(cgb_sim* s, const int32_t* lo, const int32_t* ext, double* d, int32_t* owner) {
    if (!s || !lo || !ext) return CGB_EINVAL;
    DevArgs& a = s->a;
    const int L[3] = {a.nx, a.ny, a.nz};
    for (int c = 0; c < 3; c++)
        if (lo[c] < 0 || ext[c] < 1 || (long long)lo[c] + ext[c] > L[c]) FAIL(s, CGB_EINVAL, "box outside the lattice");
    int rc = cgb_sync(s);
    if (rc && rc != CGB_EUNSTABLE) return rc;
    const long long nb = (long long)ext[0] * ext[1] * ext[2];
    const size_t bytes = 19 * (size_t)nb * 8 + (size_t)nb * 4;
    int rc2 = ensure_tmp(s, bytes);
    if (rc2) return rc2;
    bind_buffers(s);
    const int lo3[3] = {lo[0], lo[1], lo[2]}, ex3[3] = {ext[0], ext[1], ext[2]};
    int* own = (int*)(s->tmp + 19 * nb);
    HIPCHK(s, launch_decode_box(a, lo3, ex3, s->tmp, own, s->st));
    if (d) HIPCHK(s, hipMemcpyAsync(d, s->tmp, 19 * (size_t)nb * 8, hipMemcpyDeviceToHost, s->st));
    if (owner) HIPCHK(s, hipMemcpyAsync(owner, own, (size_t)nb * 4, hipMemcpyDeviceToHost, s->st));
    HIPCHK(s, hipStreamSynchronize(s->st));
    return CGB_OK;
}

int cgb_get_mixture_box(cgb_sim* s, const int32_t* lo, const int32_t* ext, double* u) {
    if (!s || !lo || !ext || !u) return CGB_EINVAL;
    DevArgs& a = s->a;
    const int L[3] = {a.nx, a.ny, a.nz};
    for (int c = 0; c < 3; c++)
        if (lo[c] < 0 || ext[c] < 1 || (long long)lo[c] + ext[c] > L[c]) FAIL(s, CGB_EINVAL, "box outside the lattice");
    int rc = cgb_sync(s);
    if (rc && rc != CGB_EUNSTABLE) return rc;
    const long long nb = (long long)ext[0] * ext[1] * ext[2];
    int rc2 = ensure_tmp(s, 3 * (size_t)nb * 8);
    if (rc2) return rc2;
    bind_buffers(s);
    const int lo3[3] = {lo[0], lo[1], lo[2]}, ex3[3] = {ext[0], ext[1], ext[2]};
    HIPCHK(s, launch_mixture_box(a, lo3, ex3, s->tmp, s->st));
    HIPCHK(s, hipMemcpyAsync(u, s->tmp, 3 * (size_t)nb * 8, hipMemcpyDeviceToHost, s->st));
    HIPCHK(s, hipStreamSynchronize(s->st));
    return CGB_OK;
}

int cgb_get_fields(cgb_sim* s, double* rho, double* u) {
    if (!s) return CGB_EINVAL;
    int rc = cgb_sync(s);
    if (rc && rc != CGB_EUNSTABLE) return rc;
    DevArgs& a = s->a;
    const size_t nsb = (size_t)a.ns * 8;
    int rc2 = ensure_tmp(s, 4 * nsb);
    if (rc2) return rc2;
    bind_buffers(s);
    HIPCHK(s, launch_fields(a, s->tmp, s->tmp + a.ns, s->st));
    if (rho) HIPCHK(s, hipMemcpyAsync(rho, s->tmp, nsb, hipMemcpyDeviceToHost, s->st));
    if (u) HIPCHK(s, hipMemcpyAsync(u, s->tmp + a.ns, 3 * nsb, hipMemcpyDeviceToHost, s->st));
    HIPCHK(s, hipStreamSynchronize(s->st));
    return CGB_OK;
}

int cgb_get_particles(cgb_sim* s, double* X, double* q, double* V, double* L) {
    if (!s) return CGB_EINVAL;
    int rc = cgb_sync(s);
    if (rc && rc != CGB_EUNSTABLE) return rc;
    const size_t n = (size_t)s->a.n;
    if (n) {
        if (X) HIPCHK(s, hipMemcpyAsync(X, s->a.X, 3 * n * 8, hipMemcpyDeviceToHost, s->st));
        if (q) HIPCHK(s, hipMemcpyAsync(q, s->a.q, 4 * n * 8, hipMemcpyDeviceToHost, s->st));
        if (V) HIPCHK(s, hipMemcpyAsync(V, s->a.V, 3 * n * 8, hipMemcpyDeviceToHost, s->st));
        if (L) HIPCHK(s, hipMemcpyAsync(L, s->a.L, 3 * n * 8, hipMemcpyDeviceToHost, s->st));
        HIPCHK(s, hipStreamSynchronize(s->st));
    }
    return CGB_OK;
}

int cgb_get_forces(cgb_sim* s, double* Fh, double* Th, double* Fp, double* Tp) {
    if (!s) return CGB_EINVAL;
    int rc = cgb_sync(s);
    if (rc && rc != CGB_EUNSTABLE) return rc;
    const size_t n = (size_t)s->a.n;
    if (!n) return CGB_OK;
    std::vector<double> h(6 * n), pp(6 * n);
    HIPCHK(s, hipMemcpyAsync(h.data(), s->a.FTh, 6 * n * 8, hipMemcpyDeviceToHost, s->st));
    HIPCHK(s, hipMemcpyAsync(pp.data(), s->a.FTp, 6 * n * 8, hipMemcpyDeviceToHost, s->st));
    HIPCHK(s, hipStreamSynchronize(s->st));
    for (size_t i = 0; i < n; i++)
        for (int c = 0; c < 3; c++) {
            if (Fh) Fh[3 * i + c] = h[6 * i + c];
            if (Th) Th[3 * i + c] = h[6 * i + 3 + c];
            if (Fp) Fp[3 * i + c] = pp[6 * i + c];
            if (Tp) Tp[3 * i + c] = pp[6 * i + 3 + c];
        }
    return CGB_OK;
}

int cgb_get_owner(cgb_sim* s, int32_t* owner) {
    if (!s || !owner) return CGB_EINVAL;
    int rc = cgb_sync(s);
    if (rc && rc != CGB_EUNSTABLE) return rc;
    HIPCHK(s, hipMemcpyAsync(owner, s->a.owner, (size_t)s->a.ns * 4, hipMemcpyDeviceToHost, s->st));
    HIPCHK(s, hipStreamSynchronize(s->st));
    return CGB_OK;
}

int cgb_get_link_mask(cgb_sim* s, uint32_t* mask) {
    if (!s || !mask) return CGB_EINVAL;
    int rc = cgb_sync(s);
    if (rc && rc != CGB_EUNSTABLE) return rc;
    HIPCHK(s, hipMemcpyAsync(mask, s->a.flags, (size_t)s->a.ns * 4, hipMemcpyDeviceToHost, s->st));
    HIPCHK(s, hipStreamSynchronize(s->st));
    for (long long i = 0; i < s->a.ns; i++) mask[i] = (mask[i] & NONFLUID) ? 0u : (mask[i] & LINKBITS);
    return CGB_OK;
}

int cgb_get_pairs(cgb_sim* s, int32_t* ij, int64_t cap, int64_t* n) {
    if (!s || !n) return CGB_EINVAL;
    int rc = cgb_sync(s);
    if (rc && rc != CGB_EUNSTABLE) return rc;
    DevArgs& a = s->a;
    const int want = std::max(1024, 64 * a.n);
    if (want > s->pair_cap && s->mem_mode == MEM_OWN) {
        dfree(s, s->pair_buf);
        s->pair_buf = nullptr;
        if (!s->pair_cnt) HIPCHK(s, dalloc(s, &s->pair_cnt, 16));
        HIPCHK(s, dalloc(s, &s->pair_buf, (size_t)want * 2 * 4));
        s->pair_cap = want;
    }
    HIPCHK(s, launch_cells(a, s->st));
    HIPCHK(s, launch_pairs(a, s->pair_buf, s->pair_cnt, s->pair_cap, s->st));
    int cnt = 0;
    HIPCHK(s, hipMemcpyAsync(&cnt, s->pair_cnt, 4, hipMemcpyDeviceToHost, s->st));
    HIPCHK(s, hipStreamSynchronize(s->st));
    if (cnt > s->pair_cap) FAIL(s, CGB_ENOMEM, "pair buffer overflow (%d pairs)", cnt);
    std::vector<int> buf(2 * (size_t)cnt);
    if (cnt) HIPCHK(s, hipMemcpy(buf.data(), s->pair_buf, 2 * (size_t)cnt * 4, hipMemcpyDeviceToHost));
    std::vector<std::pair<int, int>> pr((size_t)cnt);
    for (int k = 0; k < cnt; k++) pr[(size_t)k] = {buf[2 * (size_t)k], buf[2 * (size_t)k + 1]};
    std::sort(pr.begin(), pr.end());
    *n = cnt;
    if (ij)
        for (int64_t k = 0; k < std::min<int64_t>(cap, cnt); k++) {
            ij[2 * k] = pr[(size_t)k].first;
            ij[2 * k + 1] = pr[(size_t)k].second;
        }
    return CGB_OK;
}

int cgb_get_observables(cgb_sim* s, double* out) {
    if (!s || !out) return CGB_EINVAL;
    int rc = cgb_sync(s);
    if (rc && rc != CGB_EUNSTABLE) return rc;
    DevArgs& a = s->a;
    bind_buffers(s);
    HIPCHK(s, launch_observables(a, s->obs_partial, s->obs_nblk, s->st));
    std::vector<double> part((size_t)s->obs_nblk * 8);
    const int nbb = (a.n + 255) / 256;
    std::vector<double> bpart(3 * (size_t)std::max(nbb, 1), 0.0);
    double bp[3] = {0, 0, 0};
    int bad = 0;
    HIPCHK(s, hipMemcpyAsync(part.data(), s->obs_partial, part.size() * 8, hipMemcpyDeviceToHost, s->st));
    if (nbb) HIPCHK(s, hipMemcpyAsync(bpart.data(), a.body_part, 3 * (size_t)nbb * 8, hipMemcpyDeviceToHost, s->st));
    HIPCHK(s, hipMemcpyAsync(&bad, a.bad_step, 4, hipMemcpyDeviceToHost, s->st));
    std::vector<double> V(3 * (size_t)a.n);
    std::vector<uint8_t> fx((size_t)a.n);
    if (a.n) {
        HIPCHK(s, hipMemcpyAsync(V.data(), a.V, V.size() * 8, hipMemcpyDeviceToHost, s->st));
        HIPCHK(s, hipMemcpyAsync(fx.data(), a.fixed, fx.size(), hipMemcpyDeviceToHost, s->st));
    }
    HIPCHK(s, hipStreamSynchronize(s->st));
    for (int b = 0; b < nbb; b++)
        for (int c = 0; c < 3; c++) bp[c] += bpart[3 * (size_t)b + c];
    double acc[8] = {0};
    for (int b = 0; b < s->obs_nblk; b++)
        for (int k = 0; k < 8; k++) acc[k] += part[8 * (size_t)b + k];
    double pm[3] = {0, 0, 0};
    for (int i = 0; i < a.n; i++)
        if (!fx[(size_t)i]) for (int c = 0; c < 3; c++) pm[c] += a.M * V[3 * (size_t)i + c];
    out[0] = acc[0];
    for (int c = 0; c < 3; c++) {
        out[1 + c] = acc[1 + c];
        out[4 + c] = pm[c];
        out[8 + c] = (s->step > 0 ? acc[5 + c] : 0.0) + bp[c];
    }
    out[7] = acc[4];
    out[11] = (double)s->step;
    out[12] = bad == 0x7fffffff ? -1.0 : (double)bad;
    return CGB_OK;
}

int cgb_get_profile(cgb_sim* s, int32_t axis, double* prof) {
    if (!s || !prof || axis < 0 || axis > 2) return CGB_EINVAL;
    int rc = cgb_sync(s);
    if (rc && rc != CGB_EUNSTABLE) return rc;
    DevArgs& a = s->a;
    const int np = axis == 0 ? a.nx : (axis == 1 ? a.ny : a.nz);
    int rc2 = ensure_tmp(s, 2 * (size_t)np * 8);
    if (rc2) return rc2;
    bind_buffers(s);
    HIPCHK(s, launch_kin(a, s->st));
    HIPCHK(s, launch_fill_f64(s->tmp, 2 * (long long)np, 0.0, s->st));
    HIPCHK(s, launch_profile_z(a, s->tmp, s->tmp + np, s->st, axis));
    std::vector<double> h(2 * (size_t)np);
    HIPCHK(s, hipMemcpyAsync(h.data(), s->tmp, h.size() * 8, hipMemcpyDeviceToHost, s->st));
    HIPCHK(s, hipStreamSynchronize(s->st));
    for (int k = 0; k < np; k++) prof[k] = h[(size_t)np + k] > 0 ? h[(size_t)k] / h[(size_t)np + k] : 0.0;
    return CGB_OK;
}

int cgb_get_profile_z(cgb_sim* s, double* prof) { return cgb_get_profile(s, 1, prof); }

int cgb_get_le_flux(cgb_sim* s, double* out, int32_t cap, int32_t* n) {
    if (!s || !n || cap < 0 || (cap > 0 && !out)) return CGB_EINVAL;
    HIPCHK(s, hipStreamSynchronize(s->st));
    const DevArgs& a = s->a;
    if (a.le_u == 0.0) FAIL(s, CGB_EINVAL, "not a viscometer lattice (le_u = 0)");
    int cnt = 0;
    HIPCHK(s, hipMemcpy(&cnt, a.track_n, 4, hipMemcpyDeviceToHost));
    *n = std::min(cnt, a.track_cap);
    const int m = std::min(*n, (int)cap);
    if (m > 0 && a.le_rec) HIPCHK(s, hipMemcpy(out, a.le_rec, (size_t)m * 8, hipMemcpyDeviceToHost));
    return CGB_OK;
}

int cgb_mu_app_le(const double* flux, int32_t n, int32_t first, const double* prof_x, int32_t nx, int32_t ny,
                  int32_t nz, double rho0, double tau, double* mu_rel) {
    if (!flux || !prof_x || !mu_rel || first < 0 || n <= first || nx < 4 || ny < 1 || nz < 1 || !(rho0 > 0) ||
        !(tau > 0.5))
        return CGB_EINVAL;
    // least-squares slope of the profile over the central half of the planes
    const int x0 = nx / 4, x1 = 3 * nx / 4;
    double sx = 0, sy = 0, sxx = 0, sxy = 0;
    const double m = x1 - x0;
    for (int x = x0; x < x1; x++) { sx += x; sy += prof_x[x]; sxx += (double)x * x; sxy += x * prof_x[x]; }
    const double gd = (m * sxy - sx * sy) / (m * sxx - sx * sx);
    double dp = 0;
    for (int t = first; t < n; t++) dp += flux[t];
    dp /= (n - first);
    const double nu = (2.0 * tau - 1.0) / 6.0;
    *mu_rel = dp / ((double)ny * nz * gd) / (rho0 * nu);
    return CGB_OK;
}

int cgb_set_concurrency(cgb_sim* s, int on) {
    if (!s) return CGB_EINVAL;
    HIPCHK(s, hipStreamSynchronize(s->st));
    s->fork = on != 0;
    return CGB_OK;
}

int cgb_profile(cgb_sim* s, int enable) {
    if (!s) return CGB_EINVAL;
    HIPCHK(s, hipStreamSynchronize(s->st));
    harvest(s);
    if (enable) {
        for (int k = 0; k < K_NKIND; k++) { s->ktime[k] = 0; s->kcount[k] = 0; }
    }
    s->prof = enable != 0;
    return CGB_OK;
}

int cgb_kernel_times(cgb_sim* s, char* names, double* ms, int64_t* count, int32_t cap, int32_t* n) {
    if (!s || !n) return CGB_EINVAL;
    HIPCHK(s, hipStreamSynchronize(s->st));
    harvest(s);
    int k = 0;
    for (; k < K_NKIND && k < cap; k++) {
        if (names) { memset(names + 64 * k, 0, 64); strncpy(names + 64 * k, kKindNames[k], 63); }
        if (ms) ms[k] = s->ktime[k];
        if (count) count[k] = s->kcount[k];
    }
    *n = k;
    return CGB_OK;
}

// ---------------------------------------------------------------- tiles
int cgb_set_tiles(cgb_sim* s, int32_t bx, int32_t by, int32_t tz) {
    if (!s) return CGB_EINVAL;
    const int nt = by == 0 ? bx : bx * by;  // by = 0: plane-linear tiles of bx sites
    if (bx < 1 || by < 0 || nt > 256 || nt % 64 != 0 || !(tz == 4 || tz == 8 || tz == 16 || tz == 32))
        FAIL(s, CGB_EINVAL, "tile %dx%dx%d: need bx*by (bx when by = 0) a multiple of 64, at most 256, tz in {4,8,16,32}", bx, by, tz);
    if (by == 0 && s->a.tau != 1.0)
        FAIL(s, CGB_EINVAL, "tile %dx0x%d: plane-linear tiles need tau = 1", bx, tz);
    if ((s->a.big || s->a.cidx) && tz != 16)
        FAIL(s, CGB_EINVAL, "tile %dx%dx%d: the large-lattice and indexed layouts sweep 16 nodes (tz = 16)", bx, by, tz);
    HIPCHK(s, hipStreamSynchronize(s->st));
    set_tiles(s, LaunchCfg{bx, by, tz});
    // more LB blocks than mixture-record partials: own memory grows; in
    // caller-provided memory the record falls back to its own pass
    const long long nb = lb_blocks(s->a);
    if (s->mem_mode == MEM_OWN && nb > s->a.track_slots && nb < (1LL << 31)) {
        double* np = nullptr;
        HIPCHK(s, dalloc(s, &np, (size_t)nb * 2 * 8));
        dfree(s, s->a.track_part);
        s->a.track_part = np;
        s->a.track_slots = (int)nb;
    }
    return CGB_OK;
}

// Times the fused LB kernel alone on the current state: it reads the current
// populations, flags and boundary velocities and writes only buffers that the
// next step rewrites before reading (the other population buffer and its
// density field), so the state is unchanged.
int cgb_time_lb(cgb_sim* s, int32_t reps, double* ms_avg) {
    if (!s || reps < 1 || !ms_avg) return CGB_EINVAL;
    if (!s->fluid_ready) FAIL(s, CGB_ESTATE, "fluid not initialised");
    HIPCHK(s, hipStreamSynchronize(s->st));
    if (s->prof) harvest(s);
    bind_buffers(s);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    for (int k = 0; k < 2 && e == hipSuccess; k++) e = launch_lb(s->a, s->lbcfg, s->st);
    if (e == hipSuccess) e = hipEventRecord(e0, s->st);
    for (int k = 0; k < reps && e == hipSuccess; k++) e = launch_lb(s->a, s->lbcfg, s->st);
    if (e == hipSuccess) e = hipEventRecord(e1, s->st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    HIPCHK(s, e);
    *ms_avg = (double)ms / reps;
    return CGB_OK;
}

// ---------------------------------------------------------------- mixture record
int cgb_track(cgb_sim* s, int32_t cap) {
    if (!s || cap < 0) return CGB_EINVAL;
    HIPCHK(s, hipStreamSynchronize(s->st));
    DevArgs& a = s->a;
    if (s->mem_mode != MEM_OWN) {
        if (cap > s->track_max) FAIL(s, CGB_EINVAL, "%d steps exceed the arena's record of %d", cap, s->track_max);
        a.track = cap > 0 ? s->track_buf : nullptr;
        a.le_rec = cap > 0 ? s->le_rec_buf : nullptr;
        a.track_cap = cap;
    } else {
        dfree(s, a.track);
        dfree(s, a.le_rec);
        a.track = nullptr;
        a.le_rec = nullptr;
        a.track_cap = 0;
        if (cap > 0) {
            HIPCHK(s, dalloc(s, &a.track, 2 * (size_t)cap * 8));
            if (a.le_u != 0.0) HIPCHK(s, dalloc(s, &a.le_rec, (size_t)cap * 8));
            a.track_cap = cap;
        }
    }
    HIPCHK(s, launch_fill_i32(a.track_n, 1, 0, s->st));
    HIPCHK(s, hipStreamSynchronize(s->st));
    return CGB_OK;
}

int cgb_get_track(cgb_sim* s, double* out, int32_t cap, int32_t* n) {
    if (!s || !n || cap < 0 || (cap > 0 && !out)) return CGB_EINVAL;
    HIPCHK(s, hipStreamSynchronize(s->st));
    const DevArgs& a = s->a;
    int cnt = 0;
    HIPCHK(s, hipMemcpy(&cnt, a.track_n, 4, hipMemcpyDeviceToHost));
    const int m = std::min(std::min(cnt, a.track_cap), (int)cap);
    *n = std::min(cnt, a.track_cap);
    if (m > 0) {
        HIPCHK(s, hipMemcpy(out, a.track, 2 * (size_t)m * 8, hipMemcpyDeviceToHost));
        for (int k = 0; k < m; k++) {
            out[2 * k] *= 2.0 / s->n_nonwall;
            out[2 * k + 1] /= s->n_nonwall;
        }
    }
    return CGB_OK;
}

int cgb_mu_rel_kolmogorov(const double* A, int32_t n, int32_t first, double f0, double rho0, int32_t ny, double* mu) {
    if (!A || !mu || first < 0 || n - 1 <= first || ny < 3 || !(rho0 > 0)) return CGB_EINVAL;
    const double k = 2.0 * M_PI / ny, ck = cos(k);
    double sum = 0.0;
    for (int t = first; t < n - 1; t++)
        sum += (f0 * (5.0 + ck) / (6.0 * rho0) - (A[t + 1] - A[t])) / (A[t] * (1.0 - ck) / 3.0);
    *mu = sum / (n - 1 - first);
    return CGB_OK;
}

int cgb_mu_rel_slit(const double* ubar, int32_t n, int32_t first, double g, double tau, int32_t ny, double* mu) {
    if (!ubar || !mu || first < 0 || n <= first || ny < 3 || !(tau > 0.5)) return CGB_EINVAL;
    double u = 0.0;
    for (int t = first; t < n; t++) u += ubar[t];
    u /= (n - first);
    const double nf = ny - 2, nu = (2.0 * tau - 1.0) / 6.0, lam = (tau - 0.5) * (tau - 0.5);
    *mu = g * (nf * nf + 8.0 * lam - 1.0) / (12.0 * nu * u);
    return CGB_OK;
}

int cgb_mu_rel(cgb_sim* s, int32_t first, double* mu) {
    if (!s || !mu) return CGB_EINVAL;
    const cgb_params& P = s->P;
    if (P.le_u != 0.0) {
        int n = 0;
        int rc = cgb_get_le_flux(s, nullptr, 0, &n);
        if (rc) return rc;
        std::vector<double> fl((size_t)std::max(n, 1)), prof((size_t)P.nx);
        rc = cgb_get_le_flux(s, fl.data(), n, &n);
        if (!rc) rc = cgb_get_profile(s, 0, prof.data());
        if (rc) return rc;
        rc = cgb_mu_app_le(fl.data(), n, first, prof.data(), P.nx, P.ny, P.nz, P.rho0, P.tau, mu);
        if (rc) FAIL(s, rc, "too few recorded steps (%d) after step %d", n, first);
        return CGB_OK;
    }
    const bool kolm = P.force_mode == 2 && !P.wall_y;
    const bool slit = P.force_mode == 1 && P.wall_y && P.g[0] == 0.0 && P.g[1] == 0.0 && P.g[2] != 0.0 &&
                      !(P.force_zhi > P.force_zlo);
    if (!kolm && !slit) FAIL(s, CGB_EINVAL, "no apparent-viscosity estimator for this driving");
    // the Kolmogorov estimator's one-step map (decay (1 - cos k)/3, forcing
    // (5 + cos k)/6) is the exact map at tau = 1 only
    if (kolm && P.tau != 1.0) FAIL(s, CGB_EINVAL, "the Kolmogorov estimator holds at tau = 1 only (tau = %g)", P.tau);
    int n = 0;
    int rc = cgb_get_track(s, nullptr, 0, &n);
    if (rc) return rc;
    std::vector<double> tr(2 * (size_t)std::max(n, 1));
    rc = cgb_get_track(s, tr.data(), n, &n);
    if (rc) return rc;
    std::vector<double> series((size_t)std::max(n, 1));
    for (int k = 0; k < n; k++) series[(size_t)k] = tr[2 * (size_t)k + (kolm ? 0 : 1)];
    rc = kolm ? cgb_mu_rel_kolmogorov(series.data(), n, first, P.f0, P.rho0, P.ny, mu)
              : cgb_mu_rel_slit(series.data(), n, first, P.g[2], P.tau, P.ny, mu);
    if (rc) FAIL(s, rc, "too few recorded steps (%d) after step %d", n, first);
    return CGB_OK;
}

int cgb_get_tiles(cgb_sim* s, int32_t* t) {
    if (!s || !t) return CGB_EINVAL;
    t[0] = s->lbcfg.bx; t[1] = s->lbcfg.by; t[2] = s->lbcfg.tz;
    return CGB_OK;
}

// ---------------------------------------------------------------- checkpoint
static const char kMagic[8] = {'C', 'G', 'B', 'C', 'K', 'P', 'T', '1'};

int cgb_save(cgb_sim* s, const char* path) {
    if (!s || !path) return CGB_EINVAL;
    int rc = cgb_sync(s);
    if (rc) return rc;
    DevArgs& a = s->a;
    FILE* f = fopen(path, "wb");
    if (!f) FAIL(s, CGB_EINVAL, "cannot open %s", path);
    const size_t popb = 19 * (size_t)a.pstride * s->esize, rhob = (size_t)a.pstride * s->esize;
    std::vector<char> buf(std::max(popb, (size_t)a.ns * 4));
    bool ok = fwrite(kMagic, 1, 8, f) == 8 && fwrite(&s->P, sizeof s->P, 1, f) == 1 &&
              fwrite(&a.n, 4, 1, f) == 1 && fwrite(&s->step, 8, 1, f) == 1;
    auto dump = [&](const void* dev, size_t bytes) {
        if (!ok) return;
        if (hipMemcpy(buf.data(), dev, bytes, hipMemcpyDeviceToHost) != hipSuccess) { ok = false; return; }
        ok = fwrite(buf.data(), 1, bytes, f) == bytes;
    };
    dump(s->pop[s->cur], popb);
    dump(s->rho[s->cur], rhob);
    dump(a.owner, (size_t)a.ns * 4);
    dump(a.flags, (size_t)a.ns * 4);
    if (a.n) {
        const size_t n = (size_t)a.n;
        dump(a.X, 3 * n * 8); dump(a.q, 4 * n * 8); dump(a.V, 3 * n * 8); dump(a.L, 3 * n * 8);
        dump(a.fixed, n); dump(a.Xprev, 3 * n * 8); dump(a.Hprev, 3 * n * 8);
    }
    fclose(f);
    if (!ok) FAIL(s, CGB_EDEVICE, "write to %s failed", path);
    return CGB_OK;
}

int cgb_load(cgb_sim* s, const char* path) {
    if (!s || !path) return CGB_EINVAL;
    HIPCHK(s, hipStreamSynchronize(s->st));
    DevArgs& a = s->a;
    FILE* f = fopen(path, "rb");
    if (!f) FAIL(s, CGB_EINVAL, "cannot open %s", path);
    char mg[8];
    cgb_params P;
    int n = 0;
    long long step = 0;
    bool ok = fread(mg, 1, 8, f) == 8 && memcmp(mg, kMagic, 8) == 0 && fread(&P, sizeof P, 1, f) == 1 &&
              fread(&n, 4, 1, f) == 1 && fread(&step, 8, 1, f) == 1;
    if (!ok || P.nx != s->P.nx || P.ny != s->P.ny || P.nz != s->P.nz || P.precision != s->P.precision) {
        fclose(f);
        FAIL(s, CGB_EINVAL, "checkpoint %s does not match this lattice", path);
    }
    if (n > s->ncap) {
        if (s->mem_mode != MEM_OWN) { fclose(f); FAIL(s, CGB_EINVAL, "%d cells exceed the arena's %d", n, s->ncap); }
        int rc = alloc_particles(s, n);
        if (!rc) rc = init_particle_buffers(s);
        if (rc) { fclose(f); return rc; }
    }
    a.n = n;
    const size_t popb = 19 * (size_t)a.pstride * s->esize, rhob = (size_t)a.pstride * s->esize;
    std::vector<char> buf(std::max(popb, (size_t)a.ns * 4));
    auto load = [&](void* dev, size_t bytes) {
        if (!ok) return;
        ok = fread(buf.data(), 1, bytes, f) == bytes;
        if (ok) ok = hipMemcpy(dev, buf.data(), bytes, hipMemcpyHostToDevice) == hipSuccess;
    };
    load(s->pop[s->cur], popb);
    load(s->rho[s->cur], rhob);
    load(a.owner, (size_t)a.ns * 4);
    load(a.flags, (size_t)a.ns * 4);
    if (n) {
        const size_t nn = (size_t)n;
        load(a.X, 3 * nn * 8); load(a.q, 4 * nn * 8); load(a.V, 3 * nn * 8); load(a.L, 3 * nn * 8);
        load(a.fixed, nn); load(a.Xprev, 3 * nn * 8); load(a.Hprev, 3 * nn * 8);
    }
    fclose(f);
    if (!ok) FAIL(s, CGB_EINVAL, "checkpoint %s is truncated", path);
    s->step = step;
    s->fluid_ready = true;
    bind_buffers(s);
    HIPCHK(s, launch_fill_i32(a.dstep, 1, (int)step - 1, s->st));
    HIPCHK(s, launch_fill_i32(a.cand, a.ns, NO_CAND, s->st));
    HIPCHK(s, launch_cells(a, s->st));
    // boundary data of the loaded state (the next step recomputes it; a timed
    // LB launch before that step reads it)
    HIPCHK(s, launch_kin(a, s->st));
    HIPCHK(s, a.lmom ? launch_lmom(a, s->st) : launch_usol(a, s->st, true));
    HIPCHK(s, hipStreamSynchronize(s->st));
    return CGB_OK;
}

}  // extern "C"

namespace cgb {
int sim_set_tiles(cgb_sim* s, LaunchCfg cfg) { return cgb_set_tiles(s, cfg.bx, cfg.by, cfg.tz); }
void sim_bind(cgb_sim* s) { bind_buffers(s); }
}  // namespace cgb
