// lb.hip -- fused pull stream + bounce-back + BGK collision + momentum exchange.
//
// For a fluid node x and each direction r the pulled population is
// n*_r(x - c_r) when the source is fluid (Eq. 2); when the source is a wall or
// a cell node it is the node's own post-collision n*_rbar(x) (mid-link
// bounce-back, Eq. 9) plus, for a moving boundary, the correction of Eq. 10,
// C = 6 w_r rho(x) (c_r . v_b), with rho(x) the node's density at the time of
// the bounced populations.  For a cell, v_b = V + Omega x (x - c_r/2 - X) at
// the link midpoint; since c_r . (Omega x c_r) = 0 this equals c_r . U with
// U = V + Omega x (x - X), the rigid-body velocity at the fluid node, which is
// computed once per (node, cell).  The transferred momentum (2 n*_rbar + C)
// c_rbar (Eq. 12) is summed per cell in FP64.  Only its part (2 d_rbar + C)
// c_rbar that depends on the deviations d = n* - w rho0 is summed: the
// constant part 2 w rho0 c_rbar, together with the particle-particle and
// particle-wall link forces of Eqs. 13-14, sums to exactly zero over the
// closed surface of a cell's node set (the sums of w c and of (x - X) x w c
// over the outward links of any node set vanish), so the two forms are the
// same force.  Collision: Eqs. 1, 4, 5 with the Guo forcing term,
// u = (sum n c + g/2)/rho.
//
// Work decomposition: a workgroup owns a tile of BX x BY x TZ nodes; each
// thread sweeps TZ nodes along z.  Momentum exchange: each lane keeps one
// (cell, F, T) accumulator that follows it along z; when the cell changes the
// accumulator is added into a per-workgroup LDS hash table (FP64 LDS atomics).
// At the end the table is written, with plain stores, to a per-cell slot
// indexed by the tile's position relative to the cell's footprint (no device
// atomics); a gather kernel sums the slots of each cell.
#include "cgb_dev.h"

namespace cgb {

constexpr int TAB_CAP = 512;

// velocity components of a direction known only at run time, from bit masks
// of the directions with component +1 and -1
__host__ __device__ constexpr uint32_t comp_mask(int axis, int sign) {
    uint32_t m = 0;
    for (int r = 0; r < 19; r++) {
        const int c = axis == 0 ? CX(r) : (axis == 1 ? CY(r) : CZ(r));
        if (c == sign) m |= 1u << r;
    }
    return m;
}
// direction sets for the link geometry: axis links (|c| = 1) and diagonal
// links with component +1 / -1 along each axis, and diagonals by the sign of
// the product of two components
__host__ __device__ constexpr uint32_t dir_mask(int axis, int sign, bool diag) {
    uint32_t m = 0;
    for (int r = 1; r < 19; r++) {
        const int c = axis == 0 ? CX(r) : (axis == 1 ? CY(r) : CZ(r));
        const bool is_diag = r >= 7;
        if (c == sign && is_diag == diag) m |= 1u << r;
    }
    return m;
}
__host__ __device__ constexpr uint32_t prod_mask(int a0, int a1, int sign) {
    uint32_t m = 0;
    for (int r = 1; r < 19; r++) {
        const int c0 = a0 == 0 ? CX(r) : (a0 == 1 ? CY(r) : CZ(r));
        const int c1 = a1 == 0 ? CX(r) : (a1 == 1 ? CY(r) : CZ(r));
        if (c0 * c1 == sign) m |= 1u << r;
    }
    return m;
}
constexpr uint32_t AXP0 = dir_mask(0, 1, false), AXM0 = dir_mask(0, -1, false);
constexpr uint32_t AXP1 = dir_mask(1, 1, false), AXM1 = dir_mask(1, -1, false);
constexpr uint32_t AXP2 = dir_mask(2, 1, false), AXM2 = dir_mask(2, -1, false);
constexpr uint32_t DGP0 = dir_mask(0, 1, true), DGM0 = dir_mask(0, -1, true);
constexpr uint32_t DGP1 = dir_mask(1, 1, true), DGM1 = dir_mask(1, -1, true);
constexpr uint32_t DGP2 = dir_mask(2, 1, true), DGM2 = dir_mask(2, -1, true);
constexpr uint32_t SXYP = prod_mask(0, 1, 1), SXYM = prod_mask(0, 1, -1);
constexpr uint32_t SXZP = prod_mask(0, 2, 1), SXZM = prod_mask(0, 2, -1);
constexpr uint32_t SYZP = prod_mask(1, 2, 1), SYZM = prod_mask(1, 2, -1);

__device__ inline int cxr(int r) { return (int)((comp_mask(0, 1) >> r) & 1u) - (int)((comp_mask(0, -1) >> r) & 1u); }
__device__ inline int cyr(int r) { return (int)((comp_mask(1, 1) >> r) & 1u) - (int)((comp_mask(1, -1) >> r) & 1u); }
__device__ inline int czr(int r) { return (int)((comp_mask(2, 1) >> r) & 1u) - (int)((comp_mask(2, -1) >> r) & 1u); }

__device__ inline unsigned tab_hash(int p) { return ((unsigned)p * 2654435761u) >> (32 - 9); }

struct LdsTable {
    int key[TAB_CAP];
    double val[6][TAB_CAP];
};

// tile offset of the block relative to the footprint of cell p (one axis)
__device__ inline int foot_lo(const DevArgs& a, int axis, double Xc) {
    const int n = axis == 0 ? a.nx : (axis == 1 ? a.ny : a.nz);
    int lo = (int)floor(Xc - a.Rb) - 1;
    if (axis == 1 && a.wall_y) return lo < 0 ? 0 : lo;
    lo %= n;
    return lo < 0 ? lo + n : lo;
}

__device__ inline int slot_of(const DevArgs& a, int p, const int* tile) {
    const double* k = a.kin + 12 * (long long)p;
    int slot = 0, mul = 1;
    for (int c = 0; c < 3; c++) {
        const int t0 = foot_lo(a, c, k[c]) / a.tile[c];
        int off = tile[c] - t0;
        if (off < 0) off += a.ntile[c];
        if (off >= a.slots[c]) return -1;
        slot += off * mul;
        mul *= a.slots[c];
    }
    return slot;
}

__device__ inline void global_add6(const DevArgs& a, int p, const double* v) {
    double* F = a.FTh + 6 * (long long)p;
    for (int c = 0; c < 6; c++) unsafeAtomicAdd(F + c, v[c]);
}

__device__ inline void table_add(LdsTable& tb, const DevArgs& a, int p, const double* v) {
    unsigned h = tab_hash(p);
    for (int probe = 0; probe < TAB_CAP; probe++) {
        int old = __hip_atomic_load(&tb.key[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (old == -1) old = atomicCAS(&tb.key[h], -1, p);
        if (old == -1 || old == p) {
            for (int c = 0; c < 6; c++) unsafeAtomicAdd(&tb.val[c][h], v[c]);
            return;
        }
        h = (h + 1) & (TAB_CAP - 1);
    }
    global_add6(a, p, v);  // table full: direct device atomics
}

template <int P, int TZ>
__global__ void __launch_bounds__(256) lb_kernel_tau(DevArgs a) {
    using Cd = Codec<P>;
    using T = typename Cd::T;
    using R = typename Cd::R;
    __shared__ LdsTable tb;
    const int nthr = blockDim.x * blockDim.y;
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    for (int e = tid; e < TAB_CAP; e += nthr) {
        tb.key[e] = -1;
        for (int c = 0; c < 6; c++) tb.val[c][e] = 0.0;
    }
    __syncthreads();

    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z0 = blockIdx.z * TZ;
    const bool inb = (x < a.nx) && (y < a.ny);
    const unsigned nx = (unsigned)a.nx;
    const unsigned plane = (unsigned)a.nx * (unsigned)a.ny;
    const T* __restrict__ A = (const T*)a.A;
    T* __restrict__ B = (T*)a.B;
    const unsigned ps = (unsigned)a.pstride;  // 19 * pstride < 2^32 (checked at create)
    // offset from x to the pull source x - c along each axis (periodic wrap);
    // index 0: c = -1, 1: c = 0, 2: c = +1
    const int ox[3] = {x == a.nx - 1 ? -(a.nx - 1) : 1, 0, x == 0 ? a.nx - 1 : -1};
    const int oy[3] = {y == a.ny - 1 ? -(int)((a.ny - 1) * nx) : (int)nx, 0, y == 0 ? (int)((a.ny - 1) * nx) : -(int)nx};
    double gy[3];
    body_force(a, (double)y, gy);
    const R gx = (R)gy[0], gyy = (R)gy[1], gz = (R)gy[2];
    const R omega = (R)(1.0 / a.tau);
    const R pref = (R)(1.0 - 0.5 / a.tau);

    int spid = -1;
    double acc[6] = {0, 0, 0, 0, 0, 0};

    for (int zz = 0; zz < TZ; zz++) {
        const int z = z0 + zz;
        if (z >= a.nz) break;
        const unsigned i = (unsigned)x + nx * (unsigned)y + plane * (unsigned)z;
        const uint32_t f = inb ? a.flags[i] : NONFLUID;
        if (f & NONFLUID) continue;
        const int oz[3] = {z == a.nz - 1 ? -(int)((a.nz - 1) * plane) : (int)plane, 0,
                           z == 0 ? (int)((a.nz - 1) * plane) : -(int)plane};
#define SRC(r) (i + (unsigned)(ox[CX(r) + 1] + oy[CY(r) + 1] + oz[CZ(r) + 1]))

        // pull; a non-fluid source bounces the node's own opposite population
        R d[19];
#pragma unroll
        for (int r = 0; r < 19; r++) {
            const bool bb = (f >> r) & 1u;
            const T v = A[bb ? (unsigned)OPP(r) * ps + i : (unsigned)r * ps + SRC(r)];
            d[r] = Cd::dec(v, dec_scale<P>(a, r));
        }

        const uint32_t links = f & LINKBITS;
        if (links) {
            // link bits whose source belongs to a cell (walls are the rest);
            // walked bit by bit so that no source address stays live
            uint32_t pmask = 0;
            for (uint32_t m = links; m; m &= m - 1) {
                const int r = __builtin_ctz(m);
                if (a.owner[i + (unsigned)(ox[1 + cxr(r)] + oy[1 + cyr(r)] + oz[1 + czr(r)])] >= 0) pmask |= 1u << r;
            }
            const uint32_t wl = a.moving_walls ? (links & ~pmask) : 0u;
            double rho_x = 0.0;
            if (pmask | wl) rho_x = a.rho0 + (double)Cd::dec(((const T*)a.rhoA)[i], rho_dec_scale<P>(a));
            while (pmask) {
                // the cell behind the lowest remaining link and all of its links
                const int r0 = __builtin_ctz(pmask);
                const int p = a.owner[i + (unsigned)(ox[1 + cxr(r0)] + oy[1 + cyr(r0)] + oz[1 + czr(r0)])];
                uint32_t sub = 1u << r0;
                for (uint32_t m = pmask & (pmask - 1); m; m &= m - 1) {
                    const int r = __builtin_ctz(m);
                    if (a.owner[i + (unsigned)(ox[1 + cxr(r)] + oy[1 + cyr(r)] + oz[1 + czr(r)])] == p) sub |= 1u << r;
                }
                pmask &= ~sub;
                const double* k = a.kin + 12 * (size_t)p;
                const double l0 = min_image((double)x - k[0], (double)a.nx);
                const double l1 = a.wall_y ? ((double)y - k[1]) : min_image((double)y - k[1], (double)a.ny);
                const double l2 = min_image((double)z - k[2], (double)a.nz);
                const double U0 = k[3] + (k[7] * l2 - k[8] * l1);
                const double U1 = k[4] + (k[8] * l0 - k[6] * l2);
                const double U2 = k[5] + (k[6] * l1 - k[7] * l0);
                const double rc = 6.0 * rho_x;
                double F0 = 0.0, F1 = 0.0, F2 = 0.0;
#pragma unroll
                for (int r = 1; r < 19; r++) {
                    if ((sub >> r) & 1u) {
                        const double cu = CX(r) * U0 + CY(r) * U1 + CZ(r) * U2;
                        const double C = WD(r) * rc * cu;
                        const double dyn = 2.0 * (double)d[r] + C;
                        F0 -= dyn * CX(r); F1 -= dyn * CY(r); F2 -= dyn * CZ(r);
                        d[r] = d[r] + (R)C;
                    }
                }
                if (p != spid) {
                    if (spid >= 0) table_add(tb, a, spid, acc);
                    spid = p;
#pragma unroll
                    for (int c = 0; c < 6; c++) acc[c] = 0.0;
                }
                acc[0] += F0; acc[1] += F1; acc[2] += F2;
                acc[3] += l1 * F2 - l2 * F1;
                acc[4] += l2 * F0 - l0 * F2;
                acc[5] += l0 * F1 - l1 * F0;
            }
            if (wl) {
#pragma unroll
                for (int r = 1; r < 19; r++) {
                    if ((wl >> r) & 1u) {
                        const int ys = y - CY(r);
                        const bool bot = a.wall_y && ys == 0, top = a.wall_y && ys == a.ny - 1;
                        if (bot || top) {
                            const double w0 = bot ? a.wvb[0] : a.wvt[0];
                            const double w1 = bot ? a.wvb[1] : a.wvt[1];
                            const double w2 = bot ? a.wvb[2] : a.wvt[2];
                            d[r] = d[r] + (R)(6.0 * WD(r) * rho_x * (CX(r) * w0 + CY(r) * w1 + CZ(r) * w2));
                        }
                    }
                }
            }
        }
#undef SRC

        // BGK collision with Guo forcing
        R drho = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
        for (int r = 0; r < 19; r++) {
            drho += d[r];
            if (CX(r)) jx += CX(r) * d[r];
            if (CY(r)) jy += CY(r) * d[r];
            if (CZ(r)) jz += CZ(r) * d[r];
        }
        const R rho = (R)a.rho0 + drho;
        const R irho = (R)1 / rho;
        const R ux = (jx + (R)0.5 * gx) * irho, uy = (jy + (R)0.5 * gyy) * irho, uz = (jz + (R)0.5 * gz) * irho;
        const R usq = ux * ux + uy * uy + uz * uz;
        const R ug = ux * gx + uy * gyy + uz * gz;
        R rsum = 0;
#pragma unroll
        for (int r = 0; r < 19; r++) {
            const R w = (R)WD(r);
            const R cu = CX(r) * ux + CY(r) * uy + CZ(r) * uz;
            const R cg = CX(r) * gx + CY(r) * gyy + CZ(r) * gz;
            const R poly = (R)3 * cu + (R)4.5 * cu * cu - (R)1.5 * usq + (R)4.5 * cu * cu * cu - (R)4.5 * usq * cu;
            const R eq = w * (drho + rho * poly);
            const R Fr = pref * w * ((R)3 * (cg - ug) + (R)9 * cu * cg);
            const R out = d[r] - (d[r] - eq) * omega + Fr;
            const T st = Cd::enc(out, enc_scale<P>(a, r));
            B[(unsigned)r * ps + i] = st;
            rsum += Cd::dec(st, dec_scale<P>(a, r));
        }
        ((T*)a.rhoB)[i] = Cd::enc(rsum, rho_enc_scale<P>(a));
        if (!(usq <= (R)0.16)) {
            atomicOr(a.status, ST_UNSTABLE);
            atomicMin(a.bad_step, *a.dstep);
        }
    }
    if (spid >= 0) table_add(tb, a, spid, acc);
    __syncthreads();

    // table -> per-cell slots (plain stores)
    const int tile[3] = {(int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z};
    const int stamp = *a.dstep + 1;
    for (int e = tid; e < TAB_CAP; e += nthr) {
        const int p = tb.key[e];
        if (p < 0) continue;
        double v[6];
        for (int c = 0; c < 6; c++) v[c] = tb.val[c][e];
        const int s = slot_of(a, p, tile);
        if (s < 0) {
            global_add6(a, p, v);
            continue;
        }
        const long long q = (long long)p * a.nslot + s;
        double* dst = a.FTpart + 6 * q;
        for (int c = 0; c < 6; c++) dst[c] = v[c];
        a.stamp[q] = stamp;
    }
}

// One cell's share of a fluid node's links (mask = its link bits): with
// C_r = 6 w_r rho (c_r . U), U the rigid-body velocity at the node,
//   sum_r C_r     = 6 rho (sum w_r c_r) . U,
//   sum_r C_r c_r = 6 rho (sum w_r c_r c_r^T) U,
// and the momentum to the cell is -(2 sum own_r c_r + sum C_r c_r), where
// own_r is the node's bounced population.  The per-node arithmetic runs in the
// compute precision M of the storage mode (FP64 for P64, FP32 otherwise); the
// per-cell sums are FP64.
// kinematics of cell p needed at a fluid node: X, V, Omega
struct Kin {
    double X0, X1, X2, V0, V1, V2, W0, W1, W2;
};
__device__ inline Kin load_kin(const DevArgs& a, int p) {
    const double* k = a.kin + 12 * (size_t)(p < 0 ? 0 : p);
    return Kin{k[0], k[1], k[2], k[3], k[4], k[5], k[6], k[7], k[8]};
}

template <class M>
__device__ inline void cell_links(const DevArgs& a, int x, int y, int z, const Kin& k, uint32_t mask, M rho_x,
                                  M s0, M s1, M s2, M* cm, M* FT) {
    const M l0 = (M)min_image((double)x - k.X0, (double)a.nx);
    const M l1 = (M)(a.wall_y ? ((double)y - k.X1) : min_image((double)y - k.X1, (double)a.ny));
    const M l2 = (M)min_image((double)z - k.X2, (double)a.nz);
    const M V0 = (M)k.V0, V1 = (M)k.V1, V2 = (M)k.V2, W0 = (M)k.W0, W1 = (M)k.W1, W2 = (M)k.W2;
    const M U0 = V0 + (W1 * l2 - W2 * l1);
    const M U1 = V1 + (W2 * l0 - W0 * l2);
    const M U2 = V2 + (W0 * l1 - W1 * l0);
    // geometric sums in units of 1/36 (36 w = 2 on axis links, 1 on diagonals)
    const int ax0 = 2 * (__popc(mask & AXP0) - __popc(mask & AXM0)) + (__popc(mask & DGP0) - __popc(mask & DGM0));
    const int ax1 = 2 * (__popc(mask & AXP1) - __popc(mask & AXM1)) + (__popc(mask & DGP1) - __popc(mask & DGM1));
    const int ax2 = 2 * (__popc(mask & AXP2) - __popc(mask & AXM2)) + (__popc(mask & DGP2) - __popc(mask & DGM2));
    const int mxx = 2 * __popc(mask & (AXP0 | AXM0)) + __popc(mask & (DGP0 | DGM0));
    const int myy = 2 * __popc(mask & (AXP1 | AXM1)) + __popc(mask & (DGP1 | DGM1));
    const int mzz = 2 * __popc(mask & (AXP2 | AXM2)) + __popc(mask & (DGP2 | DGM2));
    const int mxy = __popc(mask & SXYP) - __popc(mask & SXYM);
    const int mxz = __popc(mask & SXZP) - __popc(mask & SXZM);
    const int myz = __popc(mask & SYZP) - __popc(mask & SYZM);
    const M rc = (M)6 * rho_x * (M)(1.0 / 36.0);
    const M sc = rc * ((M)ax0 * U0 + (M)ax1 * U1 + (M)ax2 * U2);
    const M c0 = rc * ((M)mxx * U0 + (M)mxy * U1 + (M)mxz * U2);
    const M c1 = rc * ((M)mxy * U0 + (M)myy * U1 + (M)myz * U2);
    const M c2 = rc * ((M)mxz * U0 + (M)myz * U1 + (M)mzz * U2);
    cm[0] += sc; cm[1] += c0; cm[2] += c1; cm[3] += c2;
    const M F0 = -((M)2 * s0 + c0), F1 = -((M)2 * s1 + c1), F2 = -((M)2 * s2 + c2);
    FT[0] = F0; FT[1] = F1; FT[2] = F2;
    FT[3] = l1 * F2 - l2 * F1;
    FT[4] = l2 * F0 - l0 * F2;
    FT[5] = l0 * F1 - l1 * F0;
}

template <class M>
__device__ inline void table_add_m(LdsTable& tb, const DevArgs& a, int p, const M* v) {
    double d[6];
#pragma unroll
    for (int c = 0; c < 6; c++) d[c] = (double)v[c];
    table_add(tb, a, p, d);
}

// tau = 1 (the paper's operating point, Sec. IV): the post-collision state is
// n^eq(rho, u) plus the forcing term, a function of the moments alone, so the
// pulled populations are folded into rho and j as they arrive and never held.
template <int P, int TZ>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) lb_kernel_tau1(DevArgs a) {
    using Cd = Codec<P>;
    using T = typename Cd::T;
    using R = typename Cd::R;
    using M = R;
    __shared__ LdsTable tb;
    const int nthr = blockDim.x * blockDim.y;
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    for (int e = tid; e < TAB_CAP; e += nthr) {
        tb.key[e] = -1;
        for (int c = 0; c < 6; c++) tb.val[c][e] = 0.0;
    }
    __syncthreads();

    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z0 = blockIdx.z * TZ;
    const bool inb = (x < a.nx) && (y < a.ny);
    const unsigned nx = (unsigned)a.nx;
    const unsigned plane = (unsigned)a.nx * (unsigned)a.ny;
    const unsigned ps = (unsigned)a.pstride;  // 19 * pstride * sizeof(T) < 2^32 (checked at create)
    constexpr unsigned ES = sizeof(T);
    const auto rA = make_rsrc(a.A, 19ull * ps * ES);
    const auto rB = make_rsrc(a.B, 19ull * ps * ES);
    const auto rRA = make_rsrc(a.rhoA, (unsigned long long)ps * ES);
    const auto rRB = make_rsrc(a.rhoB, (unsigned long long)ps * ES);
    const auto rOwn = make_rsrc(a.owner, (unsigned long long)a.ns * 4);
    const auto rFl = make_rsrc(a.flags, (unsigned long long)a.ns * 4);
    const int ox[3] = {x == a.nx - 1 ? -(a.nx - 1) : 1, 0, x == 0 ? a.nx - 1 : -1};
    const int oy[3] = {y == a.ny - 1 ? -(int)((a.ny - 1) * nx) : (int)nx, 0, y == 0 ? (int)((a.ny - 1) * nx) : -(int)nx};
    double gyd[3];
    body_force(a, (double)y, gyd);
    const R gx = (R)gyd[0], gy = (R)gyd[1], gz = (R)gyd[2];

    // two (cell, F, T) accumulators per lane; a cell not held by either
    // evicts the older one into the table
    int spa = -1, spb = -1;
    M aa0 = 0, aa1 = 0, aa2 = 0, aa3 = 0, aa4 = 0, aa5 = 0;
    M ab0 = 0, ab1 = 0, ab2 = 0, ab3 = 0, ab4 = 0, ab5 = 0;
#define CGB_ACCUM(P_, FT_)                                                                      \
    do {                                                                                        \
        const int p_ = (P_);                                                                    \
        if (p_ == spa) {                                                                        \
            aa0 += FT_[0]; aa1 += FT_[1]; aa2 += FT_[2]; aa3 += FT_[3]; aa4 += FT_[4]; aa5 += FT_[5]; \
        } else if (p_ == spb) {                                                                 \
            ab0 += FT_[0]; ab1 += FT_[1]; ab2 += FT_[2]; ab3 += FT_[3]; ab4 += FT_[4]; ab5 += FT_[5]; \
        } else {                                                                                \
            if (spb >= 0) {                                                                     \
                const M ev_[6] = {ab0, ab1, ab2, ab3, ab4, ab5};                                \
                table_add_m<M>(tb, a, spb, ev_);                                                \
            }                                                                                   \
            spb = spa; ab0 = aa0; ab1 = aa1; ab2 = aa2; ab3 = aa3; ab4 = aa4; ab5 = aa5;        \
            spa = p_; aa0 = FT_[0]; aa1 = FT_[1]; aa2 = FT_[2]; aa3 = FT_[3]; aa4 = FT_[4]; aa5 = FT_[5]; \
        }                                                                                       \
    } while (0)

    // flags of the first node; each step prefetches the next node's flags
    uint32_t fnext = (inb && z0 < a.nz) ? bload<uint32_t>(rFl, 4u * ((unsigned)x + nx * (unsigned)y + plane * (unsigned)z0)) : NONFLUID;
    for (int zz = 0; zz < TZ; zz++) {
        const int z = z0 + zz;
        if (z >= a.nz) break;
        const unsigned i = (unsigned)x + nx * (unsigned)y + plane * (unsigned)z;
        const uint32_t f = fnext;
        fnext = (inb && zz + 1 < TZ && z + 1 < a.nz) ? bload<uint32_t>(rFl, 4u * (i + plane)) : NONFLUID;
        if (f & NONFLUID) continue;
        const int oz[3] = {z == a.nz - 1 ? -(int)((a.nz - 1) * plane) : (int)plane, 0,
                           z == 0 ? (int)((a.nz - 1) * plane) : -(int)plane};
#define SRC(r) (i + (unsigned)(ox[CX(r) + 1] + oy[CY(r) + 1] + oz[CZ(r) + 1]))

        // issue the 19 pulls (non-fluid source: bounce-back) and the owner
        // loads of the link directions together; loads for non-link
        // directions use an offset past the end of the buffer, which reads 0
        // without touching memory
        const uint32_t links = f & LINKBITS;
        T v[19];
#pragma unroll
        for (int r = 0; r < 19; r++) {
            const bool bb = (f >> r) & 1u;
            v[r] = bload<T>(rA, ES * (bb ? (unsigned)OPP(r) * ps + i : (unsigned)r * ps + SRC(r)));
        }
        int ow[19];
#pragma unroll
        for (int r = 1; r < 19; r++) {
            const bool lk = (links >> r) & 1u;
            ow[r] = bload<int>(rOwn, lk ? 4u * SRC(r) : 0xfffffff0u);
        }
        // owners: first cell p1, second cell p2, the rest
        int p1 = -1, p2 = -1;
        uint32_t pm1 = 0, pm2 = 0, pm3 = 0;
#pragma unroll
        for (int r = 1; r < 19; r++) {
            const int o = ((links >> r) & 1u) ? ow[r] : -1;
            if (o >= 0) {
                if (p1 < 0 || o == p1) { p1 = o; pm1 |= 1u << r; }
                else if (p2 < 0 || o == p2) { p2 = o; pm2 |= 1u << r; }
                else pm3 |= 1u << r;
            }
        }
        // cell kinematics requested before the pulls are consumed
        Kin k1{}, k2{};
        if (pm1) k1 = load_kin(a, p1);
        if (pm2) k2 = load_kin(a, p2);

        // moments; sums of own_r c_r over the links of p1 and of p2
        R drho = 0, jx = 0, jy = 0, jz = 0;
        R s10 = 0, s11 = 0, s12 = 0, s20 = 0, s21 = 0, s22 = 0;
#pragma unroll
        for (int r = 0; r < 19; r++) {
            const R dv = Cd::dec(v[r], dec_scale<P>(a, r));
            drho += dv;
            if (CX(r)) jx += CX(r) * dv;
            if (CY(r)) jy += CY(r) * dv;
            if (CZ(r)) jz += CZ(r) * dv;
            if (r > 0) {
                const R d1 = ((pm1 >> r) & 1u) ? dv : (R)0;
                const R d2 = ((pm2 >> r) & 1u) ? dv : (R)0;
                if (CX(r)) { s10 += CX(r) * d1; s20 += CX(r) * d2; }
                if (CY(r)) { s11 += CY(r) * d1; s21 += CY(r) * d2; }
                if (CZ(r)) { s12 += CZ(r) * d1; s22 += CZ(r) * d2; }
            }
        }

        if (links) {
            const uint32_t pall = pm1 | pm2 | pm3;
            const uint32_t wl = a.moving_walls ? (links & ~pall) : 0u;
            M rho_x = 0;
            if (pall | wl) rho_x = (M)a.rho0 + (M)Cd::dec(bload<T>(rRA, ES * i), rho_dec_scale<P>(a));
            M cm[4] = {0, 0, 0, 0};
            M FT[6];
            if (pm1) {
                cell_links<M>(a, x, y, z, k1, pm1, rho_x, s10, s11, s12, cm, FT);
                CGB_ACCUM(p1, FT);
            }
            if (pm2) {
                cell_links<M>(a, x, y, z, k2, pm2, rho_x, s20, s21, s22, cm, FT);
                CGB_ACCUM(p2, FT);
            }
            while (pm3) {
                // third and further cells (rare): one cell per pass
                const int r0 = __builtin_ctz(pm3);
                const int p = bload<int>(rOwn, 4u * (i + (unsigned)(ox[1 + cxr(r0)] + oy[1 + cyr(r0)] + oz[1 + czr(r0)])));
                uint32_t sub = 0;
                R t0 = 0, t1 = 0, t2 = 0;
#pragma unroll
                for (int r = 1; r < 19; r++) {
                    const bool m = (pm3 >> r) & 1u;
                    const int ov = bload<int>(rOwn, m ? 4u * SRC(r) : 0xfffffff0u);
                    const T v = bload<T>(rA, m ? ES * ((unsigned)OPP(r) * ps + i) : 0xfffffff0u);
                    if (m && ov == p) {
                        sub |= 1u << r;
                        const R dv = Cd::dec(v, dec_scale<P>(a, r));
                        if (CX(r)) t0 += CX(r) * dv;
                        if (CY(r)) t1 += CY(r) * dv;
                        if (CZ(r)) t2 += CZ(r) * dv;
                    }
                }
                pm3 &= ~sub;
                cell_links<M>(a, x, y, z, load_kin(a, p), sub, rho_x, t0, t1, t2, cm, FT);
                table_add_m<M>(tb, a, p, FT);
            }
            if (wl) {
                // moving wall planes: the corrections with the wall velocity
#pragma unroll
                for (int r = 1; r < 19; r++) {
                    if ((wl >> r) & 1u) {
                        const int ys = y - CY(r);
                        const bool bot = a.wall_y && ys == 0, top = a.wall_y && ys == a.ny - 1;
                        if (bot || top) {
                            const M w0 = (M)(bot ? a.wvb[0] : a.wvt[0]);
                            const M w1 = (M)(bot ? a.wvb[1] : a.wvt[1]);
                            const M w2 = (M)(bot ? a.wvb[2] : a.wvt[2]);
                            const M C = (M)6 * (M)WD(r) * rho_x * (CX(r) * w0 + CY(r) * w1 + CZ(r) * w2);
                            cm[0] += C; cm[1] += C * CX(r); cm[2] += C * CY(r); cm[3] += C * CZ(r);
                        }
                    }
                }
            }
            drho += (R)cm[0]; jx += (R)cm[1]; jy += (R)cm[2]; jz += (R)cm[3];
        }
#undef SRC

        // n* = n^eq(rho, u) + Guo term (tau = 1), for opposite pairs r, rbar:
        // even part E = 4.5 cu^2 - 1.5 u^2 (+ forcing 0.5 w (9 cu cg - 3 u.g)),
        // odd part O = 3 cu + 4.5 cu^3 - 4.5 u^2 cu (+ forcing 1.5 w cg)
        const R rho = (R)a.rho0 + drho;
        const R irho = (R)1 / rho;
        const R ux = (jx + (R)0.5 * gx) * irho, uy = (jy + (R)0.5 * gy) * irho, uz = (jz + (R)0.5 * gz) * irho;
        const R usq = ux * ux + uy * uy + uz * uz;
        const R ug = ux * gx + uy * gy + uz * gz;
        {
            const R w0 = (R)(1.0 / 3.0);
            const R out0 = w0 * (drho - rho * (R)1.5 * usq) - (R)1.5 * w0 * ug;
            bstore<T>(Cd::enc(out0, enc_scale<P>(a, 0)), rB, ES * i);
        }
#pragma unroll
        for (int r = 1; r < 19; r += 2) {
            const R w = (R)WD(r);
            const R cu = CX(r) * ux + CY(r) * uy + CZ(r) * uz;
            const R cg = CX(r) * gx + CY(r) * gy + CZ(r) * gz;
            const R cu2 = cu * cu;
            const R ev = w * (drho + rho * ((R)4.5 * cu2 - (R)1.5 * usq)) + (R)0.5 * w * ((R)9 * cu * cg - (R)3 * ug);
            const R od = w * rho * cu * ((R)3 + (R)4.5 * cu2 - (R)4.5 * usq) + (R)1.5 * w * cg;
            bstore<T>(Cd::enc(ev + od, enc_scale<P>(a, r)), rB, ES * ((unsigned)r * ps + i));
            bstore<T>(Cd::enc(ev - od, enc_scale<P>(a, r + 1)), rB, ES * ((unsigned)(r + 1) * ps + i));
        }
        // the collision conserves mass: the density deviation of n* is drho
        bstore<T>(Cd::enc(drho, rho_enc_scale<P>(a)), rRB, ES * i);
        if (!(usq <= (R)0.16)) {
            atomicOr(a.status, ST_UNSTABLE);
            atomicMin(a.bad_step, *a.dstep);
        }
    }
    if (spa >= 0) { const M ev[6] = {aa0, aa1, aa2, aa3, aa4, aa5}; table_add_m<M>(tb, a, spa, ev); }
    if (spb >= 0) { const M ev[6] = {ab0, ab1, ab2, ab3, ab4, ab5}; table_add_m<M>(tb, a, spb, ev); }
#undef CGB_ACCUM
    __syncthreads();

    const int tile[3] = {(int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z};
    const int stamp = *a.dstep + 1;
    for (int e = tid; e < TAB_CAP; e += nthr) {
        const int p = tb.key[e];
        if (p < 0) continue;
        double v[6];
        for (int c = 0; c < 6; c++) v[c] = tb.val[c][e];
        const int s = slot_of(a, p, tile);
        if (s < 0) {
            global_add6(a, p, v);
            continue;
        }
        const long long q = (long long)p * a.nslot + s;
        double* dst = a.FTpart + 6 * q;
        for (int c = 0; c < 6; c++) dst[c] = v[c];
        a.stamp[q] = stamp;
    }
}

// sum the stamped slots of every cell into its hydrodynamic force and torque
__global__ void mem_gather_kernel(DevArgs a) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    const double* k = a.kin + 12 * (long long)p;
    int cnt[3], t0[3];
    for (int c = 0; c < 3; c++) {
        const int n = c == 0 ? a.nx : (c == 1 ? a.ny : a.nz);
        const int lo = foot_lo(a, c, k[c]);
        const int ext = (int)ceil(k[c] + a.Rb) + 1 - ((int)floor(k[c] - a.Rb) - 1) + 1;
        t0[c] = lo / a.tile[c];
        // tiles touched by the ext nodes starting at lo (wrapping)
        int m = 1, prev = t0[c];
        for (int s = 1; s < ext; s++) {
            int node = lo + s;
            if (c == 1 && a.wall_y) { if (node >= n) break; }
            else if (node >= n) node -= n;
            const int t = node / a.tile[c];
            if (t != prev) { m++; prev = t; }
        }
        cnt[c] = m < a.slots[c] ? m : a.slots[c];
    }
    const int stamp = *a.dstep + 1;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int oz = 0; oz < cnt[2]; oz++)
        for (int oy = 0; oy < cnt[1]; oy++)
            for (int ox = 0; ox < cnt[0]; ox++) {
                const int s = ox + a.slots[0] * (oy + a.slots[1] * oz);
                const long long q = (long long)p * a.nslot + s;
                if (a.stamp[q] != stamp) continue;
                const double* src = a.FTpart + 6 * q;
                for (int c = 0; c < 6; c++) acc[c] += src[c];
            }
    double* F = a.FTh + 6 * (long long)p;
    for (int c = 0; c < 6; c++) F[c] += acc[c];
}

template <int P>
static hipError_t launch_lb_p(const DevArgs& a, LaunchCfg cfg, hipStream_t st) {
    dim3 blk(cfg.bx, cfg.by, 1);
    dim3 grd((a.nx + cfg.bx - 1) / cfg.bx, (a.ny + cfg.by - 1) / cfg.by, (a.nz + cfg.tz - 1) / cfg.tz);
    const bool t1 = a.tau == 1.0;
    switch (cfg.tz) {
        case 4:
            if (t1) hipLaunchKernelGGL((lb_kernel_tau1<P, 4>), grd, blk, 0, st, a);
            else hipLaunchKernelGGL((lb_kernel_tau<P, 4>), grd, blk, 0, st, a);
            break;
        case 8:
            if (t1) hipLaunchKernelGGL((lb_kernel_tau1<P, 8>), grd, blk, 0, st, a);
            else hipLaunchKernelGGL((lb_kernel_tau<P, 8>), grd, blk, 0, st, a);
            break;
        case 16:
            if (t1) hipLaunchKernelGGL((lb_kernel_tau1<P, 16>), grd, blk, 0, st, a);
            else hipLaunchKernelGGL((lb_kernel_tau<P, 16>), grd, blk, 0, st, a);
            break;
        case 32:
            if (t1) hipLaunchKernelGGL((lb_kernel_tau1<P, 32>), grd, blk, 0, st, a);
            else hipLaunchKernelGGL((lb_kernel_tau<P, 32>), grd, blk, 0, st, a);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_lb(const DevArgs& a, LaunchCfg cfg, hipStream_t st) {
    if (cfg.bx != a.tile[0] || cfg.by != a.tile[1] || cfg.tz != a.tile[2]) return hipErrorInvalidValue;
    hipError_t e;
    switch (a.precision) {
        case CGB_P64: e = launch_lb_p<CGB_P64>(a, cfg, st); break;
        case CGB_P32: e = launch_lb_p<CGB_P32>(a, cfg, st); break;
        case CGB_PMX16: e = launch_lb_p<CGB_PMX16>(a, cfg, st); break;
        case CGB_PMXBF16: e = launch_lb_p<CGB_PMXBF16>(a, cfg, st); break;
        default: return hipErrorInvalidValue;
    }
    return e;
}

hipError_t launch_mem_gather(const DevArgs& a, hipStream_t st) {
    if (a.n == 0) return hipSuccess;
    hipLaunchKernelGGL(mem_gather_kernel, dim3((a.n + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace cgb
