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
        const int old = atomicCAS(&tb.key[h], -1, p);
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
            atomicMin(a.bad_step, (int)a.step);
        }
    }
    if (spid >= 0) table_add(tb, a, spid, acc);
    __syncthreads();

    // table -> per-cell slots (plain stores)
    const int tile[3] = {(int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z};
    const int stamp = (int)a.step + 1;
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
// own_r is the node's bounced population.  sown = sum own_r c_r over mask.
template <int P>
__device__ inline void cell_links(const DevArgs& a, int x, int y, int z, int p, uint32_t mask, double rho_x,
                                  const double* sown, double* cm /* dC rho, dC j */, double* F, double* Tq,
                                  double* lev) {
    const double* k = a.kin + 12 * (size_t)p;
    const double l0 = min_image((double)x - k[0], (double)a.nx);
    const double l1 = a.wall_y ? ((double)y - k[1]) : min_image((double)y - k[1], (double)a.ny);
    const double l2 = min_image((double)z - k[2], (double)a.nz);
    const double U0 = k[3] + (k[7] * l2 - k[8] * l1);
    const double U1 = k[4] + (k[8] * l0 - k[6] * l2);
    const double U2 = k[5] + (k[6] * l1 - k[7] * l0);
    // geometric sums over the link set (constants of the lattice)
    double a0 = 0, a1 = 0, a2 = 0, mxx = 0, myy = 0, mzz = 0, mxy = 0, mxz = 0, myz = 0;
#pragma unroll
    for (int r = 1; r < 19; r++) {
        if ((mask >> r) & 1u) {
            const double w = WD(r);
            a0 += w * CX(r); a1 += w * CY(r); a2 += w * CZ(r);
            mxx += w * (CX(r) * CX(r)); myy += w * (CY(r) * CY(r)); mzz += w * (CZ(r) * CZ(r));
            mxy += w * (CX(r) * CY(r)); mxz += w * (CX(r) * CZ(r)); myz += w * (CY(r) * CZ(r));
        }
    }
    const double rc = 6.0 * rho_x;
    const double sc = rc * (a0 * U0 + a1 * U1 + a2 * U2);
    const double c0 = rc * (mxx * U0 + mxy * U1 + mxz * U2);
    const double c1 = rc * (mxy * U0 + myy * U1 + myz * U2);
    const double c2 = rc * (mxz * U0 + myz * U1 + mzz * U2);
    cm[0] += sc; cm[1] += c0; cm[2] += c1; cm[3] += c2;
    F[0] = -(2.0 * sown[0] + c0);
    F[1] = -(2.0 * sown[1] + c1);
    F[2] = -(2.0 * sown[2] + c2);
    Tq[0] = l1 * F[2] - l2 * F[1];
    Tq[1] = l2 * F[0] - l0 * F[2];
    Tq[2] = l0 * F[1] - l1 * F[0];
    lev[0] = l0; lev[1] = l1; lev[2] = l2;
}

// tau = 1 (the paper's operating point, Sec. IV): the post-collision state is
// n^eq(rho, u) plus the forcing term, a function of the moments alone, so the
// pulled populations are folded into rho and j as they arrive and never held.
template <int P, int TZ>
__global__ void __launch_bounds__(256) lb_kernel_tau1(DevArgs a) {
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

    int spid = -1;
    double acc[6] = {0, 0, 0, 0, 0, 0};

    for (int zz = 0; zz < TZ; zz++) {
        const int z = z0 + zz;
        if (z >= a.nz) break;
        const unsigned i = (unsigned)x + nx * (unsigned)y + plane * (unsigned)z;
        const uint32_t f = inb ? bload<uint32_t>(rFl, 4u * i) : NONFLUID;
        if (f & NONFLUID) continue;
        const int oz[3] = {z == a.nz - 1 ? -(int)((a.nz - 1) * plane) : (int)plane, 0,
                           z == 0 ? (int)((a.nz - 1) * plane) : -(int)plane};
#define SRC(r) (i + (unsigned)(ox[CX(r) + 1] + oy[CY(r) + 1] + oz[CZ(r) + 1]))

        // owners behind the links: the first cell p1 and its links, other cells
        const uint32_t links = f & LINKBITS;
        int p1 = -1;
        uint32_t pm1 = 0, pmo = 0;
        if (links) {
#pragma unroll
            for (int r = 1; r < 19; r++) {
                if ((links >> r) & 1u) {
                    const int o = bload<int>(rOwn, 4u * SRC(r));
                    if (o >= 0) {
                        if (p1 < 0) p1 = o;
                        if (o == p1) pm1 |= 1u << r;
                        else pmo |= 1u << r;
                    }
                }
            }
        }

        // moments of the pulled populations (non-fluid source: bounce-back);
        // sum of own_r c_r over p1's links on the way
        R drho = 0, jx = 0, jy = 0, jz = 0;
        double so0 = 0.0, so1 = 0.0, so2 = 0.0;
#pragma unroll
        for (int r = 0; r < 19; r++) {
            const bool bb = (f >> r) & 1u;
            const T v = bload<T>(rA, ES * (bb ? (unsigned)OPP(r) * ps + i : (unsigned)r * ps + SRC(r)));
            const R dv = Cd::dec(v, dec_scale<P>(a, r));
            drho += dv;
            if (CX(r)) jx += CX(r) * dv;
            if (CY(r)) jy += CY(r) * dv;
            if (CZ(r)) jz += CZ(r) * dv;
            if (r > 0 && ((pm1 >> r) & 1u)) {
                const double dd = (double)dv;
                if (CX(r)) so0 += CX(r) * dd;
                if (CY(r)) so1 += CY(r) * dd;
                if (CZ(r)) so2 += CZ(r) * dd;
            }
        }

        if (links) {
            const uint32_t wl = a.moving_walls ? (links & ~(pm1 | pmo)) : 0u;
            double rho_x = 0.0;
            if (pm1 | wl) rho_x = a.rho0 + (double)Cd::dec(bload<T>(rRA, ES * i), rho_dec_scale<P>(a));
            double cm[4] = {0, 0, 0, 0};
            int p = p1;
            uint32_t mask = pm1;
            double sown[3] = {so0, so1, so2};
            while (mask) {
                double F[3], Tq[3], lev[3];
                cell_links<P>(a, x, y, z, p, mask, rho_x, sown, cm, F, Tq, lev);
                if (p != spid) {
                    if (spid >= 0) table_add(tb, a, spid, acc);
                    spid = p;
#pragma unroll
                    for (int c = 0; c < 6; c++) acc[c] = 0.0;
                }
                acc[0] += F[0]; acc[1] += F[1]; acc[2] += F[2];
                acc[3] += Tq[0]; acc[4] += Tq[1]; acc[5] += Tq[2];
                // next cell among the remaining links (rare): reload from cache
                mask = 0;
                if (pmo) {
                    p = bload<int>(rOwn, 4u * (i + (unsigned)(ox[1 + cxr(__builtin_ctz(pmo))] + oy[1 + cyr(__builtin_ctz(pmo))] +
                                                               oz[1 + czr(__builtin_ctz(pmo))])));
                    sown[0] = sown[1] = sown[2] = 0.0;
                    for (uint32_t m = pmo; m; m &= m - 1) {
                        const int r = __builtin_ctz(m);
                        const int cx = cxr(r), cy = cyr(r), cz = czr(r);
                        if (bload<int>(rOwn, 4u * (i + (unsigned)(ox[1 + cx] + oy[1 + cy] + oz[1 + cz]))) != p) continue;
                        mask |= 1u << r;
                        const unsigned rb = (unsigned)(r + ((r & 1) ? 1 : -1));
                        const double dd = (double)Cd::dec(bload<T>(rA, ES * (rb * ps + i)), dec_scale<P>(a, r));
                        sown[0] += cx * dd; sown[1] += cy * dd; sown[2] += cz * dd;
                    }
                    pmo &= ~mask;
                }
            }
            if (wl) {
                // moving wall planes: same sums with the wall velocity
#pragma unroll
                for (int r = 1; r < 19; r++) {
                    if ((wl >> r) & 1u) {
                        const int ys = y - CY(r);
                        const bool bot = a.wall_y && ys == 0, top = a.wall_y && ys == a.ny - 1;
                        if (bot || top) {
                            const double w0 = bot ? a.wvb[0] : a.wvt[0];
                            const double w1 = bot ? a.wvb[1] : a.wvt[1];
                            const double w2 = bot ? a.wvb[2] : a.wvt[2];
                            const double C = 6.0 * WD(r) * rho_x * (CX(r) * w0 + CY(r) * w1 + CZ(r) * w2);
                            cm[0] += C; cm[1] += C * CX(r); cm[2] += C * CY(r); cm[3] += C * CZ(r);
                        }
                    }
                }
            }
            drho += (R)cm[0]; jx += (R)cm[1]; jy += (R)cm[2]; jz += (R)cm[3];
        }
#undef SRC

        // n* = n^eq(rho, u) + Guo term (tau = 1)
        const R rho = (R)a.rho0 + drho;
        const R irho = (R)1 / rho;
        const R ux = (jx + (R)0.5 * gx) * irho, uy = (jy + (R)0.5 * gy) * irho, uz = (jz + (R)0.5 * gz) * irho;
        const R usq = ux * ux + uy * uy + uz * uz;
        const R ug = ux * gx + uy * gy + uz * gz;
        R rsum = 0;
#pragma unroll
        for (int r = 0; r < 19; r++) {
            const R w = (R)WD(r);
            const R cu = CX(r) * ux + CY(r) * uy + CZ(r) * uz;
            const R cg = CX(r) * gx + CY(r) * gy + CZ(r) * gz;
            const R poly = (R)3 * cu + (R)4.5 * cu * cu - (R)1.5 * usq + (R)4.5 * cu * cu * cu - (R)4.5 * usq * cu;
            const R out = w * (drho + rho * poly) + (R)0.5 * w * ((R)3 * (cg - ug) + (R)9 * cu * cg);
            const T st = Cd::enc(out, enc_scale<P>(a, r));
            bstore<T>(st, rB, ES * ((unsigned)r * ps + i));
            rsum += Cd::dec(st, dec_scale<P>(a, r));
        }
        bstore<T>(Cd::enc(rsum, rho_enc_scale<P>(a)), rRB, ES * i);
        if (!(usq <= (R)0.16)) {
            atomicOr(a.status, ST_UNSTABLE);
            atomicMin(a.bad_step, (int)a.step);
        }
    }
    if (spid >= 0) table_add(tb, a, spid, acc);
    __syncthreads();

    const int tile[3] = {(int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z};
    const int stamp = (int)a.step + 1;
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
    const int stamp = (int)a.step + 1;
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
