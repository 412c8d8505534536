// lb.hip -- fused pull stream + bounce-back + BGK collision + momentum exchange.
//
// One thread per lattice node.  For a fluid node x and each direction r the
// pulled population is n*_r(x - c_r) when the source is fluid (Eq. 2);
// when the source is a wall or a cell node it is the node's own post-collision
// n*_rbar(x) (mid-link bounce-back, Eq. 9) plus, for a moving boundary, the
// correction C = 6 w_r rho(x) (c_r . v_b) of Eq. 10 with rho(x) the node's
// density at the time of the bounced populations.  The transferred momentum
// (2 n*_rbar + C) c_rbar (Eq. 12) is summed per cell in FP64.  Only its part
// (2 d_rbar + C) c_rbar that depends on the deviations d = n* - w rho0 is
// summed: the constant part 2 w rho0 c_rbar, together with the particle-
// particle and particle-wall link forces of Eqs. 13-14, sums to exactly zero
// over the closed surface of a cell's node set (sum of w c over the outward
// links of any node set vanishes, and so does the sum of (x - X) x w c), so
// the two forms are the same force.  Collision: Eqs. 1, 4, 5 with the Guo
// forcing term, u = (sum n c + g/2)/rho.
//
// Per-cell sums: each lane keeps one (cell, F, T) slot; lanes of a wave are
// combined with a segmented wave reduction (one FP64 atomic per distinct cell
// and component per wave).
#include "cgb_dev.h"

namespace cgb {

template <int P>
__global__ void __launch_bounds__(256) lb_kernel(DevArgs a) {
    using Cd = Codec<P>;
    using T = typename Cd::T;
    using R = typename Cd::R;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    const bool inb = (x < a.nx) && (y < a.ny);
    const long long plane = (long long)a.nx * a.ny;
    const long long i = inb ? (long long)x + (long long)a.nx * y + plane * z : 0;
    const uint32_t f = inb ? a.flags[i] : NONFLUID;
    const bool act = !(f & NONFLUID);

    int spid = -1;
    double sF0 = 0, sF1 = 0, sF2 = 0, sT0 = 0, sT1 = 0, sT2 = 0;

    if (act) {
        const T* __restrict__ A = (const T*)a.A;
        T* __restrict__ B = (T*)a.B;
        const long long ps = a.pstride;
        const int xm = wrap(x - 1, a.nx), xp = wrap(x + 1, a.nx);
        const int ym = wrap(y - 1, a.ny), yp = wrap(y + 1, a.ny);
        const int zm = wrap(z - 1, a.nz), zp = wrap(z + 1, a.nz);
        // source coordinate along an axis for velocity component c: x - c
        const int sxv[3] = {xp, x, xm};
        const long long syv[3] = {(long long)a.nx * yp, (long long)a.nx * y, (long long)a.nx * ym};
        const long long szv[3] = {plane * zp, plane * z, plane * zm};

        R d[19];
#pragma unroll
        for (int r = 0; r < 19; r++) {
            const long long j = sxv[CX(r) + 1] + syv[CY(r) + 1] + szv[CZ(r) + 1];
            d[r] = (f & (1u << r)) ? (R)0 : Cd::dec(A[r * ps + j], dec_scale<P>(a, r));
        }

        if (f & LINKBITS) {
            const double rho_x = a.rho0 + (double)Cd::dec(((const T*)a.rhoA)[i], rho_dec_scale<P>(a));
#pragma unroll
            for (int r = 1; r < 19; r++) {
                if (!(f & (1u << r))) continue;
                const long long j = sxv[CX(r) + 1] + syv[CY(r) + 1] + szv[CZ(r) + 1];
                const int o = a.owner[j];
                const int rb = OPP(r);
                const R own = Cd::dec(A[rb * ps + i], dec_scale<P>(a, rb));
                double C = 0.0;
                if (o >= 0) {
                    const double* k = a.kin + 12 * (long long)o;
                    // boundary velocity at the link midpoint x - c_r/2
                    double b[3];
                    b[0] = min_image((double)x - 0.5 * CX(r) - k[0], (double)a.nx);
                    b[1] = a.wall_y ? ((double)y - 0.5 * CY(r) - k[1])
                                    : min_image((double)y - 0.5 * CY(r) - k[1], (double)a.ny);
                    b[2] = min_image((double)z - 0.5 * CZ(r) - k[2], (double)a.nz);
                    const double vb0 = k[3] + (k[7] * b[2] - k[8] * b[1]);
                    const double vb1 = k[4] + (k[8] * b[0] - k[6] * b[2]);
                    const double vb2 = k[5] + (k[6] * b[1] - k[7] * b[0]);
                    const double cv = CX(r) * vb0 + CY(r) * vb1 + CZ(r) * vb2;
                    C = 6.0 * WD(r) * rho_x * cv;
                    // momentum to the cell: (2 d_rbar + C) c_rbar = -(2 d_rbar + C) c_r
                    const double dyn = 2.0 * (double)own + C;
                    const double f0 = -dyn * CX(r), f1 = -dyn * CY(r), f2 = -dyn * CZ(r);
                    double l[3];
                    l[0] = min_image((double)x - k[0], (double)a.nx);
                    l[1] = a.wall_y ? ((double)y - k[1]) : min_image((double)y - k[1], (double)a.ny);
                    l[2] = min_image((double)z - k[2], (double)a.nz);
                    if (o != spid) {
                        if (spid >= 0) {
                            double* F = a.FTh + 6 * (long long)spid;
                            unsafeAtomicAdd(F + 0, sF0); unsafeAtomicAdd(F + 1, sF1); unsafeAtomicAdd(F + 2, sF2);
                            unsafeAtomicAdd(F + 3, sT0); unsafeAtomicAdd(F + 4, sT1); unsafeAtomicAdd(F + 5, sT2);
                        }
                        spid = o;
                        sF0 = sF1 = sF2 = sT0 = sT1 = sT2 = 0.0;
                    }
                    sF0 += f0; sF1 += f1; sF2 += f2;
                    sT0 += l[1] * f2 - l[2] * f1;
                    sT1 += l[2] * f0 - l[0] * f2;
                    sT2 += l[0] * f1 - l[1] * f0;
                } else if (a.moving_walls) {
                    const int ys = y - CY(r);
                    const bool bot = a.wall_y && ys == 0, top = a.wall_y && ys == a.ny - 1;
                    if (bot || top) {
                        const double w0 = bot ? a.wvb[0] : a.wvt[0];
                        const double w1 = bot ? a.wvb[1] : a.wvt[1];
                        const double w2 = bot ? a.wvb[2] : a.wvt[2];
                        C = 6.0 * WD(r) * rho_x * (CX(r) * w0 + CY(r) * w1 + CZ(r) * w2);
                    }
                }
                d[r] = own + (R)C;
            }
        }

        // collision with Guo forcing
        R drho = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
        for (int r = 0; r < 19; r++) {
            drho += d[r];
            if (CX(r)) jx += CX(r) * d[r];
            if (CY(r)) jy += CY(r) * d[r];
            if (CZ(r)) jz += CZ(r) * d[r];
        }
        double gd[3];
        body_force(a, (double)y, gd);
        const R gx = (R)gd[0], gy = (R)gd[1], gz = (R)gd[2];
        const R rho = (R)a.rho0 + drho;
        const R irho = (R)1 / rho;
        const R ux = (jx + (R)0.5 * gx) * irho, uy = (jy + (R)0.5 * gy) * irho, uz = (jz + (R)0.5 * gz) * irho;
        const R usq = ux * ux + uy * uy + uz * uz;
        const R omega = (R)(1.0 / a.tau);
        const R pref = (R)(1.0 - 0.5 / a.tau);
        const R ug = ux * gx + uy * gy + uz * gz;
        T* __restrict__ Bo = B;
        R rsum = 0;
#pragma unroll
        for (int r = 0; r < 19; r++) {
            const R w = (R)WD(r);
            const R cu = CX(r) * ux + CY(r) * uy + CZ(r) * uz;
            const R cg = CX(r) * gx + CY(r) * gy + CZ(r) * gz;
            const R poly = (R)3 * cu + (R)4.5 * cu * cu - (R)1.5 * usq + (R)4.5 * cu * cu * cu - (R)4.5 * usq * cu;
            const R eq = w * (drho + rho * poly);
            const R Fr = pref * w * ((R)3 * (cg - ug) + (R)9 * cu * cg);
            const R out = d[r] - (d[r] - eq) * omega + Fr;
            const T st = Cd::enc(out, enc_scale<P>(a, r));
            Bo[r * a.pstride + i] = st;
            rsum += Cd::dec(st, dec_scale<P>(a, r));
        }
        ((T*)a.rhoB)[i] = Cd::enc(rsum, rho_enc_scale<P>(a));
        if (!(usq <= (R)0.16)) {
            atomicOr(a.status, ST_UNSTABLE);
            atomicMin(a.bad_step, (int)a.step);
        }
    }

    // segmented wave reduction of the (cell, F, T) slots
    const int lane = __lane_id();
    while (true) {
        const unsigned long long act_mask = __ballot(spid >= 0);
        if (act_mask == 0ull) break;
        const int leader = __ffsll((long long)act_mask) - 1;
        const int lp = __shfl(spid, leader, 64);
        const bool mine = (spid == lp);
        double v0 = wave_sum(mine ? sF0 : 0.0);
        double v1 = wave_sum(mine ? sF1 : 0.0);
        double v2 = wave_sum(mine ? sF2 : 0.0);
        double v3 = wave_sum(mine ? sT0 : 0.0);
        double v4 = wave_sum(mine ? sT1 : 0.0);
        double v5 = wave_sum(mine ? sT2 : 0.0);
        if (lane == leader) {
            double* F = a.FTh + 6 * (long long)lp;
            unsafeAtomicAdd(F + 0, v0); unsafeAtomicAdd(F + 1, v1); unsafeAtomicAdd(F + 2, v2);
            unsafeAtomicAdd(F + 3, v3); unsafeAtomicAdd(F + 4, v4); unsafeAtomicAdd(F + 5, v5);
        }
        if (mine) spid = -1;
    }
}

hipError_t launch_lb(const DevArgs& a, LaunchCfg cfg, hipStream_t st) {
    dim3 blk(cfg.bx, cfg.by, 1);
    dim3 grd((a.nx + cfg.bx - 1) / cfg.bx, (a.ny + cfg.by - 1) / cfg.by, a.nz);
    switch (a.precision) {
        case CGB_P64: hipLaunchKernelGGL(lb_kernel<CGB_P64>, grd, blk, 0, st, a); break;
        case CGB_P32: hipLaunchKernelGGL(lb_kernel<CGB_P32>, grd, blk, 0, st, a); break;
        case CGB_PMX16: hipLaunchKernelGGL(lb_kernel<CGB_PMX16>, grd, blk, 0, st, a); break;
        case CGB_PMXBF16: hipLaunchKernelGGL(lb_kernel<CGB_PMXBF16>, grd, blk, 0, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace cgb
