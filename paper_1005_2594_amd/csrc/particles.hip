// particles.hip -- cell-side kernels of the time step.
//
//  prep         axis o = R(q) e_z and space-frame angular velocity of each cell
//  raster       (1) claims, over each cell's bounding box: every node inside
//               the discretised ellipsoid (Sec. II: half axes R_par along o,
//               R_perp across) that the cell does not own records the lowest
//               covering index; (2) resolve, one thread per node: the owner
//               keeps a node while it is still inside it (single occupancy,
//               first arrival keeps the node), otherwise the lowest claimer
//               takes it, otherwise it becomes fluid; a claimed fluid node
//               goes to the lowest claimer.  Changes go to a transition list.
//  transitions  apply owner changes, update node flags, and balance the deleted
//               (covered) or created (freed, Eq. 5 at rho0 and the rigid-body
//               velocity) fluid momentum with a force and torque on the cell.
//  cells        cell list with bin edge >= cut-off (counting sort, bins sorted
//               by index for a deterministic order).
//  potentials   Berne-Pechukas pair forces (Eqs. 15-18) and cell-wall forces
//               (Eqs. 19-20), one thread per cell over its 27 neighbour bins.
//  integrate    FP64 leap-frog: V += F/M, X += V, L += T, quaternion rotation
//               by an explicit midpoint step.
#include "cgb_dev.h"

namespace cgb {

// ------------------------------------------------------------------ prep
// integer displacement d = s - b of a node from the node b nearest to a cell
// centre X (f = X - b), moved to the periodic image in which s - X is nearest
__device__ inline int image_shift(int d, float f, int n) {
    const float e = (float)d - f;
    if (e >= 0.5f * (float)n) return d - n;
    if (e < -0.5f * (float)n) return d + n;
    return d;
}

// kinematics of cell p into k (X, V, Omega, o) and the tables; every input is
// loaded before the first store and nothing stored is read back, so the
// loads of a wave are in flight together
__device__ void prep_one(const DevArgs& a, int p, bool zero_forces, double* k) {
    double q[4], L[3];
    for (int c = 0; c < 4; c++) q[c] = a.q[4 * p + c];
    for (int c = 0; c < 3; c++) {
        L[c] = a.L[3 * p + c];
        k[c] = a.X[3 * p + c];
        k[3 + c] = a.V[3 * p + c];
    }
    double o[3];
    axis_of(q, o);
    const double oL = o[0] * L[0] + o[1] * L[1] + o[2] * L[2];
    const double kk = 1.0 / a.Ipar - 1.0 / a.Iperp;
    for (int c = 0; c < 3; c++) {
        k[6 + c] = L[c] / a.Iperp + kk * oL * o[c];
        k[9 + c] = o[c];
    }
    // FP32 form for the node-velocity stencils: u(s) = U0 + Omega x (s - b)
    // with b the lattice node nearest to X (s - b a small integer vector)
    const int L3[3] = {a.nx, a.ny, a.nz};
    int b[3];
    double U0[3];
    double db[3];
    for (int c = 0; c < 3; c++) {
        b[c] = (int)floor(k[c] + 0.5);
        db[c] = (double)b[c] - k[c];
        if (c == 1 && a.wall_y) continue;  // no periodic image across the walls
        if (b[c] >= L3[c]) b[c] -= L3[c];
        if (b[c] < 0) b[c] += L3[c];
    }
    cross3(k + 6, db, U0);
    double* kd = a.kin + 12 * (long long)p;
    for (int c = 0; c < 12; c++) kd[c] = k[c];
    float* kf = a.kinf + 12 * (long long)p;
    for (int c = 0; c < 3; c++) {
        kf[c] = (float)(k[3 + c] + U0[c]);
        kf[3 + c] = (float)k[6 + c];
    }
    kf[6] = __int_as_float(b[0] | (b[1] << 16));
    kf[7] = __int_as_float(b[2]);
    for (int c = 0; c < 3; c++) kf[8 + c] = (float)(-db[c]);  // X - b, in [-1/2, 1/2]
    kf[11] = 0.0f;
    if (zero_forces) {
        for (int c = 0; c < 6; c++) { a.FTh[6 * p + c] = 0.0; a.FTp[6 * p + c] = 0.0; }
        for (int c = 0; c < 12; c++) a.FTt[12 * (long long)p + c] = 0ull;
    }
}

__global__ void prep_kernel(DevArgs a, int zero_forces) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    double k[12];
    prep_one(a, p, zero_forces != 0, k);
}

hipError_t launch_prep(const DevArgs& a, hipStream_t st) {
    if (a.n == 0) return hipSuccess;
    hipLaunchKernelGGL(prep_kernel, dim3((a.n + 255) / 256), dim3(256), 0, st, a, 1);
    return hipGetLastError();
}

hipError_t launch_kin(const DevArgs& a, hipStream_t st) {
    if (a.n == 0) return hipSuccess;
    hipLaunchKernelGGL(prep_kernel, dim3((a.n + 255) / 256), dim3(256), 0, st, a, 0);
    return hipGetLastError();
}

// all cell nodes become fluid at rest (rho0); used before a fresh rasterisation
template <int P>
__global__ void clear_cells_kernel(DevArgs a) {
    using Cd = Codec<P>;
    using T = typename Cd::T;
    using R = typename Cd::R;
    const long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (s >= a.ns) return;
    a.cand[s] = NO_CAND;
    if (a.owner[s] < 0) return;
    a.owner[s] = OWN_FLUID;
    T* A = (T*)a.A;
    const long long c = sidx(a, s);
    for (int r = 0; r < 19; r++) A[r * a.pstride + c] = Cd::enc((R)0, enc_scale<P>(a, r));
    ((T*)a.rhoA)[c] = Cd::enc((R)0, rho_enc_scale<P>(a));
}

hipError_t launch_clear_cells(const DevArgs& a, hipStream_t st) {
    dim3 g((unsigned)((a.ns + 255) / 256)), b(256);
    switch (a.precision) {
        case CGB_P64: hipLaunchKernelGGL(clear_cells_kernel<CGB_P64>, g, b, 0, st, a); break;
        case CGB_P32: hipLaunchKernelGGL(clear_cells_kernel<CGB_P32>, g, b, 0, st, a); break;
        case CGB_PMX16: hipLaunchKernelGGL(clear_cells_kernel<CGB_PMX16>, g, b, 0, st, a); break;
        case CGB_PMXBF16: hipLaunchKernelGGL(clear_cells_kernel<CGB_PMXBF16>, g, b, 0, st, a); break;
        case CGB_PMX16S: hipLaunchKernelGGL(clear_cells_kernel<CGB_PMX16S>, g, b, 0, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ raster
// Axis-aligned half extents of the ellipsoid with axis o: along axis a every
// inside node has |x_a - X_a| < sqrt(R_perp^2 - (R_perp^2 - R_par^2) o_a^2);
// a small margin keeps nodes whose inside test rounds the other way.
__device__ inline void half_extents(const DevArgs& a, const double* o, double* h) {
    const double rp2 = 1.0 / a.iRperp2, rl2 = 1.0 / a.iRpar2;
    for (int c = 0; c < 3; c++) h[c] = sqrt(fmax(rp2 - (rp2 - rl2) * o[c] * o[c], 0.0)) + 1e-6;
}

// the box of the previous rasterisation: centre and half extents
struct PrevBox {
    double X[3], H[3];
};

__device__ inline PrevBox prev_box(const DevArgs& a, int p) {
    PrevBox b;
    for (int c = 0; c < 3; c++) { b.X[c] = a.Xprev[3 * p + c]; b.H[c] = a.Hprev[3 * p + c]; }
    return b;
}

// Node box of the current rasterisation (k: the cell's kinematics, h: its
// half extents) in lo, ext.  Returns false (and flags instability) when the
// union of that box with the box of the previous rasterisation (pb) is not
// finite or wider than a cell moving less than half a node per step can
// span, so that no state of the cells can send a walk outside the lattice.
__device__ inline bool cell_box(const DevArgs& a, const double* k, const double* h, const PrevBox& pb, int* lo, int* ext) {
    const int maxext = 2 * (int)ceil(a.Rb) + 6;
    for (int c = 0; c < 3; c++) {
        double x0 = pb.X[c];
        const double x1 = k[c];
        const double Lb = c == 0 ? a.nx : (c == 1 ? a.ny : a.nz);
        if (c != 1 || !a.wall_y) {
            // a cell that crossed the periodic boundary: unwrap the old position
            const double d = x0 - x1;
            if (d > 0.5 * Lb) x0 -= Lb;
            else if (d < -0.5 * Lb) x0 += Lb;
        }
        const double hp = pb.H[c];
        const double mn = fmin(x0 - hp, x1 - h[c]), mx = fmax(x0 + hp, x1 + h[c]);
        if (!(mn > -Lb && mx < 2.0 * Lb && mx - mn < (double)maxext)) {
            atomicOr(a.status, ST_UNSTABLE);
            return false;
        }
        lo[c] = (int)floor(x1 - h[c]);
        ext[c] = (int)ceil(x1 + h[c]) - lo[c] + 1;
    }
    return true;
}

__device__ inline bool covers(const DevArgs& a, const CellRec& c, int x, int y, int z) {
    double d[3];
    node_disp(a, x, y, z, c.X, d);
    return inside_test(a, d, c.o);
}

// cell records in cell-list order (the order of the previous cell list; any
// permutation of the cells gives the same results): record k describes cell p, whose
// kinematics are kp and whose previous box is pb (loaded by the caller
// before this overwrites it with the box of this rasterisation)
__device__ void record_one(const DevArgs& a, int k, int p, const double* kp, const PrevBox& pb) {
    CellRec c;
    for (int i = 0; i < 3; i++) { c.X[i] = kp[i]; c.V[i] = kp[3 + i]; c.W[i] = kp[6 + i]; c.o[i] = kp[9 + i]; }
    c.p = p;
    double h[3];
    half_extents(a, kp + 9, h);
    c.ok = cell_box(a, kp, h, pb, c.lo, c.ext) ? 1 : 0;
    if (!c.ok) {
        for (int i = 0; i < 3; i++) { c.lo[i] = 0; c.ext[i] = 0; }
    } else {
        for (int i = 0; i < 3; i++) { a.Xprev[3 * p + i] = kp[i]; a.Hprev[3 * p + i] = h[i]; }
    }
    ((CellRec*)a.crec)[k] = c;
}

__global__ void cellrec_kernel(DevArgs a) {
    const int k = xcd_block((int)blockIdx.x, (int)gridDim.x) * (int)blockDim.x + (int)threadIdx.x;
    if (k >= a.n) return;
    const int p = a.bin_idx[k];
    double kp[12];
    for (int c = 0; c < 12; c++) kp[c] = a.kin[12 * (long long)p + c];
    const PrevBox pb = prev_box(a, p);
    record_one(a, k, p, kp, pb);
}

hipError_t launch_cellrec(const DevArgs& a, hipStream_t st) {
    if (a.n == 0) return hipSuccess;
    hipLaunchKernelGGL(cellrec_kernel, dim3((a.n + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

// Claim pass: one wave per cell, CPW cells (waves) per workgroup: lane
// (ix, iy) of an 8 x 8 footprint walks z in slabs of ZB nodes whose loads are
// issued together.  Every node inside the cell that it does not own records
// the lowest covering index (the owner keeps a node it still covers, so it
// needs no claim), and every node inside the cell is appended to the cell's
// list (kept at the cell's record position, so that the momentum sum can load
// it without waiting for the record), in the fixed order (footprint, slab,
// plane, lane): after the resolve
// pass the nodes a cell owns are the listed nodes whose owner it is, which
// the momentum exchange walks instead of the box.  The waves of a workgroup
// work independently.
constexpr int ZB = 8;
constexpr int CPW = 4;
constexpr unsigned LIST_OWNED = 0x80000000u;  // list entry of a node its cell already owned

__device__ __forceinline__ void claim_kernel_body(const DevArgs& a, const KCtx& G) {
    const unsigned nx = (unsigned)a.nx, plane = (unsigned)a.nx * (unsigned)a.ny;
    const int lane = threadIdx.x & 63;
    const int k = __builtin_amdgcn_readfirstlane(xcd_block((int)G.bx, (int)G.gx) * CPW + (int)(threadIdx.x >> 6));
    if (k >= a.n) return;
    // cells in cell-list order: neighbouring waves touch neighbouring nodes
    const CellRec cr = ((const CellRec*)a.crec)[k];
    if (!cr.ok) return;  // the record kernel has flagged the state as unstable
    const int p = cr.p;
    const int lo[3] = {cr.lo[0], cr.lo[1], cr.lo[2]};
    const int ext[3] = {cr.ext[0], cr.ext[1], cr.ext[2]};
    unsigned* lst = a.clist + (size_t)k * (size_t)a.lcap;
    int cnt = 0;  // the same in every lane
    for (int bx = 0; bx < ext[0]; bx += 8)
        for (int by = 0; by < ext[1]; by += 8) {
            const int ix = bx + (lane & 7), iy = by + (lane >> 3);
            bool col = ix < ext[0] && iy < ext[1];
            const int x = wrap(lo[0] + ix, a.nx);
            int y = lo[1] + iy;
            if (a.wall_y) col = col && y >= 0 && y < a.ny;
            else y = wrap(y, a.ny);
            for (int z0 = 0; z0 < ext[2]; z0 += ZB) {
                unsigned sj[ZB];
                int ow[ZB];
#pragma unroll
                for (int j = 0; j < ZB; j++) {
                    const bool ok = col && z0 + j < ext[2];
                    sj[j] = (unsigned)x + nx * (unsigned)y + plane * (unsigned)wrap(lo[2] + z0 + j, a.nz);
                    ow[j] = ok ? a.owner[sj[j]] : OWN_WALL;
                }
#pragma unroll
                for (int j = 0; j < ZB; j++) {
                    const int o = ow[j];
                    const int z = wrap(lo[2] + z0 + j, a.nz);
                    const bool in = o != OWN_WALL && covers(a, cr, x, y, z);
                    if (in && o != p) atomicMin(a.cand + sj[j], p);
                    // the viscometer's sheared planes must stay fluid
                    if (in && a.le_u != 0.0 && (x == 0 || x == a.nx - 1)) atomicOr(a.status, ST_LE_SEAM);
                    const unsigned long long m = __ballot(in);
                    if (in) {
                        // bit 31 marks a node the cell already owns: it keeps it
                        // (it still covers it), so the momentum exchange need not
                        // look its owner up (sites < 2^31)
                        const int e = cnt + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
                        if (e < a.lcap) lst[e] = sj[j] | (o == p ? LIST_OWNED : 0u);
                    }
                    cnt += __popcll(m);
                }
            }
        }
    if (lane == 0) {
        a.ccount[k] = cnt < a.lcap ? cnt : a.lcap;
        if (cnt > a.lcap) atomicOr(a.status, ST_LIST_OVERFLOW);
    }
}
__global__ void __launch_bounds__(64 * CPW) claim_kernel(DevArgs a) { claim_kernel_body(a, hw_ctx()); }
__global__ void __launch_bounds__(64 * CPW) claim_kernel_multi(const DevArgs* __restrict__ as, const ChanGrid* __restrict__ cg, int nch) {
    const int c = chan_of(cg, nch);
    claim_kernel_body(as[c], chan_ctx(cg[c]));
}


// Resolve pass, one thread per node, after every cell's claims: a cell node
// stays with its owner while the owner still covers it (single occupancy,
// first arrival keeps the node), otherwise goes to the lowest claimer,
// otherwise becomes fluid; a claimed fluid node goes to the lowest claimer.
// Changes go to the transition list (one reservation per wave) and the claims
// are cleared for the next step.  Every node a cell owns or claims is visited
// once, in lattice order, so the loads are coalesced and no box is walked.
__device__ __forceinline__ void resolve_kernel_body(const DevArgs& a, const KCtx& G) {
    const long long si = (long long)G.bx * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const bool in = si < a.ns;
    const unsigned s = in ? (unsigned)si : 0u;
    const int o = in ? a.owner[s] : OWN_WALL;
    const int c = in ? a.cand[s] : NO_CAND;
    int nw = o;
    if (o >= 0) {
        const double* k = a.kin + 12 * (long long)o;
        const double X[3] = {k[0], k[1], k[2]}, ax[3] = {k[9], k[10], k[11]};
        const unsigned nx = (unsigned)a.nx, ny = (unsigned)a.ny;
        double d[3];
        node_disp(a, (int)(s % nx), (int)((s / nx) % ny), (int)(s / (nx * ny)), X, d);
        nw = inside_test(a, d, ax) ? o : (c != NO_CAND ? c : OWN_FLUID);
    } else if (o == OWN_FLUID && c != NO_CAND) {
        nw = c;
    }
    if (c != NO_CAND) a.cand[s] = NO_CAND;
    const bool tr = nw != o;
    const unsigned long long m = __ballot(tr);
    if (m) {
        const int first = __ffsll((long long)m) - 1;
        int base = 0;
        const int seg = (int)(G.bx % TSEG);
        if (lane == first) base = atomicAdd(a.ntrans + seg, __popcll(m));
        base = __shfl(base, first, 64);
        if (tr) {
            const int t = base + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
            if (t < a.trans_cap) {
                const long long e = (long long)seg * a.trans_cap + t;
                a.trans[3 * e] = (int)s;
                a.trans[3 * e + 1] = o;
                a.trans[3 * e + 2] = nw;
            } else {
                atomicOr(a.status, ST_TRANS_OVERFLOW);
            }
        }
    }
}
__global__ void __launch_bounds__(256) resolve_kernel(DevArgs a) { resolve_kernel_body(a, hw_ctx()); }
__global__ void __launch_bounds__(256) resolve_kernel_multi(const DevArgs* __restrict__ as, const ChanGrid* __restrict__ cg, int nch) {
    const int c = chan_of(cg, nch);
    resolve_kernel_body(as[c], chan_ctx(cg[c]));
}


static inline unsigned cell_grid(int n) { return (unsigned)((n + CPW - 1) / CPW); }

// ------------------------------------------------------------------ momentum exchange
// Force and torque on each cell from its links (Eq. 12).  The LB kernel has
// stored, at every cell node s, the momentum m_s the links of s carried to the
// cell in this step (the deviation part of sum_r (2 n*_rbar + C_r) c_rbar over
// its fluid neighbours; the constant part and the solid links of Eqs. 13-14
// cancel over the closed surface of the cell's node set).  The transferred
// momentum of a link is parallel to c_r, so any point of the link line is a
// lever point; s is used: the torque is sum_s (s - X) x m_s.
// Two cells per wave (lanes 0-31 and 32-63), cells in cell-list order: each
// half walks its cell's list of covered nodes (written by the claim pass) and
// keeps the nodes the cell owns after the resolve pass; FP64 sums in list
// order, then over the half (the order is fixed: the result does not depend
// on scheduling).  The cover/uncover sums of the transitions are added.
__device__ __forceinline__ void mem_reduce_kernel_body(const DevArgs& a, const KCtx& G) {
    const int lane = threadIdx.x & 63, half = lane >> 5, hl = lane & 31;
    const int wv = threadIdx.x >> 6;
    const int k = 2 * __builtin_amdgcn_readfirstlane(xcd_block((int)G.bx, (int)G.gx) * CPW + wv) + half;
    if (2 * (k >> 1) >= a.n) return;  // whole wave: no cell
    const bool live = k < a.n;        // the second half of the last wave may have none
    const int kr = live ? k : k - 1;
    // the record, the list length and the first 32 list entries sit at the
    // record position: their loads go out together (entries past the length
    // are loaded and not used)
    const unsigned* lst = a.clist + (size_t)kr * (size_t)a.lcap;
    const unsigned ent0 = hl < a.lcap ? lst[hl] : 0u;
    const int cnt0 = a.ccount[kr];
    const CellRec cr = ((const CellRec*)a.crec)[kr];
    const int p = cr.p;
    // the record kernel flags a cell whose box is not valid; its list was not written
    int cnt = (live && cr.ok) ? cnt0 : 0;
    if (cnt > a.lcap) cnt = a.lcap;
    // the cover/uncover sums of the transitions, loaded beside the node momenta
    double ftt[6];
    {
        const unsigned long long* Ft = a.FTt + 12 * (long long)p;
#pragma unroll
        for (int c = 0; c < 6; c++) ftt[c] = fx_value(Ft + 2 * c);
    }
    const unsigned nx = (unsigned)a.nx, plane = (unsigned)a.nx * (unsigned)a.ny;
    double FT[6] = {0, 0, 0, 0, 0, 0};
    unsigned nxt = ent0;
    for (int e = hl; e < cnt; e += 32) {
        const unsigned ent = nxt;
        if (e + 32 < cnt) nxt = lst[e + 32];  // the lane's next entry, one pass ahead
        const unsigned s = ent & ~LIST_OWNED;
        const int o = (ent & LIST_OWNED) ? p : a.owner[s];
        double2 m01;
        double m2;
        if (a.big) {
            // large-lattice layout: the LB kernel left the momentum in the
            // node's own output slots
            const int es = a.precision == CGB_P64 ? 8 : (a.precision == CGB_P32 ? 4 : 2);
            m01.x = mom_from_slots(a.B, es, a.pstride, s, 0);
            m01.y = mom_from_slots(a.B, es, a.pstride, s, 1);
            m2 = mom_from_slots(a.B, es, a.pstride, s, 2);
        } else {
            const double* Fn = a.fnode + 3 * (size_t)sidx(a, s);
            m01.x = Fn[0];
            m01.y = Fn[1];
            m2 = Fn[2];
        }
        if (o != p) continue;
        double d[3];
        node_disp(a, (int)(s % nx), (int)((s / nx) % (unsigned)a.ny), (int)(s / plane), cr.X, d);
        FT[0] += m01.x; FT[1] += m01.y; FT[2] += m2;
        FT[3] += d[1] * m2 - d[2] * m01.y;
        FT[4] += d[2] * m01.x - d[0] * m2;
        FT[5] += d[0] * m01.y - d[1] * m01.x;
    }
    // sums over each half of the wave
#pragma unroll
    for (int c = 0; c < 6; c++)
#pragma unroll
        for (int off = 16; off >= 1; off >>= 1) FT[c] += __shfl_xor(FT[c], off, 64);
    if (hl == 0 && live) {
        double* F = a.FTh + 6 * (long long)p;
#pragma unroll
        for (int c = 0; c < 6; c++) F[c] = FT[c] + ftt[c];
    }
}
__global__ void __launch_bounds__(64 * CPW) mem_reduce_kernel(DevArgs a) { mem_reduce_kernel_body(a, hw_ctx()); }
__global__ void __launch_bounds__(64 * CPW) mem_reduce_kernel_multi(const DevArgs* __restrict__ as, const ChanGrid* __restrict__ cg, int nch) {
    const int c = chan_of(cg, nch);
    mem_reduce_kernel_body(as[c], chan_ctx(cg[c]));
}


hipError_t launch_mem_reduce(const DevArgs& a, hipStream_t st) {
    if (a.n == 0) return hipSuccess;
    hipLaunchKernelGGL(mem_reduce_kernel, dim3(cell_grid((a.n + 1) / 2)), dim3(64 * CPW), 0, st, a);
    return hipGetLastError();
}

// Boundary velocity field: a cell node gets the rigid-body velocity of its
// cell, V + Omega x (s - X) (the moving-boundary term of Eq. 10 uses it), a
// wall node its plane velocity (zero for resting walls), a fluid node zero.
// Runs after the occupancy update of the step.
// ALL: every node (at set-up).  Otherwise only groups of 32 consecutive nodes
// along x (one 128-byte line of an FP32 component plane) that hold a cell
// node are written, whole: the field is read only at non-fluid nodes, and
// wall nodes keep the values written at set-up.  Layout [3][pstride].
template <class M, bool ALL>
__global__ void __launch_bounds__(256) usol_kernel(DevArgs a) {
    const int lane = (int)(threadIdx.x & 63);
    const int x = (int)blockIdx.x * 64 + lane;
    const int y = (int)blockIdx.y * 4 + (int)(threadIdx.x >> 6);
    const int z = (int)blockIdx.z;
    const bool in = x < a.nx && y < a.ny;  // uniform over each wave in y, not in x
    const unsigned s = (unsigned)x + (unsigned)a.nx * ((unsigned)y + (unsigned)a.ny * (unsigned)z);
    const int o = in ? a.owner[s] : OWN_FLUID;
    bool wr = in;
    if (!ALL) {
        const unsigned long long m = __ballot(o >= 0);
        wr = in && ((m >> (lane & ~31)) & 0xffffffffull) != 0ull;
    }
    if (!wr) return;
    double u[3] = {0, 0, 0};
    if (o >= 0) {
        if constexpr (sizeof(M) == 4) {
            // FP32 link type: from the compact table, u = U0 + Omega x (s - b),
            // s - b taken to the periodic image nearest to the cell centre
            const float* kf = a.kinf + 12 * (long long)o;
            const float4 k0 = *(const float4*)kf, k1 = *(const float4*)(kf + 4), k2 = *(const float4*)(kf + 8);
            const int bxy = __float_as_int(k1.z);
            int d0 = x - (bxy & 0xffff), d1 = y - (bxy >> 16), d2 = z - __float_as_int(k1.w);
            d0 = image_shift(d0, k2.x, a.nx);
            if (!a.wall_y) d1 = image_shift(d1, k2.y, a.ny);
            d2 = image_shift(d2, k2.z, a.nz);
            const float e0 = (float)d0, e1 = (float)d1, e2 = (float)d2;
            // Omega = (k0.w, k1.x, k1.y)
            u[0] = k0.x + (k1.x * e2 - k1.y * e1);
            u[1] = k0.y + (k1.y * e0 - k0.w * e2);
            u[2] = k0.z + (k0.w * e1 - k1.x * e0);
        } else {
            const double* k = a.kin + 12 * (long long)o;
            double d[3];
            node_disp(a, x, y, z, k, d);
            cross3(k + 6, d, u);
            for (int c = 0; c < 3; c++) u[c] += k[3 + c];
        }
    } else if (o == OWN_WALL && a.wall_y) {
        if (y == 0) { u[0] = a.wvb[0]; u[1] = a.wvb[1]; u[2] = a.wvb[2]; }
        else if (y == a.ny - 1) { u[0] = a.wvt[0]; u[1] = a.wvt[1]; u[2] = a.wvt[2]; }
    }
    M* U = (M*)a.usol;
    const size_t ps = (size_t)a.pstride;
    U[s] = (M)u[0];
    U[ps + s] = (M)u[1];
    U[2 * ps + s] = (M)u[2];
}

hipError_t launch_usol(const DevArgs& a, hipStream_t st, bool all) {
    const dim3 g((unsigned)((a.nx + 63) / 64), (unsigned)((a.ny + 3) / 4), (unsigned)a.nz), b(256);
    if (a.precision == CGB_P64) {
        if (all) hipLaunchKernelGGL((usol_kernel<double, true>), g, b, 0, st, a);
        else hipLaunchKernelGGL((usol_kernel<double, false>), g, b, 0, st, a);
    } else {
        if (all) hipLaunchKernelGGL((usol_kernel<float, true>), g, b, 0, st, a);
        else hipLaunchKernelGGL((usol_kernel<float, false>), g, b, 0, st, a);
    }
    return hipGetLastError();
}

// tau = 1: moments of the moving-boundary corrections of every fluid node
// with links.  C_r = 6 w_r rho(x) (c_r . u(s_r)) (Eq. 10, u(s) the velocity of
// the non-fluid source s_r = x - c_r) enters the tau = 1 collision only
// through sum_r C_r and sum_r C_r c_r, and rho(x) factors out: the node needs
// K = (sum_r w_r q_r, sum_r w_r c_r q_r), q_r = c_r . u(s_r), over its links.
// A workgroup covers a TX x (256 / TX) patch and sweeps tz planes; the velocity
// of the patch and a one-node halo is built in LDS from the owner map and the
// cells' kinematics (the per-cell FP32 table for the FP32 link type, FP64
// kinematics for FP64), in a ring of four planes (three are read while the
// next is built), so the link sources are read from LDS.
// At a cell node the first three planes hold instead the rigid-body velocity
// u(s) of the node (the LB kernel's momentum exchange reads it there).
// Groups of 32 nodes along x (one 128-byte line of an FP32 plane) that hold a
// node with links or a cell node are written whole; layout [4][pstride].
// patch: TX x (256 / TX) nodes of an x-y plane, swept over tz planes
template <int TX>
struct LmShape {
    static constexpr int TY = 256 / TX, HX = TX + 2, HY = TY + 2, NP = HX * HY;
    static_assert(NP <= 512, "two positions per thread");
};


// site of halo'd plane position q of the patch at (x0, y0), plane z
template <int TX>
__device__ inline unsigned lm_site(const DevArgs& a, int q, int x0, int y0, int z, int* x, int* y) {
    using S = LmShape<TX>;
    const int hx = q % S::HX, hy = q / S::HX;
    *x = wrap_halo(x0 - 1 + hx, a.nx);
    *y = wrap_halo(y0 - 1 + hy, a.ny);
    return (unsigned)*x + (unsigned)a.nx * ((unsigned)*y + (unsigned)a.ny * (unsigned)z);
}

// velocity of position q with owner o, written to the plane in slot sl
// (NC = 4: the decoded stored density deviation dr of the split codec too)
template <class M, int TX, int NC>
__device__ inline void lm_vel(const DevArgs& a, M* U, int sl, int q, int o, uint32_t dr, int x, int y, int z) {
    using S = LmShape<TX>;
    double u[3] = {0, 0, 0};
    if (o >= 0) {
        if constexpr (sizeof(M) == 4) {
            // FP32 link type: from the compact table, u = U0 + Omega x (s - b),
            // s - b taken to the periodic image nearest to the cell centre
            const float* kf = a.kinf + 12 * (long long)o;
            const float4 k0 = *(const float4*)kf, k1 = *(const float4*)(kf + 4), k2 = *(const float4*)(kf + 8);
            const int bxy = __float_as_int(k1.z);
            int d0 = x - (bxy & 0xffff), d1 = y - (bxy >> 16), d2 = z - __float_as_int(k1.w);
            d0 = image_shift(d0, k2.x, a.nx);
            if (!a.wall_y) d1 = image_shift(d1, k2.y, a.ny);
            d2 = image_shift(d2, k2.z, a.nz);
            const float e0 = (float)d0, e1 = (float)d1, e2 = (float)d2;
            // Omega = (k0.w, k1.x, k1.y)
            u[0] = k0.x + (k1.x * e2 - k1.y * e1);
            u[1] = k0.y + (k1.y * e0 - k0.w * e2);
            u[2] = k0.z + (k0.w * e1 - k1.x * e0);
        } else {
            const double* k = a.kin + 12 * (long long)o;
            double d[3];
            node_disp(a, x, y, z, k, d);
            cross3(k + 6, d, u);
            for (int c = 0; c < 3; c++) u[c] += k[3 + c];
        }
    } else if (o == OWN_WALL && a.wall_y) {
        if (y == 0) { u[0] = a.wvb[0]; u[1] = a.wvb[1]; u[2] = a.wvb[2]; }
        else if (y == a.ny - 1) { u[0] = a.wvt[0]; u[1] = a.wvt[1]; u[2] = a.wvt[2]; }
    }
    M* P = U + (size_t)sl * NC * S::NP;
    P[q] = (M)u[0];
    P[S::NP + q] = (M)u[1];
    P[2 * S::NP + q] = (M)u[2];
    if constexpr (NC == 4) P[3 * S::NP + q] = (M)((float)__builtin_bit_cast(_Float16, (unsigned short)dr) * a.pmx_inv);
}

// owners (and, NC = 4, stored FP16 density deviations) of the two positions
// of this thread in plane z
template <int TX, int NC>
__device__ inline void lm_owners(const DevArgs& a, int x0, int y0, int z, int* o0, int* o1, uint32_t* d0, uint32_t* d1) {
    int x, y;
    const int q0 = (int)threadIdx.x, q1 = (int)threadIdx.x + 256;
    const unsigned s0 = lm_site<TX>(a, q0, x0, y0, z, &x, &y);
    const unsigned s1 = q1 < LmShape<TX>::NP ? lm_site<TX>(a, q1, x0, y0, z, &x, &y) : s0;
    *o0 = a.owner[s0];
    *o1 = q1 < LmShape<TX>::NP ? a.owner[s1] : OWN_FLUID;
    if constexpr (NC == 4) {
        // (walls of the indexed layout hold no density: 0, like the stored
        // zeros of a wall in the dense layout)
        const unsigned short* D = (const unsigned short*)a.rhoA;
        const long long c0 = sidx(a, s0), c1 = sidx(a, s1);
        *d0 = c0 >= 0 ? D[c0] : 0u;
        *d1 = c1 >= 0 ? D[c1] : 0u;
    }
}

template <class M, int TX, int NC>
__device__ inline void lm_build(const DevArgs& a, M* U, int sl, int x0, int y0, int z, int o0, int o1, uint32_t d0, uint32_t d1) {
    int x, y;
    const int q0 = (int)threadIdx.x, q1 = (int)threadIdx.x + 256;
    lm_site<TX>(a, q0, x0, y0, z, &x, &y);
    lm_vel<M, TX, NC>(a, U, sl, q0, o0, d0, x, y, z);
    if (q1 < LmShape<TX>::NP) {
        lm_site<TX>(a, q1, x0, y0, z, &x, &y);
        lm_vel<M, TX, NC>(a, U, sl, q1, o1, d1, x, y, z);
    }
}

// workgroup barrier that waits for this wave's LDS accesses only: global
// loads in flight (the prefetched owners and flags) stay in flight
__device__ inline void lm_lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// NC = 4 (split FP16 codec): besides the link moments, each fluid node gets
// the density parts of its pulled populations, T = (sum_r w_r D_r,
// sum_r w_r c_r D_r) with D_r the stored density deviation of the source of
// direction r (the node's own for the rest direction and for a bounced
// population), and stores E = 6 rho(x) K + T, which the LB adds to its sums
// of the FP16 residuals; every site is written (zeros at non-fluid nodes).
// NT: the moments are stored non-temporally (the split codec's form, which
// writes every site, on lattices whose output outgrows the last-level cache,
// see nt_out); the LB, a later launch, reads them
template <class M, int TX, int NC, bool NT = false>
__device__ __forceinline__ void lmom_kernel_body(const DevArgs& a, const KCtx& G, int tz) {
    using S = LmShape<TX>;
    __shared__ M U[4 * NC * S::NP];  // [slot][component][HY][HX]
    const int tx = (int)(threadIdx.x % TX), ty = (int)(threadIdx.x / TX);
    const int x0 = (int)G.bx * TX, y0 = (int)G.by * S::TY, z0 = (int)G.bz * tz;
    const int x = x0 + tx, y = y0 + ty;
    const bool in = x < a.nx && y < a.ny;
    const int zend = a.nz - z0 < tz ? a.nz - z0 : tz;
    M* K = (M*)a.lmom;
    const size_t ps = (size_t)a.pstride;
    const int lane = (int)(threadIdx.x & 63);
    const unsigned s0 = (unsigned)x + (unsigned)a.nx * ((unsigned)y + (unsigned)a.ny * (unsigned)z0);
    const unsigned plane = (unsigned)a.nx * (unsigned)a.ny;
    // plane p lives in slot (p - z0 + 1) & 3 of a four-plane ring: at step z
    // planes z - 1, z, z + 1 are read while plane z + 2 is written, so one
    // barrier per step suffices; owners are read one plane ahead and the
    // node's flags one step ahead, and stay in flight across the barrier
    int o0, o1, n0, n1;
    uint32_t e0 = 0, e1 = 0, m0 = 0, m1 = 0;
    lm_owners<TX, NC>(a, x0, y0, wrap_halo(z0 - 1, a.nz), &o0, &o1, &e0, &e1);
    lm_owners<TX, NC>(a, x0, y0, z0, &n0, &n1, &m0, &m1);
    lm_build<M, TX, NC>(a, U, 0, x0, y0, wrap_halo(z0 - 1, a.nz), o0, o1, e0, e1);
    lm_owners<TX, NC>(a, x0, y0, wrap_halo(z0 + 1, a.nz), &o0, &o1, &e0, &e1);
    lm_build<M, TX, NC>(a, U, 1, x0, y0, z0, n0, n1, m0, m1);
    uint32_t fnext = in ? a.flags[s0] : NONFLUID;
    for (int zz = 0; zz < zend; zz++) {
        const int z = z0 + zz;
        const unsigned s = s0 + plane * (unsigned)zz;
        const uint32_t f = fnext;
        fnext = (in && zz + 1 < zend) ? a.flags[s + plane] : NONFLUID;
        if (zz + 1 < zend) lm_owners<TX, NC>(a, x0, y0, wrap_halo(z + 2, a.nz), &n0, &n1, &m0, &m1);
        lm_build<M, TX, NC>(a, U, (zz + 2) & 3, x0, y0, wrap_halo(z + 1, a.nz), o0, o1, e0, e1);
        o0 = n0; o1 = n1; e0 = m0; e1 = m1;
        lm_lds_barrier();
        const bool fl = !(f & NONFLUID);
        const bool lk = fl && (f & LINKBITS) != 0u;
        const bool cn = (f & NONFLUID) && !(f & WALLNODE);  // a cell node (lanes outside read NONFLUID | 0)
        const unsigned long long m = __ballot(NC == 4 ? fl : (lk || (in && cn)));
        if (in && (NC == 4 || ((m >> (lane & ~31)) & 0xffffffffull) != 0ull)) {
            // sums over the links (directions that are not links weigh 0)
            M k0 = 0, k1 = 0, k2 = 0, k3 = 0;
            M t0 = 0, t1 = 0, t2 = 0, t3 = 0;
            M Dx = 0;
            if constexpr (NC == 4) {
                Dx = U[(size_t)((zz + 1) & 3) * NC * S::NP + 3 * S::NP + (ty + 1) * S::HX + (tx + 1)];
                t0 = (M)(1.0 / 3.0) * Dx;
            }
            if constexpr (NC == 4) {
                // density parts first, then the link sums (fewer values live at once)
#pragma unroll
                for (int r = 1; r < 19; r++) {
                    const M* P = U + (size_t)((zz + 1 - CZ(r)) & 3) * NC * S::NP + (ty + 1 - CY(r)) * S::HX + (tx + 1 - CX(r));
                    const M wd = (M)WD(r) * (((f >> r) & 1u) ? Dx : P[3 * S::NP]);
                    t0 += wd;
                    if (CX(r)) t1 += (M)CX(r) * wd;
                    if (CY(r)) t2 += (M)CY(r) * wd;
                    if (CZ(r)) t3 += (M)CZ(r) * wd;
                }
                __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int r = 1; r < 19; r++) {
                const M* P = U + (size_t)((zz + 1 - CZ(r)) & 3) * NC * S::NP + (ty + 1 - CY(r)) * S::HX + (tx + 1 - CX(r));
                M q = 0;
                if (CX(r)) q += (M)CX(r) * P[0];
                if (CY(r)) q += (M)CY(r) * P[S::NP];
                if (CZ(r)) q += (M)CZ(r) * P[2 * S::NP];
                const bool bb = (f >> r) & 1u;
                const M wq = (lk && bb) ? (M)WD(r) * q : (M)0;
                k0 += wq;
                if (CX(r)) k1 += (M)CX(r) * wq;
                if (CY(r)) k2 += (M)CY(r) * wq;
                if (CZ(r)) k3 += (M)CZ(r) * wq;
            }
            if constexpr (NC == 4) {
                const M rho6 = (M)6 * ((M)a.rho0 + Dx);
                k0 = fl ? rho6 * k0 + t0 : (M)0;
                k1 = fl ? rho6 * k1 + t1 : (M)0;
                k2 = fl ? rho6 * k2 + t2 : (M)0;
                k3 = fl ? rho6 * k3 + t3 : (M)0;
            }
            if (cn) {
                const M* P = U + (size_t)((zz + 1) & 3) * NC * S::NP + (ty + 1) * S::HX + (tx + 1);
                k0 = P[0]; k1 = P[S::NP]; k2 = P[2 * S::NP]; k3 = (M)0;
            }
            const long long c = sidx(a, s);
            if (c >= 0) {
                if constexpr (NT) {
                    __builtin_nontemporal_store(k0, K + c);
                    __builtin_nontemporal_store(k1, K + ps + c);
                    __builtin_nontemporal_store(k2, K + 2 * ps + c);
                    __builtin_nontemporal_store(k3, K + 3 * ps + c);
                } else {
                    K[c] = k0;
                    K[ps + c] = k1;
                    K[2 * ps + c] = k2;
                    K[3 * ps + c] = k3;
                }
            }
        }
    }
}
// waves per SIMD each form holds without spilling (the split codec's form
// needs 80 registers: asking for 6 keeps it there, where 8 left it at 81 and
// so at 5 waves)
template <class M, int NC>
constexpr int LM_WAVES = sizeof(M) == 4 ? (NC == 4 ? 6 : 8) : 5;
template <class M, int TX, int NC, bool NT = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(LM_WAVES<M, NC>))) lmom_kernel(DevArgs a, int tz) { lmom_kernel_body<M, TX, NC, NT>(a, hw_ctx(), tz); }
template <class M, int TX, int NC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(LM_WAVES<M, NC>))) lmom_kernel_multi(const DevArgs* __restrict__ as, const ChanGrid* __restrict__ cg, int nch) {
    unsigned t;
    const int c = chan_of_xcd(cg, nch, &t);
    lmom_kernel_body<M, TX, NC>(as[c], chan_ctx_at(cg[c], t), cg[c].arg);
}


// workgroups of a link-moment kernel resident on the whole device at once
// (0 if the runtime cannot say); fixed per process
template <class M, int TX, int NC>
static int lm_resident() {
    static const int n = [] {
        int dev = 0, ncu = 0, per = 0;
        if (hipGetDevice(&dev) != hipSuccess) return 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, lmom_kernel<M, TX, NC>, 256, 0) != hipSuccess) return 0;
        return ncu * per;
    }();
    return n;
}

// Patches 32 nodes wide and 8 rows deep on every lattice: against 64 x 4
// they build fewer halo nodes per node (340 against 396 per 256) and leave
// no more lanes idle on any width (fewer on widths between 65 and 96, the
// batch's wider channels: its step took 3.25 against 3.33 ms; at 256^3 the
// two tie).  A large lattice is swept in
// as few slabs as fill the device with one round of resident workgroups (each
// workgroup builds two planes before its first node, so long sweeps cost
// less, and a second, partial round would leave the device part idle); a
// short sweep when long sweeps would leave the device with few workgroups.
template <class M, int TX, int NC>
static dim3 lm_grid(const DevArgs& a, int* tzo, bool batch = false) {
    const int ty = 256 / TX;
    if (batch) {
        // a launch for every channel of a batch fills the device by itself:
        // sweeps of 16 planes (each node's moments do not depend on the sweep)
        *tzo = 16;
        return dim3((unsigned)((a.nx + TX - 1) / TX), (unsigned)((a.ny + ty - 1) / ty), (unsigned)((a.nz + 15) / 16));
    }
    const long long patches = (long long)((a.nx + TX - 1) / TX) * ((a.ny + ty - 1) / ty);
    int tz = 4;
    if (patches * ((a.nz + 15) / 16) >= 2048) {
        tz = 16;
        const long long slabs = lm_resident<M, TX, NC>() / patches;
        if (slabs >= 1) {
            const long long t = (a.nz + slabs - 1) / slabs;
            if (t >= 8) tz = (int)t;
        }
    }
    *tzo = tz;
    return dim3((unsigned)((a.nx + TX - 1) / TX), (unsigned)((a.ny + ty - 1) / ty), (unsigned)((a.nz + tz - 1) / tz));
}

template <class M, int TX, int NC>
static void lm_launch(const DevArgs& a, hipStream_t st) {
    int tz = 0;
    const dim3 g = lm_grid<M, TX, NC>(a, &tz);
    if (NC == 4 && a.nt_out) hipLaunchKernelGGL((lmom_kernel<M, TX, NC, true>), g, dim3(256), 0, st, a, tz);
    else hipLaunchKernelGGL((lmom_kernel<M, TX, NC>), g, dim3(256), 0, st, a, tz);
}

hipError_t launch_lmom(const DevArgs& a, hipStream_t st) {
    if (a.precision == CGB_P64) lm_launch<double, 32, 3>(a, st);
    else if (a.precision == CGB_PMX16S) lm_launch<float, 32, 4>(a, st);
    else lm_launch<float, 32, 3>(a, st);
    return hipGetLastError();
}

__global__ void zero_int_kernel(int* p) { *p = 0; }

// start of a time step: clear the transition list and advance the device-side
// step index (kernels read the step from device memory, so a captured step
// sequence stays correct when it is replayed)
__global__ void step_begin_kernel(int* ntrans, int* dstep, int advance) {
    if (threadIdx.x < TSEG) ntrans[threadIdx.x] = 0;
    if (threadIdx.x == 0 && advance) *dstep += 1;
}

// Start of a time step in one launch: clear the transition list and advance
// the device-side step index (block 0), and for each cell its axis, angular
// velocity and FP32 velocity table, zeroed force sums and its record, written
// at the cell's position in the previous cell list (the thread that computes
// a cell's kinematics writes its record, so the two need no separate passes).
__device__ __forceinline__ void step_prep_kernel_body(const DevArgs& a, const KCtx& G) {
    if (G.bx == 0) {
        if (threadIdx.x < TSEG) a.ntrans[threadIdx.x] = 0;
        if (threadIdx.x == 0) *a.dstep += 1;
    }
    const int p = G.bx * blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    // the record's inputs are loaded before prep_one stores
    const int rk = a.rank[p];
    const PrevBox pb = prev_box(a, p);
    double k[12];
    prep_one(a, p, true, k);
    record_one(a, rk, p, k, pb);
}
__global__ void step_prep_kernel(DevArgs a) { step_prep_kernel_body(a, hw_ctx()); }
__global__ void step_prep_kernel_multi(const DevArgs* __restrict__ as, const ChanGrid* __restrict__ cg, int nch) {
    const int c = chan_of(cg, nch);
    step_prep_kernel_body(as[c], chan_ctx(cg[c]));
}


hipError_t launch_step_prep(const DevArgs& a, hipStream_t st) {
    if (a.n == 0) hipLaunchKernelGGL(step_begin_kernel, dim3(1), dim3(TSEG), 0, st, a.ntrans, a.dstep, 1);
    else hipLaunchKernelGGL(step_prep_kernel, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

// records: the set-up path builds the step-begin state and the records here;
// a time step has them from launch_step_prep
hipError_t launch_raster(const DevArgs& a, hipStream_t st, bool fresh, bool records) {
    if (records) hipLaunchKernelGGL(step_begin_kernel, dim3(1), dim3(TSEG), 0, st, a.ntrans, a.dstep, fresh ? 0 : 1);
    if (a.n == 0) return hipGetLastError();
    if (records) hipLaunchKernelGGL(cellrec_kernel, dim3((a.n + 255) / 256), dim3(256), 0, st, a);
    hipLaunchKernelGGL(claim_kernel, dim3(cell_grid(a.n)), dim3(64 * CPW), 0, st, a);
    hipLaunchKernelGGL(resolve_kernel, dim3((unsigned)((a.ns + 255) / 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

// ------------------------------------------------------------------ transitions
template <int P>
__device__ void transition_one(const DevArgs& a, int t, bool book) {
    using Cd = Codec<P>;
    using T = typename Cd::T;
    using R = typename Cd::R;
    const long long s = a.trans[3 * t];
    const int o = a.trans[3 * t + 1], nw = a.trans[3 * t + 2];
    const int x = (int)(s % a.nx), y = (int)((s / a.nx) % a.ny), z = (int)(s / ((long long)a.nx * a.ny));
    T* A = (T*)a.A;
    const long long c = sidx(a, s);  // storage index (a transition never involves a wall)
    a.owner[s] = nw;
    const bool was_fluid = (o == OWN_FLUID), is_fluid = (nw == OWN_FLUID);
    if (was_fluid != is_fluid) {
        atomicXor(a.flags + s, NONFLUID);
        for (int r = 1; r < 19; r++) {
            const int xn = wrap(x + CX(r), a.nx), yn = wrap(y + CY(r), a.ny), zn = wrap(z + CZ(r), a.nz);
            const long long tn = xn + (long long)a.nx * (yn + (long long)a.ny * zn);
            atomicXor(a.flags + tn, 1u << r);
        }
    }
    if (was_fluid && !is_fluid) {
        if (!book) return;
        // covered: the deleted fluid momentum goes to the cell
        double m[3] = {0, 0, 0};
        const R Ds = rho_dec<P>(a, ((const T*)a.rhoA)[c]);
        for (int r = 0; r < 19; r++) {
            const double v = (double)pop_dec<P>(a, A[r * a.pstride + c], r, Ds);
            m[0] += v * CX(r); m[1] += v * CY(r); m[2] += v * CZ(r);
        }
        double d[3], tq[3];
        node_disp(a, x, y, z, a.kin + 12 * (long long)nw, d);
        cross3(d, m, tq);
        unsigned long long* F = a.FTt + 12 * (long long)nw;
        for (int c = 0; c < 3; c++) { fx_add(F + 2 * c, m[c]); fx_add(F + 6 + 2 * c, tq[c]); }
    } else if (!was_fluid && is_fluid) {
        if (!book) {
            for (int r = 0; r < 19; r++) A[r * a.pstride + c] = Cd::enc((R)0, enc_scale<P>(a, r));
            ((T*)a.rhoA)[c] = Cd::enc((R)0, rho_enc_scale<P>(a));
            return;
        }
        // freed: fluid at rho0 with the rigid-body velocity of the cell
        const double* k = a.kin + 12 * (long long)o;
        double d[3], us[3];
        node_disp(a, x, y, z, k, d);
        cross3(k + 6, d, us);
        for (int c = 0; c < 3; c++) us[c] += k[3 + c];
        const double usq = us[0] * us[0] + us[1] * us[1] + us[2] * us[2];
        double m[3] = {0, 0, 0};
        R rs = 0;
        for (int r = 0; r < 19; r++) {
            const double cu = CX(r) * us[0] + CY(r) * us[1] + CZ(r) * us[2];
            const double poly = 3.0 * cu + 4.5 * cu * cu - 1.5 * usq + 4.5 * cu * cu * cu - 4.5 * usq * cu;
            const double eq = WD(r) * (0.0 + a.rho0 * poly);
            // split codec: the density deviation of the new fluid is 0
            const T stv = pop_enc<P>(a, (R)eq, r, (R)0);
            A[r * a.pstride + c] = stv;
            const R back = pop_dec<P>(a, stv, r, (R)0);
            rs += back;
            m[0] += (double)back * CX(r); m[1] += (double)back * CY(r); m[2] += (double)back * CZ(r);
        }
        ((T*)a.rhoA)[c] = Cd::enc(Cd::SPLIT ? (R)0 : rs, rho_enc_scale<P>(a));
        double tq[3];
        cross3(d, m, tq);
        unsigned long long* F = a.FTt + 12 * (long long)o;
        for (int c = 0; c < 3; c++) { fx_add(F + 2 * c, -m[c]); fx_add(F + 6 + 2 * c, -tq[c]); }
    }
}

// TSEG x 8 blocks: block b takes segment b % TSEG
template <int P>
__device__ __forceinline__ void transitions_kernel_body(const DevArgs& a, const KCtx& G, int book) {
    const int seg = G.bx % TSEG, part = G.bx / TSEG, nparts = G.gx / TSEG;
    const int cnt = min(a.ntrans[seg], a.trans_cap);
    for (int t = part * blockDim.x + threadIdx.x; t < cnt; t += nparts * blockDim.x)
        transition_one<P>(a, (int)((long long)seg * a.trans_cap + t), book != 0);
}
template <int P>
__global__ void transitions_kernel(DevArgs a, int book) { transitions_kernel_body<P>(a, hw_ctx(), book); }
template <int P>
__global__ void transitions_kernel_multi(const DevArgs* __restrict__ as, const ChanGrid* __restrict__ cg, int nch, int book) {
    const int c = chan_of(cg, nch);
    transitions_kernel_body<P>(as[c], chan_ctx(cg[c]), book);
}


hipError_t launch_transitions(const DevArgs& a, hipStream_t st, bool book) {
    dim3 g(TSEG * 8), b(256);
    switch (a.precision) {
        case CGB_P64: hipLaunchKernelGGL(transitions_kernel<CGB_P64>, g, b, 0, st, a, (int)book); break;
        case CGB_P32: hipLaunchKernelGGL(transitions_kernel<CGB_P32>, g, b, 0, st, a, (int)book); break;
        case CGB_PMX16: hipLaunchKernelGGL(transitions_kernel<CGB_PMX16>, g, b, 0, st, a, (int)book); break;
        case CGB_PMXBF16: hipLaunchKernelGGL(transitions_kernel<CGB_PMXBF16>, g, b, 0, st, a, (int)book); break;
        case CGB_PMX16S: hipLaunchKernelGGL(transitions_kernel<CGB_PMX16S>, g, b, 0, st, a, (int)book); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ flags
__global__ void flags_rebuild_kernel(DevArgs a) {
    const long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (s >= a.ns) return;
    const int x = (int)(s % a.nx), y = (int)((s / a.nx) % a.ny), z = (int)(s / ((long long)a.nx * a.ny));
    const int own = a.owner[s];
    uint32_t f = (own != OWN_FLUID) ? NONFLUID : 0u;
    if (own == OWN_WALL) f |= WALLNODE;
    for (int r = 1; r < 19; r++) {
        const int xs = wrap(x - CX(r), a.nx), ys = wrap(y - CY(r), a.ny), zs = wrap(z - CZ(r), a.nz);
        if (a.owner[xs + (long long)a.nx * (ys + (long long)a.ny * zs)] != OWN_FLUID) f |= 1u << r;
    }
    a.flags[s] = f;
}

hipError_t launch_flags_rebuild(const DevArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(flags_rebuild_kernel, dim3((unsigned)((a.ns + 255) / 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

// ------------------------------------------------------------------ fills
__global__ void fill_i32_kernel(int* p, long long n, int v) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void fill_f64_kernel(double* p, long long n, double v) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) p[i] = v;
}
hipError_t launch_fill_i32(int* p, long long n, int v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    long long nb = (n + 255) / 256;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)nb), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}
hipError_t launch_fill_f64(double* p, long long n, double v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    long long nb = (n + 255) / 256;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(fill_f64_kernel, dim3((unsigned)nb), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

// ------------------------------------------------------------------ cell list
__device__ inline int bin_coord(const DevArgs& a, int c, double v) {
    if (!(v == v)) return 0;
    int b = (int)floor(v / a.bedge[c]);
    if (b < 0) b = 0;
    if (b >= a.nb[c]) b = a.nb[c] - 1;
    return b;
}

__device__ __forceinline__ void bin_clear_kernel_body(const DevArgs& a, const KCtx& G) {
    const int b = G.bx * blockDim.x + threadIdx.x;
    if (b < a.nbins) a.bin_count[b] = 0;
}
__global__ void bin_clear_kernel(DevArgs a) { bin_clear_kernel_body(a, hw_ctx()); }
__global__ void bin_clear_kernel_multi(const DevArgs* __restrict__ as, const ChanGrid* __restrict__ cg, int nch) {
    const int c = chan_of(cg, nch);
    bin_clear_kernel_body(as[c], chan_ctx(cg[c]));
}


__device__ __forceinline__ void bin_count_kernel_body(const DevArgs& a, const KCtx& G) {
    const int p = G.bx * blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    const int bx = bin_coord(a, 0, a.X[3 * p]), by = bin_coord(a, 1, a.X[3 * p + 1]), bz = bin_coord(a, 2, a.X[3 * p + 2]);
    const int b = bx + a.nb[0] * (by + a.nb[1] * bz);
    a.pbin[p] = b;
    atomicAdd(a.bin_count + b, 1);
}
__global__ void bin_count_kernel(DevArgs a) { bin_count_kernel_body(a, hw_ctx()); }
__global__ void bin_count_kernel_multi(const DevArgs* __restrict__ as, const ChanGrid* __restrict__ cg, int nch) {
    const int c = chan_of(cg, nch);
    bin_count_kernel_body(as[c], chan_ctx(cg[c]));
}


// exclusive scan of bin_count into bin_start[0..nbins]: (1) each block of 256
// threads scans 4096 bins (16 per thread) and records its total, (2) one block
// scans the block totals, (3) each block adds its offset
constexpr int SCAN_PER_BLOCK = 4096;
__device__ __forceinline__ void scan_local_kernel_body(const DevArgs& a, const KCtx& G) {
    __shared__ int tot[256];
    int* block_tot = a.scan_tmp;
    const int base = G.bx * SCAN_PER_BLOCK + threadIdx.x * 16;
    int v[16], s = 0;
    for (int k = 0; k < 16; k++) {
        const int b = base + k;
        v[k] = b < a.nbins ? a.bin_count[b] : 0;
        s += v[k];
    }
    tot[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int t = threadIdx.x >= off ? tot[threadIdx.x - off] : 0;
        __syncthreads();
        tot[threadIdx.x] += t;
        __syncthreads();
    }
    int run = threadIdx.x ? tot[threadIdx.x - 1] : 0;
    for (int k = 0; k < 16; k++) {
        const int b = base + k;
        if (b < a.nbins) { a.bin_start[b] = run; a.bin_fill[b] = 0; }
        run += v[k];
    }
    if (threadIdx.x == 255) block_tot[G.bx] = tot[255];
}
__global__ void __launch_bounds__(256) scan_local_kernel(DevArgs a) { scan_local_kernel_body(a, hw_ctx()); }
__global__ void __launch_bounds__(256) scan_local_kernel_multi(const DevArgs* __restrict__ as, const ChanGrid* __restrict__ cg, int nch) {
    const int c = chan_of(cg, nch);
    scan_local_kernel_body(as[c], chan_ctx(cg[c]));
}


__device__ __forceinline__ void scan_top_kernel_body(const DevArgs& a, const KCtx& G) {
    __shared__ int tot[1024];
    int* block_tot = a.scan_tmp;
    const int nblk = (a.nbins + SCAN_PER_BLOCK - 1) / SCAN_PER_BLOCK;
    int* total_out = a.bin_start + a.nbins;
    const int chunk = (nblk + 1023) / 1024;
    const int t = threadIdx.x;
    int s = 0;
    for (int k = 0; k < chunk; k++) { const int b = t * chunk + k; if (b < nblk) s += block_tot[b]; }
    tot[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int v = t >= off ? tot[t - off] : 0;
        __syncthreads();
        tot[t] += v;
        __syncthreads();
    }
    int run = t ? tot[t - 1] : 0;
    for (int k = 0; k < chunk; k++) {
        const int b = t * chunk + k;
        if (b < nblk) { const int v = block_tot[b]; block_tot[b] = run; run += v; }
    }
    if (t == 1023) *total_out = tot[1023];
}
__global__ void __launch_bounds__(1024) scan_top_kernel(DevArgs a) { scan_top_kernel_body(a, hw_ctx()); }
__global__ void __launch_bounds__(1024) scan_top_kernel_multi(const DevArgs* __restrict__ as, const ChanGrid* __restrict__ cg, int nch) {
    const int c = chan_of(cg, nch);
    scan_top_kernel_body(as[c], chan_ctx(cg[c]));
}


__device__ __forceinline__ void scan_add_kernel_body(const DevArgs& a, const KCtx& G) {
    const int* block_off = a.scan_tmp;
    const int b = G.bx * blockDim.x + threadIdx.x;
    if (b < a.nbins) a.bin_start[b] += block_off[b / SCAN_PER_BLOCK];
}
__global__ void scan_add_kernel(DevArgs a) { scan_add_kernel_body(a, hw_ctx()); }
__global__ void scan_add_kernel_multi(const DevArgs* __restrict__ as, const ChanGrid* __restrict__ cg, int nch) {
    const int c = chan_of(cg, nch);
    scan_add_kernel_body(as[c], chan_ctx(cg[c]));
}


__device__ __forceinline__ void bin_fill_kernel_body(const DevArgs& a, const KCtx& G) {
    const int p = G.bx * blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    const int b = a.pbin[p];
    const int pos = a.bin_start[b] + atomicAdd(a.bin_fill + b, 1);
    a.bin_idx[pos] = p;
}
__global__ void bin_fill_kernel(DevArgs a) { bin_fill_kernel_body(a, hw_ctx()); }
__global__ void bin_fill_kernel_multi(const DevArgs* __restrict__ as, const ChanGrid* __restrict__ cg, int nch) {
    const int c = chan_of(cg, nch);
    bin_fill_kernel_body(as[c], chan_ctx(cg[c]));
}


__device__ __forceinline__ void bin_sort_kernel_body(const DevArgs& a, const KCtx& G) {
    const int b = G.bx * blockDim.x + threadIdx.x;
    if (b >= a.nbins) return;
    const int s = a.bin_start[b], e = a.bin_start[b + 1];
    for (int i = s + 1; i < e; i++) {
        const int v = a.bin_idx[i];
        int j = i - 1;
        while (j >= s && a.bin_idx[j] > v) { a.bin_idx[j + 1] = a.bin_idx[j]; j--; }
        a.bin_idx[j + 1] = v;
    }
}
__global__ void bin_sort_kernel(DevArgs a) { bin_sort_kernel_body(a, hw_ctx()); }
__global__ void bin_sort_kernel_multi(const DevArgs* __restrict__ as, const ChanGrid* __restrict__ cg, int nch) {
    const int c = chan_of(cg, nch);
    bin_sort_kernel_body(as[c], chan_ctx(cg[c]));
}


// positions in cell-list order with the cell's index (exact in a double), so
// that a candidate is one independent 32-byte load
struct alignas(32) SortedPos {
    double x, y, z, id;
};

__device__ __forceinline__ void sorted_pos_kernel_body(const DevArgs& a, const KCtx& G) {
    const int t = G.bx * blockDim.x + threadIdx.x;
    if (t >= a.n) return;
    const int j = a.bin_idx[t];
    ((SortedPos*)a.Xs)[t] = SortedPos{a.X[3 * j], a.X[3 * j + 1], a.X[3 * j + 2], (double)j};
    a.rank[j] = t;
}
__global__ void sorted_pos_kernel(DevArgs a) { sorted_pos_kernel_body(a, hw_ctx()); }
__global__ void sorted_pos_kernel_multi(const DevArgs* __restrict__ as, const ChanGrid* __restrict__ cg, int nch) {
    const int c = chan_of(cg, nch);
    sorted_pos_kernel_body(as[c], chan_ctx(cg[c]));
}


hipError_t launch_cells(const DevArgs& a, hipStream_t st) {
    if (a.n == 0) return hipSuccess;
    hipLaunchKernelGGL(bin_clear_kernel, dim3((a.nbins + 255) / 256), dim3(256), 0, st, a);
    hipLaunchKernelGGL(bin_count_kernel, dim3((a.n + 255) / 256), dim3(256), 0, st, a);
    const int nblk = (a.nbins + SCAN_PER_BLOCK - 1) / SCAN_PER_BLOCK;
    hipLaunchKernelGGL(scan_local_kernel, dim3(nblk), dim3(256), 0, st, a);
    hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(1024), 0, st, a);
    hipLaunchKernelGGL(scan_add_kernel, dim3((a.nbins + 255) / 256), dim3(256), 0, st, a);
    hipLaunchKernelGGL(bin_fill_kernel, dim3((a.n + 255) / 256), dim3(256), 0, st, a);
    hipLaunchKernelGGL(bin_sort_kernel, dim3((a.nbins + 255) / 256), dim3(256), 0, st, a);
    hipLaunchKernelGGL(sorted_pos_kernel, dim3((a.n + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

// element i < 3 of a 3-array by selects (a dynamically indexed local array
// would live in scratch memory)
__device__ inline int pick3(const int* v, int i) { return i == 0 ? v[0] : (i == 1 ? v[1] : v[2]); }

// neighbour bin offsets along one axis (deduplicated for fewer than 3 bins;
// clipped at the wall planes)
__device__ inline int axis_bins(const DevArgs& a, int c, int b, int* out) {
    // written with constant indices only, so that out[] stays in registers
    const int nb = a.nb[c];
    const bool periodic = !(c == 1 && a.wall_y);
    if (!periodic) {
        const bool lo = b - 1 >= 0, hi = b + 1 < nb;
        out[0] = lo ? b - 1 : b;
        out[1] = lo ? b : (hi ? b + 1 : b);
        out[2] = b + 1;
        return 1 + (lo ? 1 : 0) + (hi ? 1 : 0);
    }
    if (nb >= 3) { out[0] = wrap(b - 1, nb); out[1] = b; out[2] = wrap(b + 1, nb); return 3; }
    out[0] = 0; out[1] = 1; out[2] = 2;
    return nb;
}

// squared length evaluated exactly as written (pair membership is decided
// bit-identically to a reference evaluating the same expression)
__device__ inline double dist2_exact(const double* rv) {
#pragma clang fp contract(off)
    return rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2];
}

// ------------------------------------------------------------------ potentials
// Berne-Pechukas pair term for rvec = X_i - X_j.  U = eps (1 - r/sigma)^2,
// eps = eps-bar / sqrt(1 - chi^2 g^2) (Eq. 16), sigma = sigma-bar /
// sqrt(1 - chi/2 [(a+b)^2/(1+chi g) + (a-b)^2/(1-chi g)]) (Eq. 17) with
// a = r.o_i, b = r.o_j, g = o_i.o_j.  Returns -dU/dX_i and -o_i x dU/do_i.
__device__ void pair_term(const DevArgs& a, const double* rv, const double* oi, const double* oj,
                          double* F, double* Ti) {
    // fused multiply-adds only within one expression, so that the term rounds
    // alike wherever it is inlined
#pragma clang fp contract(on)
    const double r2 = rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2];
    if (r2 == 0.0) return;
    const double r = sqrt(r2);
    const double ir = 1.0 / r;
    const double e[3] = {rv[0] * ir, rv[1] * ir, rv[2] * ir};
    const double sp2 = a.sig_perp * a.sig_perp, sl2 = a.sig_par * a.sig_par;
    const double chi = (sl2 - sp2) / (sl2 + sp2);
    const double sbar = 2.0 * a.sig_perp;
    const double ca = e[0] * oi[0] + e[1] * oi[1] + e[2] * oi[2];
    const double cb = e[0] * oj[0] + e[1] * oj[1] + e[2] * oj[2];
    const double g = oi[0] * oj[0] + oi[1] * oj[1] + oi[2] * oj[2];
    const double ip = 1.0 / (1.0 + chi * g), iq = 1.0 / (1.0 - chi * g);
    const double sp = ca + cb, sm = ca - cb;
    const double S = sp * sp * ip + sm * sm * iq;
    const double sigma = sbar / sqrt(1.0 - 0.5 * chi * S);
    if (r >= sigma) return;
    const double e1 = 1.0 - chi * chi * g * g;
    const double eps = a.eps / sqrt(e1);
    const double s = 1.0 - r / sigma;
    const double dUdr = -2.0 * eps * s / sigma;
    // dU/dS through sigma: (2 eps s r / sigma^2) * chi sigma^3 / (4 sbar^2)
    const double K = (2.0 * eps * s * r / (sigma * sigma)) * (0.25 * chi * sigma * sigma * sigma / (sbar * sbar));
    const double Sa = 2.0 * sp * ip + 2.0 * sm * iq;
    const double Sb = 2.0 * sp * ip - 2.0 * sm * iq;
    const double Sg = -chi * sp * sp * ip * ip + chi * sm * sm * iq * iq;
    const double deps = a.eps * chi * chi * g / (e1 * sqrt(e1));
    for (int c = 0; c < 3; c++)
        F[c] -= dUdr * e[c] + K * (Sa * (oi[c] - ca * e[c]) + Sb * (oj[c] - cb * e[c])) * ir;
    double gi[3];
    for (int c = 0; c < 3; c++) gi[c] = K * (Sa * e[c] + Sg * oj[c]) + s * s * deps * oj[c];
    double t[3];
    cross3(oi, gi, t);
    for (int c = 0; c < 3; c++) Ti[c] -= t[c];
}

// cell-wall term for rvec = X_i - x_wall (Eqs. 19-20)
__device__ void wall_term(const DevArgs& a, const double* rv, const double* o, double* F, double* Ti) {
    const double r2 = rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2];
    if (r2 == 0.0) return;
    const double r = sqrt(r2);
    const double ir = 1.0 / r;
    const double e[3] = {rv[0] * ir, rv[1] * ir, rv[2] * ir};
    const double sp2 = a.sig_perp * a.sig_perp, sl2 = a.sig_par * a.sig_par, sw2 = a.sig_w * a.sig_w;
    const double sbw = sqrt(sp2 + sw2);
    const double chiw = (sl2 - sp2) / (sl2 + sw2);
    const double ca = e[0] * o[0] + e[1] * o[1] + e[2] * o[2];
    const double den = 1.0 - chiw * ca * ca;
    if (den <= 0.0) return;
    const double sigma = sbw / sqrt(den);
    if (r >= sigma) return;
    const double s = 1.0 - r / sigma;
    const double dUdr = -2.0 * a.eps_w * s / sigma;
    const double K = (2.0 * a.eps_w * s * r / (sigma * sigma)) * (chiw * ca * sigma * sigma * sigma / (sbw * sbw));
    for (int c = 0; c < 3; c++) F[c] -= dUdr * e[c] + K * (o[c] - ca * e[c]) * ir;
    double ke[3] = {K * e[0], K * e[1], K * e[2]}, t[3];
    cross3(o, ke, t);
    for (int c = 0; c < 3; c++) Ti[c] -= t[c];
}

constexpr int POT_BLOCK = 128;

// The three x-neighbour bins of a bin row are contiguous in the cell list
// unless they wrap: ranges [r[0], r[1]) and [r[2], r[3]) of x-bin indices
// (the second empty when the row does not wrap).
__device__ inline void row_xranges(const DevArgs& a, int bxi, int* r) {
    int lx[3];
    const int nxb = axis_bins(a, 0, bxi, lx);
    r[2] = r[3] = 0;
    if (nxb < 3) { r[0] = 0; r[1] = nxb; return; }
    if (lx[0] < lx[2]) { r[0] = lx[0]; r[1] = lx[2] + 1; return; }
    if (lx[1] == 0) { r[0] = 0; r[1] = 2; r[2] = lx[0]; r[3] = lx[0] + 1; }
    else { r[0] = lx[0]; r[1] = lx[1] + 1; r[2] = 0; r[3] = 1; }
}

__device__ inline void pair_rv(const DevArgs& a, const double* Xi, const SortedPos& e, double* rv) {
    rv[0] = min_image(Xi[0] - e.x, (double)a.nx);
    rv[1] = a.wall_y ? (Xi[1] - e.y) : min_image(Xi[1] - e.y, (double)a.ny);
    rv[2] = min_image(Xi[2] - e.z, (double)a.nz);
}

__device__ inline void wall_vec(const DevArgs& a, const double* Xi, unsigned w, double* rv) {
    // site indices are below 2^32 (checked at create)
    const unsigned nx = (unsigned)a.nx, ny = (unsigned)a.ny;
    const int wx = (int)(w % nx), wy = (int)((w / nx) % ny), wz = (int)(w / (nx * ny));
    double nd[3];
    node_disp(a, wx, wy, wz, Xi, nd);
    rv[0] = -nd[0]; rv[1] = -nd[1]; rv[2] = -nd[2];
}

// Pair forces (Eqs. 16-18) on lattices without walls: one thread per cell,
// cells in cell-list order (neighbouring threads share neighbour bins).  The
// bounds of the up to 18 candidate ranges (9 bin rows, each in one or two
// parts) are loaded together; the candidates of all ranges are then walked
// as one sequence, CB at a time with independent loads, in the order (z row,
// y row, part, position).  The partners in range are listed first (LDS, per
// thread) and evaluated after the walk in that order, so that a wave runs the
// pair term about as often as its busiest cell has partners, not once per
// candidate; a full list is evaluated on the spot, in order.
constexpr int CB = 2;
constexpr int NRANGE = 18;
constexpr int PLIST = 16;
__device__ __forceinline__ void potentials_kernel_body(const DevArgs& a, const KCtx& G) {
    __shared__ int plt[PLIST][POT_BLOCK];  // [slot][thread]: list position of a partner
    __shared__ int plj[PLIST][POT_BLOCK];  // and its cell index
    const int tid = (int)threadIdx.x;
    const int k = xcd_block((int)G.bx, (int)G.gx) * (int)blockDim.x + tid;
    if (k >= a.n) return;  // no barrier below: each thread uses its own list column
    const SortedPos* S = (const SortedPos*)a.Xs;
    const SortedPos me = S[k];
    const int i = (int)me.id;
    const double Xi[3] = {me.x, me.y, me.z};
    const double* ki = a.kin + 12 * (long long)i;
    const double oi[3] = {ki[9], ki[10], ki[11]};
    double F[3] = {0, 0, 0}, T[3] = {0, 0, 0};
    const int b = a.pbin[i];
    const int bxi = b % a.nb[0], byi = (b / a.nb[0]) % a.nb[1], bzi = b / (a.nb[0] * a.nb[1]);
    int xr[4], ly[3] = {0, 0, 0}, lz[3] = {0, 0, 0};
    row_xranges(a, bxi, xr);
    const int nyb = axis_bins(a, 1, byi, ly), nzb = axis_bins(a, 2, bzi, lz);
    // range q = 6 iz + 2 iy + h: first list position and start in the sequence
    int t0[NRANGE], pre[NRANGE + 1];
#pragma unroll
    for (int q = 0; q < NRANGE; q++) {
        const int iz = q / 6, iy = (q / 2) % 3, h = q & 1;
        const int x0 = h ? xr[2] : xr[0], x1 = h ? xr[3] : xr[1];
        const int row = a.nb[0] * (pick3(ly, iy) + a.nb[1] * pick3(lz, iz));
        const bool on = iz < nzb && iy < nyb && x1 > x0;
        t0[q] = on ? a.bin_start[row + x0] : 0;
        pre[q + 1] = on ? a.bin_start[row + x1] : 0;  // end, until the prefix below
    }
    pre[0] = 0;
#pragma unroll
    for (int q = 0; q < NRANGE; q++) pre[q + 1] = pre[q] + (pre[q + 1] - t0[q]);
    const int total = pre[NRANGE];
    int np = 0;
    // the listed partners, in list order
    auto evaluate = [&]() {
        for (int s = 0; s < np; s++) {
            const SortedPos e = S[plt[s][tid]];
            const double* kj = a.kin + 12 * (long long)plj[s][tid];
            const double oj[3] = {kj[9], kj[10], kj[11]};
            double rv[3];
            pair_rv(a, Xi, e, rv);
            pair_term(a, rv, oi, oj, F, T);
        }
        np = 0;
    };
    for (int u = 0; u < total; u += CB) {
        SortedPos e[CB];
        int tc[CB];
#pragma unroll
        for (int c = 0; c < CB; c++) {
            const int w = u + c;
            int t = k;  // past the sequence: the cell's own entry, not used
#pragma unroll
            for (int q = 0; q < NRANGE; q++)
                if (w >= pre[q] && w < pre[q + 1]) t = t0[q] + (w - pre[q]);
            tc[c] = t;
            e[c] = S[t];
        }
#pragma unroll
        for (int c = 0; c < CB; c++) {
            const int j = (int)e[c].id;
            if (u + c >= total || j == i) continue;
            double rv[3];
            pair_rv(a, Xi, e[c], rv);
            if (!(dist2_exact(rv) < a.r_cut2)) continue;
            if (np == PLIST) evaluate();
            plt[np][tid] = tc[c];
            plj[np][tid] = j;
            np++;
        }
    }
    evaluate();
    for (int c = 0; c < 3; c++) { a.FTp[6 * i + c] = F[c]; a.FTp[6 * i + 3 + c] = T[c]; }
}
__global__ void __launch_bounds__(POT_BLOCK) potentials_kernel(DevArgs a) { potentials_kernel_body(a, hw_ctx()); }
__global__ void __launch_bounds__(POT_BLOCK) potentials_kernel_multi(const DevArgs* __restrict__ as, const ChanGrid* __restrict__ cg, int nch) {
    const int c = chan_of(cg, nch);
    potentials_kernel_body(as[c], chan_ctx(cg[c]));
}


// Pair and wall forces (Eqs. 16-20) on lattices with walls, PG lanes per
// cell: a cell next to a wall screens some hundred wall nodes of its
// neighbour bins.  Lane g of a group takes every PG-th candidate (cell or
// wall node) of each bin row and lists the ones in range (its own order, so
// the sums are deterministic); the group then evaluates the lists and sums
// over its lanes in a fixed order.  A list that overflows evaluates its
// extra entries on the spot.
constexpr int PG = 8;
constexpr int PG_LIST = 8;
static_assert(PG >= 6 && PG <= 64 && (PG & (PG - 1)) == 0, "a group's lanes 0-5 write the six sums");

__device__ __forceinline__ void potentials_grp_kernel_body(const DevArgs& a, const KCtx& G) {
    // [slot][thread]: a partner j >= 0, or ~t for wall entry t
    __shared__ int plist[PG_LIST][POT_BLOCK];
    const int k = (int)(((unsigned)xcd_block((int)G.bx, (int)G.gx) * (unsigned)POT_BLOCK + threadIdx.x) / PG);
    const int g = (int)(threadIdx.x % PG);
    const bool live = k < a.n;  // uniform over each group; groups do not meet
    const SortedPos* S = (const SortedPos*)a.Xs;
    const SortedPos me = S[live ? k : 0];
    const int i = (int)me.id;
    const double Xi[3] = {me.x, me.y, me.z};
    const double* ki = a.kin + 12 * (long long)i;
    const double oi[3] = {ki[9], ki[10], ki[11]};
    double F[3] = {0, 0, 0}, T[3] = {0, 0, 0};
    const int b = a.pbin[i];
    const int bxi = b % a.nb[0], byi = (b / a.nb[0]) % a.nb[1], bzi = b / (a.nb[0] * a.nb[1]);
    int xr[4], ly[3], lz[3];
    row_xranges(a, bxi, xr);
    const int nyb = axis_bins(a, 1, byi, ly), nzb = live ? axis_bins(a, 2, bzi, lz) : 0;
    int np = 0;
    for (int iz = 0; iz < nzb; iz++)
        for (int iy = 0; iy < nyb; iy++) {
            const int row = a.nb[0] * (pick3(ly, iy) + a.nb[1] * pick3(lz, iz));
            for (int h = 0; h < 2; h++) {
                const int x0 = h ? xr[2] : xr[0], x1 = h ? xr[3] : xr[1];
                if (x1 <= x0) continue;
                const int t0 = a.bin_start[row + x0], t1 = a.bin_start[row + x1];
                for (int t = t0 + g; t < t1; t += PG) {
                    const SortedPos e = S[t];
                    const int j = (int)e.id;
                    if (j == i) continue;
                    double rv[3];
                    pair_rv(a, Xi, e, rv);
                    if (!(dist2_exact(rv) < a.r_cut2)) continue;
                    if (np < PG_LIST) {
                        plist[np][threadIdx.x] = t;
                    } else {
                        const double* kj = a.kin + 12 * (long long)j;
                        const double oj[3] = {kj[9], kj[10], kj[11]};
                        pair_term(a, rv, oi, oj, F, T);
                    }
                    np++;
                }
                const int w0 = a.wall_start[row + x0], w1 = a.wall_start[row + x1];
                for (int t = w0 + g; t < w1; t += PG) {
                    double rv[3];
                    wall_vec(a, Xi, (unsigned)a.wall_idx[t], rv);
                    const double r2 = rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2];
                    if (!(r2 < a.wall_range2)) continue;
                    if (np < PG_LIST) plist[np][threadIdx.x] = ~t;
                    else wall_term(a, rv, oi, F, T);
                    np++;
                }
            }
        }
    const int nl = np < PG_LIST ? np : PG_LIST;
    for (int q = 0; q < nl; q++) {
        const int e = plist[q][threadIdx.x];
        double rv[3];
        if (e >= 0) {
            const SortedPos p = S[e];
            pair_rv(a, Xi, p, rv);
            const double* kj = a.kin + 12 * (long long)p.id;
            const double oj[3] = {kj[9], kj[10], kj[11]};
            pair_term(a, rv, oi, oj, F, T);
        } else {
            wall_vec(a, Xi, (unsigned)a.wall_idx[~e], rv);
            wall_term(a, rv, oi, F, T);
        }
    }
#pragma unroll
    for (int off = 1; off < PG; off <<= 1)
#pragma unroll
        for (int c = 0; c < 3; c++) {
            F[c] += __shfl_xor(F[c], off, 64);
            T[c] += __shfl_xor(T[c], off, 64);
        }
    if (live && g < 6) {
        const double v = g == 0 ? F[0] : (g == 1 ? F[1] : (g == 2 ? F[2] : (g == 3 ? T[0] : (g == 4 ? T[1] : T[2]))));
        a.FTp[6 * i + g] = v;
    }
}
__global__ void __launch_bounds__(POT_BLOCK) potentials_grp_kernel(DevArgs a) { potentials_grp_kernel_body(a, hw_ctx()); }
__global__ void __launch_bounds__(POT_BLOCK) potentials_grp_kernel_multi(const DevArgs* __restrict__ as, const ChanGrid* __restrict__ cg, int nch) {
    const int c = chan_of(cg, nch);
    potentials_grp_kernel_body(as[c], chan_ctx(cg[c]));
}


hipError_t launch_potentials(const DevArgs& a, hipStream_t st) {
    if (a.n == 0) return hipSuccess;
    if (a.nsw > 0)
        hipLaunchKernelGGL(potentials_grp_kernel, dim3((unsigned)(((long long)a.n * PG + POT_BLOCK - 1) / POT_BLOCK)), dim3(POT_BLOCK), 0, st, a);
    else
        hipLaunchKernelGGL(potentials_kernel, dim3((a.n + POT_BLOCK - 1) / POT_BLOCK), dim3(POT_BLOCK), 0, st, a);
    return hipGetLastError();
}

__global__ void pairs_kernel(DevArgs a, int* out, int* count, int cap) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const double Xi[3] = {a.X[3 * i], a.X[3 * i + 1], a.X[3 * i + 2]};
    const int b = a.pbin[i];
    const int bxi = b % a.nb[0], byi = (b / a.nb[0]) % a.nb[1], bzi = b / (a.nb[0] * a.nb[1]);
    int lx[3], ly[3], lz[3];
    const int nxb = axis_bins(a, 0, bxi, lx), nyb = axis_bins(a, 1, byi, ly), nzb = axis_bins(a, 2, bzi, lz);
    for (int iz = 0; iz < nzb; iz++)
        for (int iy = 0; iy < nyb; iy++)
            for (int ix = 0; ix < nxb; ix++) {
                const int bb = pick3(lx, ix) + a.nb[0] * (pick3(ly, iy) + a.nb[1] * pick3(lz, iz));
                for (int t = a.bin_start[bb]; t < a.bin_start[bb + 1]; t++) {
                    const int j = a.bin_idx[t];
                    if (j <= i) continue;
                    double rv[3];
                    rv[0] = min_image(Xi[0] - a.X[3 * j], (double)a.nx);
                    rv[1] = a.wall_y ? (Xi[1] - a.X[3 * j + 1]) : min_image(Xi[1] - a.X[3 * j + 1], (double)a.ny);
                    rv[2] = min_image(Xi[2] - a.X[3 * j + 2], (double)a.nz);
                    if (!(dist2_exact(rv) < a.r_cut2)) continue;
                    const int pos = atomicAdd(count, 1);
                    if (pos < cap) { out[2 * pos] = i; out[2 * pos + 1] = j; }
                }
            }
}

hipError_t launch_pairs(const DevArgs& a, int* out, int* count, int cap, hipStream_t st) {
    hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, st, count);
    if (a.n == 0) return hipGetLastError();
    hipLaunchKernelGGL(pairs_kernel, dim3((a.n + 127) / 128), dim3(128), 0, st, a, out, count, cap);
    return hipGetLastError();
}

// ------------------------------------------------------------------ integrate
__device__ inline void qmul(const double* a, const double* b, double* c) {
    c[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    c[1] = a[0] * b[1] + b[0] * a[1] + a[2] * b[3] - a[3] * b[2];
    c[2] = a[0] * b[2] + b[0] * a[2] + a[3] * b[1] - a[1] * b[3];
    c[3] = a[0] * b[3] + b[0] * a[3] + a[1] * b[2] - a[2] * b[1];
}
__device__ inline void qrot(const double* w, double h, double* dq) {
    const double wn = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    if (wn == 0.0) { dq[0] = 1; dq[1] = dq[2] = dq[3] = 0; return; }
    const double ang = 0.5 * wn * h;
    const double sn = sin(ang) / wn;
    dq[0] = cos(ang); dq[1] = sn * w[0]; dq[2] = sn * w[1]; dq[3] = sn * w[2];
}
__device__ inline void qnormalise(double* q) {
    const double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int c = 0; c < 4; c++) q[c] /= n;
}
__device__ inline void omega_sym(const DevArgs& a, const double* o, const double* L, double* w) {
    const double oL = o[0] * L[0] + o[1] * L[1] + o[2] * L[2];
    const double kk = 1.0 / a.Ipar - 1.0 / a.Iperp;
    for (int c = 0; c < 3; c++) w[c] = L[c] / a.Iperp + kk * oL * o[c];
}

__device__ void integrate_one(const DevArgs& a, int p, double* bf);

// one thread per cell; the body force added to the cells is reduced per block
// (no same-address atomics) into body_part[3 * block]
__device__ __forceinline__ void integrate_kernel_body(const DevArgs& a, const KCtx& G) {
    __shared__ double red[3][256];
    const int p = G.bx * blockDim.x + threadIdx.x;
    double bf[3] = {0, 0, 0};
    if (p < a.n) integrate_one(a, p, bf);
    for (int c = 0; c < 3; c++) red[c][threadIdx.x] = bf[c];
    __syncthreads();
    for (int off = 128; off >= 1; off >>= 1) {
        if ((int)threadIdx.x < off)
            for (int c = 0; c < 3; c++) red[c][threadIdx.x] += red[c][threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int c = 0; c < 3; c++) a.body_part[3 * G.bx + c] = red[c][0];
}
__global__ void __launch_bounds__(256) integrate_kernel(DevArgs a) { integrate_kernel_body(a, hw_ctx()); }
__global__ void __launch_bounds__(256) integrate_kernel_multi(const DevArgs* __restrict__ as, const ChanGrid* __restrict__ cg, int nch) {
    const int c = chan_of(cg, nch);
    integrate_kernel_body(as[c], chan_ctx(cg[c]));
}


__device__ void integrate_one(const DevArgs& a, int p, double* bf) {
    if (a.fixed[p]) {
        for (int c = 0; c < 3; c++) { a.V[3 * p + c] = 0.0; a.L[3 * p + c] = 0.0; }
        return;
    }
    // the state is loaded before the first store (the stores could alias the
    // loads as far as the compiler knows), so the loads are in flight together
    double X[3], q[4];
    for (int c = 0; c < 3; c++) X[c] = a.X[3 * p + c];
    for (int c = 0; c < 4; c++) q[c] = a.q[4 * p + c];
    double gb[3] = {0, 0, 0};
    if (a.force_on_particles) body_force(a, X[1], X[2], gb);
    bool bad = false;
    double Lnew[3], Vn[3];
    for (int c = 0; c < 3; c++) {
        const double F = a.FTh[6 * p + c] + a.FTp[6 * p + c] + a.Mdrive * gb[c];
        Vn[c] = a.V[3 * p + c] + F / a.M;
        Lnew[c] = a.L[3 * p + c] + (a.FTh[6 * p + 3 + c] + a.FTp[6 * p + 3 + c]);
        if (!(fabs(Vn[c]) < 0.5) || !(fabs(Lnew[c]) < 1e30)) bad = true;
    }
    if (bad) {
        // unstable: flag it and leave the cell where it is, inside the box
        atomicOr(a.status, ST_UNSTABLE);
        atomicMin(a.bad_step, *a.dstep);
        return;
    }
    for (int c = 0; c < 3; c++) {
        a.V[3 * p + c] = Vn[c];
        a.L[3 * p + c] = Lnew[c];
        double xn = X[c] + Vn[c];
        if (!(c == 1 && a.wall_y)) {
            const double Lb = c == 0 ? a.nx : (c == 1 ? a.ny : a.nz);
            if (xn >= Lb) xn -= Lb;
            else if (xn < 0.0) xn += Lb;
        }
        a.X[3 * p + c] = xn;
    }
    // viscometer (Sec. IV): a cell whose centre has come closer than sigma_perp
    // to one of the sheared side planes (the node planes x = 0 and nx - 1)
    // while moving towards it has its normal velocity negated
    if (a.le_u != 0.0) {
        const double xc = a.X[3 * p];
        if ((xc < a.sig_perp && Vn[0] < 0.0) || ((double)(a.nx - 1) - xc < a.sig_perp && Vn[0] > 0.0))
            a.V[3 * p] = -Vn[0];
    }
    bf[0] = a.Mdrive * gb[0]; bf[1] = a.Mdrive * gb[1]; bf[2] = a.Mdrive * gb[2];
    // quaternion: half-step predictor, then full step with the midpoint rate
    double o[3], w[3], dq[4], qh[4], qn[4];
    axis_of(q, o);
    omega_sym(a, o, Lnew, w);
    qrot(w, 0.5, dq);
    qmul(dq, q, qh);
    qnormalise(qh);
    axis_of(qh, o);
    omega_sym(a, o, Lnew, w);
    qrot(w, 1.0, dq);
    qmul(dq, q, qn);
    qnormalise(qn);
    for (int c = 0; c < 4; c++) a.q[4 * p + c] = qn[c];
    if (!(qn[0] == qn[0])) {
        atomicOr(a.status, ST_UNSTABLE);
        atomicMin(a.bad_step, *a.dstep);
    }
}

hipError_t launch_integrate(const DevArgs& a, hipStream_t st) {
    if (a.n == 0) return hipSuccess;
    hipLaunchKernelGGL(integrate_kernel, dim3((a.n + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace cgb

namespace cgb {

// ------------------------------------------------------------ batch launches
// lmom variant: the link-moment type as the single launch chooses it
static int lm_variant(const DevArgs& a) {
    if (a.precision == CGB_P64) return 0;
    if (a.precision == CGB_PMX16S) return 1;
    return 2;
}

bool multi_grid_particles(int kind, const DevArgs& a, int* variant, unsigned* bx, unsigned* by, dim3* grid, int* arg) {
    *variant = 0;
    *bx = 256;
    *by = 1;
    *arg = 0;
    const unsigned n = (unsigned)a.n;
    switch (kind) {
        case MK_PREP: *grid = dim3(n ? (n + 255) / 256 : 1); return true;  // block 0 also starts the step
        case MK_CLAIM: *bx = 64 * CPW; *grid = dim3(cell_grid(a.n)); return n > 0;
        case MK_RESOLVE: *grid = dim3((unsigned)((a.ns + 255) / 256)); return n > 0;
        case MK_TRANS: *variant = a.precision; *grid = dim3(TSEG * 8); return true;
        case MK_LMOM: {
            if (!a.lmom) return false;
            const int v = lm_variant(a);
            *variant = v;
            int tz = 0;
            switch (v) {
                case 0: *grid = lm_grid<double, 32, 3>(a, &tz, true); break;
                case 1: *grid = lm_grid<float, 32, 4>(a, &tz, true); break;
                default: *grid = lm_grid<float, 32, 3>(a, &tz, true); break;
            }
            *arg = tz;
            return true;
        }
        case MK_MEM: *bx = 64 * CPW; *grid = dim3(cell_grid((a.n + 1) / 2)); return n > 0;
        case MK_BIN_CLEAR: *grid = dim3((unsigned)((a.nbins + 255) / 256)); return n > 0;
        case MK_BIN_COUNT: *grid = dim3((n + 255) / 256); return n > 0;
        case MK_SCAN_LOCAL: *grid = dim3((unsigned)((a.nbins + SCAN_PER_BLOCK - 1) / SCAN_PER_BLOCK)); return n > 0;
        case MK_SCAN_TOP: *bx = 1024; *grid = dim3(1); return n > 0;
        case MK_SCAN_ADD: *grid = dim3((unsigned)((a.nbins + 255) / 256)); return n > 0;
        case MK_BIN_FILL: *grid = dim3((n + 255) / 256); return n > 0;
        case MK_BIN_SORT: *grid = dim3((unsigned)((a.nbins + 255) / 256)); return n > 0;
        case MK_SORTED_POS: *grid = dim3((n + 255) / 256); return n > 0;
        case MK_POT:
            *bx = POT_BLOCK;
            *variant = a.nsw > 0 ? 1 : 0;
            *grid = a.nsw > 0 ? dim3((unsigned)(((long long)a.n * PG + POT_BLOCK - 1) / POT_BLOCK))
                              : dim3((n + POT_BLOCK - 1) / POT_BLOCK);
            return n > 0;
        case MK_INT: *grid = dim3((n + 255) / 256); return n > 0;
        default: return false;
    }
}

#define CGB_MULTI_GO(K) hipLaunchKernelGGL(K, dim3(m.blocks), dim3(m.bx, m.by), 0, st, args, m.cg, m.nch)
hipError_t launch_multi_particles(const MultiLaunch& m, const DevArgs* args, hipStream_t st) {
    switch (m.kind) {
        case MK_PREP: CGB_MULTI_GO(step_prep_kernel_multi); break;
        case MK_CLAIM: CGB_MULTI_GO(claim_kernel_multi); break;
        case MK_RESOLVE: CGB_MULTI_GO(resolve_kernel_multi); break;
        case MK_TRANS:
            switch (m.variant) {
                case CGB_P64: hipLaunchKernelGGL(transitions_kernel_multi<CGB_P64>, dim3(m.blocks), dim3(m.bx), 0, st, args, m.cg, m.nch, 1); break;
                case CGB_P32: hipLaunchKernelGGL(transitions_kernel_multi<CGB_P32>, dim3(m.blocks), dim3(m.bx), 0, st, args, m.cg, m.nch, 1); break;
                case CGB_PMX16: hipLaunchKernelGGL(transitions_kernel_multi<CGB_PMX16>, dim3(m.blocks), dim3(m.bx), 0, st, args, m.cg, m.nch, 1); break;
                case CGB_PMXBF16: hipLaunchKernelGGL(transitions_kernel_multi<CGB_PMXBF16>, dim3(m.blocks), dim3(m.bx), 0, st, args, m.cg, m.nch, 1); break;
                case CGB_PMX16S: hipLaunchKernelGGL(transitions_kernel_multi<CGB_PMX16S>, dim3(m.blocks), dim3(m.bx), 0, st, args, m.cg, m.nch, 1); break;
                default: return hipErrorInvalidValue;
            }
            break;
        case MK_LMOM:
            switch (m.variant) {
                case 0: CGB_MULTI_GO((lmom_kernel_multi<double, 32, 3>)); break;
                case 1: CGB_MULTI_GO((lmom_kernel_multi<float, 32, 4>)); break;
                default: CGB_MULTI_GO((lmom_kernel_multi<float, 32, 3>)); break;
            }
            break;
        case MK_MEM: CGB_MULTI_GO(mem_reduce_kernel_multi); break;
        case MK_BIN_CLEAR: CGB_MULTI_GO(bin_clear_kernel_multi); break;
        case MK_BIN_COUNT: CGB_MULTI_GO(bin_count_kernel_multi); break;
        case MK_SCAN_LOCAL: CGB_MULTI_GO(scan_local_kernel_multi); break;
        case MK_SCAN_TOP: CGB_MULTI_GO(scan_top_kernel_multi); break;
        case MK_SCAN_ADD: CGB_MULTI_GO(scan_add_kernel_multi); break;
        case MK_BIN_FILL: CGB_MULTI_GO(bin_fill_kernel_multi); break;
        case MK_BIN_SORT: CGB_MULTI_GO(bin_sort_kernel_multi); break;
        case MK_SORTED_POS: CGB_MULTI_GO(sorted_pos_kernel_multi); break;
        case MK_POT:
            if (m.variant) {
                CGB_MULTI_GO(potentials_grp_kernel_multi);
            } else {
                CGB_MULTI_GO(potentials_kernel_multi);
            }
            break;
        case MK_INT: CGB_MULTI_GO(integrate_kernel_multi); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
#undef CGB_MULTI_GO

}  // namespace cgb
