// lb.hip -- fused pull stream + moving bounce-back + BGK collision.
//
// For a fluid node x and each direction r the pulled population is
// n*_r(x - c_r) when the source is fluid (Eq. 2).  When the source
// s = x - c_r is a wall or a cell node it is the node's own post-collision
// n*_rbar(x) (mid-link bounce-back, Eq. 9) plus the correction of Eq. 10,
// C_r = 6 w_r rho(x) (c_r . v_b), with rho(x) the node's density at the time
// of the bounced populations (the stored density deviation field).  For a
// cell, v_b = V + Omega x (x - c_r/2 - X) at the link midpoint; because
// c_r . (Omega x c_r) = 0, c_r . v_b equals c_r . u(s) with
// u(s) = V + Omega x (s - X), the rigid-body velocity at the source node.
// At tau = 1 the corrections enter only through their sums over the links,
// sum C_r = 6 rho(x) sum w_r q_r and sum C_r c_r = 6 rho(x) sum w_r c_r q_r
// (q_r = c_r . u(s_r)): a stencil kernel stores these moments at each fluid
// node with links after the occupancy update, and the LB reads them with one
// coalesced load.  With the split FP16 codec the same kernel also sums, at
// every fluid node, the density parts w_r D of the pulled populations (D of
// each population's source node), so that the LB decodes only the residuals.
// For general tau the per-direction values are needed: a
// node-parallel kernel stores u(s) for every cell node and walls hold their
// plane velocity, and the LB gathers the velocity of each link's source.  In
// neither case does a link need to know which body is behind it.
//
// Momentum exchange (Eq. 12): the lanes of cell nodes, which have no
// populations of their own, form the momentum their links carry to the cell,
// sum_r (2 n*_rbar(x) + C_r) c_rbar over the fluid neighbours x = s + c_r,
// from the populations and densities the fluid lanes of the same kernel load
// for their bounce-back (so those lines are on chip), in FP64, and store it
// per node; a per-cell pass sums the nodes of each cell and their torques.
//
// Collision: Eqs. 1, 4, 5 with the Guo forcing term, u = (sum n c + g/2)/rho.
// Work decomposition: a workgroup of BX x BY threads covers a patch of an x-y
// plane; each thread sweeps TZ nodes along z.
#include "cgb_dev.h"

namespace cgb {

// the nonzero velocity components of direction r, in the order x, y, z:
// first and second component index (second = -1 on axis directions)
__host__ __device__ constexpr int comp1(int r) { return CX(r) ? 0 : (CY(r) ? 1 : 2); }
__host__ __device__ constexpr int comp2(int r) {
    return (CX(r) && CY(r)) ? 1 : ((CX(r) || CY(r)) && CZ(r) ? 2 : -1);
}
__host__ __device__ constexpr int compv(int r, int c) { return c == 0 ? CX(r) : (c == 1 ? CY(r) : CZ(r)); }

constexpr unsigned OOB = 0xfffffff0u;  // byte offset past every buffer: loads read 0, stores are dropped

// source-node velocity components along the nonzero components of c_r, for
// the link directions (the other directions load from the out-of-range
// offset and read 0); u(s) is stored as three component planes [3][pstride]
// in the link type M, so that the lanes of a wave gathering one component
// from a row of source nodes touch few cache lines
template <class M>
struct LinkVel {
    M a[19], b[19];
};

template <class M, class SrcF>
__device__ inline void issue_link_loads(__amdgpu_buffer_rsrc_t rU, unsigned ps, uint32_t links, SrcF src, LinkVel<M>& lv) {
#pragma unroll
    for (int r = 1; r < 19; r++) {
        const bool lk = (links >> r) & 1u;
        const unsigned sr = src(r);
        lv.a[r] = bload<M>(rU, lk ? (unsigned)sizeof(M) * ((unsigned)comp1(r) * ps + sr) : OOB);
        if (comp2(r) >= 0) lv.b[r] = bload<M>(rU, lk ? (unsigned)sizeof(M) * ((unsigned)comp2(r) * ps + sr) : OOB);
    }
}

// c_r . u(s)
template <class M>
__device__ inline M link_cu(const LinkVel<M>& lv, int r) {
    M cu = (M)compv(r, comp1(r)) * lv.a[r];
    if (comp2(r) >= 0) cu += (M)compv(r, comp2(r)) * lv.b[r];
    return cu;
}

// Momentum the links of cell node s (site i, flags f, rigid-body velocity
// u = V + Omega x (s - X) at the node) carry to its cell in this step
// (Eq. 12): the fluid neighbour x = s + c_r bounces its own n*_rbar(x) into
// direction r and the correction C_r = 6 w_r rho(x) (c_r . u) (Eq. 10) is
// added, so the link transfers (2 n*_rbar(x) + C_r) c_rbar.  Only the part of
// the deviations d = n* - w rho0 is summed: the constant part 2 w rho0 c_rbar,
// with the link forces of Eqs. 13-14 between cells and from walls, cancels
// over the closed surface of any node set.  Populations and densities are
// decoded in the codec's precision (the values the fluid lanes bounce), C,
// the link momenta and their sum are FP64.  ox, oy, oz: offsets to x - c along
// each axis at index c + 1 (so x + c_r is at index 1 - c_r).
// links R0 <= r < R1 of the cell node: loads issued together, then summed
template <int P, int R0, int R1>
__device__ inline void cell_links_part(const DevArgs& a, __amdgpu_buffer_rsrc_t rA, __amdgpu_buffer_rsrc_t rRA,
                                       unsigned i, uint32_t f, const int* ox, const int* oy, const int* oz,
                                       const double* us, double* m) {
    using Cd = Codec<P>;
    using T = typename Cd::T;
    using R = typename Cd::R;
    constexpr unsigned ES = sizeof(T);
    const unsigned ps = (unsigned)a.pstride;
    T dv[R1 - R0], rv[R1 - R0];
#pragma unroll
    for (int r = R0; r < R1; r++) {
        // s + c_r is fluid: bit OPP(r) of the flags (source s - c_OPP(r)) is clear
        const bool lk = !((f >> OPP(r)) & 1u);
        const unsigned xi = i + (unsigned)(ox[1 - CX(r)] + oy[1 - CY(r)] + oz[1 - CZ(r)]);
        dv[r - R0] = bload<T>(rA, lk ? ES * ((unsigned)OPP(r) * ps + xi) : OOB);
        rv[r - R0] = bload<T>(rRA, lk ? ES * xi : OOB);
    }
#pragma unroll
    for (int r = R0; r < R1; r++) {
        const bool lk = !((f >> OPP(r)) & 1u);
        const R Dx = rho_dec<P>(a, rv[r - R0]);
        const double rho_x = a.rho0 + (double)Dx;
        double cu = 0;
        if (CX(r)) cu += CX(r) * us[0];
        if (CY(r)) cu += CY(r) * us[1];
        if (CZ(r)) cu += CZ(r) * us[2];
        const double C = 6.0 * WD(r) * rho_x * cu;
        const double mr = lk ? -(2.0 * (double)pop_dec<P>(a, dv[r - R0], OPP(r), Dx) + C) : 0.0;
        if (CX(r)) m[0] += CX(r) * mr;
        if (CY(r)) m[1] += CY(r) * mr;
        if (CZ(r)) m[2] += CZ(r) * mr;
    }
}

// Momentum the links of cell node s (site i, flags f, rigid-body velocity
// u = V + Omega x (s - X) at the node) carry to its cell in this step
// (Eq. 12): the fluid neighbour x = s + c_r bounces its own n*_rbar(x) into
// direction r and the correction C_r = 6 w_r rho(x) (c_r . u) (Eq. 10) is
// added, so the link transfers (2 n*_rbar(x) + C_r) c_rbar.  Only the part of
// the deviations d = n* - w rho0 is summed: the constant part 2 w rho0 c_rbar,
// with the link forces of Eqs. 13-14 between cells and from walls, cancels
// over the closed surface of any node set.  Populations and densities are
// decoded in the codec's precision (the values the fluid lanes bounce), C,
// the link momenta and their sum are FP64.  ox, oy, oz: offsets to x - c along
// each axis at index c + 1 (so x + c_r is at index 1 - c_r).  The links are
// taken in three groups of six, each group's loads in flight together, so that
// this path needs no more registers than the fluid path beside it.
template <int P, class M>
__device__ inline void cell_node_links(const DevArgs& a, __amdgpu_buffer_rsrc_t rA, __amdgpu_buffer_rsrc_t rRA,
                                       unsigned i, uint32_t f, const int* oxi, const int* oyi, const int* oz,
                                       M u0, M u1, M u2) {
    // the x and y offsets do not change along a thread's z sweep; made
    // opaque here, so that the compiler forms the 18 neighbour offsets on
    // this path instead of keeping them in registers across the whole sweep
    int ox[3] = {oxi[0], 0, oxi[2]}, oy[3] = {oyi[0], 0, oyi[2]};
    asm volatile("" : "+v"(ox[0]), "+v"(ox[2]), "+v"(oy[0]), "+v"(oy[2]));
    const double us[3] = {(double)u0, (double)u1, (double)u2};
    double m[3] = {0, 0, 0};
    cell_links_part<P, 1, 7>(a, rA, rRA, i, f, ox, oy, oz, us, m);
    __builtin_amdgcn_sched_barrier(0);
    cell_links_part<P, 7, 13>(a, rA, rRA, i, f, ox, oy, oz, us, m);
    __builtin_amdgcn_sched_barrier(0);
    cell_links_part<P, 13, 19>(a, rA, rRA, i, f, ox, oy, oz, us, m);
    double* F = a.fnode + 3 * (size_t)i;
    F[0] = m[0];
    F[1] = m[1];
    F[2] = m[2];
}

// ---------------------------------------------------------------- viscometer seam
// Plane-Couette viscometer (Sec. IV): Lees-Edwards shear across the periodic
// seam of x.  The image of the box beyond x = nx - 1 moves at +U e_z and is
// shifted by Delta = U t along z (t: steps completed before this one); the
// image below x = 0 moves at -U e_z, shifted by -Delta.  A population pulled
// across the seam comes from the image: into x = 0 along c_x = +1 from the
// node (nx - 1, y - c_y) at z - c_z + Delta, into x = nx - 1 along c_x = -1
// from (0, y - c_y) at z - c_z - Delta, linearly interpolated between the two
// nodes that bracket that z, and carried into this box's frame by the
// Galilean shift n^eq(rho_s, u_s -/+ U e_z) - n^eq(rho_s, u_s) of the
// interpolated source's moments.  The sheared planes never hold cell nodes
// (cells are reflected before they reach them), so every source is fluid.
// One thread per node of the two seam planes computes its five crossing
// populations (FP64, stored in the compute precision) and its share of
// Delta p_LE,z: the z momentum carried across the seam in -x, the mean of its
// values before and after the shift (the frames of the two sides).

// the directions with c_x = +1 (side 0) and c_x = -1 (side 1), k = 0..4
__host__ __device__ constexpr int le_dir(int side, int k) {
    constexpr int d0[5] = {1, 7, 9, 11, 13}, d1[5] = {2, 8, 10, 12, 14};
    return side == 0 ? d0[k] : d1[k];
}
// the index k of direction r among its side's crossing directions
__host__ __device__ constexpr int le_slot(int r) {
    return (r == 1 || r == 2) ? 0 : ((r == 7 || r == 8) ? 1 : ((r == 9 || r == 10) ? 2 : ((r == 11 || r == 12) ? 3 : 4)));
}

template <int P>
__global__ void __launch_bounds__(LE_BLOCK) le_kernel(DevArgs a) {
    using Cd = Codec<P>;
    using T = typename Cd::T;
    using R = typename Cd::R;
    __shared__ double red[LE_BLOCK];
    const int nyz = a.ny * a.nz;
    const int t = (int)(blockIdx.x * LE_BLOCK + threadIdx.x);
    double flux = 0.0;
    if (t < 2 * nyz) {
        const int side = t / nyz, rem = t % nyz;
        const int y = rem % a.ny, z = rem / a.ny;
        const int xs = side == 0 ? a.nx - 1 : 0;
        const double delta = fmod(a.le_u * (double)(*a.dstep), (double)a.nz);
        const T* A = (const T*)a.A;
        const T* RA = (const T*)a.rhoA;
        R* out = (R*)a.le_buf;
        for (int k = 0; k < 5; k++) {
            const int r = le_dir(side, k);
            const int ys = wrap(y - CY(r), a.ny);
            double zf = fmod((double)(z - CZ(r)) + (side == 0 ? delta : -delta), (double)a.nz);
            if (zf < 0.0) zf += a.nz;
            const double zl = floor(zf), w = zf - zl;
            const int z0 = wrap((int)zl, a.nz), z1 = wrap((int)zl + 1, a.nz);
            const long long i0 = xs + (long long)a.nx * (ys + (long long)a.ny * z0);
            const long long i1 = xs + (long long)a.nx * (ys + (long long)a.ny * z1);
            const R D0 = rho_dec<P>(a, RA[i0]), D1 = rho_dec<P>(a, RA[i1]);
            double drho = 0.0, j[3] = {0.0, 0.0, 0.0}, nr = 0.0;
            for (int q = 0; q < 19; q++) {
                const double v0 = (double)pop_dec<P>(a, A[q * a.pstride + i0], q, D0);
                const double v1 = (double)pop_dec<P>(a, A[q * a.pstride + i1], q, D1);
                const double n = (1.0 - w) * v0 + w * v1;
                drho += n;
                j[0] += CX(q) * n; j[1] += CY(q) * n; j[2] += CZ(q) * n;
                if (q == r) nr = n;
            }
            const double rho = a.rho0 + drho;
            const double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
            const double du = side == 0 ? -a.le_u : a.le_u;
            // n^eq(rho, u + du e_z) - n^eq(rho, u) of direction r (Eq. 5)
            const double cu0 = CX(r) * u[0] + CY(r) * u[1] + CZ(r) * u[2];
            const double cu1 = cu0 + CZ(r) * du;
            const double us0 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
            const double us1 = u[0] * u[0] + u[1] * u[1] + (u[2] + du) * (u[2] + du);
            const double p0 = 3.0 * cu0 + 4.5 * cu0 * cu0 - 1.5 * us0 + 4.5 * cu0 * cu0 * cu0 - 4.5 * us0 * cu0;
            const double p1 = 3.0 * cu1 + 4.5 * cu1 * cu1 - 1.5 * us1 + 4.5 * cu1 * cu1 * cu1 - 4.5 * us1 * cu1;
            const double shifted = nr + WD(r) * rho * (p1 - p0);
            out[(size_t)(side * 5 + k) * nyz + rem] = (R)shifted;
            flux += -0.5 * CX(r) * CZ(r) * (nr + shifted);
        }
    }
    red[threadIdx.x] = flux;
    __syncthreads();
    for (int off = LE_BLOCK / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) a.le_part[blockIdx.x] = red[0];
}

// Delta p_LE,z of the step into the record (at the track record's next slot;
// the track kernels advance the count after this)
__global__ void le_finish_kernel(DevArgs a, int nblk) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int b = 0; b < nblk; b++) s += a.le_part[b];
    const int n = *a.track_n;
    if (a.le_rec && n < a.track_cap) a.le_rec[n] = s;
}

hipError_t launch_le(const DevArgs& a, hipStream_t st) {
    if (a.le_u == 0.0) return hipSuccess;
    const dim3 g((unsigned)le_blocks(a)), b(LE_BLOCK);
    switch (a.precision) {
        case CGB_P64: hipLaunchKernelGGL(le_kernel<CGB_P64>, g, b, 0, st, a); break;
        case CGB_P32: hipLaunchKernelGGL(le_kernel<CGB_P32>, g, b, 0, st, a); break;
        case CGB_PMX16: hipLaunchKernelGGL(le_kernel<CGB_PMX16>, g, b, 0, st, a); break;
        case CGB_PMXBF16: hipLaunchKernelGGL(le_kernel<CGB_PMXBF16>, g, b, 0, st, a); break;
        default: return hipErrorInvalidValue;  // the split codec is refused at creation
    }
    if (a.track) hipLaunchKernelGGL(le_finish_kernel, dim3(1), dim3(64), 0, st, a, le_blocks(a));
    return hipGetLastError();
}

// the seam side of a node (0: x = 0, 1: x = nx - 1) when the viscometer is on, else -1
__device__ inline int le_side(const DevArgs& a, int x) {
    if (a.le_u == 0.0) return -1;
    return x == 0 ? 0 : (x == a.nx - 1 ? 1 : -1);
}
// direction r crosses the seam into a node of side `side`
__host__ __device__ constexpr bool le_crosses(int side, int r) { return side == 0 ? CX(r) == 1 : CX(r) == -1; }

// general tau: populations are kept per direction
template <int P, int TZ>
__global__ void __launch_bounds__(256) lb_kernel_tau(DevArgs a) {
    using Cd = Codec<P>;
    using T = typename Cd::T;
    using R = typename Cd::R;
    using M = R;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z0 = blockIdx.z * TZ;
    const bool inb = (x < a.nx) && (y < a.ny);
    const unsigned nx = (unsigned)a.nx;
    const unsigned plane = (unsigned)a.nx * (unsigned)a.ny;
    const unsigned ps = (unsigned)a.pstride;
    constexpr unsigned ES = sizeof(T);
    const auto rA = make_rsrc(a.A, 19ull * ps * ES);
    const auto rB = make_rsrc(a.B, 19ull * ps * ES);
    const auto rRA = make_rsrc(a.rhoA, (unsigned long long)ps * ES);
    const auto rRB = make_rsrc(a.rhoB, (unsigned long long)ps * ES);
    const auto rU = make_rsrc(a.usol, 3ull * ps * sizeof(M));
    // offset from x to the pull source x - c along each axis (periodic wrap);
    // index 0: c = -1, 1: c = 0, 2: c = +1
    const int ox[3] = {x == a.nx - 1 ? -(a.nx - 1) : 1, 0, x == 0 ? a.nx - 1 : -1};
    const int oy[3] = {y == a.ny - 1 ? -(int)((a.ny - 1) * nx) : (int)nx, 0, y == 0 ? (int)((a.ny - 1) * nx) : -(int)nx};
    // body force at this plane: constant, or f0 sin(2 pi y/ny) from the table
    const int yc = y < a.ny ? y : a.ny - 1;
    const R gx0 = a.force_mode == 1 ? (R)a.g[0] : (R)0;
    const R gy0 = a.force_mode == 1 ? (R)a.g[1] : (R)0;
    const R gz0 = a.force_mode == 1 ? (R)a.g[2] : (a.force_mode == 2 ? (R)(a.f0 * a.ysin[yc]) : (R)0);
    const R omega = (R)(1.0 / a.tau);
    const R pref = (R)(1.0 - 0.5 / a.tau);

#pragma unroll 1
    for (int zz = 0; zz < TZ; zz++) {
        const int z = z0 + zz;
        if (z >= a.nz) break;
        // a constant force confined to a slab of z acts there only (uniform over the step)
        const bool fon = !a.fregion || (z >= a.fzlo && z < a.fzhi);
        const R gx = fon ? gx0 : (R)0, gy = fon ? gy0 : (R)0, gz = fon ? gz0 : (R)0;
        const unsigned i = (unsigned)x + nx * (unsigned)y + plane * (unsigned)z;
        const uint32_t f = inb ? a.flags[i] : NONFLUID;
        // outputs of the node; a non-fluid node stores zeros.  The stores
        // below are shared by all lanes of the wave, so that each wave store
        // writes its lines whole (stores issued separately by the fluid and
        // non-fluid lanes would each write part of the same lines)
        T ob[19], orho;
#pragma unroll
        for (int r = 0; r < 19; r++) ob[r] = Cd::enc((R)0, (R)1);
        orho = Cd::enc((R)0, (R)1);
        if (!(f & NONFLUID)) {
        const int oz[3] = {z == a.nz - 1 ? -(int)((a.nz - 1) * plane) : (int)plane, 0,
                           z == 0 ? (int)((a.nz - 1) * plane) : -(int)plane};
        auto src = [&](int r) { return i + (unsigned)(ox[CX(r) + 1] + oy[CY(r) + 1] + oz[CZ(r) + 1]); };
        const uint32_t links = f & LINKBITS;

        // pull; a non-fluid source bounces the node's own opposite population
        T v[19];
#pragma unroll
        for (int r = 0; r < 19; r++) {
            const bool bb = (f >> r) & 1u;
            v[r] = bload<T>(rA, ES * (bb ? (unsigned)OPP(r) * ps + i : (unsigned)r * ps + src(r)));
        }
        // split codec: the density of each pulled population's source node
        T vs[19];
        if constexpr (Cd::SPLIT) {
#pragma unroll
            for (int r = 1; r < 19; r++) vs[r] = bload<T>(rRA, ((f >> r) & 1u) ? OOB : ES * src(r));
        }
        LinkVel<M> lv;
        issue_link_loads<M>(rU, ps, links, src, lv);
        const T rstored = bload<T>(rRA, (links || Cd::SPLIT) ? ES * i : OOB);
        const R Down = rho_dec<P>(a, rstored);

        R d[19];
#pragma unroll
        for (int r = 0; r < 19; r++) {
            R Ds = Down;
            if constexpr (Cd::SPLIT) if (r > 0 && !((f >> r) & 1u)) Ds = rho_dec<P>(a, vs[r]);
            d[r] = pop_dec<P>(a, v[r], r, Ds);
        }
        // viscometer seam: the populations pulled across it come from the sheared image
        const int side = le_side(a, x);
        if (side >= 0) {
            const R* L = (const R*)a.le_buf;
            const size_t nyz = (size_t)a.ny * a.nz, q = (size_t)y + (size_t)a.ny * z;
#pragma unroll
            for (int r = 1; r < 19; r++)
                if (le_crosses(side, r)) d[r] = L[(size_t)(side * 5 + le_slot(r)) * nyz + q];
        }
        if (links) {
            const M rho_x = (M)a.rho0 + (M)Down;
#pragma unroll
            for (int r = 1; r < 19; r++) d[r] += (R)((M)(6.0 * WD(r)) * rho_x * link_cu<M>(lv, r));
        }

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
        const R ux = (jx + (R)0.5 * gx) * irho, uy = (jy + (R)0.5 * gy) * irho, uz = (jz + (R)0.5 * gz) * irho;
        const R usq = ux * ux + uy * uy + uz * uz;
        const R ug = ux * gx + uy * gy + uz * gz;
        // split codec: the density is stored first and the residuals are
        // taken against its decoded value (the collision conserves mass);
        // otherwise the density of the stored populations is stored
        R Dq = 0;
        if constexpr (Cd::SPLIT) {
            orho = Cd::enc(drho, rho_enc_scale<P>(a));
            Dq = rho_dec<P>(a, orho);
        }
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
            const T st = pop_enc<P>(a, out, r, Dq);
            ob[r] = st;
            if constexpr (!Cd::SPLIT) rsum += Cd::dec(st, dec_scale<P>(a, r));
        }
        if constexpr (!Cd::SPLIT) orho = Cd::enc(rsum, rho_enc_scale<P>(a));
        if (!(usq <= (R)0.16)) {
            atomicOr(a.status, ST_UNSTABLE);
            atomicMin(a.bad_step, *a.dstep);
        }
        } else if (inb && !(f & WALLNODE)) {
            // a cell node: the boundary velocity field holds its rigid-body velocity
            const int oz[3] = {z == a.nz - 1 ? -(int)((a.nz - 1) * plane) : (int)plane, 0,
                               z == 0 ? (int)((a.nz - 1) * plane) : -(int)plane};
            const M u0 = bload<M>(rU, (unsigned)sizeof(M) * i), u1 = bload<M>(rU, (unsigned)sizeof(M) * (ps + i)),
                    u2 = bload<M>(rU, (unsigned)sizeof(M) * (2 * ps + i));
            cell_node_links<P, M>(a, rA, rRA, i, f, ox, oy, oz, u0, u1, u2);
        }
        if (inb) {
#pragma unroll
            for (int r = 0; r < 19; r++) bstore<T>(ob[r], rB, ES * ((unsigned)r * ps + i));
            bstore<T>(orho, rRB, ES * i);
        }
    }
}

// Memory access of the tau = 1 kernel.  Narrow: raw buffer accesses, one
// scalar resource per array and a 32-bit byte offset per lane; a lane that
// loads nothing passes an offset past the buffer and reads 0.  Wide (the
// large-lattice layout, arrays past 4 GB): global accesses with a 64-bit
// address per lane; a lane that loads nothing reads a zeroed word instead.
// Element indices are 32-bit in the narrow form and 64-bit in the wide one.
template <bool W> struct LbMem;
template <> struct LbMem<false> {
    using I = unsigned;
    __amdgpu_buffer_rsrc_t r;
    __device__ LbMem(const void* p, unsigned long long bytes, const void*) : r(make_rsrc(p, bytes)) {}
    template <class T> __device__ T ld(I e, bool on) const { return bload<T>(r, on ? e * (I)sizeof(T) : OOB); }
    template <class T> __device__ void st(T v, I e) const { bstore<T>(v, r, e * (I)sizeof(T)); }
    template <class T> __device__ void stnt(T v, I e) const { bstore_nt<T>(v, r, e * (I)sizeof(T)); }
};
template <> struct LbMem<true> {
    using I = unsigned long long;
    char* p;
    const char* z;
    __device__ LbMem(const void* q, unsigned long long, const void* zero)
        : p((char*)const_cast<void*>(q)), z((const char*)zero) {}
    template <class T> __device__ T ld(I e, bool on) const { return *(const T*)(on ? p + e * sizeof(T) : z); }
    template <class T> __device__ void st(T v, I e) const { *(T*)(p + e * sizeof(T)) = v; }
    template <class T> __device__ void stnt(T v, I e) const { __builtin_nontemporal_store(v, (T*)(p + e * sizeof(T))); }
};

// tau = 1 (the paper's operating point, Sec. IV): the post-collision state is
// n^eq(rho, u) plus the forcing term, a function of the moments alone, so the
// pulled populations are folded into rho and j as they arrive.  LAY: the
// storage layout.  LAY_DENSE: every site stored.  LAY_BIG, the large-lattice
// layout: 64-bit lane addresses; a cell node's momentum goes to its own
// output slots instead of the node-momentum array.  LAY_IDX, the indexed
// layout of sparse geometries: only non-wall nodes are stored, each site's
// storage index comes from the map cidx (one load per neighbour), walls
// store nothing.
constexpr int LAY_DENSE = 0, LAY_BIG = 1, LAY_IDX = 2;

// The block's share of the mixture record (the quantity of the track pass:
// u_z of the collision at fluid nodes, the cell's rigid-body u_z at cell
// nodes, summed over the non-wall nodes with weights sin(2 pi y/ny) and 1):
// t is the thread's sum over its sweep at row y.  Butterfly sums within each
// wave, then the waves in order: a fixed order, so the record is
// deterministic.  Partial slot: the block's index in its lattice's grid.
__device__ __forceinline__ void lb_track_partial(const DevArgs& a, const KCtx& G, double t, int y) {
    __shared__ double red[2][4];
    double p0 = t * a.ysin[y], p1 = t;
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
        p0 += __shfl_xor(p0, m, 64);
        p1 += __shfl_xor(p1, m, 64);
    }
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    const int nw = (blockDim.x * blockDim.y) / 64;
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = p0;
        red[1][tid >> 6] = p1;
    }
    __syncthreads();
    if (tid == 0) {
        double s0 = 0.0, s1 = 0.0;
        for (int w = 0; w < nw; w++) {
            s0 += red[0][w];
            s1 += red[1][w];
        }
        const long long slot = G.bx + (long long)G.gx * (G.by + (long long)G.gy * G.bz);
        a.track_part[2 * slot] = s0;
        a.track_part[2 * slot + 1] = s1;
    }
}
// NT: the populations and densities are stored non-temporally (lattices
// whose output outgrows the last-level cache, see nt_out)
template <int P, int TZ, int LAY, bool NT = false>
__device__ __forceinline__ void lb_kernel_tau1_body(const DevArgs& a, const KCtx& G) {
    using Cd = Codec<P>;
    using T = typename Cd::T;
    using R = typename Cd::R;
    using M = R;
    constexpr bool BIG = LAY == LAY_BIG, IDX = LAY == LAY_IDX;
    using Mem = LbMem<BIG>;
    using I = typename Mem::I;
    // the thread's column (x, y): from a bx x by patch, or (plane-linear
    // tiles, by = 0) from bx consecutive sites of the flattened x-y plane
    int x, y;
    bool inb;
    if (a.tile[1] == 0) {
        const int q = (int)(G.bx * blockDim.x + threadIdx.x);
        y = q / a.nx;
        x = q - y * a.nx;
        inb = y < a.ny;
    } else {
        x = (int)(G.bx * blockDim.x + threadIdx.x);
        y = (int)(G.by * blockDim.y + threadIdx.y);
        inb = (x < a.nx) && (y < a.ny);
    }
    const int z0 = G.bz * TZ;
    const I nx = (I)a.nx;
    const I plane = (I)a.nx * (I)a.ny;
    const I ps = (I)a.pstride;  // narrow: every offset fits 32 bits (checked at create)
    const Mem mA(a.A, 19ull * (unsigned long long)a.pstride * sizeof(T), a.zero);
    const Mem mB(a.B, 19ull * (unsigned long long)a.pstride * sizeof(T), a.zero);
    const Mem mRA(a.rhoA, (unsigned long long)a.pstride * sizeof(T), a.zero);
    const Mem mRB(a.rhoB, (unsigned long long)a.pstride * sizeof(T), a.zero);
    const Mem mFl(a.flags, (unsigned long long)a.ns * 4, a.zero);
    const Mem mK(a.lmom, 4ull * (unsigned long long)a.pstride * sizeof(M), a.zero);
    const Mem mC(a.cidx, (unsigned long long)a.ns * 4, a.zero);
    const int oxs[3] = {x == a.nx - 1 ? -(a.nx - 1) : 1, 0, x == 0 ? a.nx - 1 : -1};
    const int oys[3] = {y == a.ny - 1 ? -(int)((a.ny - 1) * a.nx) : a.nx, 0, y == 0 ? (int)((a.ny - 1) * a.nx) : -a.nx};
    // body force at this plane: constant, or f0 sin(2 pi y/ny) from the table
    const int yc = y < a.ny ? y : a.ny - 1;
    const R gx0 = a.force_mode == 1 ? (R)a.g[0] : (R)0;
    const R gy0 = a.force_mode == 1 ? (R)a.g[1] : (R)0;
    const R gz0 = a.force_mode == 1 ? (R)a.g[2] : (a.force_mode == 2 ? (R)(a.f0 * a.ysin[yc]) : (R)0);

    // flags of the first node; each step prefetches the next node's flags
    const bool f0on = inb && z0 < a.nz;
    const uint32_t f0v = mFl.template ld<uint32_t>((I)x + nx * (I)y + plane * (I)z0, f0on);
    uint32_t fnext = f0on ? f0v : NONFLUID;
    // mixture record: this thread's sum of u_z over its nodes (y is fixed)
    R tacc = 0;
    // indexed layout: the storage indices a node needs, loaded one node
    // ahead.  mc[0] is the node's own, mc[q] that of its neighbour x - c_q: a
    // fluid lane pulls direction r from mc[r], a cell lane's link along c_r
    // reads the node x + c_r = mc[rbar].  The set does not depend on the
    // node's flags, so the next node's loads are issued while this node is
    // computed (masked at walls by the prefetched flag word).
    int mc[19];
    // (ox, oy: the x and y offsets of x - c, index c + 1; their middle entries are 0)
    auto map_loads = [&](const int* ox, const int* oy, I iq, int zq, bool on, int* out) {
        const int ozq[3] = {zq == a.nz - 1 ? -(int)((a.nz - 1) * plane) : (int)plane, 0,
                            zq == 0 ? (int)((a.nz - 1) * plane) : -(int)plane};
#pragma unroll
        for (int q = 0; q < 19; q++)
            out[q] = mC.template ld<int>(iq + (I)(ox[CX(q) + 1] + oy[CY(q) + 1] + ozq[CZ(q) + 1]), on);
    };
    if constexpr (IDX) map_loads(oxs, oys, (I)x + nx * (I)y + plane * (I)z0, z0, f0on && !(f0v & WALLNODE), mc);
#pragma unroll 1
    for (int zz = 0; zz < TZ; zz++) {
        const int z = z0 + zz;
        if (z >= a.nz) break;
        // a constant force confined to a slab of z acts there only (uniform over the step)
        const bool fon = !a.fregion || (z >= a.fzlo && z < a.fzhi);
        const R gx = fon ? gx0 : (R)0, gy = fon ? gy0 : (R)0, gz = fon ? gz0 : (R)0;
        const I i = (I)x + nx * (I)y + plane * (I)z;
        const uint32_t f = fnext;
        const bool fnon = inb && zz + 1 < TZ && z + 1 < a.nz;
        const uint32_t fnv = mFl.template ld<uint32_t>(i + plane, fnon);
        fnext = fnon ? fnv : NONFLUID;
        // outputs of the node; a non-fluid node stores zeros (a cell node in
        // the large-lattice layout its momentum).  The stores below are shared
        // by all lanes of the wave, so that each wave store writes its lines
        // whole (stores issued separately by the fluid and non-fluid lanes
        // would each write part of the same lines)
        const int oz[3] = {z == a.nz - 1 ? -(int)((a.nz - 1) * plane) : (int)plane, 0,
                           z == 0 ? (int)((a.nz - 1) * plane) : -(int)plane};
        const bool fl = !(f & NONFLUID);
        const bool cn = inb && (f & NONFLUID) && !(f & WALLNODE);  // a cell node
        const uint32_t links = f & LINKBITS;
        // the x and y offsets do not change along the sweep; made opaque in
        // each step, so that the compiler forms the per-direction offsets here
        // instead of keeping some thirty of them in registers for the sweep
        int ox[3] = {oxs[0], 0, oxs[2]}, oy[3] = {oys[0], 0, oys[2]};
        asm volatile("" : "+v"(ox[0]), "+v"(ox[2]), "+v"(oy[0]), "+v"(oy[2]));
        // One set of loads serves both kinds of lanes, so that their loads are
        // in flight together.  Slot r: a fluid lane pulls n*_r(x - c_r), or
        // bounces its own n*_rbar(x) when the source is not fluid (Eq. 9); a
        // cell lane loads the population its link along c_r carries,
        // n*_rbar(s + c_r), when s + c_r is fluid (Eq. 12).
        // indexed layout: the node's storage index (-1 at a wall or outside)
        I ci = i;
        int cw = 0;
        if constexpr (IDX) {
            cw = (inb && !(f & WALLNODE)) ? mc[0] : -1;
            ci = (I)cw;
        }
        T v[19];
#pragma unroll
        for (int r = 0; r < 19; r++) {
            const bool bb = (f >> r) & 1u;
            const bool lnk = r > 0 && cn && !((f >> OPP(r)) & 1u);
            I e;
            bool on;
            if constexpr (IDX) {
                const int nb = lnk ? mc[OPP(r)] : mc[r];
                e = lnk ? (I)OPP(r) * ps + (I)nb : (bb ? (I)OPP(r) * ps + ci : (I)r * ps + (I)nb);
                on = lnk || fl;
            } else {
                e = bb ? (I)OPP(r) * ps + i : (I)r * ps + i + (I)(ox[CX(r) + 1] + oy[CY(r) + 1] + oz[CZ(r) + 1]);
                on = fl;
                if (lnk) {
                    e = (I)OPP(r) * ps + i + (I)(ox[1 - CX(r)] + oy[1 - CY(r)] + oz[1 - CZ(r)]);
                    on = true;
                }
            }
            v[r] = mA.template ld<T>(e, on);
        }
        // fluid lanes: their link moments (the split codec's hold every fluid
        // node's density parts too, see below); cell lanes: planes 0-2 hold
        // the node's rigid-body velocity
        M km[4];
        const bool kon = (fl && (links || Cd::SPLIT)) || cn;
#pragma unroll
        for (int c = 0; c < 4; c++) km[c] = mK.template ld<M>((I)c * ps + ci, kon);
        // cell lanes: the densities of their links' fluid nodes
        T dn[19];
#pragma unroll
        for (int r = 1; r < 19; r++) {
            const bool lnk = cn && !((f >> OPP(r)) & 1u);
            if constexpr (IDX) dn[r] = mRA.template ld<T>((I)mc[OPP(r)], lnk);
            else dn[r] = mRA.template ld<T>(i + (I)(ox[1 - CX(r)] + oy[1 - CY(r)] + oz[1 - CZ(r)]), lnk);
        }
        int mn[19];
        if constexpr (IDX) map_loads(ox, oy, i + plane, z + 1, fnon && !(fnv & WALLNODE), mn);
        double m0 = 0, m1 = 0, m2 = 0;
        if (cn) {
            // fused multiply-adds only within one expression, so that every
            // compiled variant of this kernel rounds the sums below alike
#pragma clang fp contract(on)
            // the momentum the node's links carry to its cell (Eq. 12): the
            // neighbour x = s + c_r bounces n*_rbar(x) into direction r and the
            // correction C_r = 6 w_r rho(x) (c_r . u(s)) (Eq. 10) is added, so the
            // link transfers (2 n*_rbar(x) + C_r) c_rbar; deviation part only (the
            // constant part and the solid links of Eqs. 13-14 cancel over the
            // closed surface of a node set); FP64 from the decoded values
            const double us[3] = {(double)km[0], (double)km[1], (double)km[2]};
#pragma unroll
            for (int r = 1; r < 19; r++) {
                const bool lk = !((f >> OPP(r)) & 1u);
                const R Dx = rho_dec<P>(a, dn[r]);
                const double rho_x = a.rho0 + (double)Dx;
                double cu = 0;
                if (CX(r)) cu += CX(r) * us[0];
                if (CY(r)) cu += CY(r) * us[1];
                if (CZ(r)) cu += CZ(r) * us[2];
                const double C = 6.0 * WD(r) * rho_x * cu;
                const double mr = lk ? -(2.0 * (double)pop_dec<P>(a, v[r], OPP(r), Dx) + C) : 0.0;
                if (CX(r)) m0 += CX(r) * mr;
                if (CY(r)) m1 += CY(r) * mr;
                if (CZ(r)) m2 += CZ(r) * mr;
            }
            if constexpr (!BIG) {
                double* F = a.fnode + 3 * (size_t)ci;
                F[0] = m0;
                F[1] = m1;
                F[2] = m2;
            }
            tacc += (R)km[2];  // the rigid-body u_z the bounce-back used
        }
        T ob[19], orho;
#pragma unroll
        for (int r = 0; r < 19; r++) ob[r] = Cd::enc((R)0, (R)1);
        orho = Cd::enc((R)0, (R)1);
        if constexpr (BIG) {
            if (cn) {
                const double m[3] = {m0, m1, m2};
#pragma unroll
                for (int k = 0; k < 24 / (int)sizeof(T); k++) ob[k] = mom_piece<T>(m, k);
            }
        }
        if (fl) {
        R Down = 0;  // the node's stored density deviation (for C; not needed by the split codec)
        R drho = 0, jx = 0, jy = 0, jz = 0;
        if constexpr (!Cd::SPLIT) Down = rho_dec<P>(a, mRA.template ld<T>(ci, links != 0u));
        // viscometer seam: the populations pulled across it come from the
        // sheared image (the split codec is refused with the viscometer)
        const int side = le_side(a, x);
        const R* L = (const R*)a.le_buf;
        const size_t nyz = (size_t)a.ny * a.nz, q = (size_t)y + (size_t)a.ny * z;
#pragma unroll
        for (int r = 0; r < 19; r++) {
            // split codec: the residual parts w_r h_r only
            R dv = pop_dec<P>(a, v[r], r, (R)0);
            if (r > 0 && side >= 0 && le_crosses(side, r)) dv = L[(size_t)(side * 5 + le_slot(r)) * nyz + q];
            drho += dv;
            if (CX(r)) jx += CX(r) * dv;
            if (CY(r)) jy += CY(r) * dv;
            if (CZ(r)) jz += CZ(r) * dv;
        }
        if constexpr (Cd::SPLIT) {
            // the density parts of the pulled populations (w_r D of each
            // population's source, the node's own for a bounced one) and the
            // moving-boundary corrections, summed by the link-moment kernel
            drho += (R)km[0]; jx += (R)km[1]; jy += (R)km[2]; jz += (R)km[3];
        } else if (links) {
            // moving-boundary corrections summed over the links:
            // sum C_r = 6 rho(x) K0, sum C_r c_r = 6 rho(x) (K1, K2, K3)
            const M rho6 = (M)6 * ((M)a.rho0 + (M)Down);
            drho += (R)(rho6 * km[0]); jx += (R)(rho6 * km[1]); jy += (R)(rho6 * km[2]); jz += (R)(rho6 * km[3]);
        }

        // n* = n^eq(rho, u) + Guo term (tau = 1), for opposite pairs r, rbar:
        // even part E = 4.5 cu^2 - 1.5 u^2 (+ forcing 0.5 w (9 cu cg - 3 u.g)),
        // odd part O = 3 cu + 4.5 cu^3 - 4.5 u^2 cu (+ forcing 1.5 w cg)
        const R rho = (R)a.rho0 + drho;
        const R irho = (R)1 / rho;
        const R ux = (jx + (R)0.5 * gx) * irho, uy = (jy + (R)0.5 * gy) * irho, uz = (jz + (R)0.5 * gz) * irho;
        const R usq = ux * ux + uy * uy + uz * uz;
        const R ug = ux * gx + uy * gy + uz * gz;
        tacc += uz;
        // the collision conserves mass: the density deviation of n* is drho.
        // Split codec: the stored outputs are n*_r - w_r (rho0 + Dq), with Dq
        // the decoded stored density, so drho enters as drho - Dq
        orho = Cd::enc(drho, rho_enc_scale<P>(a));
        R dres = drho;
        if constexpr (Cd::SPLIT) dres = drho - rho_dec<P>(a, orho);
        {
            const R w0 = (R)(1.0 / 3.0);
            const R out0 = w0 * (dres - rho * (R)1.5 * usq) - (R)1.5 * w0 * ug;
            ob[0] = Cd::enc(out0, enc_scale<P>(a, 0));
        }
#pragma unroll
        for (int r = 1; r < 19; r += 2) {
            const R w = (R)WD(r);
            const R cu = CX(r) * ux + CY(r) * uy + CZ(r) * uz;
            const R cg = CX(r) * gx + CY(r) * gy + CZ(r) * gz;
            const R cu2 = cu * cu;
            const R ev = w * (dres + rho * ((R)4.5 * cu2 - (R)1.5 * usq)) + (R)0.5 * w * ((R)9 * cu * cg - (R)3 * ug);
            const R od = w * rho * cu * ((R)3 + (R)4.5 * cu2 - (R)4.5 * usq) + (R)1.5 * w * cg;
            ob[r] = Cd::enc(ev + od, enc_scale<P>(a, r));
            ob[r + 1] = Cd::enc(ev - od, enc_scale<P>(a, r + 1));
        }
        if (!(usq <= (R)0.16)) {
            atomicOr(a.status, ST_UNSTABLE);
            atomicMin(a.bad_step, *a.dstep);
        }
        }
        if (inb && cw >= 0) {  // (walls of the indexed layout store nothing)
            if constexpr (NT) {
#pragma unroll
                for (int r = 0; r < 19; r++) mB.template stnt<T>(ob[r], (I)r * ps + ci);
                mRB.template stnt<T>(orho, ci);
            } else {
#pragma unroll
                for (int r = 0; r < 19; r++) mB.template st<T>(ob[r], (I)r * ps + ci);
                mRB.template st<T>(orho, ci);
            }
        }
        if constexpr (IDX) {
#pragma unroll
            for (int q = 0; q < 19; q++) mc[q] = mn[q];
        }
    }
    if (track_in_lb(a)) lb_track_partial(a, G, inb ? (double)tacc : 0.0, yc);
}
template <int P, int TZ, int LAY, bool NT = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(LAY == LAY_DENSE ? 4 : 3))) lb_kernel_tau1(DevArgs a) { lb_kernel_tau1_body<P, TZ, LAY, NT>(a, hw_ctx()); }
template <int P, int TZ, int LAY>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(LAY == LAY_DENSE ? 4 : 3))) lb_kernel_tau1_multi(const DevArgs* __restrict__ as, const ChanGrid* __restrict__ cg, int nch) {
    unsigned t;
    const int c = chan_of_xcd(cg, nch, &t);
    lb_kernel_tau1_body<P, TZ, LAY>(as[c], chan_ctx_at(cg[c], t));
}


template <int P>
static hipError_t launch_lb_p(const DevArgs& a, LaunchCfg cfg, hipStream_t st) {
    const bool lin = cfg.by == 0;  // plane-linear tiles (tau = 1, checked when set)
    dim3 blk(cfg.bx, lin ? 1 : cfg.by, 1);
    dim3 grd(lin ? (unsigned)(((long long)a.nx * a.ny + cfg.bx - 1) / cfg.bx) : (unsigned)((a.nx + cfg.bx - 1) / cfg.bx),
             lin ? 1u : (unsigned)((a.ny + cfg.by - 1) / cfg.by), (a.nz + cfg.tz - 1) / cfg.tz);
    const bool t1 = a.tau == 1.0;
    if (lin && !t1) return hipErrorInvalidValue;
    if (a.big || a.cidx) {
        // the large-lattice and indexed layouts: tau = 1 and 16-node sweeps
        // only (checked when the handle is created and when tiles are set)
        if (!t1 || cfg.tz != 16) return hipErrorInvalidValue;
        if (a.big && a.nt_out) hipLaunchKernelGGL((lb_kernel_tau1<P, 16, LAY_BIG, true>), grd, blk, 0, st, a);
        else if (a.big) hipLaunchKernelGGL((lb_kernel_tau1<P, 16, LAY_BIG>), grd, blk, 0, st, a);
        else hipLaunchKernelGGL((lb_kernel_tau1<P, 16, LAY_IDX>), grd, blk, 0, st, a);
        return hipGetLastError();
    }
    switch (cfg.tz) {
        case 4:
            if (t1 && a.nt_out) hipLaunchKernelGGL((lb_kernel_tau1<P, 4, LAY_DENSE, true>), grd, blk, 0, st, a);
            else if (t1) hipLaunchKernelGGL((lb_kernel_tau1<P, 4, LAY_DENSE>), grd, blk, 0, st, a);
            else hipLaunchKernelGGL((lb_kernel_tau<P, 4>), grd, blk, 0, st, a);
            break;
        case 8:
            if (t1 && a.nt_out) hipLaunchKernelGGL((lb_kernel_tau1<P, 8, LAY_DENSE, true>), grd, blk, 0, st, a);
            else if (t1) hipLaunchKernelGGL((lb_kernel_tau1<P, 8, LAY_DENSE>), grd, blk, 0, st, a);
            else hipLaunchKernelGGL((lb_kernel_tau<P, 8>), grd, blk, 0, st, a);
            break;
        case 16:
            if (t1 && a.nt_out) hipLaunchKernelGGL((lb_kernel_tau1<P, 16, LAY_DENSE, true>), grd, blk, 0, st, a);
            else if (t1) hipLaunchKernelGGL((lb_kernel_tau1<P, 16, LAY_DENSE>), grd, blk, 0, st, a);
            else hipLaunchKernelGGL((lb_kernel_tau<P, 16>), grd, blk, 0, st, a);
            break;
        case 32:
            if (t1 && a.nt_out) hipLaunchKernelGGL((lb_kernel_tau1<P, 32, LAY_DENSE, true>), grd, blk, 0, st, a);
            else if (t1) hipLaunchKernelGGL((lb_kernel_tau1<P, 32, LAY_DENSE>), grd, blk, 0, st, a);
            else hipLaunchKernelGGL((lb_kernel_tau<P, 32>), grd, blk, 0, st, a);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// batch: the dense tau = 1 kernel for every channel of a tile group; the
// variant is (precision, sweep depth)
bool multi_grid_lb(const DevArgs& a, LaunchCfg cfg, int* variant, unsigned* bx, unsigned* by, dim3* grid) {
    if (a.tau != 1.0 || a.big || a.cidx || a.le_u != 0.0) return false;
    *variant = a.precision * 64 + cfg.tz;
    *bx = (unsigned)cfg.bx;
    *by = (unsigned)cfg.by;  // 0: plane-linear tiles (a launch of its own, blocks of bx x 1)
    if (cfg.by == 0)
        *grid = dim3((unsigned)(((long long)a.nx * a.ny + cfg.bx - 1) / cfg.bx), 1, (a.nz + cfg.tz - 1) / cfg.tz);
    else
        *grid = dim3((a.nx + cfg.bx - 1) / cfg.bx, (a.ny + cfg.by - 1) / cfg.by, (a.nz + cfg.tz - 1) / cfg.tz);
    return true;
}

template <int P>
static hipError_t launch_multi_lb_p(const MultiLaunch& m, const DevArgs* args, hipStream_t st, int tz) {
    const dim3 g(m.blocks), b(m.bx, m.by ? m.by : 1);
    switch (tz) {
        case 4: hipLaunchKernelGGL((lb_kernel_tau1_multi<P, 4, LAY_DENSE>), g, b, 0, st, args, m.cg, m.nch); break;
        case 8: hipLaunchKernelGGL((lb_kernel_tau1_multi<P, 8, LAY_DENSE>), g, b, 0, st, args, m.cg, m.nch); break;
        case 16: hipLaunchKernelGGL((lb_kernel_tau1_multi<P, 16, LAY_DENSE>), g, b, 0, st, args, m.cg, m.nch); break;
        case 32: hipLaunchKernelGGL((lb_kernel_tau1_multi<P, 32, LAY_DENSE>), g, b, 0, st, args, m.cg, m.nch); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_multi_lb(const MultiLaunch& m, const DevArgs* args, hipStream_t st) {
    const int tz = m.variant % 64;
    switch (m.variant / 64) {
        case CGB_P64: return launch_multi_lb_p<CGB_P64>(m, args, st, tz);
        case CGB_P32: return launch_multi_lb_p<CGB_P32>(m, args, st, tz);
        case CGB_PMX16: return launch_multi_lb_p<CGB_PMX16>(m, args, st, tz);
        case CGB_PMXBF16: return launch_multi_lb_p<CGB_PMXBF16>(m, args, st, tz);
        case CGB_PMX16S: return launch_multi_lb_p<CGB_PMX16S>(m, args, st, tz);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_lb(const DevArgs& a, LaunchCfg cfg, hipStream_t st) {
    if (cfg.bx != a.tile[0] || cfg.by != a.tile[1] || cfg.tz != a.tile[2]) return hipErrorInvalidValue;
    switch (a.precision) {
        case CGB_P64: return launch_lb_p<CGB_P64>(a, cfg, st);
        case CGB_P32: return launch_lb_p<CGB_P32>(a, cfg, st);
        case CGB_PMX16: return launch_lb_p<CGB_PMX16>(a, cfg, st);
        case CGB_PMXBF16: return launch_lb_p<CGB_PMXBF16>(a, cfg, st);
        case CGB_PMX16S: return launch_lb_p<CGB_PMX16S>(a, cfg, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace cgb
