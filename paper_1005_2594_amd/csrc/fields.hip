// fields.hip -- population codec, equilibrium initialisation and read-out
// reductions (moments of Eqs. 7-8, mass, momentum, velocity profile).
#include "cgb_dev.h"

namespace cgb {

// FP64 deviations [19][ns] -> storage, and the density deviation field
template <int P>
__global__ void encode_kernel(DevArgs a, const double* d) {
    using Cd = Codec<P>;
    using T = typename Cd::T;
    using R = typename Cd::R;
    const long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (s >= a.ns) return;
    const long long c = sidx(a, s);
    if (c < 0) return;  // a wall of the indexed layout holds nothing
    T* A = (T*)a.A;
    R Dq = 0;
    if constexpr (Cd::SPLIT) {
        // the density first; the residuals are taken against its decoded value
        double dr = 0;
        for (int r = 0; r < 19; r++) dr += d[r * a.ns + s];
        const T st = Cd::enc((R)dr, rho_enc_scale<P>(a));
        ((T*)a.rhoA)[c] = st;
        Dq = rho_dec<P>(a, st);
    }
    R rs = 0;
    for (int r = 0; r < 19; r++) {
        const T v = pop_enc<P>(a, (R)d[r * a.ns + s], r, Dq);
        A[r * a.pstride + c] = v;
        rs += pop_dec<P>(a, v, r, Dq);
    }
    if constexpr (!Cd::SPLIT) ((T*)a.rhoA)[c] = Cd::enc(rs, rho_enc_scale<P>(a));
}

template <int P>
__global__ void decode_kernel(DevArgs a, double* d) {
    using Cd = Codec<P>;
    using T = typename Cd::T;
    const long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (s >= a.ns) return;
    const T* A = (const T*)a.A;
    // non-fluid nodes hold no populations (their slots are never read; with
    // the large-lattice layout a cell node's slots carry its momentum)
    if (a.owner[s] != OWN_FLUID) {
        for (int r = 0; r < 19; r++) d[r * a.ns + s] = 0.0;
        return;
    }
    const long long c = sidx(a, s);
    const auto Ds = rho_dec<P>(a, ((const T*)a.rhoA)[c]);
    for (int r = 0; r < 19; r++) d[r * a.ns + s] = (double)pop_dec<P>(a, A[r * a.pstride + c], r, Ds);
}

// the populations (FP64 deviations, 0 at non-fluid nodes) and the owners of
// the box lo + [0, ext): out[r * nb + k] and own[k], k = x' + ext0 (y' + ext1 z')
template <int P>
__global__ void decode_box_kernel(DevArgs a, int lx, int ly, int lz, int ex, int ey, int ez, double* out, int* own) {
    using Cd = Codec<P>;
    using T = typename Cd::T;
    const long long nb = (long long)ex * ey * ez;
    const long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (k >= nb) return;
    const int x = lx + (int)(k % ex), y = ly + (int)((k / ex) % ey), z = lz + (int)(k / ((long long)ex * ey));
    const long long s = x + (long long)a.nx * (y + (long long)a.ny * z);
    const int o = a.owner[s];
    own[k] = o;
    if (o != OWN_FLUID) {
        for (int r = 0; r < 19; r++) out[r * nb + k] = 0.0;
        return;
    }
    const T* A = (const T*)a.A;
    const long long c = sidx(a, s);
    const auto Ds = rho_dec<P>(a, ((const T*)a.rhoA)[c]);
    for (int r = 0; r < 19; r++) out[r * nb + k] = (double)pop_dec<P>(a, A[r * a.pstride + c], r, Ds);
}

// the mixture velocity of the box lo + [0, ext): fluid nodes the velocity of
// the last collision, (sum n c - g/2) / rho; cell nodes the rigid-body
// velocity of their cell as the last bounce-back used it, V + Omega x (s - X);
// walls 0.  u[3 k + c], k = x' + ext0 (y' + ext1 z')
template <int P>
__global__ void mixture_box_kernel(DevArgs a, int lx, int ly, int lz, int ex, int ey, int ez, double* u) {
    using Cd = Codec<P>;
    using T = typename Cd::T;
    const long long nb = (long long)ex * ey * ez;
    const long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (k >= nb) return;
    const int x = lx + (int)(k % ex), y = ly + (int)((k / ex) % ey), z = lz + (int)(k / ((long long)ex * ey));
    const long long s = x + (long long)a.nx * (y + (long long)a.ny * z);
    const int o = a.owner[s];
    double v[3] = {0.0, 0.0, 0.0};
    if (o == OWN_FLUID) {
        const T* A = (const T*)a.A;
        const long long c = sidx(a, s);
        const auto Ds = rho_dec<P>(a, ((const T*)a.rhoA)[c]);
        double drho = 0, j[3] = {0, 0, 0};
        for (int r = 0; r < 19; r++) {
            const double d = (double)pop_dec<P>(a, A[r * a.pstride + c], r, Ds);
            drho += d;
            j[0] += d * CX(r); j[1] += d * CY(r); j[2] += d * CZ(r);
        }
        double g[3];
        body_force(a, (double)y, (double)z, g);
        for (int c = 0; c < 3; c++) v[c] = (j[c] - 0.5 * g[c]) / (a.rho0 + drho);
    } else if (o >= 0) {
        const double* kp = a.kin + 12 * (long long)o;
        double d[3], w[3];
        node_disp(a, x, y, z, kp, d);
        cross3(kp + 6, d, w);
        for (int c = 0; c < 3; c++) v[c] = kp[3 + c] + w[c];
    }
    for (int c = 0; c < 3; c++) u[3 * k + c] = v[c];
}

// Eq. 5 at (rho, u) on every non-wall node, written as n^eq - w rho0
template <int P>
__global__ void equilibrium_kernel(DevArgs a, const double* rho, const double* u) {
    using Cd = Codec<P>;
    using T = typename Cd::T;
    using R = typename Cd::R;
    const long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (s >= a.ns) return;
    T* A = (T*)a.A;
    const bool wall = a.owner[s] == OWN_WALL;
    const long long c = sidx(a, s);
    if (c < 0) return;  // a wall of the indexed layout holds nothing
    const double rr = rho ? rho[s] : a.rho0;
    const double ux = u ? u[3 * s] : 0.0, uy = u ? u[3 * s + 1] : 0.0, uz = u ? u[3 * s + 2] : 0.0;
    const double usq = ux * ux + uy * uy + uz * uz;
    R Dq = 0;
    if constexpr (Cd::SPLIT) {
        // Eq. 5 conserves the density: the density deviation is rho - rho0
        const T st = Cd::enc(wall ? (R)0 : (R)(rr - a.rho0), rho_enc_scale<P>(a));
        ((T*)a.rhoA)[c] = st;
        Dq = rho_dec<P>(a, st);
    }
    R rs = 0;
    for (int r = 0; r < 19; r++) {
        const double cu = CX(r) * ux + CY(r) * uy + CZ(r) * uz;
        const double poly = 3.0 * cu + 4.5 * cu * cu - 1.5 * usq + 4.5 * cu * cu * cu - 4.5 * usq * cu;
        const double eq = wall ? 0.0 : WD(r) * ((rr - a.rho0) + rr * poly);
        const T v = pop_enc<P>(a, (R)eq, r, Dq);
        A[r * a.pstride + c] = v;
        rs += pop_dec<P>(a, v, r, Dq);
    }
    if constexpr (!Cd::SPLIT) ((T*)a.rhoA)[c] = Cd::enc(rs, rho_enc_scale<P>(a));
}

// rho = rho0 + sum d, u = (sum d c - g/2) / rho on fluid nodes
template <int P>
__global__ void fields_kernel(DevArgs a, double* rho, double* u) {
    using Cd = Codec<P>;
    using T = typename Cd::T;
    const long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (s >= a.ns) return;
    if (a.owner[s] != OWN_FLUID) {
        if (rho) rho[s] = 0.0;
        if (u) { u[3 * s] = 0.0; u[3 * s + 1] = 0.0; u[3 * s + 2] = 0.0; }
        return;
    }
    const T* A = (const T*)a.A;
    const long long c = sidx(a, s);
    const auto Ds = rho_dec<P>(a, ((const T*)a.rhoA)[c]);
    double drho = 0, j[3] = {0, 0, 0};
    for (int r = 0; r < 19; r++) {
        const double v = (double)pop_dec<P>(a, A[r * a.pstride + c], r, Ds);
        drho += v;
        j[0] += v * CX(r); j[1] += v * CY(r); j[2] += v * CZ(r);
    }
    const double rr = a.rho0 + drho;
    double g[3];
    body_force(a, (double)((s / a.nx) % a.ny), (double)(s / ((long long)a.nx * a.ny)), g);
    if (rho) rho[s] = rr;
    if (u) for (int c = 0; c < 3; c++) u[3 * s + c] = (j[c] - 0.5 * g[c]) / rr;
}

// per-block partial sums: mass, momentum (3), fluid count, body force (3)
template <int P>
__global__ void __launch_bounds__(256) observables_kernel(DevArgs a, double* partial) {
    using Cd = Codec<P>;
    using T = typename Cd::T;
    __shared__ double red[8][256];
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const T* A = (const T*)a.A;
    for (long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x; s < a.ns; s += (long long)gridDim.x * blockDim.x) {
        if (a.owner[s] != OWN_FLUID) continue;
        const long long c = sidx(a, s);
        const auto Ds = rho_dec<P>(a, ((const T*)a.rhoA)[c]);
        double drho = 0;
        for (int r = 0; r < 19; r++) {
            const double v = (double)pop_dec<P>(a, A[r * a.pstride + c], r, Ds);
            drho += v;
            acc[1] += v * CX(r); acc[2] += v * CY(r); acc[3] += v * CZ(r);
        }
        acc[0] += a.rho0 + drho;
        acc[4] += 1.0;
        double g[3];
        body_force(a, (double)((s / a.nx) % a.ny), (double)(s / ((long long)a.nx * a.ny)), g);
        acc[5] += g[0]; acc[6] += g[1]; acc[7] += g[2];
    }
    for (int k = 0; k < 8; k++) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int off = 128; off >= 1; off >>= 1) {
        if ((int)threadIdx.x < off)
            for (int k = 0; k < 8; k++) red[k][threadIdx.x] += red[k][threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 8; k++) partial[8 * blockIdx.x + k] = red[k][0];
}

// mixture z velocity summed per plane normal to `axis`, and the node count per plane
template <int P>
__global__ void profile_kernel(DevArgs a, double* prof, double* cnt, int axis) {
    using Cd = Codec<P>;
    using T = typename Cd::T;
    const long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (s >= a.ns) return;
    const int o = a.owner[s];
    if (o == OWN_WALL) return;
    const int x = (int)(s % a.nx), y = (int)((s / a.nx) % a.ny), z = (int)(s / ((long long)a.nx * a.ny));
    double uz;
    if (o == OWN_FLUID) {
        const T* A = (const T*)a.A;
        const long long c = sidx(a, s);
        const auto Ds = rho_dec<P>(a, ((const T*)a.rhoA)[c]);
        double drho = 0, jz = 0;
        for (int r = 0; r < 19; r++) {
            const double v = (double)pop_dec<P>(a, A[r * a.pstride + c], r, Ds);
            drho += v;
            jz += v * CZ(r);
        }
        double g[3];
        body_force(a, (double)y, (double)z, g);
        uz = (jz - 0.5 * g[2]) / (a.rho0 + drho);
    } else {
        const double* k = a.kin + 12 * (long long)o;
        double d[3];
        node_disp(a, x, y, z, k, d);
        uz = k[5] + (k[6] * d[1] - k[7] * d[0]);
    }
    const int pl = axis == 0 ? x : (axis == 1 ? y : z);
    unsafeAtomicAdd(prof + pl, uz);
    unsafeAtomicAdd(cnt + pl, 1.0);
}

#define CGB_DISPATCH(KERNEL, GRID, BLOCK, ...)                                                       \
    switch (a.precision) {                                                                           \
        case CGB_P64: hipLaunchKernelGGL(KERNEL<CGB_P64>, GRID, BLOCK, 0, st, __VA_ARGS__); break;   \
        case CGB_P32: hipLaunchKernelGGL(KERNEL<CGB_P32>, GRID, BLOCK, 0, st, __VA_ARGS__); break;   \
        case CGB_PMX16: hipLaunchKernelGGL(KERNEL<CGB_PMX16>, GRID, BLOCK, 0, st, __VA_ARGS__); break; \
        case CGB_PMXBF16: hipLaunchKernelGGL(KERNEL<CGB_PMXBF16>, GRID, BLOCK, 0, st, __VA_ARGS__); break; \
        case CGB_PMX16S: hipLaunchKernelGGL(KERNEL<CGB_PMX16S>, GRID, BLOCK, 0, st, __VA_ARGS__); break; \
        default: return hipErrorInvalidValue;                                                        \
    }

static dim3 site_grid(const DevArgs& a) { return dim3((unsigned)((a.ns + 255) / 256)); }

// Mixture z velocity of the state just written (B, rhoB) summed over the
// non-wall nodes, weighted by sin(2 pi y/ny) and by 1: fluid nodes carry the
// velocity of the collision, u_z = (sum n* c_z - g_z/2)/rho (the forcing adds
// exactly g to sum n* c), cell nodes the rigid-body velocity of their cell
// that the bounce-back used (from the cell's kinematics, FP64).  Fixed grid and
// fixed per-thread site sets, block partials reduced in a fixed order: the
// sums are deterministic.  This pass serves the general-tau kernel (and a
// tile whose blocks outnumber the partial slots); the tau = 1 kernel sums the
// same quantity from the velocity of its own collision.
template <int P>
__device__ __forceinline__ void track_kernel_body(const DevArgs& a, const KCtx& G) {
    using Cd = Codec<P>;
    using T = typename Cd::T;
    using M = typename Cd::R;
    __shared__ double red[2][256];
    const T* B = (const T*)a.B;
    const T* RB = (const T*)a.rhoB;
    double ss = 0.0, s1 = 0.0;
    for (long long s = G.bx * 256LL + threadIdx.x; s < a.ns; s += (long long)G.gx * 256) {
        const int o = a.owner[s];
        if (o == OWN_WALL) continue;
        const int y = (int)(((unsigned)s / (unsigned)a.nx) % (unsigned)a.ny);  // sites < 2^32 (checked at create)
        double uz;
        if (o == OWN_FLUID) {
            double jz = 0.0;
            const long long c = sidx(a, s);
            const M Ds = rho_dec<P>(a, RB[c]);
#pragma unroll
            for (int r = 5; r < 19; r++)
                if (CZ(r)) jz += CZ(r) * (double)pop_dec<P>(a, B[r * a.pstride + c], r, Ds);
            const double drho = (double)Ds;
            double g[3];
            body_force(a, (double)y, (double)((unsigned)s / ((unsigned)a.nx * (unsigned)a.ny)), g);
            const double gz = g[2];
            uz = (jz - 0.5 * gz) / (a.rho0 + drho);
        } else {
            // the rigid-body velocity of the node's cell
            const double* k = a.kin + 12 * (long long)o;
            const int x = (int)((unsigned)s % (unsigned)a.nx), z = (int)((unsigned)s / ((unsigned)a.nx * (unsigned)a.ny));
            double d[3];
            node_disp(a, x, y, z, k, d);
            uz = k[5] + (k[6] * d[1] - k[7] * d[0]);
        }
        ss += uz * a.ysin[y];
        s1 += uz;
    }
    red[0][threadIdx.x] = ss;
    red[1][threadIdx.x] = s1;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            red[0][threadIdx.x] += red[0][threadIdx.x + off];
            red[1][threadIdx.x] += red[1][threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.track_part[2 * G.bx] = red[0][0];
        a.track_part[2 * G.bx + 1] = red[1][0];
    }
}
template <int P>
__global__ void __launch_bounds__(256) track_kernel(DevArgs a) { track_kernel_body<P>(a, hw_ctx()); }
template <int P>
__global__ void __launch_bounds__(256) track_kernel_multi(const DevArgs* __restrict__ as, const ChanGrid* __restrict__ cg, int nch) {
    const int c = chan_of(cg, nch);
    track_kernel_body<P>(as[c], chan_ctx(cg[c]));
}


// One workgroup of FIN_THREADS adds the partials: thread t the partials t,
// t + FIN_THREADS, ... in that order (loads issued eight at a time), then the
// threads in a fixed tree: the record is deterministic.
constexpr int FIN_THREADS = 1024;
__device__ __forceinline__ void track_finish_kernel_body(const DevArgs& a, const KCtx& G) {
    __shared__ double red[2][FIN_THREADS / 64];
    double ss = 0.0, s1 = 0.0;
    const long long nparts = track_in_lb(a) ? lb_blocks(a) : track_blocks(a.ns);
    const double2* P = (const double2*)a.track_part;
    long long b = threadIdx.x;
    for (; b + 7LL * FIN_THREADS < nparts; b += 8LL * FIN_THREADS) {
        double2 v[8];
#pragma unroll
        for (int u = 0; u < 8; u++) v[u] = P[b + (long long)u * FIN_THREADS];
#pragma unroll
        for (int u = 0; u < 8; u++) {
            ss += v[u].x;
            s1 += v[u].y;
        }
    }
    for (; b < nparts; b += FIN_THREADS) {
        ss += P[b].x;
        s1 += P[b].y;
    }
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
        ss += __shfl_xor(ss, m, 64);
        s1 += __shfl_xor(s1, m, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = ss;
        red[1][threadIdx.x >> 6] = s1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t0 = 0.0, t1 = 0.0;
        for (int w = 0; w < FIN_THREADS / 64; w++) {
            t0 += red[0][w];
            t1 += red[1][w];
        }
        const int n = *a.track_n;
        if (n < a.track_cap) {
            a.track[2 * n] = t0;
            a.track[2 * n + 1] = t1;
        }
        *a.track_n = n + 1;
    }
}
__global__ void __launch_bounds__(FIN_THREADS) track_finish_kernel(DevArgs a) { track_finish_kernel_body(a, hw_ctx()); }
__global__ void __launch_bounds__(FIN_THREADS) track_finish_kernel_multi(const DevArgs* __restrict__ as, const ChanGrid* __restrict__ cg, int nch) {
    const int c = chan_of(cg, nch);
    track_finish_kernel_body(as[c], chan_ctx(cg[c]));
}


hipError_t launch_track(const DevArgs& a, hipStream_t st) {
    if (!a.track) return hipSuccess;
    if (!track_in_lb(a)) CGB_DISPATCH(track_kernel, dim3(track_blocks(a.ns)), dim3(256), a);
    hipLaunchKernelGGL(track_finish_kernel, dim3(1), dim3(FIN_THREADS), 0, st, a);
    return hipGetLastError();
}

// batch: the mixture record of every channel
bool multi_grid_fields(int kind, const DevArgs& a, int* variant, unsigned* bx, unsigned* by, dim3* grid, int* arg) {
    *variant = a.precision;
    *bx = 256;
    *by = 1;
    *arg = 0;
    if (!a.track) return false;
    if (kind == MK_TRACK) {
        if (track_in_lb(a)) return false;  // the LB kernel sums this channel's record
        *grid = dim3(track_blocks(a.ns));
        return true;
    }
    if (kind == MK_TRACK_FIN) { *bx = FIN_THREADS; *grid = dim3(1); return true; }
    return false;
}

hipError_t launch_multi_fields(const MultiLaunch& m, const DevArgs* args, hipStream_t st) {
    if (m.kind == MK_TRACK_FIN) {
        hipLaunchKernelGGL(track_finish_kernel_multi, dim3(m.blocks), dim3(FIN_THREADS), 0, st, args, m.cg, m.nch);
        return hipGetLastError();
    }
    switch (m.variant) {
        case CGB_P64: hipLaunchKernelGGL(track_kernel_multi<CGB_P64>, dim3(m.blocks), dim3(256), 0, st, args, m.cg, m.nch); break;
        case CGB_P32: hipLaunchKernelGGL(track_kernel_multi<CGB_P32>, dim3(m.blocks), dim3(256), 0, st, args, m.cg, m.nch); break;
        case CGB_PMX16: hipLaunchKernelGGL(track_kernel_multi<CGB_PMX16>, dim3(m.blocks), dim3(256), 0, st, args, m.cg, m.nch); break;
        case CGB_PMXBF16: hipLaunchKernelGGL(track_kernel_multi<CGB_PMXBF16>, dim3(m.blocks), dim3(256), 0, st, args, m.cg, m.nch); break;
        case CGB_PMX16S: hipLaunchKernelGGL(track_kernel_multi<CGB_PMX16S>, dim3(m.blocks), dim3(256), 0, st, args, m.cg, m.nch); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_encode(const DevArgs& a, const double* d, hipStream_t st) {
    CGB_DISPATCH(encode_kernel, site_grid(a), dim3(256), a, d);
    return hipGetLastError();
}
hipError_t launch_decode(const DevArgs& a, double* d, hipStream_t st) {
    CGB_DISPATCH(decode_kernel, site_grid(a), dim3(256), a, d);
    return hipGetLastError();
}
hipError_t launch_equilibrium_fill(const DevArgs& a, const double* rho, const double* u, hipStream_t st) {
    CGB_DISPATCH(equilibrium_kernel, site_grid(a), dim3(256), a, rho, u);
    return hipGetLastError();
}
hipError_t launch_decode_box(const DevArgs& a, const int* lo, const int* ext, double* d, int* own, hipStream_t st) {
    const long long nb = (long long)ext[0] * ext[1] * ext[2];
    const dim3 g((unsigned)((nb + 255) / 256)), b(256);
    CGB_DISPATCH(decode_box_kernel, g, b, a, lo[0], lo[1], lo[2], ext[0], ext[1], ext[2], d, own);
    return hipGetLastError();
}

hipError_t launch_mixture_box(const DevArgs& a, const int* lo, const int* ext, double* u, hipStream_t st) {
    const long long nb = (long long)ext[0] * ext[1] * ext[2];
    const dim3 g((unsigned)((nb + 255) / 256)), b(256);
    CGB_DISPATCH(mixture_box_kernel, g, b, a, lo[0], lo[1], lo[2], ext[0], ext[1], ext[2], u);
    return hipGetLastError();
}

hipError_t launch_fields(const DevArgs& a, double* rho, double* u, hipStream_t st) {
    CGB_DISPATCH(fields_kernel, site_grid(a), dim3(256), a, rho, u);
    return hipGetLastError();
}
hipError_t launch_observables(const DevArgs& a, double* partial, int nblk, hipStream_t st) {
    CGB_DISPATCH(observables_kernel, dim3(nblk), dim3(256), a, partial);
    return hipGetLastError();
}
hipError_t launch_profile_z(const DevArgs& a, double* prof, double* cnt, hipStream_t st, int axis) {
    CGB_DISPATCH(profile_kernel, site_grid(a), dim3(256), a, prof, cnt, axis);
    return hipGetLastError();
}

}  // namespace cgb
