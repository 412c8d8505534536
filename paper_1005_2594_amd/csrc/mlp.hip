// mlp.hip -- learned closure for the apparent viscosity: an ensemble of
// multilayer perceptrons 3 -> 64 -> 64 -> 1 with SiLU activations, trained on
// the device (mean-squared error, Adam) and evaluated on the device.
//
// Parameters of one member (FP32 master copy, 4481 values): W1 [64][3],
// b1 [64], W2 [64][64], b2 [64], W3 [64], b3.  The weights enter the
// arithmetic rounded to bfloat16 (round to nearest even); the 64 x 64 layer
// and its two backward products run on the matrix cores
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation), the 3-wide and 1-wide
// layers on the vector ALUs in FP32.
//
// Matrix-core tile (one wave, 16 x 16 x 32): lane l supplies A[l%16][k] and
// B[k][l%16] for the eight k = 8(l/16) + j, j = 0..7, and receives
// D[4(l/16)+r][l%16], r = 0..3.  (Which eight k a lane holds only has to be
// the same for A and B: the product sums over all of them.)
//
// Inputs are (hematocrit, log shear rate, width / R_perp); the network maps
// standardised inputs to the standardised log of the relative apparent
// viscosity; the handle keeps the standardisation.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/cgb.h"

namespace {

constexpr int H = 64;
constexpr int NIN = 3;
constexpr int OW1 = 0, OB1 = 192, OW2 = 256, OB2 = 4352, OW3 = 4416, OB3 = 4480, NP = 4481;
constexpr int TB = 128;  // training batch (8 tiles of 16 points)
constexpr int MAXM = 6;  // members (their staged weights share one workgroup's LDS in inference)

typedef short s8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ inline unsigned short to_bf16(float f) {
    const unsigned u = __float_as_uint(f);
    return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline float from_bf16(unsigned short h) { return __uint_as_float(((unsigned)h) << 16); }
__device__ inline float bfr(float f) { return from_bf16(to_bf16(f)); }
__device__ inline float silu(float z) { return z / (1.0f + __expf(-z)); }
__device__ inline float dsilu(float z) {
    const float s = 1.0f / (1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}
__device__ inline f4 mfma(s8 a, s8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(b8, a), __builtin_bit_cast(b8, b), c, 0, 0, 0);
}

struct Norm {
    float in_mean[NIN], in_std[NIN], out_mean, out_std;
};

// weights of one member staged in LDS: W1, b1, b2, W3 as bf16-rounded /
// plain floats, W2 as bf16 row-major
struct Stage {
    float w1[H * NIN], b1[H], b2[H], w3[H], b3;
    unsigned short w2[H * H];
};

__device__ void stage_member(Stage& S, const float* p, int tid, int nthr) {
    for (int i = tid; i < H * NIN; i += nthr) S.w1[i] = bfr(p[OW1 + i]);
    for (int i = tid; i < H; i += nthr) {
        S.b1[i] = p[OB1 + i];
        S.b2[i] = p[OB2 + i];
        S.w3[i] = bfr(p[OW3 + i]);
    }
    for (int i = tid; i < H * H; i += nthr) S.w2[i] = to_bf16(p[OW2 + i]);
    if (tid == 0) S.b3 = p[OB3];
}

// Forward pass of a 16-point tile on one wave.  x: the lane's point (l % 16),
// standardised.  Returns y for points 4(l/16) + r in all lanes of the group;
// optionally keeps h1 (A-operand layout), z2 (D layout) for the backward pass.
struct Fwd {
    s8 a[2];     // h1 as bf16, chunk kc: k = 32 kc + 8 (l/16) + j, point l%16
    f4 z2[4];    // pre-activation of layer 2, block ob: point 4(l/16)+r, o = 16 ob + l%16
    float y[4];  // outputs of points 4(l/16) + r
};

__device__ void forward_tile(const Stage& S, const float* x, int l, Fwd& F) {
#pragma unroll
    for (int kc = 0; kc < 2; kc++)
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const int k = 32 * kc + 8 * (l / 16) + j;
            const float z = S.w1[3 * k] * x[0] + S.w1[3 * k + 1] * x[1] + S.w1[3 * k + 2] * x[2] + S.b1[k];
            F.a[kc][j] = (short)to_bf16(silu(z));
        }
#pragma unroll
    for (int ob = 0; ob < 4; ob++) {
        f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kc = 0; kc < 2; kc++) {
            s8 b;
#pragma unroll
            for (int j = 0; j < 8; j++) b[j] = (short)S.w2[(16 * ob + l % 16) * H + 32 * kc + 8 * (l / 16) + j];
            acc = mfma(F.a[kc], b, acc);
        }
        const float bb = S.b2[16 * ob + l % 16];
#pragma unroll
        for (int r = 0; r < 4; r++) acc[r] += bb;
        F.z2[ob] = acc;
    }
#pragma unroll
    for (int r = 0; r < 4; r++) {
        float part = 0.f;
#pragma unroll
        for (int ob = 0; ob < 4; ob++) part += S.w3[16 * ob + l % 16] * silu(F.z2[ob][r]);
        // sum over the 16 lanes of the group (same points, the 16 outputs o)
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) part += __shfl_xor(part, off, 64);
        F.y[r] = part + S.b3;
    }
}

// ---------------------------------------------------------------- inference
// One wave per 16-point tile and member loop: mean and relative spread of the
// members' viscosities mu_m = exp(y_m sigma + mean) per point.
__global__ void __launch_bounds__(256) predict_kernel(const float* __restrict__ params, int members, Norm nm,
                                                      long long n, const float* __restrict__ xin,
                                                      float* __restrict__ mean, float* __restrict__ spread) {
    extern __shared__ unsigned char smem[];
    Stage* S = (Stage*)smem;
    const int tid = threadIdx.x;
    for (int m = 0; m < members; m++) stage_member(S[m], params + (size_t)m * NP, tid, blockDim.x);
    __syncthreads();
    const int l = tid & 63;
    const long long ntile = (n + 15) / 16;
    const long long wid = (long long)blockIdx.x * (blockDim.x / 64) + (tid >> 6);
    const long long nw = (long long)gridDim.x * (blockDim.x / 64);
    for (long long t = wid; t < ntile; t += nw) {
        const long long p = 16 * t + l % 16;
        float x[3];
#pragma unroll
        for (int i = 0; i < 3; i++) x[i] = p < n ? (xin[3 * p + i] - nm.in_mean[i]) / nm.in_std[i] : 0.f;
        float s1[4] = {0, 0, 0, 0}, s2[4] = {0, 0, 0, 0};
        for (int m = 0; m < members; m++) {
            Fwd F;
            forward_tile(S[m], x, l, F);
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const float mu = __expf(F.y[r] * nm.out_std + nm.out_mean);
                s1[r] += mu;
                s2[r] += mu * mu;
            }
        }
        if (l % 16 == 0) {
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const long long q = 16 * t + 4 * (l / 16) + r;
                if (q >= n) continue;
                const float mu = s1[r] / members;
                const float var = members > 1 ? fmaxf(s2[r] - members * mu * mu, 0.f) / (members - 1) : 0.f;
                mean[q] = mu;
                spread[q] = sqrtf(var) / mu;
            }
        }
    }
}

// raw network outputs y (standardised), for the parity tests: y[m][n]
__global__ void __launch_bounds__(256) forward_kernel(const float* __restrict__ params, long long n,
                                                      const float* __restrict__ xn, float* __restrict__ y) {
    __shared__ Stage S;
    const int m = blockIdx.y;
    stage_member(S, params + (size_t)m * NP, threadIdx.x, blockDim.x);
    __syncthreads();
    const int l = threadIdx.x & 63;
    const long long ntile = (n + 15) / 16;
    for (long long t = (long long)blockIdx.x * 4 + (threadIdx.x >> 6); t < ntile; t += (long long)gridDim.x * 4) {
        const long long p = 16 * t + l % 16;
        float x[3];
        for (int i = 0; i < 3; i++) x[i] = p < n ? xn[3 * p + i] : 0.f;
        Fwd F;
        forward_tile(S, x, l, F);
        if (l % 16 == 0)
            for (int r = 0; r < 4; r++) {
                const long long q = 16 * t + 4 * (l / 16) + r;
                if (q < n) y[(size_t)m * n + q] = F.y[r];
            }
    }
}

// ---------------------------------------------------------------- training
// One workgroup (4 waves) per member and step, batch of TB points (2 tiles
// per wave).  Backward: dy = 2 (y - t) / B; dW3 = dy . h2; dz2 = dy W3 silu'(z2);
// dW2 = dz2^T h1 and dh1 = dz2 W2 on the matrix cores; dz1 = dh1 silu'(z1);
// dW1 = dz1^T x.  mode 0: write the gradient and the loss; mode 1: Adam step.
// Every sum over the batch runs in a fixed order (over the 4 points of a lane,
// the 4 lane groups of a tile by shuffles, then the 8 tiles from LDS), so a
// step's result does not depend on scheduling.
constexpr int NTILE = TB / 16;

// sum over the 4 lane groups of a wave (points 4 g + r of a tile); every
// lane receives the same value
__device__ inline float group_sum(float v) {
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    return v;
}
struct Adam {
    float lr, b1, b2, eps, c1, c2;  // c1 = 1 - b1^t, c2 = 1 - b2^t
};

__device__ inline void adam_one(float* p, float* mm, float* vv, int i, float g, const Adam& A) {
    const float m = A.b1 * mm[i] + (1.f - A.b1) * g;
    const float v = A.b2 * vv[i] + (1.f - A.b2) * g * g;
    mm[i] = m;
    vv[i] = v;
    p[i] -= A.lr * (m / A.c1) / (sqrtf(v / A.c2) + A.eps);
}

__global__ void __launch_bounds__(256) train_kernel(float* __restrict__ params, float* __restrict__ am,
                                                    float* __restrict__ av, float* __restrict__ grad,
                                                    float* __restrict__ loss, int loss_stride, int loss_col,
                                                    const float* __restrict__ xn, const float* __restrict__ tn,
                                                    const int* __restrict__ idx, int idx_stride, int mode, Adam A) {
    __shared__ Stage S;
    __shared__ unsigned short H1[TB * H], DZ2[TB * H];
    __shared__ float xs[TB * NIN], ts[TB];
    // per-tile partial sums of the gradients of W1, b1, b2, W3, b3 and of the loss
    __shared__ float pw1[NTILE][H * NIN], pb1[NTILE][H], pb2[NTILE][H], pw3[NTILE][H], pb3[NTILE], ploss[NTILE];
    const int m = blockIdx.x;
    const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
    float* P = params + (size_t)m * NP;
    stage_member(S, P, tid, blockDim.x);
    for (int i = tid; i < TB; i += blockDim.x) {
        const int q = idx[(size_t)m * idx_stride + i];
        for (int c = 0; c < NIN; c++) xs[NIN * i + c] = xn[NIN * q + c];
        ts[i] = tn[q];
    }
    __syncthreads();

    // forward and the output-layer part of the backward pass
    for (int tt = 0; tt < 2; tt++) {
        const int tile = 2 * w + tt;
        const int pl = 16 * tile + l % 16;
        Fwd F;
        forward_tile(S, xs + NIN * pl, l, F);
#pragma unroll
        for (int kc = 0; kc < 2; kc++)
#pragma unroll
            for (int j = 0; j < 8; j++) H1[pl * H + 32 * kc + 8 * (l / 16) + j] = (unsigned short)F.a[kc][j];
        float dy[4], ls = 0.f, gd = 0.f;
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const float res = F.y[r] - ts[16 * tile + 4 * (l / 16) + r];
            dy[r] = 2.f * res / TB;
            ls += res * res;
            gd += dy[r];
        }
        ls = group_sum(ls);
        gd = group_sum(gd);
        if (l == 0) { ploss[tile] = ls; pb3[tile] = gd; }
#pragma unroll
        for (int ob = 0; ob < 4; ob++) {
            const int o = 16 * ob + l % 16;
            float g3 = 0.f, g2 = 0.f;
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const float z = F.z2[ob][r];
                g3 += dy[r] * silu(z);
                const float dz = dy[r] * S.w3[o] * dsilu(z);
                g2 += dz;
                DZ2[(16 * tile + 4 * (l / 16) + r) * H + o] = to_bf16(dz);
            }
            g3 = group_sum(g3);
            g2 = group_sum(g2);
            if (l < 16) { pw3[tile][o] = g3; pb2[tile][o] = g2; }
        }
    }
    __syncthreads();

    // dW2 = dz2^T h1: wave w computes output blocks (ob = w, kb = 0..3)
    {
        const int ob = w;
#pragma unroll
        for (int kb = 0; kb < 4; kb++) {
            f4 acc = {0.f, 0.f, 0.f, 0.f};
            for (int s = 0; s < TB / 32; s++) {
                s8 a, b;
#pragma unroll
                for (int j = 0; j < 8; j++) {
                    const int p = 32 * s + 8 * (l / 16) + j;
                    a[j] = (short)DZ2[p * H + 16 * ob + l % 16];
                    b[j] = (short)H1[p * H + 16 * kb + l % 16];
                }
                acc = mfma(a, b, acc);
            }
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int o = 16 * ob + 4 * (l / 16) + r, k = 16 * kb + l % 16;
                const int i = OW2 + o * H + k;
                if (mode == 0) grad[(size_t)m * NP + i] = acc[r];
                else adam_one(P, am + (size_t)m * NP, av + (size_t)m * NP, i, acc[r], A);
            }
        }
    }
    // dh1 = dz2 W2 for the wave's two tiles, then dz1 and the first layer
    for (int tt = 0; tt < 2; tt++) {
        const int tile = 2 * w + tt;
#pragma unroll
        for (int kb = 0; kb < 4; kb++) {
            f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < 2; s++) {
                s8 a, b;
#pragma unroll
                for (int j = 0; j < 8; j++) {
                    const int o = 32 * s + 8 * (l / 16) + j;
                    a[j] = (short)DZ2[(16 * tile + l % 16) * H + o];
                    b[j] = (short)S.w2[o * H + 16 * kb + l % 16];
                }
                acc = mfma(a, b, acc);
            }
            const int k = 16 * kb + l % 16;
            float g1[3] = {0.f, 0.f, 0.f}, gb = 0.f;
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int p = 16 * tile + 4 * (l / 16) + r;
                const float* x = xs + NIN * p;
                const float z = S.w1[3 * k] * x[0] + S.w1[3 * k + 1] * x[1] + S.w1[3 * k + 2] * x[2] + S.b1[k];
                const float dz = acc[r] * dsilu(z);
                gb += dz;
                g1[0] += dz * x[0]; g1[1] += dz * x[1]; g1[2] += dz * x[2];
            }
            gb = group_sum(gb);
            for (int c = 0; c < 3; c++) g1[c] = group_sum(g1[c]);
            if (l < 16) {
                pb1[tile][k] = gb;
                for (int c = 0; c < 3; c++) pw1[tile][3 * k + c] = g1[c];
            }
        }
    }
    __syncthreads();
    // the remaining parameters
    for (int i = tid; i < NP - H * H; i += blockDim.x) {
        int pi;
        float g = 0.f;
        if (i < H * NIN) { pi = OW1 + i; for (int t = 0; t < NTILE; t++) g += pw1[t][i]; }
        else if (i < H * NIN + H) { pi = OB1 + (i - H * NIN); for (int t = 0; t < NTILE; t++) g += pb1[t][i - H * NIN]; }
        else if (i < H * NIN + 2 * H) { pi = OB2 + (i - H * NIN - H); for (int t = 0; t < NTILE; t++) g += pb2[t][i - H * NIN - H]; }
        else if (i < H * NIN + 3 * H) { pi = OW3 + (i - H * NIN - 2 * H); for (int t = 0; t < NTILE; t++) g += pw3[t][i - H * NIN - 2 * H]; }
        else { pi = OB3; for (int t = 0; t < NTILE; t++) g += pb3[t]; }
        if (mode == 0) grad[(size_t)m * NP + pi] = g;
        else adam_one(P, am + (size_t)m * NP, av + (size_t)m * NP, pi, g, A);
    }
    if (tid == 0 && loss) {
        float ls = 0.f;
        for (int t = 0; t < NTILE; t++) ls += ploss[t];
        loss[(size_t)m * loss_stride + loss_col] = ls / TB;
    }
}

// standardise inputs and targets on the device: xn = (x - mean)/std,
// tn = (log mu - out_mean)/out_std
__global__ void standardise_kernel(Norm nm, int n, const float* x, const float* mu, float* xn, float* tn) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int c = 0; c < NIN; c++) xn[NIN * i + c] = (x[NIN * i + c] - nm.in_mean[c]) / nm.in_std[c];
    if (mu) tn[i] = (logf(mu[i]) - nm.out_mean) / nm.out_std;
}


// ---------------------------------------------------------------- allocation-free training
// Device staging of cgb_mlp_train_noalloc: raw inputs and targets, their
// standardised copies, the sample indices of every step and the per-step
// losses, at fixed offsets of one array.  Each device the library runs on
// holds its own copy until the process ends; every call on a device shares
// it, so calls that overlap on one device race.  Every section is written
// before it is read in a call, so nothing needs clearing between calls.
constexpr int NA_SAMPLES = 65536;  // samples per call
constexpr int NA_STEPS = 1024;     // Adam steps per call
constexpr size_t NA_X = 0;                                              // float [NA_SAMPLES][NIN]
constexpr size_t NA_MU = NA_X + (size_t)NA_SAMPLES * NIN * 4;           // float [NA_SAMPLES]
constexpr size_t NA_XN = NA_MU + (size_t)NA_SAMPLES * 4;                // float [NA_SAMPLES][NIN]
constexpr size_t NA_TN = NA_XN + (size_t)NA_SAMPLES * NIN * 4;          // float [NA_SAMPLES]
constexpr size_t NA_IDX = NA_TN + (size_t)NA_SAMPLES * 4;               // int [MAXM][NA_STEPS][TB]
constexpr size_t NA_LOSS = NA_IDX + (size_t)MAXM * NA_STEPS * TB * 4;   // float [MAXM][NA_STEPS]
constexpr size_t NA_BYTES = NA_LOSS + (size_t)MAXM * NA_STEPS * 4;
static_assert(NA_MU % 256 == 0 && NA_XN % 256 == 0 && NA_TN % 256 == 0 && NA_IDX % 256 == 0 && NA_LOSS % 256 == 0,
              "aligned sections");

}  // namespace

// In host code this name is a host-side stand-in, not a device address:
// kernels and copies take the address scratch_ptr() obtains per device.
static __device__ __align__(256) unsigned char scratch[NA_BYTES];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_dev[64] = {};  // device address of scratch, per device ordinal

// device address of scratch on the current device (looked up once per device)
hipError_t scratch_ptr(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

}  // namespace

struct cgb_mlp {
    int members = 0;
    void* scratch = nullptr;  // device address of the staging array on the handle's device
    float* params = nullptr;
    float* am = nullptr;
    float* av = nullptr;
    float* grad = nullptr;
    long long adam_t = 0;
    Norm nm{};
    hipStream_t st = nullptr;
    std::string err;
};

#define MFAIL(h, code, ...)                   \
    do {                                      \
        char _m[384];                         \
        snprintf(_m, sizeof _m, __VA_ARGS__); \
        (h)->err = _m;                        \
        return code;                          \
    } while (0)
#define MCHK(h, call)                                                                          \
    do {                                                                                       \
        hipError_t _e = (call);                                                                \
        if (_e != hipSuccess) MFAIL(h, CGB_EDEVICE, "%s: %s", #call, hipGetErrorString(_e));   \
    } while (0)

namespace {
// device scratch for one call, freed on every return path
struct DevBuf {
    void* p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
    hipError_t alloc(size_t b) { return hipMalloc(&p, b ? b : 8); }
    template <class T> T* as() const { return (T*)p; }
};
}  // namespace

extern "C" {

int cgb_mlp_create(int32_t members, cgb_mlp** out) {
    if (!out || members < 1 || members > MAXM) return CGB_EINVAL;
    *out = nullptr;
    cgb_mlp* h = new cgb_mlp();
    h->members = members;
    const size_t b = (size_t)members * NP * sizeof(float);
    if (hipStreamCreateWithFlags(&h->st, hipStreamNonBlocking) != hipSuccess || hipMalloc(&h->params, b) != hipSuccess ||
        hipMalloc(&h->am, b) != hipSuccess || hipMalloc(&h->av, b) != hipSuccess || hipMalloc(&h->grad, b) != hipSuccess) {
        cgb_mlp_destroy(h);
        return CGB_ENOMEM;
    }
    // the staging array of cgb_mlp_train_noalloc on this (the current) device
    if (scratch_ptr(&h->scratch) != hipSuccess) {
        cgb_mlp_destroy(h);
        return CGB_EDEVICE;
    }
    (void)hipMemsetAsync(h->params, 0, b, h->st);
    (void)hipMemsetAsync(h->am, 0, b, h->st);
    (void)hipMemsetAsync(h->av, 0, b, h->st);
    for (int c = 0; c < NIN; c++) { h->nm.in_mean[c] = 0.f; h->nm.in_std[c] = 1.f; }
    h->nm.out_mean = 0.f;
    h->nm.out_std = 1.f;
    if (hipStreamSynchronize(h->st) != hipSuccess) { cgb_mlp_destroy(h); return CGB_EDEVICE; }
    *out = h;
    return CGB_OK;
}

void cgb_mlp_destroy(cgb_mlp* h) {
    if (!h) return;
    if (h->st) (void)hipStreamSynchronize(h->st);
    for (float* p : {h->params, h->am, h->av, h->grad}) if (p) (void)hipFree(p);
    if (h->st) (void)hipStreamDestroy(h->st);
    delete h;
}

const char* cgb_mlp_last_error(const cgb_mlp* h) { return h ? h->err.c_str() : "null handle"; }

int cgb_mlp_set_params(cgb_mlp* h, const float* p) {
    if (!h || !p) return CGB_EINVAL;
    const size_t b = (size_t)h->members * NP * sizeof(float);
    MCHK(h, hipMemcpyAsync(h->params, p, b, hipMemcpyHostToDevice, h->st));
    MCHK(h, hipMemsetAsync(h->am, 0, b, h->st));
    MCHK(h, hipMemsetAsync(h->av, 0, b, h->st));
    MCHK(h, hipStreamSynchronize(h->st));
    h->adam_t = 0;
    return CGB_OK;
}

int cgb_mlp_get_params(cgb_mlp* h, float* p) {
    if (!h || !p) return CGB_EINVAL;
    MCHK(h, hipStreamSynchronize(h->st));
    MCHK(h, hipMemcpy(p, h->params, (size_t)h->members * NP * sizeof(float), hipMemcpyDeviceToHost));
    return CGB_OK;
}

int cgb_mlp_set_norm(cgb_mlp* h, const float* in_mean, const float* in_std, float out_mean, float out_std) {
    if (!h || !in_mean || !in_std || !(out_std > 0.f)) return CGB_EINVAL;
    for (int c = 0; c < NIN; c++) {
        if (!(in_std[c] > 0.f)) return CGB_EINVAL;
        h->nm.in_mean[c] = in_mean[c];
        h->nm.in_std[c] = in_std[c];
    }
    h->nm.out_mean = out_mean;
    h->nm.out_std = out_std;
    return CGB_OK;
}

int cgb_mlp_forward(cgb_mlp* h, int64_t n, const float* xn, float* y) {
    if (!h || n < 0 || (n > 0 && (!xn || !y))) return CGB_EINVAL;
    if (n == 0) return CGB_OK;
    DevBuf dx, dy;
    MCHK(h, dx.alloc((size_t)n * NIN * 4));
    MCHK(h, dy.alloc((size_t)n * h->members * 4));
    MCHK(h, hipMemcpyAsync(dx.p, xn, (size_t)n * NIN * 4, hipMemcpyHostToDevice, h->st));
    const long long nt = (n + 15) / 16;
    const unsigned gx = (unsigned)std::min<long long>((nt + 3) / 4, 4096);
    hipLaunchKernelGGL(forward_kernel, dim3(gx, h->members), dim3(256), 0, h->st, h->params, (long long)n,
                       dx.as<float>(), dy.as<float>());
    MCHK(h, hipGetLastError());
    MCHK(h, hipMemcpyAsync(y, dy.p, (size_t)n * h->members * 4, hipMemcpyDeviceToHost, h->st));
    MCHK(h, hipStreamSynchronize(h->st));
    return CGB_OK;
}

// `steps` training launches on device buffers: standardised inputs xn [n][3]
// and targets tn [n], indices [M][steps][TB], losses [M][steps]
static int train_steps(cgb_mlp* h, const float* xn, const float* tn, const int* idx, float* loss, int32_t steps,
                       float lr, int mode) {
    const int M = h->members;
    for (int s = 0; s < steps; s++) {
        Adam A{lr, 0.9f, 0.999f, 1e-8f, 0.f, 0.f};
        if (mode == 1) {
            h->adam_t++;
            A.c1 = (float)(1.0 - pow(0.9, (double)h->adam_t));
            A.c2 = (float)(1.0 - pow(0.999, (double)h->adam_t));
        }
        hipLaunchKernelGGL(train_kernel, dim3(M), dim3(256), 0, h->st, h->params, h->am, h->av, h->grad, loss, steps,
                           s, xn, tn, idx + (size_t)s * TB, steps * TB, mode, A);
        MCHK(h, hipGetLastError());
    }
    return CGB_OK;
}

static int run_train(cgb_mlp* h, int32_t n, const float* xn_h, const float* tn_h, int32_t steps, const int32_t* idx_h,
                     float lr, float* loss_h, int mode) {
    const int M = h->members;
    DevBuf dx, dt, di, dl;
    MCHK(h, dx.alloc((size_t)n * NIN * 4));
    MCHK(h, dt.alloc((size_t)n * 4));
    MCHK(h, di.alloc((size_t)M * steps * TB * 4));
    MCHK(h, dl.alloc((size_t)M * steps * 4));
    MCHK(h, hipMemcpyAsync(dx.p, xn_h, (size_t)n * NIN * 4, hipMemcpyHostToDevice, h->st));
    MCHK(h, hipMemcpyAsync(dt.p, tn_h, (size_t)n * 4, hipMemcpyHostToDevice, h->st));
    // idx_h: [M][steps][TB]; the kernel of step s reads member m's row at m * steps * TB + s * TB
    MCHK(h, hipMemcpyAsync(di.p, idx_h, (size_t)M * steps * TB * 4, hipMemcpyHostToDevice, h->st));
    int rc = train_steps(h, dx.as<float>(), dt.as<float>(), di.as<int>(), dl.as<float>(), steps, lr, mode);
    if (rc) return rc;
    if (loss_h) MCHK(h, hipMemcpyAsync(loss_h, dl.p, (size_t)M * steps * 4, hipMemcpyDeviceToHost, h->st));
    MCHK(h, hipStreamSynchronize(h->st));
    return CGB_OK;
}

static int check_idx(cgb_mlp* h, int32_t n, int32_t steps, const int32_t* idx) {
    const long long tot = (long long)h->members * steps * TB;
    for (long long i = 0; i < tot; i++)
        if (idx[i] < 0 || idx[i] >= n) MFAIL(h, CGB_EINVAL, "sample index %d out of range [0, %d)", idx[i], n);
    return CGB_OK;
}

int cgb_mlp_grad(cgb_mlp* h, int32_t n, const float* xn, const float* tn, const int32_t* idx, float* grad, float* loss) {
    if (!h || n < 1 || !xn || !tn || !idx || !grad) return CGB_EINVAL;
    int rc = check_idx(h, n, 1, idx);
    if (rc) return rc;
    rc = run_train(h, n, xn, tn, 1, idx, 0.f, loss, 0);
    if (rc) return rc;
    MCHK(h, hipMemcpy(grad, h->grad, (size_t)h->members * NP * 4, hipMemcpyDeviceToHost));
    return CGB_OK;
}

int cgb_mlp_train(cgb_mlp* h, int32_t n, const float* x, const float* mu, int32_t steps, const int32_t* idx, float lr,
                  float* loss) {
    if (!h || n < 1 || !x || !mu || steps < 1 || !idx || !(lr > 0.f)) return CGB_EINVAL;
    int rc = check_idx(h, n, steps, idx);
    if (rc) return rc;
    for (int i = 0; i < n; i++)
        if (!(mu[i] > 0.f)) MFAIL(h, CGB_EINVAL, "target %d is not positive", i);
    // standardise on the device, then train on the standardised copies
    DevBuf dx, dm, dxn, dtn;
    MCHK(h, dx.alloc((size_t)n * NIN * 4));
    MCHK(h, dm.alloc((size_t)n * 4));
    MCHK(h, dxn.alloc((size_t)n * NIN * 4));
    MCHK(h, dtn.alloc((size_t)n * 4));
    MCHK(h, hipMemcpyAsync(dx.p, x, (size_t)n * NIN * 4, hipMemcpyHostToDevice, h->st));
    MCHK(h, hipMemcpyAsync(dm.p, mu, (size_t)n * 4, hipMemcpyHostToDevice, h->st));
    hipLaunchKernelGGL(standardise_kernel, dim3((n + 255) / 256), dim3(256), 0, h->st, h->nm, n, dx.as<float>(),
                       dm.as<float>(), dxn.as<float>(), dtn.as<float>());
    MCHK(h, hipGetLastError());
    std::vector<float> xn((size_t)n * NIN), tn((size_t)n);
    MCHK(h, hipMemcpyAsync(xn.data(), dxn.p, xn.size() * 4, hipMemcpyDeviceToHost, h->st));
    MCHK(h, hipMemcpyAsync(tn.data(), dtn.p, tn.size() * 4, hipMemcpyDeviceToHost, h->st));
    MCHK(h, hipStreamSynchronize(h->st));
    return run_train(h, n, xn.data(), tn.data(), steps, idx, lr, loss, 1);
}

int cgb_mlp_train_noalloc(cgb_mlp* h, int32_t n, const float* x, const float* mu, int32_t steps, const int32_t* idx,
                          float lr, float* loss) {
    if (!h || n < 1 || !x || !mu || steps < 1 || !idx || !(lr > 0.f)) return CGB_EINVAL;
    if (n > NA_SAMPLES || steps > NA_STEPS)
        MFAIL(h, CGB_EINVAL, "%d samples / %d steps exceed the staging limits (%d samples, %d steps per call)", n, steps,
              NA_SAMPLES, NA_STEPS);
    int rc = check_idx(h, n, steps, idx);
    if (rc) return rc;
    for (int i = 0; i < n; i++)
        if (!(mu[i] > 0.f)) MFAIL(h, CGB_EINVAL, "target %d is not positive", i);
    if (!h->scratch) MFAIL(h, CGB_EDEVICE, "no staging array on this device");
    unsigned char* S = (unsigned char*)h->scratch;  // device address, never the host-side name
    float* dx = (float*)(S + NA_X);
    float* dmu = (float*)(S + NA_MU);
    float* dxn = (float*)(S + NA_XN);
    float* dtn = (float*)(S + NA_TN);
    int* di = (int*)(S + NA_IDX);
    float* dl = (float*)(S + NA_LOSS);
    const int M = h->members;
    MCHK(h, hipMemcpyAsync(dx, x, (size_t)n * NIN * 4, hipMemcpyHostToDevice, h->st));
    MCHK(h, hipMemcpyAsync(dmu, mu, (size_t)n * 4, hipMemcpyHostToDevice, h->st));
    // [M][steps][TB]: the kernel of step s reads member m's row at m * steps * TB + s * TB
    MCHK(h, hipMemcpyAsync(di, idx, (size_t)M * steps * TB * 4, hipMemcpyHostToDevice, h->st));
    hipLaunchKernelGGL(standardise_kernel, dim3((n + 255) / 256), dim3(256), 0, h->st, h->nm, n, dx, dmu, dxn, dtn);
    MCHK(h, hipGetLastError());
    rc = train_steps(h, dxn, dtn, di, dl, steps, lr, 1);
    if (rc) return rc;
    if (loss) MCHK(h, hipMemcpyAsync(loss, dl, (size_t)M * steps * 4, hipMemcpyDeviceToHost, h->st));
    MCHK(h, hipStreamSynchronize(h->st));
    return CGB_OK;
}

int cgb_mlp_predict_device(cgb_mlp* h, int64_t n, const float* x, float* mean, float* spread, void* stream) {
    if (!h || n < 0 || (n > 0 && (!x || !mean || !spread))) return CGB_EINVAL;
    if (n == 0) return CGB_OK;
    hipStream_t st = stream ? (hipStream_t)stream : h->st;
    const long long nt = (n + 15) / 16;
    const unsigned g = (unsigned)std::min<long long>((nt + 3) / 4, 2048);
    const size_t lds = sizeof(Stage) * h->members;
    hipLaunchKernelGGL(predict_kernel, dim3(g), dim3(256), lds, st, h->params, h->members, h->nm, (long long)n, x,
                       mean, spread);
    MCHK(h, hipGetLastError());
    return CGB_OK;
}

int cgb_mlp_predict(cgb_mlp* h, int64_t n, const float* x, float* mean, float* spread) {
    if (!h || n < 0 || (n > 0 && (!x || !mean || !spread))) return CGB_EINVAL;
    if (n == 0) return CGB_OK;
    DevBuf dx, dm, ds;
    MCHK(h, dx.alloc((size_t)n * NIN * 4));
    MCHK(h, dm.alloc((size_t)n * 4));
    MCHK(h, ds.alloc((size_t)n * 4));
    MCHK(h, hipMemcpyAsync(dx.p, x, (size_t)n * NIN * 4, hipMemcpyHostToDevice, h->st));
    int rc = cgb_mlp_predict_device(h, n, dx.as<float>(), dm.as<float>(), ds.as<float>(), nullptr);
    if (rc) return rc;
    MCHK(h, hipMemcpyAsync(mean, dm.p, (size_t)n * 4, hipMemcpyDeviceToHost, h->st));
    MCHK(h, hipMemcpyAsync(spread, ds.p, (size_t)n * 4, hipMemcpyDeviceToHost, h->st));
    MCHK(h, hipStreamSynchronize(h->st));
    return CGB_OK;
}

}  // extern "C"
