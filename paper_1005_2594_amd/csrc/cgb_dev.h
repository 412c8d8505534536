// cgb_dev.h -- device-side definitions shared by the HIP kernels of libcgb.
//
// D3Q19 tables (Sec. II: 19 velocities, weights 1/3, 1/18, 1/36 by |c|, Eq. 6),
// storage codecs for the population deviations, and the argument block every
// kernel receives by value.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/cgb.h"

namespace cgb {

// velocity components, order: rest, +-x, +-y, +-z, then the face diagonals
// with opposites adjacent
__host__ __device__ constexpr int CX(int r) {
    constexpr int v[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    return v[r];
}
__host__ __device__ constexpr int CY(int r) {
    constexpr int v[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    return v[r];
}
__host__ __device__ constexpr int CZ(int r) {
    constexpr int v[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    return v[r];
}
__host__ __device__ constexpr int OPP(int r) { return r == 0 ? 0 : ((r & 1) ? r + 1 : r - 1); }
__host__ __device__ constexpr double WD(int r) { return r == 0 ? 1.0 / 3.0 : (r <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }

// node flag word: bit 31 = node is not fluid (cell or wall); bit 30 = wall
// node; bit r (1..18) = the pull source x - c_r of the node is not fluid
constexpr uint32_t NONFLUID = 0x80000000u;
constexpr uint32_t WALLNODE = 0x40000000u;
constexpr uint32_t LINKBITS = 0x0007FFFEu;
constexpr int32_t OWN_WALL = -2;
constexpr int32_t OWN_FLUID = -1;
constexpr int32_t NO_CAND = 0x7fffffff;

// status word bits
constexpr int ST_UNSTABLE = 1;
constexpr int ST_TRANS_OVERFLOW = 2;
constexpr int ST_PAIR_OVERFLOW = 4;
constexpr int ST_LIST_OVERFLOW = 8;
constexpr int ST_LE_SEAM = 16;  // a cell covers a node of a sheared plane of the viscometer

constexpr int TSEG = 64;  // segments of the transition list

struct DevArgs {
    // lattice
    int nx, ny, nz;
    long long ns;       // sites
    long long pstride;  // elements between direction planes
    int wall_y;
    int moving_walls;
    double wvb[3], wvt[3];
    double tau, rho0;
    int force_mode;
    double g[3];
    double f0;
    int fregion, fzlo, fzhi;  // force_mode 1 confined to fzlo <= z < fzhi (fregion = 1)
    int force_on_particles;
    // storage
    int precision;
    float pmx_scale, pmx_inv;  // PMX: stored = d / w * scale
    void* A;        // populations read this step  [19][pstride]
    void* B;        // populations written this step
    void* rhoA;     // density deviation field read (for Eq. 10)
    void* rhoB;     // density deviation field written
    int32_t* owner;
    uint32_t* flags;
    int32_t* cand;
    // particles
    int n;
    double* X;      // n*3
    double* q;      // n*4
    double* V;      // n*3
    double* L;      // n*3
    uint8_t* fixed;
    double* Xprev;  // n*3, position of the last rasterisation
    double* Hprev;  // n*3, axis-aligned half extents at the last rasterisation
    double* kin;    // n*12: X, V, Omega, axis at the start of the step
    float* kinf;    // n*12: rigid-body velocity about the nearest node b of X, in FP32:
                    // U0 = V + Omega x (b - X) (3), Omega (3), b packed (x | y << 16, z), X - b (3), 0
    double* FTh;    // n*6 hydrodynamic force, torque of the step
    double* FTp;    // n*6 potential force, torque
    unsigned long long* FTt;  // n*12 cover/uncover force and torque of the step in
                              // two-word fixed point (fx_add): order-independent sums
    unsigned* clist;  // [n][lcap] nodes each cell covers at this step's rasterisation,
                      // at the cell's record position (cell-list order)
    int* ccount;      // n: entries of each list (by record position)
    int lcap;         // list capacity (bound on the nodes inside one cell)
    double M, Ipar, Iperp;
    double Mdrive;   // mass the body force acts on: M, or rho0 times the cell volume
    double iRpar2, iRperp2, Rb;
    // transitions
    int* trans;     // 3 ints per transition: site, old, new
    int* ntrans;    // TSEG counters: the list is split into TSEG segments of trans_cap
    int trans_cap;  // entries each, so that reservations spread over TSEG addresses
    // cell list
    int nb[3];
    double bedge[3];
    int* pbin;      // n
    int* bin_count; // nbins
    int* bin_start; // nbins+1
    int* bin_fill;  // nbins
    int* bin_idx;   // n
    int* rank;      // n: position of each cell in the cell-list order (inverse of bin_idx)
    double* Xs;     // n*4 positions in cell-list order and the cell index
    int* wall_start;// nbins+1 (surface wall nodes per bin)
    int* wall_idx;  // site indices
    int nsw;        // number of surface wall nodes
    int nbins;
    double r_cut2;
    double wall_range2;
    double sig_perp, sig_par, sig_w, eps, eps_w;
    // bookkeeping
    int* status;
    int* bad_step;
    int* dstep;        // device-side index of the current step
    long long step;
    double* body_part; // per-block partial sums of the body force on cells
    // moving bounce-back and momentum exchange (element type: FP64 for P64,
    // FP32 otherwise)
    void* lmom;        // tau = 1: [4][pstride] link moments of each fluid node
                       // with links (sum w q, sum w c q; q = c . u(source))
    void* usol;        // tau != 1: [3][pstride]: velocity planes (x, y, z) of every non-fluid
                       // node: the rigid-body velocity of its cell at the node,
                       // or the wall velocity
    void* crec;        // [n] CellRec, in cell-list order (per-cell kernels)
    double* fnode;     // [ns][3] momentum the links of each cell node carried to
                       // its cell in the step (Eq. 12), written by the LB kernel
                       // (not allocated with the large-lattice layout, see big)
    // Large-lattice layout (lattices whose arrays pass 4 GB, or on request):
    // the LB kernel addresses memory with 64-bit lane addresses instead of
    // 32-bit buffer offsets, and a cell node's momentum is stored in the
    // node's own output population slots (dead at non-fluid nodes) instead of
    // fnode: slot k of the written populations holds bytes [k ES, (k+1) ES)
    // of the three doubles (ES: the storage element size)
    int big;
    const void* zero;
    // Indexed layout (sparse geometries such as vessel networks): the
    // populations, densities, link moments and node momenta are stored for
    // the non-wall nodes only, in lattice order; cidx[s] is the storage index
    // of site s (-1 at a wall).  Null: dense storage (index = site).
    const int32_t* cidx;  // 256 zeroed bytes: the source of a 64-bit-addressed load a lane skips
    // per-step record of the mixture velocity (apparent viscosity)
    double* track;      // [track_cap][2]: sums of u_z sin(2 pi y/ny) and of u_z
    int* track_n;       // steps recorded (keeps counting past track_cap)
    int track_cap;
    double* track_part; // per-block partial sums [track_slots][2]
    int track_slots;    // partials track_part holds
    double* ysin;       // [ny] sin(2 pi y / ny)
    // plane-Couette viscometer: Lees-Edwards seam of x (le_u = 0: off)
    double le_u;
    void* le_buf;       // [2][5][ny*nz] (compute precision) populations pulled across the
                        // seam: side 0 into x = 0 along c_x = +1, side 1 into x = nx-1 along c_x = -1
    double* le_part;    // per-block partial sums of Delta p_LE,z
    double* le_rec;     // [track_cap] Delta p_LE,z per recorded step (with the track record)
    int nt_out;        // 1: the populations outgrow the 256 MB last-level cache, where the next
                       // launch would find nothing of them cached anyway: the LB (dense and
                       // large-lattice layouts) and the split codec's link moments are launched
                       // in their forms with non-temporal output stores
    int tile[3];       // LB launch shape the kernels were configured for
    int* scan_tmp;     // block totals of the bin scan
    int nbody_blk;     // blocks of the integrate kernel (body_part has 3 per block)
};

// Block coordinates a kernel body works with.  A launch over one lattice
// passes the hardware's; a launch over every channel of a batch (one launch
// per kernel for all channels) passes each block its channel's share, found
// from the per-channel table of first blocks and grids (ChanGrid).
struct KCtx {
    unsigned bx, by, bz, gx, gy, gz;
};
__device__ __forceinline__ KCtx hw_ctx() {
    return KCtx{blockIdx.x, blockIdx.y, blockIdx.z, gridDim.x, gridDim.y, gridDim.z};
}
struct ChanGrid {
    unsigned start, gx, gy, gz;  // first block of the channel in the launch, its grid
    int arg;                     // a per-channel scalar of the kernel (the link-moment sweep depth)
    int pad[3];
};
// The channel of this block: the launch's table of nch entries is followed by
// one channel index per block of the launch (one load instead of a search).
__device__ __forceinline__ int chan_of(const ChanGrid* cg, int nch) {
    const int* blk = (const int*)(cg + nch);
    return __builtin_amdgcn_readfirstlane(blk[blockIdx.x]);
}
__device__ __forceinline__ KCtx chan_ctx(const ChanGrid& q) {
    const unsigned l = blockIdx.x - q.start;
    return KCtx{l % q.gx, (l / q.gx) % q.gy, l / (q.gx * q.gy), q.gx, q.gy, q.gz};
}

// A batch advanced by one launch per kernel for every channel: the step's
// kernels in the order one lattice's step launches them.
enum MultiKind {
    MK_PREP, MK_CLAIM, MK_RESOLVE, MK_TRANS, MK_LMOM, MK_LB, MK_MEM, MK_TRACK, MK_TRACK_FIN,
    MK_BIN_CLEAR, MK_BIN_COUNT, MK_SCAN_LOCAL, MK_SCAN_TOP, MK_SCAN_ADD, MK_BIN_FILL, MK_BIN_SORT,
    MK_SORTED_POS, MK_POT, MK_INT, MK_COUNT
};
// one launch: channels that share the kernel variant and block shape
struct MultiLaunch {
    int kind, variant;
    unsigned bx, by, blocks;
    int nch;
    const ChanGrid* cg;  // device table, nch entries sorted by first block
};

// storage index of site s (see cidx); -1 at a wall of the indexed layout
__device__ inline long long sidx(const DevArgs& a, long long s) { return a.cidx ? (long long)a.cidx[s] : s; }

__host__ __device__ inline int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// what the per-cell wave kernels need of a cell, gathered once per step in
// cell-list order (one 128-byte record per wave): position, axis, velocity,
// angular velocity, the cell's index and the node box to walk (the union of
// the boxes at the previous and the current rasterisation)
struct CellRec {
    double X[3], o[3], V[3], W[3];
    int p, ok, lo[3], ext[3];
};
static_assert(sizeof(CellRec) == 128, "cell record layout");

// ------------------------------------------------------------ buffer access
// Raw buffer loads/stores take one scalar resource and a 32-bit byte offset
// per lane (no 64-bit address registers); accesses past num_records read 0 and
// drop the store.
__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void* p, unsigned long long bytes) {
    const unsigned nrec = bytes >= 0xffffffffull ? 0xffffffffu : (unsigned)bytes;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)nrec, 0x00020000);
}
template <class T> __device__ inline T bload(__amdgpu_buffer_rsrc_t r, unsigned off);
template <> __device__ inline double bload<double>(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <> __device__ inline float bload<float>(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <> __device__ inline _Float16 bload<_Float16>(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0));
}
template <> __device__ inline uint16_t bload<uint16_t>(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
}
template <> __device__ inline int bload<int>(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return (int)__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
}
template <> __device__ inline uint32_t bload<uint32_t>(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
}
template <class T> __device__ inline void bstore(T v, __amdgpu_buffer_rsrc_t r, unsigned off);
template <> __device__ inline void bstore<double>(double v, __amdgpu_buffer_rsrc_t r, unsigned off) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0u, 0, 0)), v), r, off, 0, 0);
}
template <> __device__ inline void bstore<float>(float v, __amdgpu_buffer_rsrc_t r, unsigned off) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 0);
}
template <> __device__ inline void bstore<_Float16>(_Float16 v, __amdgpu_buffer_rsrc_t r, unsigned off) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, off, 0, 0);
}
template <> __device__ inline void bstore<uint16_t>(uint16_t v, __amdgpu_buffer_rsrc_t r, unsigned off) {
    __builtin_amdgcn_raw_buffer_store_b16(v, r, off, 0, 0);
}
// the same store with the non-temporal cache policy (NT, policy bit 1): for
// streamed output that no wave of the launch reads back, so that it does not
// take the L2 lines the launch's loads reuse
template <class T> __device__ inline void bstore_nt(T v, __amdgpu_buffer_rsrc_t r, unsigned off) {
    if constexpr (sizeof(T) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0u, 0, 0)), v), r, off, 0, 2);
    else if constexpr (sizeof(T) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 2);
    else
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, off, 0, 2);
}

// A cell node's momentum in its own output slots (large-lattice layout):
// slot k holds bytes [k ES, (k + 1) ES) of the three doubles (m0, m1, m2).
template <class T>
__device__ inline T mom_piece(const double* m, int k) {
    constexpr int ES = (int)sizeof(T), PER = 8 / ES;
    const unsigned long long b = __builtin_bit_cast(unsigned long long, m[k / PER]);
    if constexpr (ES == 8) return __builtin_bit_cast(T, b);
    else if constexpr (ES == 4) return __builtin_bit_cast(T, (unsigned)(b >> (32 * (k % PER))));
    else return __builtin_bit_cast(T, (unsigned short)(b >> (16 * (k % PER))));
}
// component c of the momentum of cell node s from the slots of the
// populations B (element size es bytes, direction planes ps elements apart)
__device__ inline double mom_from_slots(const void* B, int es, long long ps, unsigned s, int c) {
    unsigned long long b = 0;
    if (es == 8) {
        b = ((const unsigned long long*)B)[(size_t)c * ps + s];
    } else if (es == 4) {
        const unsigned* P = (const unsigned*)B;
        b = (unsigned long long)P[(size_t)(2 * c) * ps + s] | ((unsigned long long)P[(size_t)(2 * c + 1) * ps + s] << 32);
    } else {
        const unsigned short* P = (const unsigned short*)B;
#pragma unroll
        for (int k = 0; k < 4; k++) b |= (unsigned long long)P[(size_t)(4 * c + k) * ps + s] << (16 * k);
    }
    return __builtin_bit_cast(double, b);
}

// Workgroup b of a launch of nb runs on XCD b mod 8 (the device deals
// workgroups to its 8 XCDs in turn, and each XCD has its own L2).  The
// per-cell kernels walk the cells in cell-list order, so that neighbouring
// waves touch neighbouring lattice lines; this bijection of [0, nb) gives each
// XCD a contiguous range of that order, so that lines that neighbouring cells
// share are fetched into one L2 rather than several (at 256^3 it halves the
// fabric traffic of the momentum exchange and the rasterisation).
__device__ inline int xcd_block(int b, int nb) {
    const int x = b & 7, k = b >> 3, q = nb >> 3, r = nb & 7;
    return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// A launch over every channel of a batch, likewise: the block index goes
// through xcd_block before the channel table is read, so each XCD takes a
// contiguous run of each channel's tiles.  The LB tiles of the batch's
// narrow channels are 32 or 64 nodes wide, so every pull along x reads a
// line its neighbouring tile reads too; with neighbouring tiles on one XCD
// that line is fetched into one L2 (the 64-channel ensemble steps 4 % faster);
// the link-moment patches share their halo rows the same way.
// A lattice 256 nodes wide, swept in whole rows, shares lines only at
// bounced populations, and its launch keeps the hardware order (there the
// mapping costs 2 %).
__device__ __forceinline__ int chan_of_xcd(const ChanGrid* cg, int nch, unsigned* t) {
    *t = (unsigned)xcd_block((int)blockIdx.x, (int)gridDim.x);
    const int* blk = (const int*)(cg + nch);
    return __builtin_amdgcn_readfirstlane(blk[*t]);
}
__device__ __forceinline__ KCtx chan_ctx_at(const ChanGrid& q, unsigned t) {
    const unsigned l = t - q.start;
    return KCtx{l % q.gx, (l / q.gx) % q.gy, l / (q.gx * q.gy), q.gx, q.gy, q.gz};
}

// v in [-1, n + patch width - 1] reduced to [0, n)
__device__ inline int wrap_halo(int v, int n) {
    if (v < 0) v += n;
    if (v >= n) v -= n;
    if (v >= n) v %= n;  // lattices narrower than a patch
    return v;
}

// ------------------------------------------------------------ codecs
// P64 / P32: plain values.  PMX: d / w_r * scale stored in FP16 or BF16 with
// round-to-nearest-even; decode multiplies by w_r / scale.  PMX16S (split):
// the node's density deviation D is stored once (the density field) and each
// direction stores (d_r / w_r - D) * scale in FP16, so d_r = w_r (D + residual);
// every reader of a population also reads the density field of the node that
// wrote it.  The density field of every mode holds the density deviation of
// the stored populations (Eq. 7 minus rho0).
__device__ inline uint16_t f32_to_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);  // NaN stays NaN
    uint32_t rounding = 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)((u + rounding) >> 16);
}
__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

template <int P> struct Codec;
template <> struct Codec<CGB_P64> {
    using T = double;
    using R = double;
    static constexpr bool SPLIT = false;
    __device__ static R dec(T v, R) { return v; }
    __device__ static T enc(R v, R) { return v; }
};
template <> struct Codec<CGB_P32> {
    using T = float;
    using R = float;
    static constexpr bool SPLIT = false;
    __device__ static R dec(T v, R) { return v; }
    __device__ static T enc(R v, R) { return v; }
};
template <> struct Codec<CGB_PMX16> {
    using T = _Float16;
    using R = float;
    static constexpr bool SPLIT = false;
    __device__ static R dec(T v, R s) { return (float)v * s; }
    __device__ static T enc(R v, R s) {
        // the product rounded to FP32, then to FP16 (RNE), in every kernel.
        // Without the barrier the compiler may fuse the two into one
        // mixed-precision rounding (v_fma_mixlo_f16) in some kernel variants
        // and not in others, and halfway cases then round differently.
        float p = v * s;
        asm volatile("" : "+v"(p));
        return (_Float16)p;
    }
};
template <> struct Codec<CGB_PMXBF16> {
    using T = uint16_t;
    using R = float;
    static constexpr bool SPLIT = false;
    __device__ static R dec(T v, R s) { return bf16_to_f32(v) * s; }
    __device__ static T enc(R v, R s) { return f32_to_bf16_rne(v * s); }
};
template <> struct Codec<CGB_PMX16S> : Codec<CGB_PMX16> {
    static constexpr bool SPLIT = true;
};

template <int P> constexpr bool is_pmx() { return P == CGB_PMX16 || P == CGB_PMXBF16 || P == CGB_PMX16S; }

// per-direction decode / encode scales
template <int P>
__device__ inline typename Codec<P>::R dec_scale(const DevArgs& a, int r) {
    using R = typename Codec<P>::R;
    if constexpr (is_pmx<P>()) return (R)(WD(r) * (double)a.pmx_inv);
    else return (R)1;
}
template <int P>
__device__ inline typename Codec<P>::R enc_scale(const DevArgs& a, int r) {
    using R = typename Codec<P>::R;
    if constexpr (is_pmx<P>()) return (R)((double)a.pmx_scale / WD(r));
    else return (R)1;
}
template <int P>
__device__ inline typename Codec<P>::R rho_dec_scale(const DevArgs& a) {
    using R = typename Codec<P>::R;
    if constexpr (is_pmx<P>()) return (R)a.pmx_inv;
    else return (R)1;
}
template <int P>
__device__ inline typename Codec<P>::R rho_enc_scale(const DevArgs& a) {
    using R = typename Codec<P>::R;
    if constexpr (is_pmx<P>()) return (R)a.pmx_scale;
    else return (R)1;
}

// density deviation D of a stored density value
template <int P>
__device__ inline typename Codec<P>::R rho_dec(const DevArgs& a, typename Codec<P>::T v) {
    return Codec<P>::dec(v, rho_dec_scale<P>(a));
}
// deviation d_r of stored population v of direction r at a node whose stored
// density deviation is D (D is ignored unless the codec splits)
template <int P>
__device__ inline typename Codec<P>::R pop_dec(const DevArgs& a, typename Codec<P>::T v, int r, typename Codec<P>::R D) {
    using R = typename Codec<P>::R;
    if constexpr (Codec<P>::SPLIT) return (R)WD(r) * (Codec<P>::dec(v, (R)a.pmx_inv) + D);
    else return Codec<P>::dec(v, dec_scale<P>(a, r));
}
// stored value of deviation d of direction r at a node whose stored density
// deviation decodes to D
template <int P>
__device__ inline typename Codec<P>::T pop_enc(const DevArgs& a, typename Codec<P>::R d, int r, typename Codec<P>::R D) {
    using R = typename Codec<P>::R;
    if constexpr (Codec<P>::SPLIT) return Codec<P>::enc(d - (R)WD(r) * D, enc_scale<P>(a, r));
    else return Codec<P>::enc(d, enc_scale<P>(a, r));
}

// ------------------------------------------------------------ geometry
// Axis o = R(q) e_z and the inside test are evaluated without contraction so
// that node ownership is bit-identical to any reference that evaluates the
// same expressions in the same order.
__device__ inline void axis_of(const double* q, double* o) {
#pragma clang fp contract(off)
    o[0] = 2.0 * (q[1] * q[3] + q[0] * q[2]);
    o[1] = 2.0 * (q[2] * q[3] - q[0] * q[1]);
    o[2] = q[0] * q[0] - q[1] * q[1] - q[2] * q[2] + q[3] * q[3];
}

__device__ inline double min_image(double d, double L) {
    if (d >= 0.5 * L) d -= L;
    else if (d < -0.5 * L) d += L;
    return d;
}

// displacement node - X (minimum image on periodic axes)
__device__ inline void node_disp(const DevArgs& a, int x, int y, int z, const double* X, double* d) {
#pragma clang fp contract(off)
    d[0] = min_image((double)x - X[0], (double)a.nx);
    d[1] = a.wall_y ? ((double)y - X[1]) : min_image((double)y - X[1], (double)a.ny);
    d[2] = min_image((double)z - X[2], (double)a.nz);
}

__device__ inline bool inside_test(const DevArgs& a, const double* d, const double* o) {
#pragma clang fp contract(off)
    double dp = d[0] * o[0] + d[1] * o[1] + d[2] * o[2];
    double dd = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double val = dp * dp * a.iRpar2 + (dd - dp * dp) * a.iRperp2;
    return val < 1.0;
}

__device__ inline void body_force(const DevArgs& a, double y, double z, double* g) {
    g[0] = g[1] = g[2] = 0.0;
    if (a.force_mode == 1 && (!a.fregion || (z >= a.fzlo && z < a.fzhi))) { g[0] = a.g[0]; g[1] = a.g[1]; g[2] = a.g[2]; }
    else if (a.force_mode == 2) g[2] = a.f0 * sin(2.0 * M_PI * y / (double)a.ny);
}

__device__ inline void cross3(const double* a, const double* b, double* c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// Order-independent accumulation of doubles: v is split into hi = round(v 2^24)
// and lo = round((v - hi 2^-24) 2^76) (the remainder is exact, |lo| <= 2^51),
// and the two integers are added with 64-bit integer atomics, whose sums do
// not depend on the order of the additions.  fx_value returns
// sum(hi) 2^-24 + sum(lo) 2^-76: the exact sum of the v rounded to multiples
// of 2^-76, up to the last rounding of that expression.  Valid for |v| < 2^27
// and fewer than 2^11 terms per accumulator.
__device__ inline void fx_add(unsigned long long* acc, double v) {
    const long long hi = __double2ll_rn(v * 0x1p24);
    const double r = v - (double)hi * 0x1p-24;
    const long long lo = __double2ll_rn(r * 0x1p76);
    atomicAdd(acc, (unsigned long long)hi);
    atomicAdd(acc + 1, (unsigned long long)lo);
}
__device__ inline double fx_value(const unsigned long long* acc) {
    return (double)(long long)acc[0] * 0x1p-24 + (double)(long long)acc[1] * 0x1p-76;
}

// 64-lane sum of a double (all lanes receive the total)
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace cgb

// host-side launchers implemented in the kernel translation units
namespace cgb {
struct LaunchCfg {
    int bx, by;  // LB workgroup: threads along x and y
    int tz;      // nodes swept along z by each thread
};
hipError_t launch_lb(const DevArgs& a, LaunchCfg cfg, hipStream_t st);
// Per channel, the grid of kind's launch in a lattice's own step (the same
// work decomposition), its launch group (variant, block shape) and scalar
// argument; false when the channel's step does not launch it.
bool multi_grid(int kind, const DevArgs& a, LaunchCfg lb, int* variant, unsigned* bx, unsigned* by, dim3* grid,
                int* arg);
hipError_t launch_multi(const MultiLaunch& m, const DevArgs* args, hipStream_t st);
bool multi_grid_particles(int kind, const DevArgs& a, int* variant, unsigned* bx, unsigned* by, dim3* grid, int* arg);
hipError_t launch_multi_particles(const MultiLaunch& m, const DevArgs* args, hipStream_t st);
bool multi_grid_fields(int kind, const DevArgs& a, int* variant, unsigned* bx, unsigned* by, dim3* grid, int* arg);
hipError_t launch_multi_fields(const MultiLaunch& m, const DevArgs* args, hipStream_t st);
bool multi_grid_lb(const DevArgs& a, LaunchCfg lb, int* variant, unsigned* bx, unsigned* by, dim3* grid);
hipError_t launch_multi_lb(const MultiLaunch& m, const DevArgs* args, hipStream_t st);
hipError_t launch_mem_reduce(const DevArgs& a, hipStream_t st);
hipError_t launch_usol(const DevArgs& a, hipStream_t st, bool all);
hipError_t launch_lmom(const DevArgs& a, hipStream_t st);
hipError_t launch_prep(const DevArgs& a, hipStream_t st);
hipError_t launch_kin(const DevArgs& a, hipStream_t st);
hipError_t launch_clear_cells(const DevArgs& a, hipStream_t st);
hipError_t launch_raster(const DevArgs& a, hipStream_t st, bool fresh, bool records = true);
hipError_t launch_step_prep(const DevArgs& a, hipStream_t st);
hipError_t launch_cellrec(const DevArgs& a, hipStream_t st);
hipError_t launch_transitions(const DevArgs& a, hipStream_t st, bool bookkeeping);
hipError_t launch_cells(const DevArgs& a, hipStream_t st);
hipError_t launch_potentials(const DevArgs& a, hipStream_t st);
hipError_t launch_integrate(const DevArgs& a, hipStream_t st);
hipError_t launch_flags_rebuild(const DevArgs& a, hipStream_t st);
hipError_t launch_fill_i32(int* p, long long n, int v, hipStream_t st);
hipError_t launch_fill_f64(double* p, long long n, double v, hipStream_t st);
hipError_t launch_encode(const DevArgs& a, const double* d, hipStream_t st);
hipError_t launch_decode(const DevArgs& a, double* d, hipStream_t st);
hipError_t launch_equilibrium_fill(const DevArgs& a, const double* rho, const double* u, hipStream_t st);
hipError_t launch_fields(const DevArgs& a, double* rho, double* u, hipStream_t st);
hipError_t launch_decode_box(const DevArgs& a, const int* lo, const int* ext, double* d, int* own, hipStream_t st);
hipError_t launch_mixture_box(const DevArgs& a, const int* lo, const int* ext, double* u, hipStream_t st);
hipError_t launch_observables(const DevArgs& a, double* partial, int nblk, hipStream_t st);
hipError_t launch_profile_z(const DevArgs& a, double* prof, double* cnt, hipStream_t st, int axis);
hipError_t launch_le(const DevArgs& a, hipStream_t st);
constexpr int LE_BLOCK = 256;
static inline int le_blocks(const DevArgs& a) { return (2 * a.ny * a.nz + LE_BLOCK - 1) / LE_BLOCK; }
constexpr int TRACK_BLOCKS = 1024;
// blocks of a lattice's mixture record: one per 4096 sites, at most TRACK_BLOCKS
__host__ __device__ inline int track_blocks(long long ns) {
    const long long b = (ns + 4095) / 4096;
    return b < 1 ? 1 : (b > TRACK_BLOCKS ? TRACK_BLOCKS : (int)b);
}
// blocks of the lattice's LB launch (its tile)
__host__ __device__ inline long long lb_blocks(const DevArgs& a) {
    if (a.tile[0] < 1 || a.tile[1] < 0 || a.tile[2] < 1) return 1LL << 62;
    const long long nz = (a.nz + a.tile[2] - 1) / a.tile[2];
    if (a.tile[1] == 0)  // plane-linear: bx consecutive sites of the x-y plane per block
        return ((long long)a.nx * a.ny + a.tile[0] - 1) / a.tile[0] * nz;
    return (long long)((a.nx + a.tile[0] - 1) / a.tile[0]) * ((a.ny + a.tile[1] - 1) / a.tile[1]) * nz;
}
// the tau = 1 LB kernel sums the mixture record itself, one partial per
// block, when its blocks' partials fit; otherwise a pass of its own does
__host__ __device__ inline bool track_in_lb(const DevArgs& a) {
    return a.track && a.tau == 1.0 && lb_blocks(a) <= a.track_slots;
}
hipError_t launch_track(const DevArgs& a, hipStream_t st);
hipError_t launch_pairs(const DevArgs& a, int* out, int* count, int cap, hipStream_t st);
}  // namespace cgb
