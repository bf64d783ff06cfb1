// Dense-path kernels for gfx950 (MI355X): staging, first iterate, diagonal
// pre-pass, the fused MFMA step (product W Delta^T + update of eq. (dyn)),
// export and residual check.
//
// Paper: Kenmoe, Smerlak, Zadorin, arXiv:2002.12872.  With W = A - I (zero
// diagonal) and C = A Delta' = Delta' + W Delta', one application of eq. (dyn) is
//   W'[n][m] = lambda (C[n][m] - C[n][n] W[n][m]) / (theta_n - theta_m),  m != n,
// and the eigenvalue readout of Sec. II.B is E_n = theta_n + lambda C[n][n].
#include <float.h>

#include <algorithm>

#include "device_common.h"
#include "dpt_internal.h"

namespace dpt {
namespace {

constexpr int kThreads = 256;

inline unsigned int grid_1d(int64_t work_items, int64_t cap = 1 << 20) {
    int64_t blocks = (work_items + kThreads - 1) / kThreads;
    if (blocks < 1) blocks = 1;
    if (blocks > cap) blocks = cap;
    return (unsigned int)blocks;
}

// ----------------------------------------------------------------- utilities
__global__ void k_zero_u64(unsigned long long *p, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

__global__ void k_fill_zero_u32(unsigned int *p, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// Up to kZeroMany buffers (word counts) cleared by one launch; blockIdx.y picks the buffer.
struct ZeroMany {
    unsigned int *p[kZeroMany];
    int64_t words[kZeroMany];
};

__global__ void k_zero_many(ZeroMany z) {
    unsigned int *p = z.p[blockIdx.y];
    const int64_t cnt = z.words[blockIdx.y];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__global__ void k_fill_zero_u32x4(uint4 *p, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

template <typename TD, typename TS>
__global__ void k_pad_copy(TD *__restrict__ dst, const TS *__restrict__ src, int64_t n, int64_t ld) {
    const int64_t total = ld * ld;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / ld, c = i - r * ld;
        dst[i] = (r < n && c < n) ? (TD)src[r * n + c] : (TD)0;
    }
}

template <typename TD, typename TS>
__global__ void k_load_state(TD *__restrict__ W, const TS *__restrict__ z0, int64_t n, int64_t ld) {
    const int64_t total = ld * ld;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / ld, c = i - r * ld;
        W[i] = (r < n && c < n && r != c) ? (TD)z0[r * n + c] : (TD)0;
    }
}

__global__ void k_cvt_f32_bf16(__bf16 *__restrict__ dst, const float *__restrict__ src, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (__bf16)src[i];
}

__global__ void k_cvt_f32_f64(double *__restrict__ dst, const float *__restrict__ src, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (double)src[i];
}

// 64x64 tiles through LDS: dst[i][j] = src[j][i].  grid = (ld/64, ld/64).
template <typename T>
__global__ __launch_bounds__(256) void k_transpose(const T *__restrict__ src, T *__restrict__ dst, int64_t ld) {
    __shared__ T tile[64][65];
    const int64_t bx = blockIdx.x, by = blockIdx.y;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4) tile[r][tx] = src[(by * 64 + r) * ld + bx * 64 + tx];
    __syncthreads();
    for (int r = ty; r < 64; r += 4) dst[(bx * 64 + r) * ld + by * 64 + tx] = tile[tx][r];
}

// Four consecutive values with 16-byte accesses (the address is a multiple of 4
// elements of a 16-byte aligned array).
__device__ __forceinline__ void load4v(const float *p, float v[4]) {
    const float4 x = *reinterpret_cast<const float4 *>(p);
    v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
}
__device__ __forceinline__ void load4v(const double *p, double v[4]) {
    const double2 x = reinterpret_cast<const double2 *>(p)[0], y = reinterpret_cast<const double2 *>(p)[1];
    v[0] = x.x; v[1] = x.y; v[2] = y.x; v[3] = y.y;
}
__device__ __forceinline__ void store4v(float *p, const float v[4]) {
    *reinterpret_cast<float4 *>(p) = make_float4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ void store4v(double *p, const double v[4]) {
    reinterpret_cast<double2 *>(p)[0] = make_double2(v[0], v[1]);
    reinterpret_cast<double2 *>(p)[1] = make_double2(v[2], v[3]);
}
__device__ __forceinline__ void store4_bf16(__bf16 *p, const float v[4]) {
    const __bf16 b4[4] = {(__bf16)v[0], (__bf16)v[1], (__bf16)v[2], (__bf16)v[3]};
    uint2 packed;
    __builtin_memcpy(&packed, b4, sizeof(packed));
    *reinterpret_cast<uint2 *>(p) = packed;
}

// Exact symmetry test on 64x64 tiles: block (bx, by) loads tile (by, bx) into
// LDS and compares it with the mirrored tile (bx, by); any difference sets
// *flag.  Thread t covers columns 4 (t & 15) .. +3 of rows (t >> 4) + 16 p.
// When bf is given, the block also writes the BF16 copy of the tile it loaded
// (every tile is loaded by exactly one block), so the copy costs no extra read.
template <typename T>
__global__ __launch_bounds__(256) void k_symmetry_check(const T *__restrict__ src, int64_t ld, unsigned int *flag,
                                                        __bf16 *__restrict__ bf) {
    __shared__ T tile[64][65];
    const int64_t bx = blockIdx.x, by = blockIdx.y;
    const int r0 = threadIdx.x >> 4, c4 = (threadIdx.x & 15) * 4;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = r0 + 16 * q;
        const int64_t g = (by * 64 + r) * ld + bx * 64 + c4;
        T v[4];
        load4v(src + g, v);
#pragma unroll
        for (int e = 0; e < 4; ++e) tile[r][c4 + e] = v[e];
        if (bf) {
            const float f[4] = {(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
            store4_bf16(bf + g, f);
        }
    }
    __syncthreads();
    bool diff = false;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        // src[bx*64 + r][by*64 + c] against its mirror src[by*64 + c][bx*64 + r]
        const int r = r0 + 16 * q;
        T u[4];
        load4v(src + (bx * 64 + r) * ld + by * 64 + c4, u);
#pragma unroll
        for (int e = 0; e < 4; ++e) diff |= !(u[e] == tile[c4 + e][r]);
    }
    if (__any(diff ? 1 : 0) && (threadIdx.x & 63) == 0) atomicOr(flag, 1u);
}

// ----------------------------------------------------------- first iterate
// F(I) = I + lambda gap * Delta'  (the Hadamard with the gap removes any diagonal).
//
// lambda d / (th_n - th_m) rounded to the state type, with the gap taken in
// FP64.  FP64 state: the correctly rounded quotient.  FP32 state: the FP64
// reciprocal of the gap from the hardware estimate and two Newton steps (each
// squares the relative error, so the product carries a few FP64 ulps), then
// one rounding to FP32; this differs from the rounded exact quotient only where
// the quotient lies within a few FP64 ulps of an FP32 rounding boundary, and
// costs a fraction of the FP64 division sequence, which bound the first
// iterate by arithmetic rather than by memory.
template <typename T>
__device__ __forceinline__ T gap_quotient(double lam_d, double th_n, double th_m) {
    const double g = th_n - th_m;
    if constexpr (sizeof(T) == 8) {
        return lam_d / g;
    } else {
        double r = __builtin_amdgcn_rcp(g);
        r = fma(r, fma(-g, r, 1.0), r);
        r = fma(r, fma(-g, r, 1.0), r);
        return (T)(lam_d * r);
    }
}

// Block (bx, by) covers columns [bx CW, bx CW + CW) of rows by R + q, (by + gy)
// R + q, ... (R = 1024 / CW rows per pass, q = thread / (CW / 4)); each thread
// holds theta of its 4 consecutive columns in registers for all its rows.  CW
// is 1024, or the padded order when that is smaller (ld is a multiple of 64);
// one statistics publish per block.
template <typename T>
__global__ __launch_bounds__(256) void k_first_iterate(StepArgs a, const T *__restrict__ dT, T *__restrict__ W,
                                                       __bf16 *__restrict__ Wb, int cw) {
    const int tpr = cw >> 2, rpb = 256 / tpr;
    const int64_t m0 = (int64_t)blockIdx.x * cw + 4 * (threadIdx.x % tpr);
    const int64_t nstride = (int64_t)gridDim.y * rpb;
    double th_m[4];
    bool col_ok[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        col_ok[q] = m0 + q < a.n;
        th_m[q] = m0 + q < a.ld ? a.theta[m0 + q] : 0.0;
    }
    T amax = (T)0;
    bool bad = false;
    if (m0 < a.ld) {
        for (int64_t n = (int64_t)blockIdx.y * rpb + threadIdx.x / tpr; n < a.ld; n += nstride) {
            const double th_n = a.theta[n];
            const bool row_ok = n < a.n;
            const int64_t idx = n * a.ld + m0;
            T d[4], w[4];
            load4v(dT + idx, d);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                w[q] = (T)0;
                if (row_ok && col_ok[q] && m0 + q != n) w[q] = gap_quotient<T>(a.lambda * (double)d[q], th_n, th_m[q]);
                const T v = w[q] < (T)0 ? -w[q] : w[q];
                amax = v > amax ? v : amax;
                bad |= !(v <= (sizeof(T) == 8 ? (T)DBL_MAX : (T)FLT_MAX));
            }
            store4v(W + idx, w);
            if (Wb) {
                const float f[4] = {(float)w[0], (float)w[1], (float)w[2], (float)w[3]};
                store4_bf16(Wb + idx, f);
            }
        }
    }
    publish_stats_block(a.stat, (double)amax, (double)amax, bad);
}

// ---------------------------------------------------------------- pre-pass
__device__ __forceinline__ void load4(const float *p, double out[4]) {
    const float4 v = *reinterpret_cast<const float4 *>(p);
    out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w;
}
__device__ __forceinline__ void load4(const double *p, double out[4]) {
    const double2 v0 = *reinterpret_cast<const double2 *>(p);
    const double2 v1 = *reinterpret_cast<const double2 *>(p + 2);
    out[0] = v0.x; out[1] = v0.y; out[2] = v1.x; out[3] = v1.y;
}

// One block per row n; fixed per-thread strides and a fixed butterfly make the
// FP64 sum deterministic.  Rows are ld-aligned and zero-padded, so the loop runs
// over the whole padded row with 4-wide loads.
// d_n = Delta[n][n] + sum_k W[n][k] Delta[n][k] in FP64 for row n with the whole
// block (fixed reduction order), E_n = theta_n + lambda d_n when E is given;
// the caller passes stat_clear to exactly one block, which clears the step's
// statistics.
template <typename TW, typename TD>
__device__ __forceinline__ void prepass_row(const TW *__restrict__ W, const TD *__restrict__ D, const StepArgs &a,
                                            double *__restrict__ d, double *__restrict__ E,
                                            unsigned long long *stat_clear, int64_t n) {
    const TW *w = W + n * a.ld;
    const TD *dl = D + n * a.ld;
    double s = 0.0;
    for (int64_t k = 4 * (int64_t)threadIdx.x; k < a.ld; k += 4 * 256) {
        double wv[4], dv[4];
        load4(w + k, wv);
        load4(dl + k, dv);
        s += wv[0] * dv[0] + wv[1] * dv[1] + wv[2] * dv[2] + wv[3] * dv[3];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double dn = (double)dl[n] + ((red[0] + red[1]) + (red[2] + red[3]));
        d[n] = dn;
        if (E) E[n] = a.theta[n] + a.lambda * dn;
        if (stat_clear) {
            stat_clear[0] = 0ull;
            stat_clear[1] = 0ull;
        }
    }
}

template <typename TW, typename TD>
__global__ __launch_bounds__(256) void k_prepass(const TW *__restrict__ W, const TD *__restrict__ D, StepArgs a,
                                                 double *__restrict__ d, double *__restrict__ E,
                                                 unsigned long long *stat_clear) {
    int64_t n = blockIdx.x;
    if (a.rowmap) {  // retired rows keep their d (not needed: they are not updated)
        n = a.rowmap[blockIdx.x];
        if (n < 0) return;
    }
    prepass_row(W, D, a, d, E, blockIdx.x == 0 ? stat_clear : nullptr, n);
}

// --------------------------------------------------------- fused MFMA step
// MFMA policies.  Operand fragments: lane l holds KPL consecutive K elements of
// row (l % MI) of its operand, from K-group (l / MI).  The accumulator layouts
// are those of the CDNA3/CDNA4 matrix instructions:
//   32x32 (16 values/lane): element r of lane l is C[(r&3) + 4*(l>>5) + 8*(r>>2)][l & 31]
//   16x16 f64 (4 values/lane): element r of lane l is C[4*r + (l>>4)][l & 15]
// Any permutation of K that is applied identically to both operands leaves the
// product unchanged; each lane's K-group therefore walks a contiguous span of
// the LDS row, which makes the LDS reads 16-byte vectors.
struct PolBF16 {
    using in_t = __bf16;
    using frag_t = bf16x8_t;
    using cvec_t = floatx16_t;
    static constexpr int MI = 32, KPL = 8, KGROUPS = 2, NACC = 16;
    static __device__ __forceinline__ cvec_t mma(frag_t x, frag_t y, cvec_t c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, y, c, 0, 0, 0);
    }
    // step s of a lane's K span held as 16-byte chunks
    static __device__ __forceinline__ frag_t frag(const u32x4_t *chunks, int s) {
        return __builtin_bit_cast(frag_t, chunks[s]);
    }
    static __device__ __forceinline__ int acc_row(int r, int lane) { return (r & 3) + ((lane >> 5) << 2) + ((r >> 2) << 3); }
    static __device__ __forceinline__ int acc_col(int lane) { return lane & 31; }
};

__device__ __forceinline__ unsigned int u32_of(const u32x4_t &c, int e) { return c[e]; }

struct PolF32 {
    using in_t = float;
    using frag_t = float;
    using cvec_t = floatx16_t;
    static constexpr int MI = 32, KPL = 1, KGROUPS = 2, NACC = 16;
    static __device__ __forceinline__ cvec_t mma(frag_t x, frag_t y, cvec_t c) {
        return __builtin_amdgcn_mfma_f32_32x32x2f32(x, y, c, 0, 0, 0);
    }
    static __device__ __forceinline__ frag_t frag(const u32x4_t *chunks, int s) {
        return __uint_as_float(u32_of(chunks[s >> 2], s & 3));
    }
    static __device__ __forceinline__ int acc_row(int r, int lane) { return (r & 3) + ((lane >> 5) << 2) + ((r >> 2) << 3); }
    static __device__ __forceinline__ int acc_col(int lane) { return lane & 31; }
};

struct PolF64 {
    using in_t = double;
    using frag_t = double;
    using cvec_t = doublex4_t;
    static constexpr int MI = 16, KPL = 1, KGROUPS = 4, NACC = 4;
    static __device__ __forceinline__ cvec_t mma(frag_t x, frag_t y, cvec_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0);
    }
    static __device__ __forceinline__ frag_t frag(const u32x4_t *chunks, int s) {
        const u32x4_t c = chunks[s >> 1];
        const unsigned long long lo = c[(s & 1) * 2], hi = c[(s & 1) * 2 + 1];
        return __longlong_as_double((long long)(lo | (hi << 32)));
    }
    // f64 16x16x4: one row per register group, i.e. register r of lane l is row 4r + (l >> 4)
    static __device__ __forceinline__ int acc_row(int r, int lane) { return (r << 2) + (lane >> 4); }
    static __device__ __forceinline__ int acc_col(int lane) { return lane & 15; }
};

// One output tile (tm, tn) of one fused step; called by the single-problem
// kernel below and by the grouped serving kernel (one tile per work item).
// PLAIN: the same product without the update, Wnew = A B^T (a plain NT GEMM of
// two ld x ld operands; deltaT and Wold are not read, no statistics).  EG: the
// elements of an accumulator block whose epilogue loads are issued together.
template <class P, int BM, int BN, int BK, int WM, int WN, typename S, bool PLAIN = false, int EG = 4>
__device__ __forceinline__ void step_tile(const typename P::in_t *__restrict__ A, const typename P::in_t *__restrict__ B,
                                          const S *__restrict__ deltaT, const S *__restrict__ Wold,
                                          S *__restrict__ Wnew, __bf16 *__restrict__ Wbnew, const StepArgs &a, int tm,
                                          int tn) {
    using in_t = typename P::in_t;
    constexpr int NT = WM * WN * 64;
    constexpr int VEC = 16 / (int)sizeof(in_t);  // elements per 16-byte chunk
    constexpr int LDK = BK + VEC;                // row pitch with 16 bytes of padding
    constexpr int WTM = BM / WM, WTN = BN / WN;  // wave tile
    constexpr int TM = WTM / P::MI, TN = WTN / P::MI;
    constexpr int KSPAN = BK / P::KGROUPS;       // K elements one lane reads per tile row
    constexpr int STEPS = KSPAN / P::KPL;        // MFMAs per block pair per K-tile
    constexpr int NV = KSPAN / VEC;
    constexpr int CPR = BK / VEC;                // 16-byte chunks per tile row
    constexpr int A_CH = BM * CPR / NT, B_CH = BN * CPR / NT;
    static_assert(WTM % P::MI == 0 && WTN % P::MI == 0, "wave tile");
    static_assert(KSPAN % VEC == 0 && KSPAN % P::KPL == 0, "K span");
    static_assert((BM * CPR) % NT == 0 && (BN * CPR) % NT == 0, "load split");

    __shared__ __attribute__((aligned(16))) in_t sA[2][BM * LDK];
    __shared__ __attribute__((aligned(16))) in_t sB[2][BN * LDK];

    const int64_t row0 = (int64_t)tm * BM, col0 = (int64_t)tn * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave / WN, wc = wave % WN;
    const int64_t ld = a.ld;
    const int ktiles = (int)(ld / BK);

    typename P::cvec_t acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < P::NACC; ++r) acc[i][j][r] = 0;

    // global -> register staging (16-byte chunks), double-buffered LDS; with a
    // row map, A row r of the tile is W row rowmap[row0 + r] (padding: row 0,
    // whose products are not stored)
    const in_t *gA = A + row0 * ld;
    const in_t *gB = B + col0 * ld;
    const in_t *pa[A_CH];
#pragma unroll
    for (int i = 0; i < A_CH; ++i) {
        const int c = tid + i * NT;
        int64_t r = row0 + c / CPR;
        if (a.rowmap) r = max(a.rowmap[r], 0);
        pa[i] = (a.rowmap ? A + r * ld : gA + (int64_t)(c / CPR) * ld) + (c % CPR) * VEC;
    }
    u32x4_t ra[A_CH], rb[B_CH];
#pragma unroll
    for (int i = 0; i < A_CH; ++i) ra[i] = *reinterpret_cast<const u32x4_t *>(pa[i]);
#pragma unroll
    for (int i = 0; i < B_CH; ++i) {
        const int c = tid + i * NT;
        rb[i] = *reinterpret_cast<const u32x4_t *>(gB + (int64_t)(c / CPR) * ld + (c % CPR) * VEC);
    }
#pragma unroll
    for (int i = 0; i < A_CH; ++i) {
        const int c = tid + i * NT;
        *reinterpret_cast<u32x4_t *>(&sA[0][(c / CPR) * LDK + (c % CPR) * VEC]) = ra[i];
    }
#pragma unroll
    for (int i = 0; i < B_CH; ++i) {
        const int c = tid + i * NT;
        *reinterpret_cast<u32x4_t *>(&sB[0][(c / CPR) * LDK + (c % CPR) * VEC]) = rb[i];
    }
    __syncthreads();

    const int grp = lane / P::MI, rr = lane % P::MI;
    const int a_off = (wr * WTM + rr) * LDK + grp * KSPAN;
    const int b_off = (wc * WTN + rr) * LDK + grp * KSPAN;
    for (int kt = 0; kt < ktiles; ++kt) {
        const int buf = kt & 1;
        const bool more = kt + 1 < ktiles;
        if (more) {
            const int64_t koff = (int64_t)(kt + 1) * BK;
#pragma unroll
            for (int i = 0; i < A_CH; ++i) ra[i] = *reinterpret_cast<const u32x4_t *>(pa[i] + koff);
#pragma unroll
            for (int i = 0; i < B_CH; ++i) {
                const int c = tid + i * NT;
                rb[i] = *reinterpret_cast<const u32x4_t *>(gB + (int64_t)(c / CPR) * ld + koff + (c % CPR) * VEC);
            }
        }
        u32x4_t fa[TM][NV], fb[TN][NV];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int v = 0; v < NV; ++v)
                fa[i][v] = *reinterpret_cast<const u32x4_t *>(&sA[buf][a_off + i * P::MI * LDK + v * VEC]);
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int v = 0; v < NV; ++v)
                fb[j][v] = *reinterpret_cast<const u32x4_t *>(&sB[buf][b_off + j * P::MI * LDK + v * VEC]);
#pragma unroll
        for (int s = 0; s < STEPS; ++s)
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) acc[i][j] = P::mma(P::frag(fa[i], s), P::frag(fb[j], s), acc[i][j]);
        if (more) {
#pragma unroll
            for (int i = 0; i < A_CH; ++i) {
                const int c = tid + i * NT;
                *reinterpret_cast<u32x4_t *>(&sA[buf ^ 1][(c / CPR) * LDK + (c % CPR) * VEC]) = ra[i];
            }
#pragma unroll
            for (int i = 0; i < B_CH; ++i) {
                const int c = tid + i * NT;
                *reinterpret_cast<u32x4_t *>(&sB[buf ^ 1][(c / CPR) * LDK + (c % CPR) * VEC]) = rb[i];
            }
        }
        __syncthreads();
    }

    if constexpr (PLAIN) {
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int64_t m = col0 + wc * WTN + j * P::MI + P::acc_col(lane);
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int r = 0; r < P::NACC; ++r)
                    Wnew[(row0 + wr * WTM + i * P::MI + P::acc_row(r, lane)) * ld + m] = (S)acc[i][j][r];
        }
        return;
    }
    // Epilogue: C = Delta^T (exact, state precision) + acc; update of eq. (dyn).
    // The quotient is formed for every element and selected (0 on the diagonal
    // and outside n, m < N).  Without a row map, the elements of an accumulator
    // block go in groups of EG: the loads of a group (Delta^T, W, theta_n, d_n)
    // are issued together, then its results computed and stored (each BF16
    // shadow value beside its FP32 one).  With a branch per element the loads
    // of an element waited for the stores of the one before (half of a 64 x 64
    // BF16 step at orders up to 1024).  The persistent grouped step takes groups
    // of 2: loading more at once takes registers from its four resident waves
    // per SIMD (a whole block of 16 raised its 64 x 64 form from 108 to 184).  For an FP32 state max|W'| and the finiteness test
    // run in FP32 (the same values: |W' - W| of two floats cannot overflow in
    // FP64, so it is infinite or NaN exactly when W' or W is).
    const S lam = (S)a.lambda;
    double dmax = 0.0;
    S wmax = (S)0;
    bool bad = false;
    auto update = [&](S c, S wo, double th_n, double th_m, S dn, bool ok) -> S {
        const S num = c - dn * wo;
        const S gap = (S)(th_n - th_m);
        const S q = lam * num / gap;
        const S w = ok ? q : (S)0;
        const double dv = fabs((double)w - (double)wo);
        dmax = fmax(dmax, dv);
        wmax = fmax(wmax, fabs(w));
        if constexpr (sizeof(S) == 4)
            bad |= !(fabsf(w) <= FLT_MAX) || !(fabsf(wo) <= FLT_MAX);
        else
            bad |= !(dv <= DBL_MAX) || !(fabs(w) <= DBL_MAX);
        return w;
    };
    if (a.rowmap) {  // per-row retirement: the listed rows only (-1: padding)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int64_t m = col0 + wc * WTN + j * P::MI + P::acc_col(lane);
            const double th_m = a.theta[m];
            const bool col_ok = m < a.n;
#pragma unroll
            for (int i = 0; i < TM; ++i) {
#pragma unroll
                for (int r = 0; r < P::NACC; ++r) {
                    const int64_t n = a.rowmap[row0 + wr * WTM + i * P::MI + P::acc_row(r, lane)];
                    if (n < 0) continue;
                    const int64_t idx = n * ld + m;
                    const S w = update((S)acc[i][j][r] + deltaT[idx], Wold[idx], a.theta[n], th_m, (S)a.d[n],
                                       n < a.n && col_ok && n != m);
                    Wnew[idx] = w;
                    if (Wbnew) Wbnew[idx] = (__bf16)(float)w;
                }
            }
        }
    } else {
        const bool shadow = Wbnew != nullptr;
        constexpr int EB = P::NACC < EG ? P::NACC : EG;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int64_t m = col0 + wc * WTN + j * P::MI + P::acc_col(lane);
            const double th_m = a.theta[m];
            const bool col_ok = m < a.n;
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const int64_t nb = row0 + wr * WTM + i * P::MI;
#pragma unroll
                for (int r0 = 0; r0 < P::NACC; r0 += EB) {
                    S dtv[EB], wov[EB];
                    double thv[EB], dv[EB];
#pragma unroll
                    for (int u = 0; u < EB; ++u) {
                        const int64_t n = nb + P::acc_row(r0 + u, lane), idx = n * ld + m;
                        dtv[u] = deltaT[idx];
                        wov[u] = Wold[idx];
                        thv[u] = a.theta[n];
                        dv[u] = a.d[n];
                    }
#pragma unroll
                    for (int u = 0; u < EB; ++u) {
                        const int64_t n = nb + P::acc_row(r0 + u, lane), idx = n * ld + m;
                        const S w = update((S)acc[i][j][r0 + u] + dtv[u], wov[u], thv[u], th_m, (S)dv[u],
                                           n < a.n && col_ok && n != m);
                        Wnew[idx] = w;
                        if (shadow) Wbnew[idx] = (__bf16)(float)w;
                    }
                }
            }
        }
    }
    publish_stats(a.stat, dmax, (double)wmax, bad);
}

template <class P, int BM, int BN, int BK, int WM, int WN, typename S>
__global__ __launch_bounds__(WM *WN * 64) void k_step_gemm(const typename P::in_t *__restrict__ A,
                                                           const typename P::in_t *__restrict__ B,
                                                           const S *__restrict__ deltaT, const S *__restrict__ Wold,
                                                           S *__restrict__ Wnew, __bf16 *__restrict__ Wbnew,
                                                           StepArgs a, int tiles_m, int tiles_n) {
    int tm, tn;
    tile_coords<8>(blockIdx.x, gridDim.x, tiles_m, tiles_n, tm, tn);
    step_tile<P, BM, BN, BK, WM, WN, S>(A, B, deltaT, Wold, Wnew, Wbnew, a, tm, tn);
}

// --------------------------------------------------- per-row retirement
// out[i] = max_m |Wn[r][m] - Wo[r][m]| of row r = rowmap[i] (one block per
// entry; -1 for padding entries).
template <typename T>
__global__ __launch_bounds__(256) void k_row_delta(const T *__restrict__ Wn, const T *__restrict__ Wo,
                                                   const int32_t *__restrict__ rowmap, int64_t ld,
                                                   double *__restrict__ out) {
    const int32_t r = rowmap[blockIdx.x];
    if (r < 0) {
        if (threadIdx.x == 0) out[blockIdx.x] = -1.0;
        return;
    }
    __shared__ double red[4];
    double m = 0.0;
    for (int64_t k = threadIdx.x; k < ld; k += 256) m = fmax(m, fabs((double)Wn[r * ld + k] - (double)Wo[r * ld + k]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// dst row rows[i] = src row rows[i] (one block per listed row).
template <typename T>
__global__ __launch_bounds__(256) void k_copy_rows(T *__restrict__ dst, const T *__restrict__ src,
                                                   const int32_t *__restrict__ rows, int64_t ld) {
    const int64_t r = rows[blockIdx.x];
    for (int64_t k = threadIdx.x; k < ld; k += 256) dst[r * ld + k] = src[r * ld + k];
}

// Plain NT product C = A B^T of ld x ld FP64 operands (basis changes of the
// homotopy continuation), on the tiles of the FP64 step.
template <int BM, int BN, int BK, int WM, int WN>
__global__ __launch_bounds__(WM *WN * 64) void k_gemm_nt_f64(const double *__restrict__ A,
                                                             const double *__restrict__ B, double *__restrict__ C,
                                                             StepArgs a, int tiles_m, int tiles_n) {
    int tm, tn;
    tile_coords<8>(blockIdx.x, gridDim.x, tiles_m, tiles_n, tm, tn);
    step_tile<PolF64, BM, BN, BK, WM, WN, double, true>(A, B, (const double *)nullptr, (const double *)nullptr, C,
                                                        (__bf16 *)nullptr, a, tm, tn);
}

// --------------------------------------------------- small problems (ld 64)
// One application of F to a 64 x 64 state held in LDS (row pitch PW elements),
// by the 4 waves of the block: the product and update of
// step_tile<P, 64, 64, 16, 2, 2, S> (wave grid 2 x 2, 32 x 32 wave tiles) with
// the same MFMAs on the same operands in the same order and the same
// per-element arithmetic, so the result is bitwise the same; the operands are
// read from LDS directly (no staging), each lane's epilogue loads are issued
// before its stores, and the quotient is formed for every element and
// selected (no branch per element).  FP64: 16x16x4 MFMAs, lane group g = lane / 16 holds K
// values 4g .. 4g + 3 of each K-tile of 16, MFMA s takes K = 4g + s.  FP32:
// 32x32x2 MFMAs, g = lane / 32 holds K values 8g .. 8g + 7, MFMA s takes
// K = 8g + s.  Wold, Dl, d, th and stat are in LDS; dT (pitch dtp) may be global.
template <typename S, int PW>
__device__ __forceinline__ void small_step_tile(const S *Wold, const S *Dl, const S *dT, int dtp, S *Wnew,
                                                const double *d, const double *th, int64_t N, double lambda,
                                                unsigned long long *stat) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, wr = wave >> 1, wc = wave & 1;
    const S lam = (S)lambda;
    double dmax = 0.0, wmax = 0.0;
    bool bad = false;
    if constexpr (sizeof(S) == 8) {
        const int grp = lane >> 4, rr = lane & 15;
        doublex4_t acc[2][2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[i][j][r] = 0.0;
        const S *a0 = Wold + (wr * 32 + rr) * PW, *b0 = Dl + (wc * 32 + rr) * PW;
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) {
#pragma unroll
            for (int v = 0; v < 2; ++v) {
                const int k = kt * 16 + grp * 4 + 2 * v;
                const double2 A0 = *reinterpret_cast<const double2 *>(a0 + k);
                const double2 A1 = *reinterpret_cast<const double2 *>(a0 + 16 * PW + k);
                const double2 B0 = *reinterpret_cast<const double2 *>(b0 + k);
                const double2 B1 = *reinterpret_cast<const double2 *>(b0 + 16 * PW + k);
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const double x0 = e ? A0.y : A0.x, x1 = e ? A1.y : A1.x;
                    const double y0 = e ? B0.y : B0.x, y1 = e ? B1.y : B1.x;
                    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, y0, acc[0][0], 0, 0, 0);
                    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, y1, acc[0][1], 0, 0, 0);
                    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, y0, acc[1][0], 0, 0, 0);
                    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, y1, acc[1][1], 0, 0, 0);
                }
            }
        }
        // register r of lane l in block (i, j): row 16 i + 4 r + (l >> 4), column 16 j + (l & 15)
        S dt[2][2][4], wo[2][2][4];
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int n = wr * 32 + 16 * i + 4 * r + (lane >> 4), m = wc * 32 + 16 * j + (lane & 15);
                    dt[i][j][r] = dT[n * dtp + m];
                    wo[i][j][r] = Wold[n * PW + m];
                }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int m = wc * 32 + 16 * j + (lane & 15);
            const double th_m = th[m];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int n = wr * 32 + 16 * i + 4 * r + (lane >> 4);
                    const S c = (S)acc[i][j][r] + dt[i][j][r];
                    const S o = wo[i][j][r];
                    const S num = c - (S)d[n] * o;
                    const S gap = (S)(th[n] - th_m);
                    const S q = lam * num / gap;
                    const S w = n < N && m < N && n != m ? q : (S)0;
                    Wnew[n * PW + m] = w;
                    const double dv = fabs((double)w - (double)o), av = fabs((double)w);
                    dmax = fmax(dmax, dv);
                    wmax = fmax(wmax, av);
                    bad |= !(dv <= DBL_MAX) || !(av <= DBL_MAX);
                }
        }
    } else {
        const int grp = lane >> 5, rr = lane & 31;
        floatx16_t acc;
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
        const S *a0 = Wold + (wr * 32 + rr) * PW, *b0 = Dl + (wc * 32 + rr) * PW;
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) {
#pragma unroll
            for (int v = 0; v < 2; ++v) {
                const int k = kt * 16 + grp * 8 + 4 * v;
                const float4 A = *reinterpret_cast<const float4 *>(a0 + k);
                const float4 B = *reinterpret_cast<const float4 *>(b0 + k);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(A.x, B.x, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(A.y, B.y, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(A.z, B.z, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(A.w, B.w, acc, 0, 0, 0);
            }
        }
        // register r of lane l: row (r & 3) + 4 (l >> 5) + 8 (r >> 2), column l & 31
        const int m = wc * 32 + (lane & 31);
        S dt[16], wo[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int n = wr * 32 + (r & 3) + ((lane >> 5) << 2) + ((r >> 2) << 3);
            dt[r] = dT[n * dtp + m];
            wo[r] = Wold[n * PW + m];
        }
        const double th_m = th[m];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int n = wr * 32 + (r & 3) + ((lane >> 5) << 2) + ((r >> 2) << 3);
            const S c = (S)acc[r] + dt[r];
            const S o = wo[r];
            const S num = c - (S)d[n] * o;
            const S gap = (S)(th[n] - th_m);
            const S q = lam * num / gap;
            const S w = n < N && m < N && n != m ? q : (S)0;
            Wnew[n * PW + m] = w;
            const double dv = fabs((double)w - (double)o), av = fabs((double)w);
            dmax = fmax(dmax, dv);
            wmax = fmax(wmax, av);
            bad |= !(dv <= DBL_MAX) || !(av <= DBL_MAX);
        }
    }
    publish_stats(stat, dmax, wmax, bad);
}

// Up to nsteps applications of F in one workgroup for ld = 64 (one 64x64 tile),
// bitwise equal to the separate first-iterate / pre-pass / step launches: the
// same per-element arithmetic and the same reduction order, with the 64 rows
// spread over the block (16 lanes per row, 4 columns per lane) instead of one
// block per row.  Delta (and Delta^T when it is not Delta itself, in FP32), theta,
// d, the step statistics and the two latest iterates stay in LDS for the whole
// batch (rows padded to PW elements against bank conflicts), so a step's
// operands never leave the CU; iterate s + 1 is also written to hist + s ld^2,
// d to the given array and the statistics to ring slot (k0 + s) mod kStatRing.
// The host picks the iterate its stopping rule ends on (the later ones are
// discarded); the batch ends early after a step whose delta is below stop_below
// or not finite, or whose max|W| exceeds blowup: the host's rule ends there or
// earlier.  The last iterate computed also replaces the state in Wcur (the host
// copies an earlier one from hist when its rule ends before).
template <typename S>
__global__ __launch_bounds__(256) void k_small_steps(S *__restrict__ Wcur, S *__restrict__ hist,
                                                     const S *__restrict__ D, const S *__restrict__ DT, StepArgs a,
                                                     unsigned long long *__restrict__ stats, int64_t k0, int nsteps,
                                                     int at_identity, double *__restrict__ d, double stop_below,
                                                     double blowup) {
    constexpr int LD = 64, PW = sizeof(S) == 8 ? 66 : 68, L2P = LD * PW;
    constexpr int VPC = 16 / (int)sizeof(S), CPR = LD / VPC;  // values per 16-byte chunk, chunks per row
    __shared__ __attribute__((aligned(16))) S sW[2][L2P];
    __shared__ __attribute__((aligned(16))) S sD[L2P];
    __shared__ __attribute__((aligned(16))) S sDT[(sizeof(S) == 4) ? L2P : 1];  // FP32 only (FP64: LDS budget)
    __shared__ double sTh[64], sd[64];
    __shared__ unsigned long long sStat[2];
    __shared__ int s_stop;
    const int t = threadIdx.x, c4 = 4 * (t & 15), r0 = t >> 4;
    const bool dt_is_d = DT == D;
    if (t < 64) sTh[t] = a.theta[t];
    for (int i = t; i < LD * CPR; i += 256) {
        const int row = i / CPR, col = (i % CPR) * VPC;
        *reinterpret_cast<u32x4_t *>(&sD[row * PW + col]) = *reinterpret_cast<const u32x4_t *>(&D[row * LD + col]);
        *reinterpret_cast<u32x4_t *>(&sW[0][row * PW + col]) =
            *reinterpret_cast<const u32x4_t *>(&Wcur[row * LD + col]);
        if (sizeof(S) == 4 && !dt_is_d)
            *reinterpret_cast<u32x4_t *>(&sDT[row * PW + col]) =
                *reinterpret_cast<const u32x4_t *>(&DT[row * LD + col]);
    }
    __syncthreads();
    // Delta^T for the epilogue and the first iterate: LDS, except an FP64
    // unsymmetric Delta^T, read from global memory (cached)
    const S *dT = dt_is_d ? (const S *)sD : (sizeof(S) == 4 ? (const S *)sDT : DT);
    const int dtp = (dt_is_d || sizeof(S) == 4) ? PW : LD;
    int done = 0;
    for (int s = 0; s < nsteps; ++s) {
        const S *Wold = sW[s & 1];
        S *Wnew = sW[(s + 1) & 1];
        if (t == 0) {
            sStat[0] = 0ull;
            sStat[1] = 0ull;
        }
        __syncthreads();
        if (s == 0 && at_identity) {
            // k_first_iterate: lane (row n, columns c4 .. c4 + 3)
            double dmax = 0.0;
            bool bad = false;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int n = r0 + 16 * q;
                const double th_n = sTh[n];
                const bool row_ok = n < a.n;
                S dv[4], w[4];
                load4v(dT + n * dtp + c4, dv);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int m = c4 + e;
                    w[e] = (S)0;
                    if (row_ok && m < a.n && m != n) w[e] = gap_quotient<S>(a.lambda * (double)dv[e], th_n, sTh[m]);
                    const double v = fabs((double)w[e]);
                    dmax = fmax(dmax, v);
                    bad |= !(v <= DBL_MAX);
                }
                store4v(Wnew + n * PW + c4, w);
            }
            publish_stats_block(sStat, dmax, dmax, bad);
        } else {
            // k_prepass: in a 64-wide block reduction only lanes 0..15 of wave 0
            // hold values for ld = 64; their xor-32 and xor-16 partners hold
            // zeros, so those two butterfly levels are additions of +0.0.  The
            // xor-8, 4, 2, 1 levels: lane 0 of each 16-lane row adds, at each
            // level, the same two partial sums as in the butterfly (up to the
            // order of the two operands of each addition, which is exact), here
            // by DPP rotations within the row instead of cross-lane shuffles
            // (≈ 2000 cycles per step less)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int n = r0 + 16 * q;
                double sum = 0.0;
                {
                    double wv[4], dv[4];
                    load4(Wold + n * PW + c4, wv);
                    load4(sD + n * PW + c4, dv);
                    sum += wv[0] * dv[0] + wv[1] * dv[1] + wv[2] * dv[2] + wv[3] * dv[3];
                }
                sum = sum + 0.0;
                sum = sum + 0.0;
                sum += dpp_f64<0x128>(sum, sum);  // rotate by 8 lanes
                sum += dpp_f64<0x124>(sum, sum);  // by 4
                sum += dpp_f64<0x122>(sum, sum);  // by 2
                sum += dpp_f64<0x121>(sum, sum);  // by 1
                if ((t & 15) == 0 && n < a.n) {
                    const double dn = (double)sD[n * PW + n] + ((sum + 0.0) + (0.0 + 0.0));
                    sd[n] = dn;
                    d[n] = dn;
                }
            }
            __syncthreads();  // d complete before the step reads it
            small_step_tile<S, PW>(Wold, sD, dT, dtp, Wnew, sd, sTh, a.n, a.lambda, sStat);
        }
        __syncthreads();  // iterate s + 1 and its statistics complete before they are stored and read
        S *out = hist + (int64_t)s * LD * LD;
        for (int i = t; i < LD * CPR; i += 256) {
            const int row = i / CPR, col = (i % CPR) * VPC;
            *reinterpret_cast<u32x4_t *>(&out[row * LD + col]) = *reinterpret_cast<const u32x4_t *>(&Wnew[row * PW + col]);
        }
        if (t == 0) {
            unsigned long long *slot = stats + 2 * ((k0 + s) % kStatRing);
            slot[0] = sStat[0];
            slot[1] = sStat[1];
            const double dl = __longlong_as_double((long long)sStat[0]);
            const double wm = __longlong_as_double((long long)sStat[1]);
            s_stop = !(dl <= DBL_MAX) || dl < stop_below || !(wm <= blowup);
        }
        __syncthreads();
        done = s + 1;
        if (s_stop) break;
    }
    const S *last = sW[done & 1];
    for (int i = t; i < LD * CPR; i += 256) {
        const int row = i / CPR, col = (i % CPR) * VPC;
        *reinterpret_cast<u32x4_t *>(&Wcur[row * LD + col]) = *reinterpret_cast<const u32x4_t *>(&last[row * PW + col]);
    }
}

// ------------------------------------------------------- grouped (serving)
// Largest j in [0, cnt) with prefix[j] <= item (prefix ascending, prefix[0] = 0).
__device__ __forceinline__ int find_segment(const int32_t *prefix, int cnt, int item) {
    int lo = 0, hi = cnt - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= item)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// sum_k w[k] dl[k] over a zero-padded row of ld (a multiple of 64) FP32 values,
// in FP64, by one wave: lane l takes the 16-byte chunks l, l + 64, ... (four
// products each, added in order), then a fixed butterfly.
__device__ __forceinline__ double group_row_dot(const float *w, const float *dl, int64_t ld, int lane) {
    const float4 *w4 = reinterpret_cast<const float4 *>(w);
    const float4 *d4 = reinterpret_cast<const float4 *>(dl);
    double sum = 0.0;
    for (int64_t k = lane; k < ld / 4; k += 64) {
        const float4 a = w4[k], b = d4[k];
        sum += (double)a.x * (double)b.x;
        sum += (double)a.y * (double)b.y;
        sum += (double)a.z * (double)b.z;
        sum += (double)a.w * (double)b.w;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o);
    return sum;
}

// One wave per (request, row): d_n = Delta[n][n] + sum_k W[n][k] Delta[n][k] in
// FP64 (group_row_dot); row 0 of every request clears its stats.
__global__ __launch_bounds__(256) void k_group_prepass(const GroupTable *__restrict__ t) {
    const int nreq = t->counts[0];
    const int total = nreq > 0 ? t->pre_prefix[nreq] : 0;
    const int lane = threadIdx.x & 63;
    const int nwaves = gridDim.x * 4;
    for (int item = blockIdx.x * 4 + (threadIdx.x >> 6); item < total; item += nwaves) {
        const int r = find_segment(t->pre_prefix, nreq, item);
        const GroupReq &q = t->reqs[r];
        const int64_t row = item - t->pre_prefix[r];
        const float *w = q.W + row * q.ld;
        const float *dl = q.D + row * q.ld;
        const double sum = group_row_dot(w, dl, q.ld, lane);
        if (lane == 0) {
            q.d[row] = (double)dl[row] + sum;
            if (row == 0) {
                q.stat[0] = 0ull;
                q.stat[1] = 0ull;
            }
        }
    }
}

// One output tile (shape SHAPE) of one request per work item; blocks stride
// over the items of every request in the list (persistent grid, fixed size).
template <int PHASE, int SHAPE>
__global__ __launch_bounds__(256) void k_group_step(const GroupTable *__restrict__ t) {
    constexpr int BM = group_shape_rows(SHAPE), BN = group_shape_cols(SHAPE);
    constexpr int L = kGroupShapes * (PHASE == PH_FP32 ? 1 : 0) + SHAPE;
    const int cnt = t->counts[1 + L];
    const int32_t *idx = t->idx[L];
    const int32_t *prefix = t->prefix[L];
    const int total = cnt > 0 ? prefix[cnt] : 0;
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int j = find_segment(prefix, cnt, item);
        const GroupReq &q = t->reqs[idx[j]];
        const int tpr = (int)(q.ld / BN);
        const int local = item - prefix[j];
        const int tm = local / tpr, tn = local - tm * tpr;
        StepArgs a;
        a.n = q.n;
        a.ld = q.ld;
        a.lambda = q.lambda;
        a.theta = q.theta;
        a.d = q.d;
        a.stat = q.stat;
        if (PHASE == PH_BF16)
            step_tile<PolBF16, BM, BN, 64, 2, 2, float, false, 2>(q.Wb, q.Db, q.DT, q.W, q.Wn, q.Wbn, a, tm, tn);
        else
            step_tile<PolF32, BM, BN, 32, 2, 2, float, false, 2>(q.W, q.D, q.DT, q.W, q.Wn, (__bf16 *)nullptr, a,
                                                                 tm, tn);
    }
}

// Admission: one 64 x 64 tile (bi, bj) of one request per work item.  Thread t
// owns column t & 63 and rows (t >> 6) + 4 k.  The source tile (rows bi, columns
// bj) goes to D and Db in place and through LDS (pitch 65: conflict-free both
// ways) to DT and the first iterate at tile (bj, bi): with state W = 0 the map
// gives W1[p][q] = lambda Delta[q][p] / (theta_p - theta_q), the same quotient
// as k_first_iterate.  Items of column tile 0 write the padded theta.
__global__ __launch_bounds__(256) void k_group_admit(const AdmitTable *__restrict__ t) {
    __shared__ float tile[64][65];
    const int nreq = t->count;
    const int total = nreq > 0 ? t->prefix[nreq] : 0;
    const int col = threadIdx.x & 63, r0 = threadIdx.x >> 6;
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int r = find_segment(t->prefix, nreq, item);
        const AdmitReq &q = t->reqs[r];
        const int64_t n = q.n, ld = q.ld;
        const int tpr = (int)(ld >> 6);
        const int local = item - t->prefix[r];
        const int bi = local / tpr, bj = local - bi * tpr;
        const int64_t j = (int64_t)bj * 64 + col;
        if (bj == 0 && r0 == 0 && q.theta != q.theta_src) {
            const int64_t k = (int64_t)bi * 64 + col;
            q.theta[k] = k < n ? q.theta_src[k] : 0.0;
        }
#pragma unroll 4
        for (int k = 0; k < 16; ++k) {
            const int rr = r0 + 4 * k;
            const int64_t i = (int64_t)bi * 64 + rr;
            float v = 0.0f;
            if (i < n && j < n)
                v = q.src_f64 ? (float)static_cast<const double *>(q.src)[i * n + j]
                              : static_cast<const float *>(q.src)[i * n + j];
            q.D[i * ld + j] = v;
            if (q.Db) q.Db[i * ld + j] = (__bf16)v;
            tile[rr][col] = v;
        }
        __syncthreads();
        // transposed tile: position (p, qc) with p = bj*64 + rr, qc = bi*64 + col
        const int64_t qc = (int64_t)bi * 64 + col;
        const double th_q = qc < n ? q.theta_src[qc] : 0.0;
        float amax = 0.0f;
        bool bad = false;
#pragma unroll 4
        for (int k = 0; k < 16; ++k) {
            const int rr = r0 + 4 * k;
            const int64_t p = (int64_t)bj * 64 + rr, idx = p * ld + qc;
            const float dt = tile[col][rr];
            if (q.DT) q.DT[idx] = dt;
            if (q.W1) {
                float w = 0.0f;
                if (p < n && qc < n && p != qc) w = gap_quotient<float>(q.lambda * (double)dt, q.theta_src[p], th_q);
                q.W1[idx] = w;
                if (q.Wb1) q.Wb1[idx] = (__bf16)w;
                const float a = fabsf(w);
                amax = a > amax ? a : amax;
                bad |= !(a <= FLT_MAX);
            }
        }
        if (q.W1) publish_stats_block(q.stat, (double)amax, (double)amax, bad);  // block-uniform
        __syncthreads();  // the tile is reused by the block's next item
    }
}

// Retirement: one wave per (request, row), the pre-pass sum of k_group_prepass
// (group_row_dot), then E_n = theta_n + lambda d_n; row 0 clears the request's
// stats.
__global__ __launch_bounds__(256) void k_group_retire(const RetireTable *__restrict__ t) {
    const int nreq = t->count;
    const int total = nreq > 0 ? t->prefix[nreq] : 0;
    const int lane = threadIdx.x & 63;
    const int nwaves = gridDim.x * 4;
    for (int item = blockIdx.x * 4 + (threadIdx.x >> 6); item < total; item += nwaves) {
        const int r = find_segment(t->prefix, nreq, item);
        const RetireReq &q = t->reqs[r];
        const int64_t row = item - t->prefix[r];
        const double sum = group_row_dot(q.W + row * q.ld, q.D + row * q.ld, q.ld, lane);
        if (lane == 0) {
            q.E[row] = q.theta[row] + q.lambda * ((double)q.D[row * q.ld + row] + sum);
            if (row == 0) {
                q.stat[0] = 0ull;
                q.stat[1] = 0ull;
            }
        }
    }
}

// ------------------------------------------------------------------ export
template <typename TW, typename TO>
__global__ void k_export(const TW *__restrict__ W, int64_t n, int64_t ld, TO *__restrict__ out) {
    const int64_t total = n * n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / n, c = i - r * n;
        out[i] = (r == c) ? (TO)1 : (TO)W[r * ld + c];
    }
}

// ---------------------------------------------------------------- residual
// grid = (nchunks, nrows); each wave computes (Delta z)[m] for rows m of the
// chunk, z = e_j + W[j][:], and accumulates |(M z)_m - E_j z_m|^2.
constexpr int kResChunk = 256;

template <typename TW, typename TD>
__global__ __launch_bounds__(256) void k_residual(const TW *__restrict__ W, const TD *__restrict__ D, StepArgs a,
                                                  const int64_t *__restrict__ rows, const double *__restrict__ E,
                                                  double *__restrict__ part) {
    const int64_t j = rows[blockIdx.y];
    const TW *wj = W + j * a.ld;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const double ej = E[j];
    double acc = 0.0;
    const int64_t m_begin = (int64_t)blockIdx.x * kResChunk;
    for (int64_t m = m_begin + wave; m < m_begin + kResChunk && m < a.n; m += 4) {
        const TD *dm = D + m * a.ld;
        double s = 0.0;
        for (int64_t l = lane; l < a.n; l += 64) {
            const double zl = (l == j) ? 1.0 : (double)wj[l];
            s += (double)dm[l] * zl;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
        const double zm = (m == j) ? 1.0 : (double)wj[m];
        const double rm = a.theta[m] * zm + a.lambda * s - ej * zm;
        acc += rm * rm;
    }
    __shared__ double red[4];
    if (lane == 0) red[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

template <class P, int BM, int BN, int BK, int WM, int WN, typename S>
hipError_t launch_gemm(const StepArgs &a, const typename P::in_t *A, const typename P::in_t *B, const S *deltaT,
                       const S *Wold, S *Wnew, __bf16 *Wbnew, hipStream_t s) {
    if (a.ld % BM || a.ld % BN || a.ld % BK) return hipErrorInvalidValue;
    if (a.rowmap && (a.rows % BM || a.rows < BM || a.rows > a.ld)) return hipErrorInvalidValue;
    const int tiles_m = (int)((a.rowmap ? a.rows : a.ld) / BM), tiles_n = (int)(a.ld / BN);
    const unsigned int blocks = (unsigned int)tiles_m * (unsigned int)tiles_n;
    hipLaunchKernelGGL((k_step_gemm<P, BM, BN, BK, WM, WN, S>), dim3(blocks), dim3(WM * WN * 64), 0, s, A, B,
                       deltaT, Wold, Wnew, Wbnew, a, tiles_m, tiles_n);
    return hipGetLastError();
}

}  // namespace

// ============================================================== launchers
hipError_t launch_zero_u64(unsigned long long *p, int64_t count, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_u64, dim3(grid_1d(count, 1024)), dim3(kThreads), 0, s, p, count);
    return hipGetLastError();
}

hipError_t launch_zero_many(void *const *ptrs, const size_t *bytes, int count, hipStream_t s) {
    if (count < 1 || count > kZeroMany) return hipErrorInvalidValue;
    ZeroMany z{};
    int64_t most = 1;
    for (int i = 0; i < count; ++i) {
        if (bytes[i] % 4) return hipErrorInvalidValue;
        z.p[i] = (unsigned int *)ptrs[i];
        z.words[i] = (int64_t)(bytes[i] / 4);
        most = std::max<int64_t>(most, z.words[i]);
    }
    hipLaunchKernelGGL(k_zero_many, dim3(grid_1d(most), (unsigned int)count), dim3(kThreads), 0, s, z);
    return hipGetLastError();
}

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s) {
    if (bytes % 4) return hipErrorInvalidValue;
    if (bytes % 16 == 0 && ((uintptr_t)p & 15) == 0) {
        const int64_t count = (int64_t)(bytes / 16);
        hipLaunchKernelGGL(k_fill_zero_u32x4, dim3(grid_1d(count)), dim3(kThreads), 0, s, (uint4 *)p, count);
        return hipGetLastError();
    }
    const int64_t count = (int64_t)(bytes / 4);
    hipLaunchKernelGGL(k_fill_zero_u32, dim3(grid_1d(count)), dim3(kThreads), 0, s, (unsigned int *)p, count);
    return hipGetLastError();
}

#define DPT_PAD_COPY(NAME, TD, TS)                                                                        \
    hipError_t NAME(TD *dst, const TS *src, int64_t n, int64_t ld, hipStream_t s) {                      \
        hipLaunchKernelGGL((k_pad_copy<TD, TS>), dim3(grid_1d(ld * ld)), dim3(kThreads), 0, s, dst, src, n, ld); \
        return hipGetLastError();                                                                         \
    }
DPT_PAD_COPY(launch_pad_copy_f32_from_f32, float, float)
DPT_PAD_COPY(launch_pad_copy_f32_from_f64, float, double)
DPT_PAD_COPY(launch_pad_copy_f64_from_f64, double, double)
DPT_PAD_COPY(launch_pad_copy_f64_from_f32, double, float)
#undef DPT_PAD_COPY

hipError_t launch_load_state_f32(float *W, const void *z0, int z0_is_f64, int64_t n, int64_t ld, hipStream_t s) {
    if (z0_is_f64)
        hipLaunchKernelGGL((k_load_state<float, double>), dim3(grid_1d(ld * ld)), dim3(kThreads), 0, s, W,
                           (const double *)z0, n, ld);
    else
        hipLaunchKernelGGL((k_load_state<float, float>), dim3(grid_1d(ld * ld)), dim3(kThreads), 0, s, W,
                           (const float *)z0, n, ld);
    return hipGetLastError();
}

hipError_t launch_load_state_f64(double *W, const void *z0, int z0_is_f64, int64_t n, int64_t ld, hipStream_t s) {
    if (z0_is_f64)
        hipLaunchKernelGGL((k_load_state<double, double>), dim3(grid_1d(ld * ld)), dim3(kThreads), 0, s, W,
                           (const double *)z0, n, ld);
    else
        hipLaunchKernelGGL((k_load_state<double, float>), dim3(grid_1d(ld * ld)), dim3(kThreads), 0, s, W,
                           (const float *)z0, n, ld);
    return hipGetLastError();
}

hipError_t launch_cvt_f32_to_bf16(__bf16 *dst, const float *src, int64_t count, hipStream_t s) {
    hipLaunchKernelGGL(k_cvt_f32_bf16, dim3(grid_1d(count)), dim3(kThreads), 0, s, dst, src, count);
    return hipGetLastError();
}

hipError_t launch_cvt_f32_to_f64(double *dst, const float *src, int64_t count, hipStream_t s) {
    hipLaunchKernelGGL(k_cvt_f32_f64, dim3(grid_1d(count)), dim3(kThreads), 0, s, dst, src, count);
    return hipGetLastError();
}

hipError_t launch_transpose_f32(float *dst, const float *src, int64_t ld, hipStream_t s) {
    if (ld % 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_transpose<float>), dim3(ld / 64, ld / 64), dim3(256), 0, s, src, dst, ld);
    return hipGetLastError();
}

hipError_t launch_transpose_f64(double *dst, const double *src, int64_t ld, hipStream_t s) {
    if (ld % 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_transpose<double>), dim3(ld / 64, ld / 64), dim3(256), 0, s, src, dst, ld);
    return hipGetLastError();
}

hipError_t launch_symmetry_check_f32(const float *src, int64_t ld, unsigned int *flag, __bf16 *bf, hipStream_t s) {
    if (ld % 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_symmetry_check<float>), dim3(ld / 64, ld / 64), dim3(256), 0, s, src, ld, flag, bf);
    return hipGetLastError();
}

hipError_t launch_symmetry_check_f64(const double *src, int64_t ld, unsigned int *flag, hipStream_t s) {
    if (ld % 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_symmetry_check<double>), dim3(ld / 64, ld / 64), dim3(256), 0, s, src, ld, flag,
                       (__bf16 *)nullptr);
    return hipGetLastError();
}

// One row per block up to 256 rows, then up to 16 rows per block, at most 1024
// blocks: enough loads in flight to stream at HBM rate with few statistics
// atomics (one publish per block).
// column chunk and grid of k_first_iterate: about 2048 blocks at large orders
// (ld is a multiple of 64, so its lowest set bit is a chunk width of at least 64)
inline int first_iterate_cw(int64_t ld) { return ld >= 1024 ? 1024 : (int)(ld & -ld); }
inline dim3 first_iterate_grid(int64_t ld, int cw) {
    const int64_t gx = (ld + cw - 1) / cw, rpb = 256 / (cw / 4);
    const int64_t gy = std::max<int64_t>(1, std::min<int64_t>((ld + rpb - 1) / rpb, 2048 / gx));
    return dim3((unsigned int)gx, (unsigned int)gy);
}

hipError_t launch_first_iterate_f32(const StepArgs &a, const float *deltaT, float *W, __bf16 *Wb, hipStream_t s) {
    const int cw = first_iterate_cw(a.ld);
    hipLaunchKernelGGL((k_first_iterate<float>), first_iterate_grid(a.ld, cw), dim3(256), 0, s, a, deltaT, W, Wb, cw);
    return hipGetLastError();
}

hipError_t launch_first_iterate_f64(const StepArgs &a, const double *deltaT, double *W, hipStream_t s) {
    const int cw = first_iterate_cw(a.ld);
    hipLaunchKernelGGL((k_first_iterate<double>), first_iterate_grid(a.ld, cw), dim3(256), 0, s, a, deltaT, W,
                       (__bf16 *)nullptr, cw);
    return hipGetLastError();
}

hipError_t launch_prepass_f32_f32(const float *W, const float *D, const StepArgs &a, double *d, double *E,
                                  unsigned long long *stat_clear, hipStream_t s) {
    hipLaunchKernelGGL((k_prepass<float, float>), dim3((unsigned int)(a.rowmap ? a.rows : a.n)), dim3(256), 0, s, W, D, a, d, E,
                       stat_clear);
    return hipGetLastError();
}

hipError_t launch_prepass_f32_f64(const float *W, const double *D, const StepArgs &a, double *d, double *E,
                                  unsigned long long *stat_clear, hipStream_t s) {
    hipLaunchKernelGGL((k_prepass<float, double>), dim3((unsigned int)(a.rowmap ? a.rows : a.n)), dim3(256), 0, s, W, D, a, d, E,
                       stat_clear);
    return hipGetLastError();
}

hipError_t launch_prepass_f64_f64(const double *W, const double *D, const StepArgs &a, double *d, double *E,
                                  unsigned long long *stat_clear, hipStream_t s) {
    hipLaunchKernelGGL((k_prepass<double, double>), dim3((unsigned int)(a.rowmap ? a.rows : a.n)), dim3(256), 0, s, W, D, a, d, E,
                       stat_clear);
    return hipGetLastError();
}

// A row-mapped step whose 128 x 128 tiles would not give each of the 256 CUs
// one (few rows still running): the 64 x 64 tiles give four times as many.
static bool few_row_tiles(const StepArgs &a) { return (a.rows / 128) * (a.ld / 128) < 256; }

// Whether a step uses the 256 x 256-tile kernels of kernels_gemm_large.hip
// ((ld / 256)^2 workgroups, one per CU at a time over 256 CUs).  Measured
// against the general 128 x 128 kernels on MI355X: the BF16 step is faster from
// ld 2048 on (3072: 2.1x; the general BF16 tiles reach 12-15 % of the BF16
// peak); the FP32 step is slower up to ld 3072, and above it wherever the last
// wave of tiles is mostly empty (6144, 7168: 10-13 % slower; 4096, 5120, 10240:
// as fast or faster), so FP32 takes it from ld 4096 when the waves of tiles are
// at least 78 % full on average.
static bool use_large_step(int64_t ld, bool bf16) {
    if (bf16) return step_large_supported(ld) && ld >= 2048;
    const int64_t tiles = (ld / 256) * (ld / 256), waves = (tiles + 255) / 256;
    return step_large_preferred(ld) && tiles * 100 >= 78 * 256 * waves;
}

// Tile configurations: large problems (ld a multiple of 256) use the big tiles,
// everything else the 64x64 tiles.
hipError_t launch_step_bf16(const StepArgs &a, const __bf16 *Wb, const __bf16 *Deltab, const float *deltaT,
                            const float *W, float *Wn, __bf16 *Wbn, hipStream_t s) {
    if (Wbn && use_large_step(a.ld, true)) return launch_step_bf16_large(a, Wb, Deltab, deltaT, W, Wn, Wbn, s);
    return launch_gemm<PolBF16, 64, 64, 64, 2, 2, float>(a, Wb, Deltab, deltaT, W, Wn, Wbn, s);
}

hipError_t launch_step_f32(const StepArgs &a, const float *W, const float *Delta, const float *deltaT, float *Wn,
                           __bf16 *Wbn, hipStream_t s) {
    // a row map runs on the general kernel's 128-row tiles (the large kernel's
    // direct-to-LDS loads assume contiguous tile rows), or its 64-row tiles when
    // 128-row ones would not give every CU a tile
    if (a.rowmap) {
        if (row_tile(a.ld) == 128 && !few_row_tiles(a))
            return launch_gemm<PolF32, 128, 128, 16, 2, 2, float>(a, W, Delta, deltaT, W, Wn, Wbn, s);
        return launch_gemm<PolF32, 64, 64, 16, 2, 2, float>(a, W, Delta, deltaT, W, Wn, Wbn, s);
    }
    if (!Wbn && use_large_step(a.ld, false)) return launch_step_f32_large(a, W, Delta, deltaT, Wn, s);
    if (a.ld % 256 == 0 && a.ld >= 1024)
        return launch_gemm<PolF32, 128, 128, 16, 2, 2, float>(a, W, Delta, deltaT, W, Wn, Wbn, s);
    return launch_gemm<PolF32, 64, 64, 16, 2, 2, float>(a, W, Delta, deltaT, W, Wn, Wbn, s);
}

// FP64: the large-tile kernel of kernels_gemm_f64.hip where it is preferred
// (from order 4096 on, a multiple of 128, and at 2048), with or without a row
// map; at orders from 4096 that are not multiples of 128 the general 128 x 128
// tiles of 8 waves (32 x 64 each, two waves per SIMD, K-tiles of 32: 139 ms per
// step at N = 16384 against 154 ms for 64 x 64 tiles), or their row-mapped form;
// below, 64 x 64 tiles (128-wide tiles leave CUs idle).
hipError_t launch_step_f64(const StepArgs &a, const double *W, const double *Delta, const double *deltaT, double *Wn,
                           hipStream_t s) {
    if (a.rowmap && few_row_tiles(a))  // the last running rows: 64-row tiles, four times as many workgroups
        return launch_gemm<PolF64, 64, 64, 16, 2, 2, double>(a, W, Delta, deltaT, W, Wn, (__bf16 *)nullptr, s);
    if (step_f64_large_preferred(a.ld)) return launch_step_f64_large(a, W, Delta, deltaT, Wn, s);
    if ((a.ld >= 4096 || a.rowmap) && row_tile(a.ld) == 128)
        return launch_gemm<PolF64, 128, 128, 32, 4, 2, double>(a, W, Delta, deltaT, W, Wn, (__bf16 *)nullptr, s);
    return launch_gemm<PolF64, 64, 64, 16, 2, 2, double>(a, W, Delta, deltaT, W, Wn, (__bf16 *)nullptr, s);
}

hipError_t launch_row_delta_f32(const float *Wn, const float *Wo, const int32_t *rowmap, int64_t rows, int64_t ld,
                                double *out, hipStream_t s) {
    if (rows < 1) return hipSuccess;
    hipLaunchKernelGGL((k_row_delta<float>), dim3((unsigned int)rows), dim3(256), 0, s, Wn, Wo, rowmap, ld, out);
    return hipGetLastError();
}

hipError_t launch_row_delta_f64(const double *Wn, const double *Wo, const int32_t *rowmap, int64_t rows, int64_t ld,
                                double *out, hipStream_t s) {
    if (rows < 1) return hipSuccess;
    hipLaunchKernelGGL((k_row_delta<double>), dim3((unsigned int)rows), dim3(256), 0, s, Wn, Wo, rowmap, ld, out);
    return hipGetLastError();
}

hipError_t launch_copy_rows_f32(float *dst, const float *src, const int32_t *rows, int64_t count, int64_t ld,
                                hipStream_t s) {
    if (count < 1) return hipSuccess;
    hipLaunchKernelGGL((k_copy_rows<float>), dim3((unsigned int)count), dim3(256), 0, s, dst, src, rows, ld);
    return hipGetLastError();
}

hipError_t launch_copy_rows_f64(double *dst, const double *src, const int32_t *rows, int64_t count, int64_t ld,
                                hipStream_t s) {
    if (count < 1) return hipSuccess;
    hipLaunchKernelGGL((k_copy_rows<double>), dim3((unsigned int)count), dim3(256), 0, s, dst, src, rows, ld);
    return hipGetLastError();
}

hipError_t launch_gemm_nt_f64(const double *A, const double *B, double *C, int64_t ld, hipStream_t s) {
    StepArgs a{};
    a.n = ld;
    a.ld = ld;
    if (ld >= 4096 && ld % 128 == 0) {
        const int t = (int)(ld / 128);
        hipLaunchKernelGGL((k_gemm_nt_f64<128, 128, 32, 4, 2>), dim3((unsigned int)(t * t)), dim3(512), 0, s, A, B, C,
                           a, t, t);
    } else {
        if (ld % 64) return hipErrorInvalidValue;
        const int t = (int)(ld / 64);
        hipLaunchKernelGGL((k_gemm_nt_f64<64, 64, 16, 2, 2>), dim3((unsigned int)(t * t)), dim3(256), 0, s, A, B, C, a,
                           t, t);
    }
    return hipGetLastError();
}

hipError_t launch_small_steps_f32(float *Wcur, float *hist, const float *D, const float *DT, const StepArgs &a,
                                  unsigned long long *stats, int64_t k0, int nsteps, int at_identity, double *d,
                                  double stop_below, double blowup, hipStream_t s) {
    if (a.ld != 64 || nsteps < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_small_steps<float>), dim3(1), dim3(256), 0, s, Wcur, hist, D, DT, a, stats, k0,
                       nsteps, at_identity, d, stop_below, blowup);
    return hipGetLastError();
}

hipError_t launch_small_steps_f64(double *Wcur, double *hist, const double *D, const double *DT,
                                  const StepArgs &a, unsigned long long *stats, int64_t k0, int nsteps,
                                  int at_identity, double *d, double stop_below, double blowup, hipStream_t s) {
    if (a.ld != 64 || nsteps < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_small_steps<double>), dim3(1), dim3(256), 0, s, Wcur, hist, D, DT, a, stats, k0,
                       nsteps, at_identity, d, stop_below, blowup);
    return hipGetLastError();
}

hipError_t launch_export_f32(const float *W, int64_t n, int64_t ld, void *out, int out_f64, hipStream_t s) {
    if (out_f64)
        hipLaunchKernelGGL((k_export<float, double>), dim3(grid_1d(n * n)), dim3(kThreads), 0, s, W, n, ld,
                           (double *)out);
    else
        hipLaunchKernelGGL((k_export<float, float>), dim3(grid_1d(n * n)), dim3(kThreads), 0, s, W, n, ld,
                           (float *)out);
    return hipGetLastError();
}

hipError_t launch_export_f64(const double *W, int64_t n, int64_t ld, void *out, int out_f64, hipStream_t s) {
    if (out_f64)
        hipLaunchKernelGGL((k_export<double, double>), dim3(grid_1d(n * n)), dim3(kThreads), 0, s, W, n, ld,
                           (double *)out);
    else
        hipLaunchKernelGGL((k_export<double, float>), dim3(grid_1d(n * n)), dim3(kThreads), 0, s, W, n, ld,
                           (float *)out);
    return hipGetLastError();
}

hipError_t launch_group_prepass(const GroupTable *t, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_group_prepass, dim3((unsigned int)grid), dim3(256), 0, s, t);
    return hipGetLastError();
}

hipError_t launch_group_step(const GroupTable *t, int phase, int shape, int grid, hipStream_t s) {
    const dim3 g((unsigned int)grid), b(256);
#define DPT_GROUP_STEP(PH, SH) hipLaunchKernelGGL((k_group_step<PH, SH>), g, b, 0, s, t)
    if (phase == PH_BF16 && shape == 0)
        DPT_GROUP_STEP(PH_BF16, 0);
    else if (phase == PH_BF16 && shape == 1)
        DPT_GROUP_STEP(PH_BF16, 1);
    else if (phase == PH_BF16 && shape == 2)
        DPT_GROUP_STEP(PH_BF16, 2);
    else if (phase == PH_FP32 && shape == 0)
        DPT_GROUP_STEP(PH_FP32, 0);
    else if (phase == PH_FP32 && shape == 1)
        DPT_GROUP_STEP(PH_FP32, 1);
    else if (phase == PH_FP32 && shape == 2)
        DPT_GROUP_STEP(PH_FP32, 2);
    else
        return hipErrorInvalidValue;
#undef DPT_GROUP_STEP
    return hipGetLastError();
}

hipError_t launch_group_admit(const AdmitTable *t, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_group_admit, dim3((unsigned int)grid), dim3(256), 0, s, t);
    return hipGetLastError();
}

hipError_t launch_group_retire(const RetireTable *t, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_group_retire, dim3((unsigned int)grid), dim3(256), 0, s, t);
    return hipGetLastError();
}

// Copy of a host-built work table (coherent pinned host memory, read through its
// device mapping) into its device copy, 8 bytes per thread.  As a kernel on the
// engine's own queue it is ordered with the kernels that read the table like
// any other launch; a host-to-device copy runs on a copy engine, and the first
// kernel after it started ≈ 15 us after the copy ended.
__global__ __launch_bounds__(256) void k_fetch_table(const unsigned long long *__restrict__ src,
                                                     unsigned long long *__restrict__ dst, int64_t words) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

hipError_t launch_fetch_table(const void *src, void *dst, size_t bytes, hipStream_t s) {
    if (bytes % 8 != 0) return hipErrorInvalidValue;
    const int64_t words = (int64_t)(bytes / 8);
    if (words == 0) return hipSuccess;
    const unsigned int blocks = (unsigned int)std::min<int64_t>((words + 255) / 256, 64);
    hipLaunchKernelGGL(k_fetch_table, dim3(blocks), dim3(256), 0, s, (const unsigned long long *)src,
                       (unsigned long long *)dst, words);
    return hipGetLastError();
}

int residual_chunks(int64_t ld) { return (int)((ld + kResChunk - 1) / kResChunk); }

hipError_t launch_residual_f32(const float *W, const void *D, int d_is_f64, const StepArgs &a, const int64_t *rows,
                               int64_t nrows, const double *E, double *part, hipStream_t s) {
    const dim3 grid(residual_chunks(a.ld), (unsigned int)nrows);
    if (d_is_f64)
        hipLaunchKernelGGL((k_residual<float, double>), grid, dim3(256), 0, s, W, (const double *)D, a, rows, E, part);
    else
        hipLaunchKernelGGL((k_residual<float, float>), grid, dim3(256), 0, s, W, (const float *)D, a, rows, E, part);
    return hipGetLastError();
}

hipError_t launch_residual_f64(const double *W, const void *D, int d_is_f64, const StepArgs &a, const int64_t *rows,
                               int64_t nrows, const double *E, double *part, hipStream_t s) {
    const dim3 grid(residual_chunks(a.ld), (unsigned int)nrows);
    if (d_is_f64)
        hipLaunchKernelGGL((k_residual<double, double>), grid, dim3(256), 0, s, W, (const double *)D, a, rows, E,
                           part);
    else
        hipLaunchKernelGGL((k_residual<double, float>), grid, dim3(256), 0, s, W, (const float *)D, a, rows, E, part);
    return hipGetLastError();
}

}  // namespace dpt
