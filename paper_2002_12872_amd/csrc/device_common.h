// Device helpers shared by the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dpt {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float floatx16_t;
typedef __attribute__((__vector_size__(4 * sizeof(double)))) double doublex4_t;
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));

constexpr unsigned long long kNanBits = 0x7ff8000000000000ull;

__device__ __forceinline__ unsigned long long dbits(double x) { return (unsigned long long)__double_as_longlong(x); }

// x of another lane by a DPP lane move (both 32-bit halves with the same
// control): lanes that the row mask leaves out, or whose source lane does not
// exist, get `old`.  CTRL: 0x00-0xff quad permutation, 0x121-0x12f rotation
// right by 1-15 lanes within a row of 16, 0x140 row mirror, 0x141 half-row
// mirror, 0x142 / 0x143 broadcast of lane 15 / 31 of a row to the next rows.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_f64(double x, double old) {
    const long long xb = __double_as_longlong(x), ob = __double_as_longlong(old);
    const int lo = __builtin_amdgcn_update_dpp((int)ob, (int)xb, CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(ob >> 32), (int)(xb >> 32), CTRL, ROW_MASK, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Max over the 64 lanes of a wave of values that are never NaN, in every lane.
// DPP moves within quads, half-rows and rows, then the row ends broadcast
// forward (lane 63 ends with the maximum), instead of six dependent
// cross-lane shuffles through the LDS crossbar (≈ 2000 cycles for two values
// in the small-problem kernel).  Max is exact in any order.
__device__ __forceinline__ double wave_max(double x) {
    x = fmax(x, dpp_f64<0xb1>(x, x));       // lanes 1 0 3 2 of each quad
    x = fmax(x, dpp_f64<0x4e>(x, x));       // lanes 2 3 0 1 of each quad
    x = fmax(x, dpp_f64<0x141>(x, x));      // half-row mirror
    x = fmax(x, dpp_f64<0x140>(x, x));      // row mirror: every lane holds its row's max
    x = fmax(x, dpp_f64<0x142, 0xa>(x, x));  // rows 1, 3 take lane 15 / 47
    x = fmax(x, dpp_f64<0x143, 0xc>(x, x));  // rows 2, 3 take lane 31
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)b, 63), hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Wave-wide max of (delta, |w|) plus a non-finite flag; lane 0 of every wave
// publishes with one atomicMax per value (max is order-independent, so the
// result is deterministic).  delta and |w| are non-negative and never NaN
// (they come from fmax, which drops NaN operands; NaNs set `bad`).  The
// current value is read first (device scope, past the non-coherent L1) and the
// atomic skipped when it cannot raise it: the slot only grows during a launch,
// so a skipped update is never lost, and kernels with 10^5-10^6 waves do not
// serialise on two addresses.  Must be reached by all 64 lanes of the wave.
__device__ __forceinline__ void publish_stats(unsigned long long *stat, double dmax, double wmax, bool bad) {
    dmax = wave_max(dmax);
    wmax = wave_max(wmax);
    const bool any_bad = __any(bad ? 1 : 0);
    if ((threadIdx.x & 63) == 0) {
        const unsigned long long vd = any_bad ? kNanBits : dbits(dmax), vw = any_bad ? kNanBits : dbits(wmax);
        if (vd > __hip_atomic_load(stat, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(stat, vd);
        if (vw > __hip_atomic_load(stat + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(stat + 1, vw);
    }
}

// Block-wide form of publish_stats: the waves' maxima meet in LDS and one lane
// publishes for the whole block, so a launch issues at most two atomics per
// block.  Device-scope atomics on one address serialise (tens of ns each), so
// per-wave publishing from thousands of waves costs tens of microseconds.
// Every thread of the block must call it (it contains a barrier); blockDim.x is
// a multiple of 64 and at most 1024.
__device__ __forceinline__ void publish_stats_block(unsigned long long *stat, double dmax, double wmax, bool bad) {
    __shared__ double s_d[16], s_w[16];
    __shared__ int s_b[16];
    dmax = wave_max(dmax);
    wmax = wave_max(wmax);
    const bool any_bad = __any(bad ? 1 : 0);
    const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_d[wave] = dmax;
        s_w[wave] = wmax;
        s_b[wave] = any_bad ? 1 : 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double d = s_d[0], w = s_w[0];
        int b = s_b[0];
        for (int i = 1; i < nwaves; ++i) {
            d = fmax(d, s_d[i]);
            w = fmax(w, s_w[i]);
            b |= s_b[i];
        }
        const unsigned long long vd = b ? kNanBits : dbits(d), vw = b ? kNanBits : dbits(w);
        if (vd > __hip_atomic_load(stat, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(stat, vd);
        if (vw > __hip_atomic_load(stat + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(stat + 1, vw);
    }
    __syncthreads();  // the arrays may be reused by the block's next publish
}

// Block -> output tile.  Workgroups are dispatched round-robin over the 8 XCDs
// (bid % 8), so first make each XCD's blocks a contiguous range of logical tile
// ids, then walk the tiles in groups of G tile-rows so that the blocks resident
// on one XCD share operand panels in that XCD's L2.
template <int G>
__device__ __forceinline__ void tile_coords(int bid, int nblocks, int tiles_m, int tiles_n, int &tm, int &tn) {
    int t = bid;
    if ((nblocks & 7) == 0) t = (bid & 7) * (nblocks >> 3) + (bid >> 3);
    const int group_size = G * tiles_n;
    const int group = t / group_size;
    const int first = group * G;
    const int gm = min(tiles_m - first, G);
    const int within = t - group * group_size;
    tm = first + within % gm;
    tn = within / gm;
}

}  // namespace dpt
