// Fused BF16 D-PT step for large problems on gfx950 (ld a multiple of 256).
//
// One application of eq. (dyn) of Kenmoe, Smerlak, Zadorin (arXiv:2002.12872)
// on the padded state W = A - I:
//     C  = Delta^T + bf16(W) bf16(Delta)^T                    (MFMA, FP32 accumulate)
//     W' = lambda (C - d_n W) / (theta_n - theta_m),  m != n  (FP32 epilogue, FP64 gaps)
// plus max|W' - W| and max|W'| for the stopping rule.
//
// Tiling: 256 x 256 output tile per workgroup of 8 waves (2 per SIMD), each wave
// 128 x 64 = 4 x 2 blocks of v_mfma_f32_32x32x16_bf16.  K advances 32 at a time
// through a 4-stage LDS ring that the waves fill with direct global->LDS loads
// (global_load_lds_dwordx4: no staging registers), so up to three K-tiles are
// in flight while one is multiplied.  Each 64-byte tile row holds four 16-byte
// chunks stored at slot c ^ ((row >> 1) & 3): the eight rows read by eight
// consecutive lanes of a fragment load then fall on eight different bank groups.
#include <float.h>

#include "device_common.h"
#include "dpt_internal.h"

namespace dpt {
namespace {

constexpr int BM = 256, BN = 256, BK = 32, STAGES = 4;
constexpr int WM = 2, WN = 4, NT = WM * WN * 64;   // 512 threads
constexpr int WTM = BM / WM, WTN = BN / WN;        // 128 x 64 per wave
constexpr int TM = WTM / 32, TN = WTN / 32;        // 4 x 2 MFMA blocks
constexpr int ROW_BYTES = BK * 2;                  // one tile row of one stage
constexpr int STAGE_BYTES = (BM + BN) * ROW_BYTES; // A tile then B tile
constexpr int LOADS_PER_STAGE = 4;                 // per thread: 2 for A, 2 for B

typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) const void gbl_void;

// Byte offset of logical 16-byte chunk c (0..3) of tile row r inside one operand tile.
__device__ __forceinline__ int swz(int r, int c) { return r * ROW_BYTES + ((c ^ ((r >> 1) & 3)) << 4); }

template <int N>
__device__ __forceinline__ void wait_vmcnt() {
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// Workgroup barrier without an implicit wait on outstanding vector-memory
// operations (the prefetched stages must stay in flight); the memory clobber
// keeps the compiler from moving LDS accesses across it.
__device__ __forceinline__ void barrier_keep_loads() { asm volatile("s_barrier" ::: "memory"); }

__global__ __launch_bounds__(NT) void k_step_bf16_v2(const __bf16 *__restrict__ A, const __bf16 *__restrict__ B,
                                                     const float *__restrict__ deltaT, const float *__restrict__ Wold,
                                                     float *__restrict__ Wnew, __bf16 *__restrict__ Wbnew, StepArgs a,
                                                     int tiles_m, int tiles_n) {
    __shared__ __attribute__((aligned(16))) unsigned char smem[STAGES * STAGE_BYTES];

    int tm, tn;
    tile_coords<8>(blockIdx.x, gridDim.x, tiles_m, tiles_n, tm, tn);
    const int64_t row0 = (int64_t)tm * BM, col0 = (int64_t)tn * BN;
    const int64_t ld = a.ld;
    const int ktiles = (int)(ld / BK);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave / WN, wc = wave % WN;

    // Load assignment: wave w fills tile rows [32w, 32w + 32) of A and of B with
    // two 16-row instructions each; lane L lands at byte 16 L of the 1 KiB group,
    // i.e. row (L >> 2), physical slot (L & 3), holding logical chunk slot ^ swz.
    const __bf16 *ga[2], *gb[2];
    int lds_row_base[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int r = 32 * wave + 16 * i + (lane >> 2);
        const int c = (lane & 3) ^ ((r >> 1) & 3);
        ga[i] = A + (row0 + r) * ld + c * 8;
        gb[i] = B + (col0 + r) * ld + c * 8;
        lds_row_base[i] = (32 * wave + 16 * i) * ROW_BYTES;  // wave-uniform
    }

#define DPT_ISSUE(KT, STAGE)                                                                                       \
    do {                                                                                                           \
        unsigned char *sb_ = smem + (STAGE) * STAGE_BYTES;                                                         \
        const int64_t ko_ = (int64_t)(KT) * BK;                                                                    \
        _Pragma("unroll") for (int i_ = 0; i_ < 2; ++i_) {                                                         \
            __builtin_amdgcn_global_load_lds((gbl_void *)(ga[i_] + ko_), (lds_void *)(sb_ + lds_row_base[i_]), 16, \
                                             0, 0);                                                                \
            __builtin_amdgcn_global_load_lds((gbl_void *)(gb[i_] + ko_),                                           \
                                             (lds_void *)(sb_ + BM * ROW_BYTES + lds_row_base[i_]), 16, 0, 0);     \
        }                                                                                                          \
    } while (0)

    floatx16_t acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    // Fragment addressing: lane (fr = lane & 31, fg = lane >> 5) supplies row fr of
    // a 32-row block and, at K-step s, logical chunk 2 fg + s of the tile row.
    // Rows 32 apart share the swizzle, so block i sits 32 * ROW_BYTES further on,
    // and K-step 1 is K-step 0 with chunk bit 0 (byte-offset bit 4) flipped.
    const int fr = lane & 31, fg = lane >> 5;
    const int a_base = swz(wr * WTM + fr, 2 * fg);
    const int b_base = BM * ROW_BYTES + swz(wc * WTN + fr, 2 * fg);

    const int pro = ktiles < STAGES - 1 ? ktiles : STAGES - 1;
    for (int s = 0; s < pro; ++s) DPT_ISSUE(s, s);

    for (int kt = 0; kt < ktiles; ++kt) {
        // tile kt must have landed; later prefetched tiles may stay in flight
        const int ahead = min(STAGES - 2, ktiles - 1 - kt);
        if (ahead >= 2)
            wait_vmcnt<2 * LOADS_PER_STAGE>();
        else if (ahead == 1)
            wait_vmcnt<LOADS_PER_STAGE>();
        else
            wait_vmcnt<0>();
        barrier_keep_loads();  // every wave's part of tile kt is in LDS; stage kt-1 is free
        if (kt + STAGES - 1 < ktiles) DPT_ISSUE(kt + STAGES - 1, (kt + STAGES - 1) % STAGES);
        const unsigned char *sb = smem + (kt % STAGES) * STAGE_BYTES;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            bf16x8_t fa[TM], fb[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i)
                fa[i] = *reinterpret_cast<const bf16x8_t *>(sb + ((a_base + i * 32 * ROW_BYTES) ^ (s << 4)));
#pragma unroll
            for (int j = 0; j < TN; ++j)
                fb[j] = *reinterpret_cast<const bf16x8_t *>(sb + ((b_base + j * 32 * ROW_BYTES) ^ (s << 4)));
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
        }
    }
#undef DPT_ISSUE

    // Epilogue through LDS, in two passes of 128 tile rows (128 x 256 FP32 =
    // the whole ring): the waves owning those rows write their accumulators
    // (32x32 layout: register r of lane l is C[(r & 3) + 4 (l >> 5) + 8 (r >> 2)][l & 31]),
    // then all threads update the rows with 16-byte coalesced accesses.
    float *tile = reinterpret_cast<float *>(smem);
    constexpr int TP = 256;  // tile row pitch (floats)
    const float lam = (float)a.lambda;
    double dmax = 0.0, wmax = 0.0;
    bool bad = false;
    __syncthreads();  // the ring is no longer read
#pragma unroll
    for (int h = 0; h < WM; ++h) {
        if (wr == h) {
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int row = i * 32 + (r & 3) + ((lane >> 5) << 2) + ((r >> 2) << 3);
                        tile[row * TP + wc * WTN + j * 32 + (lane & 31)] = acc[i][j][r];
                    }
        }
        __syncthreads();
        for (int k = 0; k < (WTM * BN / 4) / NT; ++k) {
            const int q = tid + NT * k;
            const int row = q / (BN / 4), c4 = (q % (BN / 4)) * 4;
            const int64_t n = row0 + h * WTM + row, m0 = col0 + c4;
            const int64_t idx = n * ld + m0;
            const float4 cv = *reinterpret_cast<const float4 *>(&tile[row * TP + c4]);
            const float4 dt = *reinterpret_cast<const float4 *>(&deltaT[idx]);
            const float4 wo = *reinterpret_cast<const float4 *>(&Wold[idx]);
            const double th_n = a.theta[n];
            const float dn = (float)a.d[n];
            const bool row_ok = n < a.n;
            const float cs[4] = {cv.x + dt.x, cv.y + dt.y, cv.z + dt.z, cv.w + dt.w};
            const float ws[4] = {wo.x, wo.y, wo.z, wo.w};
            float w[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t m = m0 + e;
                w[e] = 0.0f;
                if (row_ok && m < a.n && m != n) {
                    const float num = cs[e] - dn * ws[e];
                    const float gap = (float)(th_n - a.theta[m]);
                    w[e] = lam * num / gap;
                }
                const double dv = fabs((double)w[e] - (double)ws[e]), av = fabs((double)w[e]);
                dmax = fmax(dmax, dv);
                wmax = fmax(wmax, av);
                bad |= !(dv <= DBL_MAX) || !(av <= DBL_MAX);
            }
            *reinterpret_cast<float4 *>(&Wnew[idx]) = make_float4(w[0], w[1], w[2], w[3]);
            const __bf16 b4[4] = {(__bf16)w[0], (__bf16)w[1], (__bf16)w[2], (__bf16)w[3]};
            uint2 packed;
            __builtin_memcpy(&packed, b4, sizeof(packed));
            *reinterpret_cast<uint2 *>(&Wbnew[idx]) = packed;
        }
        __syncthreads();  // before the next pass overwrites the tile
    }
    publish_stats(a.stat, dmax, wmax, bad);
}

}  // namespace

bool step_bf16_v2_supported(int64_t ld) { return ld % BM == 0 && ld % BN == 0 && ld >= 1024; }

hipError_t launch_step_bf16_v2(const StepArgs &a, const __bf16 *Wb, const __bf16 *Deltab, const float *deltaT,
                               const float *W, float *Wn, __bf16 *Wbn, hipStream_t s) {
    if (!step_bf16_v2_supported(a.ld)) return hipErrorInvalidValue;
    const int tiles_m = (int)(a.ld / BM), tiles_n = (int)(a.ld / BN);
    hipLaunchKernelGGL(k_step_bf16_v2, dim3((unsigned int)(tiles_m * tiles_n)), dim3(NT), 0, s, Wb, Deltab, deltaT, W,
                       Wn, Wbn, a, tiles_m, tiles_n);
    return hipGetLastError();
}

}  // namespace dpt
