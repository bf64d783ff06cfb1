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
// chunks stored at slot c ^ ((row >> 2) & 3): the sixteen rows read by sixteen
// consecutive lanes of a fragment load (one 256-byte pass over the 64 LDS
// banks) then fall on sixteen different 16-byte bank groups.
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
// Epilogue tile: 128 rows of 256 FP32 values, row pitch 264 so that the two
// half-waves of an accumulator store (rows 4 apart) hit disjoint bank halves.
constexpr int EPI_PITCH = 264;
constexpr int SMEM_BYTES = STAGES * STAGE_BYTES > 128 * EPI_PITCH * 4 ? STAGES * STAGE_BYTES : 128 * EPI_PITCH * 4;

typedef __attribute__((address_space(3))) void lds_void;
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const void gbl_void;

// Swizzle key of tile row r, and byte offset of logical 16-byte chunk c (0..3)
// of row r inside one operand tile.
__device__ __forceinline__ int swz_key(int r) { return (r >> 2) & 3; }
__device__ __forceinline__ int swz(int r, int c) { return r * ROW_BYTES + ((c ^ swz_key(r)) << 4); }

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
    __shared__ __attribute__((aligned(16))) unsigned char smem[SMEM_BYTES];

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
        const int c = (lane & 3) ^ swz_key(r);
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

    // Epilogue through LDS, in two passes of 128 tile rows (128 x 256 FP32,
    // padded rows): the waves owning those rows write their accumulators
    // (32x32 layout: register r of lane l is C[(r & 3) + 4 (l >> 5) + 8 (r >> 2)][l & 31]),
    // then all threads update the rows with 16-byte coalesced accesses.
    float *tile = reinterpret_cast<float *>(smem);
    constexpr int TP = EPI_PITCH;
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

// ---------------------------------------------------------------------------
// v3: same tile, LDS ring and epilogue, but 4 waves (one per SIMD) with a
// 128 x 128 wave tile (4 x 4 MFMA blocks, accumulators in the AGPR half of the
// register file).  Per K-tile a wave reads 16 fragments for 64 MFMAs (v2: 12
// for 16 per two waves), which cuts LDS read traffic per flop by a third.  With
// one wave per SIMD the fragment latency is hidden inside the wave: the
// fragments of tile kt+1 are read (into the second register set) while the
// second half of tile kt's MFMAs issues, after a barrier placed mid-tile.
constexpr int WM3 = 2, WN3 = 2, NT3 = WM3 * WN3 * 64;  // 256 threads
constexpr int WTM3 = BM / WM3, WTN3 = BN / WN3;        // 128 x 128 per wave
constexpr int TM3 = WTM3 / 32, TN3 = WTN3 / 32;        // 4 x 4 MFMA blocks
constexpr int LOADS3 = 8;                              // per thread per stage: 4 for A, 4 for B
#ifndef DPT_BF16_STAGES
#define DPT_BF16_STAGES 5
#endif
constexpr int STAGES3 = DPT_BF16_STAGES;               // 5 x 32 KiB = the whole 160 KiB LDS
constexpr int SMEM3 = STAGES3 * STAGE_BYTES > 128 * EPI_PITCH * 4 ? STAGES3 * STAGE_BYTES : 128 * EPI_PITCH * 4;

__global__ __launch_bounds__(NT3) void k_step_bf16_v3(const __bf16 *__restrict__ A, const __bf16 *__restrict__ B,
                                                         const float *__restrict__ deltaT,
                                                         const float *__restrict__ Wold, float *__restrict__ Wnew,
                                                         __bf16 *__restrict__ Wbnew, StepArgs a, int tiles_m,
                                                         int tiles_n) {
    __shared__ __attribute__((aligned(16))) unsigned char smem[SMEM3];

    int tm, tn;
    tile_coords<8>(blockIdx.x, gridDim.x, tiles_m, tiles_n, tm, tn);
    const int64_t row0 = (int64_t)tm * BM, col0 = (int64_t)tn * BN;
    const int64_t ld = a.ld;
    const int ktiles = (int)(ld / BK);  // a multiple of 8
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave / WN3, wc = wave % WN3;

    // wave w fills tile rows [64w, 64w + 64) of A and of B, 16 rows per instruction
    const __bf16 *ga[4], *gb[4];
    int lds_row_base[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = 64 * wave + 16 * i + (lane >> 2);
        const int c = (lane & 3) ^ swz_key(r);
        ga[i] = A + (row0 + r) * ld + c * 8;
        gb[i] = B + (col0 + r) * ld + c * 8;
        lds_row_base[i] = (64 * wave + 16 * i) * ROW_BYTES;
    }
#define DPT_ISSUE3(KT, STAGE)                                                                                      \
    do {                                                                                                           \
        unsigned char *sb_ = smem + (STAGE) * STAGE_BYTES;                                                         \
        const int64_t ko_ = (int64_t)(KT) * BK;                                                                    \
        _Pragma("unroll") for (int i_ = 0; i_ < 4; ++i_) {                                                         \
            __builtin_amdgcn_global_load_lds((gbl_void *)(ga[i_] + ko_), (lds_void *)(sb_ + lds_row_base[i_]), 16, \
                                             0, 0);                                                                \
            __builtin_amdgcn_global_load_lds((gbl_void *)(gb[i_] + ko_),                                           \
                                             (lds_void *)(sb_ + BM * ROW_BYTES + lds_row_base[i_]), 16, 0, 0);     \
        }                                                                                                          \
    } while (0)

    floatx16_t acc[TM3][TN3];
#pragma unroll
    for (int i = 0; i < TM3; ++i)
#pragma unroll
        for (int j = 0; j < TN3; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    const int fr = lane & 31, fg = lane >> 5;
    const int a_base = swz(wr * WTM3 + fr, 2 * fg);
    const int b_base = BM * ROW_BYTES + swz(wc * WTN3 + fr, 2 * fg);

    // fragments of one K-tile: [substep][block]
    bf16x8_t fa0[2][TM3], fb0[2][TN3], fa1[2][TM3], fb1[2][TN3];
#define DPT_FRAGS3(FA, FB, KT)                                                                                       \
    do {                                                                                                             \
        const unsigned char *sb_ = smem + ((KT) % STAGES3) * STAGE_BYTES;                                             \
        _Pragma("unroll") for (int s_ = 0; s_ < 2; ++s_) {                                                           \
            _Pragma("unroll") for (int i_ = 0; i_ < TM3; ++i_) FA[s_][i_] =                                           \
                *reinterpret_cast<const bf16x8_t *>(sb_ + ((a_base + i_ * 32 * ROW_BYTES) ^ (s_ << 4)));             \
            _Pragma("unroll") for (int j_ = 0; j_ < TN3; ++j_) FB[s_][j_] =                                           \
                *reinterpret_cast<const bf16x8_t *>(sb_ + ((b_base + j_ * 32 * ROW_BYTES) ^ (s_ << 4)));             \
        }                                                                                                            \
    } while (0)
#define DPT_MMA3(FA, FB, S)                                                                                          \
    do {                                                                                                             \
        _Pragma("unroll") for (int i_ = 0; i_ < TM3; ++i_) _Pragma("unroll") for (int j_ = 0; j_ < TN3; ++j_)          \
            acc[i_][j_] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(FA[S][i_], FB[S][j_], acc[i_][j_], 0, 0, 0);       \
    } while (0)
    // One K-tile kt that has a successor: substep 0 on FC; wait until tile kt+1
    // has landed and every wave is done with tile kt; then, interleaved with
    // substep 1 on FC, refill tile kt's slot with tile kt+S (S = STAGES3) and
    // read tile kt+1 into FN.  Tiles 0..kt+S-1 have been issued at that point
    // (the prologue issues 0..S-1, tile j issues j+S), so "tile kt+1 landed" is
    // vmcnt <= 8 (S-2) (tiles kt+2..kt+S-1 in flight).  Past the end the refill
    // repeats the last tile into the freed slot, which nothing reads (the slot of
    // tile ktiles-1 is never the freed one), keeping the count uniform.
#define DPT_TILE3(FCA, FCB, FNA, FNB, KT)                                                                            \
    do {                                                                                                             \
        DPT_MMA3(FCA, FCB, 0);                                                                                       \
        __builtin_amdgcn_sched_barrier(0);                                                                           \
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");                                                          \
        wait_vmcnt<(STAGES3 - 2) * LOADS3>();                                                                        \
        barrier_keep_loads();                                                                                        \
        __builtin_amdgcn_sched_barrier(0);                                                                           \
        DPT_MMA3(FCA, FCB, 1);                                                                                       \
        DPT_ISSUE3(min((KT) + STAGES3, ktiles - 1), (KT) % STAGES3);                                                   \
        DPT_FRAGS3(FNA, FNB, (KT) + 1);                                                                              \
        _Pragma("unroll") for (int g_ = 0; g_ < 8; ++g_) {                                                           \
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);                                                       \
            __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);                                                       \
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);                                                       \
            __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);                                                       \
        }                                                                                                            \
        __builtin_amdgcn_sched_barrier(0);                                                                           \
    } while (0)

    // all slots start free: tiles 0..STAGES3-1 in flight, wait for tile 0
    for (int s = 0; s < STAGES3; ++s) DPT_ISSUE3(s, s);  // ktiles >= 32
    wait_vmcnt<(STAGES3 - 1) * LOADS3>();
    barrier_keep_loads();
    DPT_FRAGS3(fa0, fb0, 0);
    for (int kt = 0; kt < ktiles - 2; kt += 2) {
        DPT_TILE3(fa0, fb0, fa1, fb1, kt);
        DPT_TILE3(fa1, fb1, fa0, fb0, kt + 1);
    }
    DPT_TILE3(fa0, fb0, fa1, fb1, ktiles - 2);
    DPT_MMA3(fa1, fb1, 0);
    DPT_MMA3(fa1, fb1, 1);
    wait_vmcnt<0>();  // the repeated refills land before the ring becomes the epilogue tile
#undef DPT_TILE3
#undef DPT_MMA3
#undef DPT_FRAGS3
#undef DPT_ISSUE3

    // Epilogue through LDS in two passes of 128 tile rows (128 x 256 FP32,
    // padded rows); the two waves owning those rows write their accumulators.
    float *tile = reinterpret_cast<float *>(smem);
    constexpr int TP = EPI_PITCH;
    const float lam = (float)a.lambda;
    double dmax = 0.0, wmax = 0.0;
    bool bad = false;
    __syncthreads();
#pragma unroll
    for (int h = 0; h < WM3; ++h) {
        if (wr == h) {
#pragma unroll
            for (int i = 0; i < TM3; ++i)
#pragma unroll
                for (int j = 0; j < TN3; ++j)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int row = i * 32 + (r & 3) + ((lane >> 5) << 2) + ((r >> 2) << 3);
                        tile[row * TP + wc * WTN3 + j * 32 + (lane & 31)] = acc[i][j][r];
                    }
        }
        __syncthreads();
        for (int k = 0; k < (WTM3 * BN / 4) / NT3; ++k) {
            const int q = tid + NT3 * k;
            const int row = q / (BN / 4), c4 = (q % (BN / 4)) * 4;
            const int64_t n = row0 + h * WTM3 + row, m0 = col0 + c4;
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
        __syncthreads();
    }
    publish_stats(a.stat, dmax, wmax, bad);
}

// ---------------------------------------------------------------------------
// v4: v3's 4 x (128 x 128) wave tiles with K-tiles of 64: every tile row read
// from global memory is one whole 128-byte line (the operand stream from L2
// into LDS runs markedly faster with full lines than with half lines), in a
// 2-stage ring of 64 KiB stages.  A K-tile is consumed as two halves of K = 32
// whose fragments go to two register sets: half 1 is read while half 0
// multiplies; the barrier (tile kt+1 landed, tile kt fully read) sits before
// the last substep, whose MFMAs cover the refill of tile kt's slot with tile
// kt+2 and the reads of tile kt+1's first half.
constexpr int BK4 = 64, ROW4 = BK4 * 2, STAGE4 = (BM + BN) * ROW4, STAGES4 = 2;
constexpr int LOADS4 = 16;  // per thread per stage: 8 for A, 8 for B
constexpr int SMEM4 = STAGES4 * STAGE4 > 128 * EPI_PITCH * 4 ? STAGES4 * STAGE4 : 128 * EPI_PITCH * 4;

// Swizzle of 128-byte rows: physical 16-byte slot of logical chunk c in row r
// is c ^ key8(r).  Any 16 consecutive rows (aligned to 8) at a fixed logical
// chunk then cover all 64 banks once, and any 8 cover 32 banks once.
__device__ __forceinline__ int key8(int r) { return (r ^ (r >> 3)) & 7; }

__global__ __launch_bounds__(NT3) void k_step_bf16_v4(const __bf16 *__restrict__ A, const __bf16 *__restrict__ B,
                                                         const float *__restrict__ deltaT,
                                                         const float *__restrict__ Wold, float *__restrict__ Wnew,
                                                         __bf16 *__restrict__ Wbnew, StepArgs a, int tiles_m,
                                                         int tiles_n) {
    __shared__ __attribute__((aligned(16))) unsigned char smem[SMEM4];

    int tm, tn;
    tile_coords<8>(blockIdx.x, gridDim.x, tiles_m, tiles_n, tm, tn);
    const int64_t row0 = (int64_t)tm * BM, col0 = (int64_t)tn * BN;
    const int64_t ld = a.ld;
    const int ktiles = (int)(ld / BK4);  // a multiple of 4
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = wave / WN3, wc = wave % WN3;

    // Loads: wave w fills tile rows [64w, 64w + 64) of A and of B, 8 rows of
    // 128 bytes per instruction; lane L lands at byte 16 L of the 1 KiB group:
    // row L >> 3, physical slot L & 7, holding logical chunk (L & 7) ^ key8(row).
    // Row 64w + 8i + lr has key8 = lr ^ i, so the lane's element offset inside
    // instruction i's 8 rows is lr * ld + (((L & 7) ^ lr ^ i) << 3); ld is a
    // multiple of 256, so the XOR with i << 3 acts on the chunk bits alone.
    const int lr = lane >> 3;
    const int lane_off = lr * (int)ld + (((lane & 7) ^ lr) << 3);
    const __bf16 *ga0 = A + (row0 + 64 * wave) * ld, *gb0 = B + (col0 + 64 * wave) * ld;
#define DPT_ISSUE4(KT, STAGE)                                                                                      \
    do {                                                                                                           \
        unsigned char *sb_ = smem + (STAGE) * STAGE4 + 64 * wave * ROW4;                                           \
        const int64_t ko_ = (int64_t)(KT) * BK4;                                                                   \
        _Pragma("unroll") for (int i_ = 0; i_ < 8; ++i_) {                                                         \
            const int64_t off_ = ko_ + 8 * i_ * ld + (lane_off ^ (i_ << 3));                                       \
            __builtin_amdgcn_global_load_lds((gbl_void *)(ga0 + off_), (lds_void *)(sb_ + i_ * 8 * ROW4), 16, 0,   \
                                             0);                                                                   \
            __builtin_amdgcn_global_load_lds((gbl_void *)(gb0 + off_),                                             \
                                             (lds_void *)(sb_ + BM * ROW4 + i_ * 8 * ROW4), 16, 0, 0);             \
        }                                                                                                          \
    } while (0)

    floatx16_t acc[TM3][TN3];
#pragma unroll
    for (int i = 0; i < TM3; ++i)
#pragma unroll
        for (int j = 0; j < TN3; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    // Fragments: lane (fr, fg) supplies row fr of a 32-row block and, at half h
    // and substep s, logical chunk 4h + 2fg + s.  Blocks 32 rows apart differ in
    // key8 by 4 when the block index is odd.
    const int fr = lane & 31, fg = lane >> 5;
    const int ra = wr * WTM3 + fr, rb = wc * WTN3 + fr;
    const int a_base = ra * ROW4 + (((2 * fg) ^ key8(ra)) << 4);
    const int b_base = BM * ROW4 + rb * ROW4 + (((2 * fg) ^ key8(rb)) << 4);
    bf16x8_t fa0[2][TM3], fb0[2][TN3], fa1[2][TM3], fb1[2][TN3];
#define DPT_FRAGS4(FA, FB, SLOT, H)                                                                                  \
    do {                                                                                                             \
        const unsigned char *sb_ = smem + (SLOT) * STAGE4;                                                           \
        _Pragma("unroll") for (int s_ = 0; s_ < 2; ++s_) {                                                           \
            _Pragma("unroll") for (int i_ = 0; i_ < TM3; ++i_) FA[s_][i_] = *reinterpret_cast<const bf16x8_t *>(     \
                sb_ + ((a_base + i_ * 32 * ROW4) ^ (((((i_ & 1) ^ (H)) << 2) ^ s_) << 4)));                          \
            _Pragma("unroll") for (int j_ = 0; j_ < TN3; ++j_) FB[s_][j_] = *reinterpret_cast<const bf16x8_t *>(     \
                sb_ + ((b_base + j_ * 32 * ROW4) ^ (((((j_ & 1) ^ (H)) << 2) ^ s_) << 4)));                          \
        }                                                                                                            \
    } while (0)
#define DPT_MMA4(FA, FB, S)                                                                                          \
    do {                                                                                                             \
        _Pragma("unroll") for (int i_ = 0; i_ < TM3; ++i_) _Pragma("unroll") for (int j_ = 0; j_ < TN3; ++j_)        \
            acc[i_][j_] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(FA[S][i_], FB[S][j_], acc[i_][j_], 0, 0, 0);       \
    } while (0)
#define DPT_INTERLEAVE4(NVMEM)                                                                                       \
    do {                                                                                                             \
        _Pragma("unroll") for (int g_ = 0; g_ < 8; ++g_) {                                                           \
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);                                                       \
            if ((NVMEM) > 0) __builtin_amdgcn_sched_group_barrier(0x020, (NVMEM) / 8, 0);                            \
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);                                                       \
            __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);                                                       \
        }                                                                                                            \
    } while (0)

    // prologue: both slots in flight, wait for tile 0, read its first half
    DPT_ISSUE4(0, 0);
    DPT_ISSUE4(1, 1);
    wait_vmcnt<LOADS4>();
    barrier_keep_loads();
    DPT_FRAGS4(fa0, fb0, 0, 0);
    for (int kt = 0; kt < ktiles - 1; ++kt) {
        const int slot = kt & 1;
        DPT_MMA4(fa0, fb0, 0);
        __builtin_amdgcn_sched_barrier(0);
        DPT_MMA4(fa0, fb0, 1);
        DPT_FRAGS4(fa1, fb1, slot, 1);
        DPT_INTERLEAVE4(0);
        __builtin_amdgcn_sched_barrier(0);
        DPT_MMA4(fa1, fb1, 0);
        __builtin_amdgcn_sched_barrier(0);
        // every fragment of tile kt is in registers; tile kt+1 must have landed
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        wait_vmcnt<0>();
        barrier_keep_loads();
        __builtin_amdgcn_sched_barrier(0);
        DPT_MMA4(fa1, fb1, 1);
        // refill the freed slot (past the end: the last tile again, never read)
        DPT_ISSUE4(min(kt + 2, ktiles - 1), slot);
        DPT_FRAGS4(fa0, fb0, slot ^ 1, 0);
        DPT_INTERLEAVE4(16);
        __builtin_amdgcn_sched_barrier(0);
    }
    DPT_MMA4(fa0, fb0, 0);
    DPT_MMA4(fa0, fb0, 1);
    DPT_FRAGS4(fa1, fb1, (ktiles - 1) & 1, 1);
    DPT_MMA4(fa1, fb1, 0);
    DPT_MMA4(fa1, fb1, 1);
    wait_vmcnt<0>();
#undef DPT_INTERLEAVE4
#undef DPT_MMA4
#undef DPT_FRAGS4
#undef DPT_ISSUE4

    // Epilogue through LDS in two passes of 128 tile rows (128 x 256 FP32,
    // padded rows); the two waves owning those rows write their accumulators.
    // Then thread t updates columns c4..c4+3 (c4 = 4 (t & 63)) of rows
    // (t >> 6) + 4k, with the global loads of 8 rows issued before any use.
    float *tile = reinterpret_cast<float *>(smem);
    constexpr int TP = EPI_PITCH, EU = 8;
    const float lam = (float)a.lambda;
    const int c4 = (tid & 63) * 4;
    const int64_t m0 = col0 + c4;
    double dmax = 0.0, wmax = 0.0;
    bool bad = false;
    __syncthreads();
#pragma unroll
    for (int h = 0; h < WM3; ++h) {
        if (wr == h) {
#pragma unroll
            for (int i = 0; i < TM3; ++i)
#pragma unroll
                for (int j = 0; j < TN3; ++j)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int row = i * 32 + (r & 3) + ((lane >> 5) << 2) + ((r >> 2) << 3);
                        tile[row * TP + wc * WTN3 + j * 32 + (lane & 31)] = acc[i][j][r];
                    }
        }
        __syncthreads();
        for (int k0 = 0; k0 < WTM3 / 4; k0 += EU) {
            f32x4 dt[EU], wo[EU];
#pragma unroll
            for (int u = 0; u < EU; ++u) {
                const int64_t n = row0 + h * WTM3 + wave + 4 * (k0 + u);
                dt[u] = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(&deltaT[n * ld + m0]));
                wo[u] = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(&Wold[n * ld + m0]));
            }
#pragma unroll
            for (int u = 0; u < EU; ++u) {
                const int row = wave + 4 * (k0 + u);
                const int64_t n = row0 + h * WTM3 + row, idx = n * ld + m0;
                const float4 cv = *reinterpret_cast<const float4 *>(&tile[row * TP + c4]);
                const double th_n = a.theta[n];
                const float dn = (float)a.d[n];
                const bool row_ok = n < a.n;
                const float cs[4] = {cv.x + dt[u][0], cv.y + dt[u][1], cv.z + dt[u][2], cv.w + dt[u][3]};
                const float ws[4] = {wo[u][0], wo[u][1], wo[u][2], wo[u][3]};
                f32x4 w;
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
                __builtin_nontemporal_store(w, reinterpret_cast<f32x4 *>(&Wnew[idx]));
                const __bf16 b4[4] = {(__bf16)w[0], (__bf16)w[1], (__bf16)w[2], (__bf16)w[3]};
                uint2 packed;
                __builtin_memcpy(&packed, b4, sizeof(packed));
                *reinterpret_cast<uint2 *>(&Wbnew[idx]) = packed;
            }
        }
        __syncthreads();
    }
    publish_stats(a.stat, dmax, wmax, bad);
}

}  // namespace

bool step_bf16_v2_supported(int64_t ld) { return ld % BM == 0 && ld % BN == 0 && ld >= 1024; }

hipError_t launch_step_bf16_v2(const StepArgs &a, const __bf16 *Wb, const __bf16 *Deltab, const float *deltaT,
                               const float *W, float *Wn, __bf16 *Wbn, hipStream_t s) {
    if (!step_bf16_v2_supported(a.ld)) return hipErrorInvalidValue;
    const int tiles_m = (int)(a.ld / BM), tiles_n = (int)(a.ld / BN);
#if defined(DPT_BF16_V2)
    hipLaunchKernelGGL(k_step_bf16_v2, dim3((unsigned int)(tiles_m * tiles_n)), dim3(NT), 0, s, Wb, Deltab, deltaT, W,
                       Wn, Wbn, a, tiles_m, tiles_n);
#elif defined(DPT_BF16_V3)
    hipLaunchKernelGGL(k_step_bf16_v3, dim3((unsigned int)(tiles_m * tiles_n)), dim3(NT3), 0, s, Wb, Deltab,
                       deltaT, W, Wn, Wbn, a, tiles_m, tiles_n);
#else
    hipLaunchKernelGGL(k_step_bf16_v4, dim3((unsigned int)(tiles_m * tiles_n)), dim3(NT3), 0, s, Wb, Deltab,
                       deltaT, W, Wn, Wbn, a, tiles_m, tiles_n);
#endif
    return hipGetLastError();
}

}  // namespace dpt
