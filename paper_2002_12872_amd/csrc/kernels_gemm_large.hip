// Fused D-PT steps for large dense problems on gfx950 (ld a multiple of 256,
// ld >= 1024): the BF16 step and the FP32 step.
//
// One application of eq. (dyn) of Kenmoe, Smerlak, Zadorin (arXiv:2002.12872)
// on the padded state W = A - I:
//     C  = Delta^T + W Delta^T                               (MFMA, FP32 accumulate)
//     W' = lambda (C - d_n W) / (theta_n - theta_m),  m != n  (FP32 epilogue, FP64 gaps)
// plus max|W' - W| and max|W'| for the stopping rule.  The BF16 step multiplies
// bf16(W) bf16(Delta)^T and also writes the BF16 shadow of W'; the FP8 step
// multiplies block-scaled FP8 copies (OCP E4M3 values, one E8M0 power-of-two
// scale per 32 consecutive values of a row) and writes the FP8 copy of W'.
//
// Shared structure.  A 256 x 256 output tile per workgroup of 4 waves (one per
// SIMD); each wave owns a 128 x 128 wave tile as 4 x 4 blocks of 32 x 32 MFMA
// accumulators (256 registers, held in the AGPR half of the register file).
// K advances in tiles of 128 bytes per row (64 BF16 or 32 FP32 values), so each
// tile row read from global memory is one whole cache line; tiles go through a
// 2-stage LDS ring (64 KiB per stage: 256 rows of A, then 256 rows of B) filled
// by direct global->LDS loads (global_load_lds_dwordx4, no staging registers).
// In LDS the 16-byte chunk c of row r sits at slot c ^ key8(r), key8(r) =
// (r ^ (r >> 3)) & 7: any 16 (and any 8) consecutive rows read at one logical
// chunk fall on disjoint banks.  The epilogue stages the accumulators through
// the freed LDS.
#include <float.h>

#include <algorithm>

#include "device_common.h"
#include "dpt_internal.h"

namespace dpt {
namespace {

constexpr int BM = 256, BN = 256;
constexpr int ROW = 128;                  // bytes of one tile row per K-tile
constexpr int STAGE = (BM + BN) * ROW;    // 64 KiB: A tile, then B tile
constexpr int NT = 256;                   // 4 waves
constexpr int WM = 2, WN = 2;             // wave grid
constexpr int WTM = BM / WM, WTN = BN / WN;  // 128 x 128 per wave
constexpr int TM = WTM / 32, TN = WTN / 32;  // 4 x 4 MFMA blocks
constexpr int LOADS = 16;                 // global->LDS instructions per thread per stage
// Epilogue tile: 128 rows of 256 FP32 values, row pitch 264 so that the two
// half-waves of an accumulator store (rows 4 apart) hit disjoint bank halves.
constexpr int EPI_PITCH = 264;
constexpr int SMEM = 2 * STAGE > 128 * EPI_PITCH * 4 ? 2 * STAGE : 128 * EPI_PITCH * 4;

typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) const void gbl_void;
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int key8(int r) { return (r ^ (r >> 3)) & 7; }

template <int N>
__device__ __forceinline__ void wait_vmcnt() {
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// Workgroup barrier without an implicit wait on outstanding vector-memory
// operations (the prefetched stage must stay in flight); the memory clobber
// keeps the compiler from moving LDS accesses across it.
__device__ __forceinline__ void barrier_keep_loads() { asm volatile("s_barrier" ::: "memory"); }

// Global->LDS loads of one K-tile into one ring slot.  Wave w fills tile rows
// [64w, 64w + 64) of A and of B, 8 rows of 128 bytes per instruction; lane L
// lands at byte 16 L of the instruction's 1 KiB: row 8i + (L >> 3), physical
// slot L & 7, so it reads logical chunk (L & 7) ^ key8(row).  key8 of tile row
// 64w + 8i + lr is lr ^ i, so the lane's byte offset inside instruction i is
// lr * ldb + (((L & 7) ^ lr ^ i) << 4); ldb (a multiple of 512) leaves the
// chunk bits free for the XOR with i << 4.
//
// Split form (blk != 0): the operands hold two K blocks of blk bytes per row,
// A = [Wh | Wl] and B = [Dh | Dl], and logical K-tile 3p + b reads physical
// K-tile p of the block pair (h, h), (l, h), (h, l) for b = 0, 1, 2; the tiles
// read twice come back within three K-tiles, from L2.
struct TileLoader {
    const unsigned char *ga, *gb;  // row 64w of the A and B tiles (bytes)
    int64_t ldb;                   // bytes per matrix row
    int64_t blk = 0;               // split form: bytes per K block (0: plain operands)
    int lane_off;                  // lr * ldb + (((L & 7) ^ lr) << 4)
    int lds_off;                   // 64 w * ROW

    __device__ void init(const void *A, const void *B, int64_t row0, int64_t col0, int64_t ld_bytes, int wave,
                         int lane) {
        ldb = ld_bytes;
        ga = (const unsigned char *)A + (row0 + 64 * wave) * ldb;
        gb = (const unsigned char *)B + (col0 + 64 * wave) * ldb;
        const int lr = lane >> 3;
        lane_off = lr * (int)ldb + (((lane & 7) ^ lr) << 4);
        lds_off = 64 * wave * ROW;
    }
    __device__ __forceinline__ void issue(unsigned char *smem, int kt, int slot) const { issue_rows(smem, kt, slot, 0, 8); }
    // instructions i in [I0, I1) of issue(): rows 8i .. 8i + 7 of both tiles
    __device__ __forceinline__ void issue_rows(unsigned char *smem, int kt, int slot, int I0, int I1) const {
        unsigned char *sb = smem + slot * STAGE + lds_off;
        int64_t koa = (int64_t)kt * ROW, kob = koa;
        if (blk) {
            const int p = kt / 3, b = kt - 3 * p;
            koa = (int64_t)p * ROW + (b == 1 ? blk : 0);
            kob = (int64_t)p * ROW + (b == 2 ? blk : 0);
        }
        // Address = wave-uniform row base (SGPR pair) + 32-bit lane offset, the
        // saddr form of the load: no 64-bit address arithmetic per load and
        // half the address registers read at issue (0.9 % of the FP32 step's
        // main loop).  The empty asm statements keep the compiler from folding
        // the lane offset into a 64-bit vector address.
#pragma unroll
        for (int i = I0; i < I1; ++i) {
            uint32_t vo = (uint32_t)lane_off ^ (uint32_t)(i << 4);
            asm volatile("" : "+v"(vo));
            const unsigned char *ra = ga + koa + 8 * i * ldb, *rb = gb + kob + 8 * i * ldb;
            asm volatile("" : "+s"(ra), "+s"(rb));
            __builtin_amdgcn_global_load_lds((gbl_void *)(ra + vo), (lds_void *)(sb + i * 8 * ROW), 16, 0, 0);
            __builtin_amdgcn_global_load_lds((gbl_void *)(rb + vo), (lds_void *)(sb + BM * ROW + i * 8 * ROW), 16, 0,
                                             0);
        }
    }
};

// Epilogue of one tile: the accumulators (32x32 layout: register r of lane l is
// C[(r & 3) + 4 (l >> 5) + 8 (r >> 2)][l & 31]) go through LDS in two passes of
// 128 tile rows; thread t updates columns c4..c4+3 (c4 = 4 (t & 63)) of rows
// (t >> 6) + 4k in batches of EU rows, the global loads of the next batch
// issued before the current one is used.
// Block-scaled FP8 (OCP E4M3) quantisation of 32 consecutive values held 4 per
// lane by 8 consecutive lanes: the E8M0 scale 2^X is the smallest power of two
// with amax <= 448 * 2^X (448 = 0.875 * 2^9, the largest E4M3 value), so with
// amax = f 2^e, f in [0.5, 1): X = e - 9 if f <= 0.875, else e - 8 (clamped to
// the E8M0 range).  Values v / 2^X are rounded to nearest-even E4M3 by the
// hardware conversion (clamped to +-448 first: the conversion does not
// saturate).  Returns the 4 FP8 bytes packed in one word; *scale gets X + 127.
__device__ __forceinline__ unsigned quant_fp8_x4(const float v[4], unsigned *scale) {
    float amax = fmaxf(fmaxf(fabsf(v[0]), fabsf(v[1])), fmaxf(fabsf(v[2]), fabsf(v[3])));
    amax = fmaxf(amax, __shfl_xor(amax, 1));
    amax = fmaxf(amax, __shfl_xor(amax, 2));
    amax = fmaxf(amax, __shfl_xor(amax, 4));
    int e = 0;
    const float f = frexpf(amax, &e);
    int x = amax > 0.0f ? (f <= 0.875f ? e - 9 : e - 8) : -127;
    x = min(max(x, -127), 127);
    float q[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) q[k] = fminf(fmaxf(ldexpf(v[k], -x), -448.0f), 448.0f);
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(q[0], q[1], 0, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(q[2], q[3], w, true);
    *scale = (unsigned)(x + 127);
    return (unsigned)w;
}

// Output forms of the shared epilogue.
// EPI_X3 writes the split BF16 form of W' (h = bf16(w), l = bf16(w - h)) as
// row n of the N x 2N operand [h | l] (row stride 2 ld).
enum EpiOut { EPI_F32 = 0, EPI_BF16 = 1, EPI_FP8 = 2, EPI_X3 = 3 };

template <int OUT>
__device__ __forceinline__ void epilogue(unsigned char *smem, floatx16_t (&acc)[TM][TN], const float *__restrict__ deltaT,
                                         const float *__restrict__ Wold, float *__restrict__ Wnew,
                                         __bf16 *__restrict__ Wbnew, unsigned char *__restrict__ Wqnew,
                                         unsigned char *__restrict__ Wsnew, const StepArgs &a, int64_t row0,
                                         int64_t col0, int tid, int lane, int wave, int wr, int wc) {
    float *tile = reinterpret_cast<float *>(smem);
    // batches of 4 rows, double-buffered (1 for the FP8 and split outputs,
    // whose extra work would otherwise spill registers)
    constexpr int TP = EPI_PITCH, EU = (OUT == EPI_F32 || OUT == EPI_BF16) ? 4 : 1, NBP = WTM / 4 / EU;
    constexpr bool HOIST = OUT != EPI_X3;
    const int64_t ld = a.ld;
    const float lam = (float)a.lambda;
    const int c4 = (tid & 63) * 4;
    const int64_t m0 = col0 + c4;
    double thm[4];
    bool colok[4];
    double dmax = 0.0;
    float wmax = 0.0f;
    bool bad = false;
    f32x4 dt[2][EU], wo[2][EU];
    double thn[2][EU], dnv[2][EU];
    // batch b: tile rows 128 (b / NBP) + wave + 4 (k0 + u), k0 = EU (b % NBP)
#define DPT_EPI_LOAD(BUF, B)                                                                                         \
    do {                                                                                                             \
        _Pragma("unroll") for (int u_ = 0; u_ < EU; ++u_) {                                                          \
            const int64_t n_ = row0 + ((B) / NBP) * WTM + wave + 4 * (((B) % NBP) * EU + u_);                         \
            dt[BUF][u_] = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(&deltaT[n_ * ld + m0]));        \
            wo[BUF][u_] = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(&Wold[n_ * ld + m0]));          \
            thn[BUF][u_] = a.theta[n_];                                                                              \
            dnv[BUF][u_] = a.d[n_];                                                                                  \
        }                                                                                                            \
    } while (0)
    auto stage = [&](int h) {
        __syncthreads();
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
    };
    // W'[n][m] = lambda (C[n][m] - d_n W[n][m]) / (theta_n - theta_m), 0 on the
    // diagonal and outside n, m < N; max|W' - W| (exact in FP64), max|W'| and
    // whether any W or W' is not finite
    auto compute = [&](const f32x4 (&dtb)[EU], const f32x4 (&wob)[EU], const double (&thb)[EU],
                       const double (&dnb)[EU], int b) {
        const int h = b / NBP, k0 = (b % NBP) * EU;
#pragma unroll
        for (int u = 0; u < EU; ++u) {
            const int row = wave + 4 * (k0 + u);
            const int64_t n = row0 + h * WTM + row, idx = n * ld + m0;
            const float4 cv = *reinterpret_cast<const float4 *>(&tile[row * TP + c4]);
            const double th_n = thb[u];
            const float dn = (float)dnb[u];
            const bool row_ok = n < a.n;
            const float cs[4] = {cv.x + dtb[u][0], cv.y + dtb[u][1], cv.z + dtb[u][2], cv.w + dtb[u][3]};
            const float ws[4] = {wob[u][0], wob[u][1], wob[u][2], wob[u][3]};
            f32x4 w;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float num = cs[e] - dn * ws[e];
                const float gap = (float)(th_n - (HOIST ? thm[e] : a.theta[m0 + e]));
                const float q = lam * num / gap;
                w[e] = row_ok && colok[e] && m0 + e != n ? q : 0.0f;
                dmax = fmax(dmax, fabs((double)w[e] - (double)ws[e]));
                wmax = fmaxf(wmax, fabsf(w[e]));
                bad |= !(fabsf(w[e]) <= FLT_MAX) || !(fabsf(ws[e]) <= FLT_MAX);
            }
            __builtin_nontemporal_store(w, reinterpret_cast<f32x4 *>(&Wnew[idx]));
            if (OUT == EPI_BF16) {
                const __bf16 b4[4] = {(__bf16)w[0], (__bf16)w[1], (__bf16)w[2], (__bf16)w[3]};
                uint2 packed;
                __builtin_memcpy(&packed, b4, sizeof(packed));
                *reinterpret_cast<uint2 *>(&Wbnew[idx]) = packed;
            } else if (OUT == EPI_X3) {
                float hv[4], lv[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    hv[e] = (float)(__bf16)w[e];
                    lv[e] = w[e] - hv[e];
                }
                const __bf16 h4[4] = {(__bf16)hv[0], (__bf16)hv[1], (__bf16)hv[2], (__bf16)hv[3]};
                const __bf16 l4[4] = {(__bf16)lv[0], (__bf16)lv[1], (__bf16)lv[2], (__bf16)lv[3]};
                uint2 ph, pl;
                __builtin_memcpy(&ph, h4, sizeof(ph));
                __builtin_memcpy(&pl, l4, sizeof(pl));
                __bf16 *orow = Wbnew + n * (2 * ld) + m0;
                *reinterpret_cast<uint2 *>(orow) = ph;
                *reinterpret_cast<uint2 *>(orow + ld) = pl;
            } else if (OUT == EPI_FP8) {  // 8 lanes = the 32 columns of one scale block
                const float v4[4] = {w[0], w[1], w[2], w[3]};
                unsigned sc;
                *reinterpret_cast<unsigned *>(&Wqnew[idx]) = quant_fp8_x4(v4, &sc);
                if ((lane & 7) == 0) Wsnew[n * (ld / 32) + m0 / 32] = (unsigned char)sc;
            }
        }
    };
    // the first batch's loads overlap the first staging (after it for the
    // FP8 and split outputs, which have no registers to spare there)
    if (EU > 1) DPT_EPI_LOAD(0, 0);
    stage(0);
    if (EU == 1) DPT_EPI_LOAD(0, 0);
    // theta and validity of the lane's four columns hold for every row (the
    // split output reads theta per element instead, for the same reason)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        thm[e] = HOIST ? a.theta[m0 + e] : 0.0;
        colok[e] = m0 + e < a.n;
    }
    // pass 0 (its last load fetches the first batch of pass 1), then pass 1:
    // two loops, so the accumulators are dead after the second staging
#pragma unroll 1
    for (int b2 = 0; b2 < NBP / 2; ++b2) {
        DPT_EPI_LOAD(1, 2 * b2 + 1);
        compute(dt[0], wo[0], thn[0], dnv[0], 2 * b2);
        DPT_EPI_LOAD(0, 2 * b2 + 2);
        compute(dt[1], wo[1], thn[1], dnv[1], 2 * b2 + 1);
    }
    stage(1);
#pragma unroll 1
    for (int b2 = NBP / 2; b2 < NBP; ++b2) {
        DPT_EPI_LOAD(1, 2 * b2 + 1);
        compute(dt[0], wo[0], thn[0], dnv[0], 2 * b2);
        if (b2 < NBP - 1) DPT_EPI_LOAD(0, 2 * b2 + 2);
        compute(dt[1], wo[1], thn[1], dnv[1], 2 * b2 + 1);
    }
#undef DPT_EPI_LOAD
    __syncthreads();
    publish_stats(a.stat, dmax, (double)wmax, bad);
}

// ---------------------------------------------------------------------------
// BF16 step.  A K-tile (64 values) is consumed as two halves of K = 32 whose
// fragments go to two register sets (fa0/fb0, fa1/fb1): half 1 is read while
// half 0 multiplies, so after the first of the four substeps every fragment of
// tile kt is in registers.  A first barrier there frees tile kt's slot, and its
// refill with tile kt+2 runs under substeps 2 and 3 (8 loads each: issued in
// one substep, the loads of four waves back up behind the CU's vector-memory
// path and stall the MFMA issue); a second barrier before the last substep
// waits for tile kt+1, whose first half is read under that substep.  A refill
// thus has about 1.5 K-tiles of MFMA work to arrive, and up to two tiles per CU
// are in flight: the operand stream into LDS is latency-bound, and one tile in
// flight sustains about 12 TB/s against 15 TB/s for two.  Fragments: lane (fr, fg)
// supplies row fr of a 32-row block and, at half h and substep s, logical chunk
// 4h + 2fg + s; blocks 32 rows apart differ in key8 by 4 when the block index
// is odd.
//
// X3 (the split form): A = [Wh | Wl] and B = [Dh | Dl] are N x 2N (row stride
// 2 ld; h = bf16(x), l = bf16(x - h)) and the K loop runs over 3 ld, pairing the
// blocks (h, h), (l, h), (h, l) K-tile by K-tile (TileLoader), so the product is
// Wh Dh^T + Wl Dh^T + Wh Dl^T, everything but the l x l term; the epilogue
// writes the split form of W' in the layout of A.
template <bool X3>
__global__ __launch_bounds__(NT) void k_step_bf16_large(const __bf16 *__restrict__ A, const __bf16 *__restrict__ B,
                                                        const float *__restrict__ deltaT,
                                                        const float *__restrict__ Wold, float *__restrict__ Wnew,
                                                        __bf16 *__restrict__ Wbnew, StepArgs a, int tiles_m,
                                                        int tiles_n) {
    constexpr int KM = X3 ? 3 : 1;  // operand columns per state column
    __shared__ __attribute__((aligned(16))) unsigned char smem[SMEM];
    int tm, tn;
    tile_coords<8>(blockIdx.x, gridDim.x, tiles_m, tiles_n, tm, tn);
    const int64_t row0 = (int64_t)tm * BM, col0 = (int64_t)tn * BN;
    const int ktiles = (int)(KM * a.ld * 2 / ROW);  // a multiple of 4
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = wave / WN, wc = wave % WN;
    TileLoader ld;
    ld.init(A, B, row0, col0, (X3 ? 2 : 1) * a.ld * 2, wave, lane);
    if (X3) ld.blk = a.ld * 2;

    floatx16_t acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    const int fr = lane & 31, fg = lane >> 5;
    const int ra = wr * WTM + fr, rb = wc * WTN + fr;
    const int a_base = ra * ROW + (((2 * fg) ^ key8(ra)) << 4);
    const int b_base = BM * ROW + rb * ROW + (((2 * fg) ^ key8(rb)) << 4);
    bf16x8_t fa0[2][TM], fb0[2][TN], fa1[2][TM], fb1[2][TN];
#define DPT_FRAGS(FA, FB, SLOT, H)                                                                                   \
    do {                                                                                                             \
        const unsigned char *sb_ = smem + (SLOT) * STAGE;                                                            \
        _Pragma("unroll") for (int s_ = 0; s_ < 2; ++s_) {                                                           \
            _Pragma("unroll") for (int i_ = 0; i_ < TM; ++i_) FA[s_][i_] = *reinterpret_cast<const bf16x8_t *>(      \
                sb_ + ((a_base + i_ * 32 * ROW) ^ (((((i_ & 1) ^ (H)) << 2) ^ s_) << 4)));                           \
            _Pragma("unroll") for (int j_ = 0; j_ < TN; ++j_) FB[s_][j_] = *reinterpret_cast<const bf16x8_t *>(      \
                sb_ + ((b_base + j_ * 32 * ROW) ^ (((((j_ & 1) ^ (H)) << 2) ^ s_) << 4)));                           \
        }                                                                                                            \
    } while (0)
#define DPT_MMA(FA, FB, S)                                                                                           \
    do {                                                                                                             \
        _Pragma("unroll") for (int i_ = 0; i_ < TM; ++i_) _Pragma("unroll") for (int j_ = 0; j_ < TN; ++j_)          \
            acc[i_][j_] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(FA[S][i_], FB[S][j_], acc[i_][j_], 0, 0, 0);       \
    } while (0)
#define DPT_VPIN(NV)                                                                                                 \
    do {                                                                                                             \
        _Pragma("unroll") for (int g_ = 0; g_ < (NV); ++g_) {                                                        \
            __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);                                                       \
            __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);                                                       \
        }                                                                                                            \
    } while (0)
#define DPT_INTERLEAVE(NVMEM)                                                                                        \
    do {                                                                                                             \
        _Pragma("unroll") for (int g_ = 0; g_ < 8; ++g_) {                                                           \
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);                                                       \
            if ((NVMEM) > 0) __builtin_amdgcn_sched_group_barrier(0x020, (NVMEM) / 8, 0);                            \
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);                                                       \
            __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);                                                       \
        }                                                                                                            \
    } while (0)

    // prologue: tiles 0 and 1 in flight, wait for tile 0, read its first half
    ld.issue(smem, 0, 0);
    ld.issue(smem, 1, 1);
    wait_vmcnt<16>();
    barrier_keep_loads();
    DPT_FRAGS(fa0, fb0, 0, 0);
    for (int kt = 0; kt < ktiles - 1; ++kt) {
        const int slot = kt & 1;
        DPT_MMA(fa0, fb0, 0);
        DPT_FRAGS(fa1, fb1, slot, 1);
        DPT_INTERLEAVE(0);
        __builtin_amdgcn_sched_barrier(0);
        // every fragment of tile kt is in registers: its slot takes tile kt+2
        // (past the end: the last tile again, never read)
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        barrier_keep_loads();
        __builtin_amdgcn_sched_barrier(0);
        const int refill = min(kt + 2, ktiles - 1);
        DPT_MMA(fa0, fb0, 1);
        ld.issue_rows(smem, refill, slot, 0, 4);
        DPT_VPIN(8);
        __builtin_amdgcn_sched_barrier(0);
        DPT_MMA(fa1, fb1, 0);
        ld.issue_rows(smem, refill, slot, 4, 8);
        DPT_VPIN(8);
        __builtin_amdgcn_sched_barrier(0);
        // tile kt+1 must have landed (only tile kt+2's 16 loads may be pending)
        wait_vmcnt<16>();
        barrier_keep_loads();
        __builtin_amdgcn_sched_barrier(0);
        DPT_MMA(fa1, fb1, 1);
        DPT_FRAGS(fa0, fb0, slot ^ 1, 0);
        DPT_INTERLEAVE(0);
        __builtin_amdgcn_sched_barrier(0);
    }
    DPT_MMA(fa0, fb0, 0);
    DPT_MMA(fa0, fb0, 1);
    DPT_FRAGS(fa1, fb1, (ktiles - 1) & 1, 1);
    DPT_MMA(fa1, fb1, 0);
    DPT_MMA(fa1, fb1, 1);
    wait_vmcnt<0>();
#undef DPT_VPIN
#undef DPT_INTERLEAVE
#undef DPT_MMA
#undef DPT_FRAGS
    epilogue<X3 ? EPI_X3 : EPI_BF16>(smem, acc, deltaT, Wold, Wnew, Wbnew, nullptr, nullptr, a, row0, col0, tid, lane,
                                     wave, wr, wc);
}

// ---------------------------------------------------------------------------
// FP32 step with v_mfma_f32_32x32x2_f32 (K = 2 per MFMA).  The K order inside a
// group of 8 values is permuted, identically for both operands: lane (fr, fg)
// loads 4 consecutive values k0 + 4 fg .. k0 + 4 fg + 3 of its row with one
// 16-byte read, and MFMA j of the group takes element j, so MFMA j sums over
// k0 + j and k0 + 4 + j and the four MFMAs cover the group once.  A K-tile (32
// values) is 4 groups of 64 MFMAs per wave; group g + 1's fragments (the other
// register set) are read while group g multiplies, pinned among its first
// MFMAs.  The barrier (tile kt+1 landed, tile kt fully read) sits in the middle
// of group 3; its second half reads tile kt+1's group 0.  The refill of the
// freed slot with tile kt+2 is spread over that half and groups 0 and 1 of the
// next K-tile (6, 6 and 4 of the 16 loads per thread): issued together, the
// loads of the four waves back up behind the CU's vector-memory path and stall
// the waves' MFMA issue.
__global__ __launch_bounds__(NT) void k_step_f32_large(const float *__restrict__ A, const float *__restrict__ B,
                                                       const float *__restrict__ deltaT, const float *__restrict__ Wold,
                                                       float *__restrict__ Wnew, StepArgs a, int tiles_m,
                                                       int tiles_n) {
    __shared__ __attribute__((aligned(16))) unsigned char smem[SMEM];
    int tm, tn;
    tile_coords<8>(blockIdx.x, gridDim.x, tiles_m, tiles_n, tm, tn);
    const int64_t row0 = (int64_t)tm * BM, col0 = (int64_t)tn * BN;
    const int ktiles = (int)(a.ld * 4 / ROW);  // a multiple of 8
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = wave / WN, wc = wave % WN;
    TileLoader ld;
    ld.init(A, B, row0, col0, a.ld * 4, wave, lane);

    floatx16_t acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    // group g of a K-tile = logical chunks 2g + fg of the row
    const int fr = lane & 31, fg = lane >> 5;
    const int ra = wr * WTM + fr, rb = wc * WTN + fr;
    const int a_base = ra * ROW + ((fg ^ key8(ra)) << 4);
    const int b_base = BM * ROW + rb * ROW + ((fg ^ key8(rb)) << 4);
    f32x4 fa[2][TM], fb[2][TN];
#define DPT_FRAGS32(BUF, SLOT, G)                                                                                    \
    do {                                                                                                             \
        const unsigned char *sb_ = smem + (SLOT) * STAGE;                                                            \
        _Pragma("unroll") for (int i_ = 0; i_ < TM; ++i_) fa[BUF][i_] = *reinterpret_cast<const f32x4 *>(           \
            sb_ + ((a_base + i_ * 32 * ROW) ^ ((((i_ & 1) << 2) ^ (2 * (G))) << 4)));                                \
        _Pragma("unroll") for (int j_ = 0; j_ < TN; ++j_) fb[BUF][j_] = *reinterpret_cast<const f32x4 *>(           \
            sb_ + ((b_base + j_ * 32 * ROW) ^ ((((j_ & 1) << 2) ^ (2 * (G))) << 4)));                                \
    } while (0)
#define DPT_MMA32(BUF, E0, E1)                                                                                       \
    do {                                                                                                             \
        _Pragma("unroll") for (int e_ = (E0); e_ < (E1); ++e_) _Pragma("unroll") for (int i_ = 0; i_ < TM; ++i_)    \
            _Pragma("unroll") for (int j_ = 0; j_ < TN; ++j_) acc[i_][j_] =                                          \
                __builtin_amdgcn_mfma_f32_32x32x2f32(fa[BUF][i_][e_], fb[BUF][j_][e_], acc[i_][j_], 0, 0, 0);        \
    } while (0)
    // 8 fragment reads among the first 16 MFMAs, NVMEM tile loads one per 4 MFMAs
#define DPT_PIN32(NVMEM)                                                                                             \
    do {                                                                                                             \
        _Pragma("unroll") for (int g_ = 0; g_ < 8; ++g_) {                                                           \
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);                                                       \
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);                                                       \
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);                                                       \
        }                                                                                                            \
        _Pragma("unroll") for (int g_ = 0; g_ < (NVMEM); ++g_) {                                                     \
            __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);                                                       \
            __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);                                                       \
        }                                                                                                            \
    } while (0)

    // prologue: tile 0 and the first rows of tile 1 in flight, wait for tile 0,
    // read its group 0
    ld.issue(smem, 0, 0);
    ld.issue_rows(smem, 1, 1, 0, 3);
    wait_vmcnt<6>();
    barrier_keep_loads();
    DPT_FRAGS32(0, 0, 0);
    for (int kt = 0; kt < ktiles - 1; ++kt) {
        const int slot = kt & 1;
        __builtin_amdgcn_sched_barrier(0);
        DPT_MMA32(0, 0, 4);
        DPT_FRAGS32(1, slot, 1);
        ld.issue_rows(smem, kt + 1, slot ^ 1, 3, 6);
        DPT_PIN32(6);
        __builtin_amdgcn_sched_barrier(0);
        DPT_MMA32(1, 0, 4);
        DPT_FRAGS32(0, slot, 2);
        ld.issue_rows(smem, kt + 1, slot ^ 1, 6, 8);
        DPT_PIN32(4);
        __builtin_amdgcn_sched_barrier(0);
        DPT_MMA32(0, 0, 4);
        DPT_FRAGS32(1, slot, 3);
        DPT_PIN32(0);
        __builtin_amdgcn_sched_barrier(0);
        DPT_MMA32(1, 0, 2);
        __builtin_amdgcn_sched_barrier(0);
        // every fragment of tile kt is in registers; tile kt+1 must have landed
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        wait_vmcnt<0>();
        barrier_keep_loads();
        __builtin_amdgcn_sched_barrier(0);
        DPT_MMA32(1, 2, 4);
        // start the refill of the freed slot (past the end: the last tile
        // again, never read)
        DPT_FRAGS32(0, slot ^ 1, 0);
        ld.issue_rows(smem, min(kt + 2, ktiles - 1), slot, 0, 3);
        DPT_PIN32(6);
        __builtin_amdgcn_sched_barrier(0);
    }
    {
        const int slot = (ktiles - 1) & 1;
        DPT_MMA32(0, 0, 4);
        DPT_FRAGS32(1, slot, 1);
        DPT_MMA32(1, 0, 4);
        DPT_FRAGS32(0, slot, 2);
        DPT_MMA32(0, 0, 4);
        DPT_FRAGS32(1, slot, 3);
        DPT_MMA32(1, 0, 4);
    }
    wait_vmcnt<0>();
#undef DPT_PIN32
#undef DPT_MMA32
#undef DPT_FRAGS32
    epilogue<EPI_F32>(smem, acc, deltaT, Wold, Wnew, nullptr, nullptr, nullptr, a, row0, col0, tid, lane, wave, wr, wc);
}

// ---------------------------------------------------------------------------
// FP8 step with the block-scaled v_mfma_scale_f32_32x32x64_f8f6f4 (E4M3 x E4M3,
// FP32 accumulate).  A K-tile is 128 values (one 128-byte line per row) plus
// the row's four E8M0 scales (one 4-byte word per row, kept after the A and B
// tiles of the stage).  Operand layout of one 64-value MFMA window: lane (r, g)
// (r = lane & 31, g = lane >> 5) holds values 16g .. 16g + 15 and 32 + 16g ..
// 32 + 16g + 15 of row r (chunks g and 2 + g of the window), and supplies the
// scale of its row's 32-value block g; each scale multiplies the values of its
// (row, block) wherever they sit.  The two windows of a K-tile go to two
// register sets, scheduled like the BF16 step's halves.
constexpr int STAGE8 = STAGE + (BM + BN) * 4;  // + 4 scale bytes per row
constexpr int LOADS8 = LOADS + 2;
static_assert(2 * STAGE8 <= SMEM, "two FP8 stages fit the epilogue tile");
typedef int i32x8 __attribute__((ext_vector_type(8)));

__global__ __launch_bounds__(NT) void k_step_fp8_large(const unsigned char *__restrict__ Aq,
                                                       const unsigned char *__restrict__ As,
                                                       const unsigned char *__restrict__ Bq,
                                                       const unsigned char *__restrict__ Bs,
                                                       const float *__restrict__ deltaT, const float *__restrict__ Wold,
                                                       float *__restrict__ Wnew, unsigned char *__restrict__ Wqnew,
                                                       unsigned char *__restrict__ Wsnew, StepArgs a, int tiles_m,
                                                       int tiles_n) {
    __shared__ __attribute__((aligned(16))) unsigned char smem[SMEM];
    int tm, tn;
    tile_coords<8>(blockIdx.x, gridDim.x, tiles_m, tiles_n, tm, tn);
    const int64_t row0 = (int64_t)tm * BM, col0 = (int64_t)tn * BN;
    const int64_t ldsc = a.ld / 32;             // scale bytes per row
    const int ktiles = (int)(a.ld / ROW);        // a multiple of 2
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = wave / WN, wc = wave % WN;
    TileLoader ld;
    ld.init(Aq, Bq, row0, col0, a.ld, wave, lane);
    // scale words: wave w loads rows 64w + lane of A and of B (4 bytes each)
    const unsigned char *gsa = As + (row0 + 64 * wave + lane) * ldsc, *gsb = Bs + (col0 + 64 * wave + lane) * ldsc;
    auto issue8 = [&](int kt, int slot) {
        ld.issue(smem + slot * (STAGE8 - STAGE), kt, slot);  // tiles at smem + slot * STAGE8
        unsigned char *sc = smem + slot * STAGE8 + STAGE + 64 * wave * 4;
        __builtin_amdgcn_global_load_lds((gbl_void *)(gsa + 4 * kt), (lds_void *)sc, 4, 0, 0);
        __builtin_amdgcn_global_load_lds((gbl_void *)(gsb + 4 * kt), (lds_void *)(sc + BM * 4), 4, 0, 0);
    };

    floatx16_t acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    const int fr = lane & 31, fg = lane >> 5;
    const int ra = wr * WTM + fr, rb = wc * WTN + fr;
    const int a_base = ra * ROW + ((fg ^ key8(ra)) << 4);
    const int b_base = BM * ROW + rb * ROW + ((fg ^ key8(rb)) << 4);
    i32x8 fa0[TM], fb0[TN], fa1[TM], fb1[TN];
    int sa0[TM], sb0[TN], sa1[TM], sb1[TN];
    // Fragments and scales of window W of the K-tile in SLOT: chunks 4W + fg and
    // 4W + 2 + fg of the lane's row; scale byte 2W + fg of the row's word.
#define DPT_FRAGS8(FA, FB, SA, SB, SLOT, W)                                                                          \
    do {                                                                                                             \
        const unsigned char *sb_ = smem + (SLOT) * STAGE8;                                                           \
        _Pragma("unroll") for (int i_ = 0; i_ < TM; ++i_) {                                                          \
            const int o_ = a_base + i_ * 32 * ROW, x_ = ((i_ & 1) << 2) ^ (4 * (W));                                 \
            const u32x4_t lo_ = *reinterpret_cast<const u32x4_t *>(sb_ + (o_ ^ (x_ << 4)));                          \
            const u32x4_t hi_ = *reinterpret_cast<const u32x4_t *>(sb_ + (o_ ^ ((x_ ^ 2) << 4)));                    \
            FA[i_] = i32x8{(int)lo_[0], (int)lo_[1], (int)lo_[2], (int)lo_[3],                                       \
                           (int)hi_[0], (int)hi_[1], (int)hi_[2], (int)hi_[3]};                                      \
            SA[i_] = (int)((*reinterpret_cast<const unsigned *>(sb_ + STAGE + 4 * (ra + 32 * i_)) >>                 \
                            (8 * (2 * (W) + fg))) & 0xffu);                                                          \
        }                                                                                                            \
        _Pragma("unroll") for (int j_ = 0; j_ < TN; ++j_) {                                                          \
            const int o_ = b_base + j_ * 32 * ROW, x_ = ((j_ & 1) << 2) ^ (4 * (W));                                 \
            const u32x4_t lo_ = *reinterpret_cast<const u32x4_t *>(sb_ + (o_ ^ (x_ << 4)));                          \
            const u32x4_t hi_ = *reinterpret_cast<const u32x4_t *>(sb_ + (o_ ^ ((x_ ^ 2) << 4)));                    \
            FB[j_] = i32x8{(int)lo_[0], (int)lo_[1], (int)lo_[2], (int)lo_[3],                                       \
                           (int)hi_[0], (int)hi_[1], (int)hi_[2], (int)hi_[3]};                                      \
            SB[j_] = (int)((*reinterpret_cast<const unsigned *>(sb_ + STAGE + BM * 4 + 4 * (rb + 32 * j_)) >>        \
                            (8 * (2 * (W) + fg))) & 0xffu);                                                          \
        }                                                                                                            \
    } while (0)
#define DPT_MMA8(FA, FB, SA, SB, I0)                                                                                 \
    do {                                                                                                             \
        _Pragma("unroll") for (int i_ = (I0); i_ < (I0) + 2; ++i_) _Pragma("unroll") for (int j_ = 0; j_ < TN; ++j_) \
            acc[i_][j_] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(FA[i_], FB[j_], acc[i_][j_], 0, 0, 0,      \
                                                                          SA[i_], 0, SB[j_]);                        \
    } while (0)

    issue8(0, 0);
    issue8(1, 1);
    wait_vmcnt<LOADS8>();
    barrier_keep_loads();
    DPT_FRAGS8(fa0, fb0, sa0, sb0, 0, 0);
    for (int kt = 0; kt < ktiles - 1; ++kt) {
        const int slot = kt & 1;
        DPT_MMA8(fa0, fb0, sa0, sb0, 0);
        __builtin_amdgcn_sched_barrier(0);
        DPT_MMA8(fa0, fb0, sa0, sb0, 2);
        DPT_FRAGS8(fa1, fb1, sa1, sb1, slot, 1);
        __builtin_amdgcn_sched_barrier(0);
        DPT_MMA8(fa1, fb1, sa1, sb1, 0);
        __builtin_amdgcn_sched_barrier(0);
        // every fragment of tile kt is in registers; tile kt+1 must have landed
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        wait_vmcnt<0>();
        barrier_keep_loads();
        __builtin_amdgcn_sched_barrier(0);
        DPT_MMA8(fa1, fb1, sa1, sb1, 2);
        issue8(min(kt + 2, ktiles - 1), slot);  // past the end: the last tile again, never read
        DPT_FRAGS8(fa0, fb0, sa0, sb0, slot ^ 1, 0);
        __builtin_amdgcn_sched_barrier(0);
    }
    DPT_MMA8(fa0, fb0, sa0, sb0, 0);
    DPT_MMA8(fa0, fb0, sa0, sb0, 2);
    DPT_FRAGS8(fa1, fb1, sa1, sb1, (ktiles - 1) & 1, 1);
    DPT_MMA8(fa1, fb1, sa1, sb1, 0);
    DPT_MMA8(fa1, fb1, sa1, sb1, 2);
    wait_vmcnt<0>();
#undef DPT_MMA8
#undef DPT_FRAGS8
    epilogue<EPI_FP8>(smem, acc, deltaT, Wold, Wnew, nullptr, Wqnew, Wsnew, a, row0, col0, tid, lane, wave, wr, wc);
}

// Block-scaled FP8 copy of an FP32 ld x ld matrix (rows of the padded layout);
// thread t quantises 4 consecutive values, 8 lanes one 32-value block.
__global__ __launch_bounds__(256) void k_quant_fp8(const float *__restrict__ src, int64_t ld,
                                                   unsigned char *__restrict__ q, unsigned char *__restrict__ sc) {
    const int64_t quads = ld * ld / 4;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < quads; t += (int64_t)gridDim.x * blockDim.x) {
        const f32x4 v = *reinterpret_cast<const f32x4 *>(src + 4 * t);
        const float v4[4] = {v[0], v[1], v[2], v[3]};
        unsigned s;
        *reinterpret_cast<unsigned *>(q + 4 * t) = quant_fp8_x4(v4, &s);
        if ((threadIdx.x & 7) == 0) sc[t / 8] = (unsigned char)s;
    }
}

}  // namespace

bool step_large_supported(int64_t ld) { return ld % BM == 0 && ld % BN == 0 && ld >= 1024; }

// The 256 x 256 tiles give (ld / 256)^2 workgroups, one per CU at a time: below
// one full wave over the 256 CUs (ld < 4096) the 128-wide tiles of the
// general kernels keep more of the chip busy.
bool step_large_preferred(int64_t ld) { return step_large_supported(ld) && ld >= 4096; }

hipError_t launch_step_bf16_large(const StepArgs &a, const __bf16 *Wb, const __bf16 *Deltab, const float *deltaT,
                                  const float *W, float *Wn, __bf16 *Wbn, hipStream_t s) {
    if (!step_large_supported(a.ld) || !Wbn) return hipErrorInvalidValue;
    const int tiles_m = (int)(a.ld / BM), tiles_n = (int)(a.ld / BN);
    hipLaunchKernelGGL(k_step_bf16_large<false>, dim3((unsigned int)(tiles_m * tiles_n)), dim3(NT), 0, s, Wb, Deltab,
                       deltaT, W, Wn, Wbn, a, tiles_m, tiles_n);
    return hipGetLastError();
}

hipError_t launch_step_x3_large(const StepArgs &a, const __bf16 *Wx3, const __bf16 *Dx3, const float *deltaT,
                                const float *W, float *Wn, __bf16 *Wx3n, hipStream_t s) {
    if (!step_large_supported(a.ld) || !Wx3n) return hipErrorInvalidValue;
    const int tiles_m = (int)(a.ld / BM), tiles_n = (int)(a.ld / BN);
    hipLaunchKernelGGL(k_step_bf16_large<true>, dim3((unsigned int)(tiles_m * tiles_n)), dim3(NT), 0, s, Wx3, Dx3,
                       deltaT, W, Wn, Wx3n, a, tiles_m, tiles_n);
    return hipGetLastError();
}

// Split form of an ld x ld FP32 matrix into the ld x 2 ld BF16 layout [h | l].
__global__ __launch_bounds__(256) void k_split_x3(const float *__restrict__ src, int64_t ld,
                                                  __bf16 *__restrict__ dst) {
    const int64_t total = ld * ld;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / ld, c = i - r * ld;
        const float x = src[i];
        const __bf16 h = (__bf16)x;
        __bf16 *row = dst + r * (2 * ld) + c;
        row[0] = h;
        row[ld] = (__bf16)(x - (float)h);
    }
}

hipError_t launch_split_x3(const float *src, int64_t ld, __bf16 *dst, hipStream_t s) {
    const int64_t total = ld * ld;
    const unsigned int blocks = (unsigned int)std::min<int64_t>((total + 255) / 256, 1 << 16);
    hipLaunchKernelGGL(k_split_x3, dim3(blocks), dim3(256), 0, s, src, ld, dst);
    return hipGetLastError();
}

hipError_t launch_step_fp8_large(const StepArgs &a, const unsigned char *Wq, const unsigned char *Ws,
                                 const unsigned char *Dq, const unsigned char *Ds, const float *deltaT, const float *W,
                                 float *Wn, unsigned char *Wqn, unsigned char *Wsn, hipStream_t s) {
    if (!step_large_supported(a.ld)) return hipErrorInvalidValue;
    const int tiles_m = (int)(a.ld / BM), tiles_n = (int)(a.ld / BN);
    hipLaunchKernelGGL(k_step_fp8_large, dim3((unsigned int)(tiles_m * tiles_n)), dim3(NT), 0, s, Wq, Ws, Dq, Ds,
                       deltaT, W, Wn, Wqn, Wsn, a, tiles_m, tiles_n);
    return hipGetLastError();
}

hipError_t launch_quant_fp8(const float *src, int64_t ld, unsigned char *q, unsigned char *sc, hipStream_t s) {
    if (ld % 32 != 0) return hipErrorInvalidValue;
    const int64_t quads = ld * ld / 4;
    const int64_t blocks = std::min<int64_t>((quads + 255) / 256, 1 << 16);
    hipLaunchKernelGGL(k_quant_fp8, dim3((unsigned int)blocks), dim3(256), 0, s, src, ld, q, sc);
    return hipGetLastError();
}

hipError_t launch_step_f32_large(const StepArgs &a, const float *W, const float *Delta, const float *deltaT,
                                 float *Wn, hipStream_t s) {
    if (!step_large_supported(a.ld)) return hipErrorInvalidValue;
    const int tiles_m = (int)(a.ld / BM), tiles_n = (int)(a.ld / BN);
    hipLaunchKernelGGL(k_step_f32_large, dim3((unsigned int)(tiles_m * tiles_n)), dim3(NT), 0, s, W, Delta, deltaT,
                       W, Wn, a, tiles_m, tiles_n);
    return hipGetLastError();
}

}  // namespace dpt
