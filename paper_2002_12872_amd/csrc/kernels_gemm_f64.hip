// Fused FP64 D-PT step for large dense problems on gfx950 (ld a multiple of
// 128, ld >= 2048; chosen where measured faster): the optional FP64 sweeps, the
// stage solves of the homotopy continuation and FP64 solves of large problems.
//
// One application of eq. (dyn) of Kenmoe, Smerlak, Zadorin (arXiv:2002.12872)
// on the padded state W = A - I, all in FP64:
//     C  = Delta^T + W Delta^T                               (v_mfma_f64_16x16x4_f64)
//     W' = lambda (C - d_n W) / (theta_n - theta_m),  m != n
// plus max|W' - W| and max|W'| for the stopping rule.
//
// Structure.  A 128 x 128 output tile per workgroup of 4 waves, each wave a
// 64 x 64 wave tile as 4 x 4 blocks of 16 x 16 accumulators (four doubles per
// lane per block: 128 accumulator registers), so that two workgroups share a
// CU (two waves per SIMD hide each other's waits).  K advances in tiles of 16
// doubles (one 128-byte cache line per row) through a 2-stage LDS ring of
// 32 KiB per stage (128 rows of W, then 128 rows of Delta) filled by direct
// global->LDS loads; 16-byte chunk c of
// tile row r sits at slot c ^ key8(r).  Operand layout of the 16x16x4 FP64
// MFMA: lane l supplies row l % 16 of its 16-row block and the K value of group
// l / 16.  Lane group g reads chunk 4h + g (doubles 8h + 2g, 8h + 2g + 1) of
// its row in half h of the K-tile, and MFMA (h, e) takes element e: it sums
// over K = {8h + 2g + e : g = 0..3}, so the two halves and two elements cover
// the 16 values of the K-tile once, in the same order for both operands; one
// half's fragments are read while the other half multiplies.
// An FP64 MFMA takes 64 cycles, so a K-tile is 64 MFMAs (4096 cycles) per wave
// against 32 KiB of operands per workgroup: the ring has a whole K-tile of work
// to cover each refill.  The epilogue stages the accumulators through the freed
// LDS.
#include <float.h>

#include <algorithm>

#include "device_common.h"
#include "dpt_internal.h"

namespace dpt {
namespace {

constexpr int BM = 128, BN = 128;
constexpr int ROW = 128;                 // bytes of one tile row per K-tile (16 doubles)
constexpr int STAGE = (BM + BN) * ROW;   // 32 KiB
constexpr int NT = 256;                  // 4 waves
constexpr int WN = 2;                    // wave grid 2 x 2
constexpr int WTM = 64, WTN = 64;        // wave tile
constexpr int TM = WTM / 16, TN = WTN / 16;  // 4 x 4 blocks of 16 x 16
constexpr int A_LOADS = BM / 32, B_LOADS = BN / 32;  // 8-row load instructions per wave: 4 and 4
constexpr int LOADS = A_LOADS + B_LOADS;             // per thread per stage
constexpr int EPI_ROWS = 64, EPI_PITCH = 130;        // epilogue pass: 64 tile rows, padded pitch (doubles)
constexpr int SMEM = 2 * STAGE > EPI_ROWS * EPI_PITCH * 8 ? 2 * STAGE : EPI_ROWS * EPI_PITCH * 8;

typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) const void gbl_void;
typedef double f64x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int key8(int r) { return (r ^ (r >> 3)) & 7; }

template <int N>
__device__ __forceinline__ void wait_vmcnt() {
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

__device__ __forceinline__ void barrier_keep_loads() { asm volatile("s_barrier" ::: "memory"); }

// Global->LDS loads of one K-tile.  Wave w fills A rows [32w, 32w + 32) and B
// rows [32w, 32w + 32), 8 rows per instruction; lane L lands at byte 16 L of
// the instruction's 1 KiB: row 8i + (L >> 3) of the instruction's rows,
// physical slot L & 7, so it reads logical chunk (L & 7) ^ key8(row), and
// key8(32w + 8i + lr) = lr ^ ((4w + i) & 7).  Each lane keeps the source of
// its A rows, so with a row map tile row r reads W row rowmap[row0 + r] (a
// padding entry, -1, reads row 0, whose products are not stored).
struct Loader {
    const unsigned char *pa[A_LOADS];
    const unsigned char *gb;
    int64_t ldb;
    int lane_off;
    int wave;

    __device__ void init(const double *A, const double *B, const int32_t *rowmap, int64_t row0, int64_t col0,
                         int64_t ld_bytes, int w, int lane) {
        ldb = ld_bytes;
        wave = w;
        gb = (const unsigned char *)B + (col0 + 32 * w) * ldb;
        const int lr = lane >> 3;
        lane_off = lr * (int)ldb + (((lane & 7) ^ lr) << 4);
#pragma unroll
        for (int i = 0; i < A_LOADS; ++i) {
            int64_t r = row0 + 32 * w + 8 * i + lr;
            if (rowmap) r = max(rowmap[r], 0);
            pa[i] = (const unsigned char *)A + r * ldb + ((((lane & 7) ^ lr) ^ ((4 * w + i) & 7)) << 4);
        }
    }
    __device__ __forceinline__ void issue(unsigned char *smem, int kt, int slot) const {
        unsigned char *sa = smem + slot * STAGE + 32 * wave * ROW;
        unsigned char *sb = smem + slot * STAGE + BM * ROW + 32 * wave * ROW;
        const int64_t ko = (int64_t)kt * ROW;
#pragma unroll
        for (int i = 0; i < A_LOADS; ++i)
            __builtin_amdgcn_global_load_lds((gbl_void *)(pa[i] + ko), (lds_void *)(sa + i * 8 * ROW), 16, 0, 0);
#pragma unroll
        for (int i = 0; i < B_LOADS; ++i)
            __builtin_amdgcn_global_load_lds(
                (gbl_void *)(gb + ko + 8 * i * ldb + (lane_off ^ (((4 * wave + i) & 7) << 4))),
                (lds_void *)(sb + i * 8 * ROW), 16, 0, 0);
    }
};

__global__ __launch_bounds__(NT, 2) void k_step_f64_large(const double *__restrict__ A, const double *__restrict__ B,
                                                       const double *__restrict__ deltaT,
                                                       const double *__restrict__ Wold, double *__restrict__ Wnew,
                                                       StepArgs a, int tiles_m, int tiles_n) {
    __shared__ __attribute__((aligned(16))) unsigned char smem[SMEM];
    int tm, tn;
    tile_coords<8>(blockIdx.x, gridDim.x, tiles_m, tiles_n, tm, tn);
    const int64_t row0 = (int64_t)tm * BM, col0 = (int64_t)tn * BN;
    const int ktiles = (int)(a.ld * 8 / ROW);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = wave / WN, wc = wave % WN;
    Loader ld;
    ld.init(A, B, a.rowmap, row0, col0, a.ld * 8, wave, lane);

    doublex4_t acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[i][j][r] = 0.0;

    const int fr = lane & 15, fg = lane >> 4;
    const int a_row = wr * WTM + fr, b_row = wc * WTN + fr;
    // two fragment sets: half h of a K-tile goes to set h, read while the other
    // set multiplies
    f64x2 fa[2][TM], fb[2][TN];
#define DPT_FRAGS64(SET, SLOT, H)                                                                                    \
    do {                                                                                                             \
        const unsigned char *sb_ = smem + (SLOT) * STAGE;                                                            \
        _Pragma("unroll") for (int i_ = 0; i_ < TM; ++i_) {                                                          \
            const int r_ = a_row + 16 * i_;                                                                          \
            fa[SET][i_] = *reinterpret_cast<const f64x2 *>(sb_ + r_ * ROW + (((4 * (H) + fg) ^ key8(r_)) << 4));   \
        }                                                                                                            \
        _Pragma("unroll") for (int j_ = 0; j_ < TN; ++j_) {                                                          \
            const int r_ = b_row + 16 * j_;                                                                          \
            fb[SET][j_] =                                                                                            \
                *reinterpret_cast<const f64x2 *>(sb_ + BM * ROW + r_ * ROW + (((4 * (H) + fg) ^ key8(r_)) << 4));   \
        }                                                                                                            \
    } while (0)
#define DPT_MMA64(SET)                                                                                               \
    do {                                                                                                             \
        _Pragma("unroll") for (int e_ = 0; e_ < 2; ++e_) _Pragma("unroll") for (int i_ = 0; i_ < TM; ++i_)          \
            _Pragma("unroll") for (int j_ = 0; j_ < TN; ++j_) acc[i_][j_] =                                          \
                __builtin_amdgcn_mfma_f64_16x16x4f64(fa[SET][i_][e_], fb[SET][j_][e_], acc[i_][j_], 0, 0, 0);        \
    } while (0)

    ld.issue(smem, 0, 0);
    if (ktiles > 1) ld.issue(smem, 1, 1);
    if (ktiles > 1)
        wait_vmcnt<LOADS>();
    else
        wait_vmcnt<0>();
    barrier_keep_loads();
    DPT_FRAGS64(0, 0, 0);
    for (int kt = 0; kt < ktiles; ++kt) {
        const int slot = kt & 1;
        DPT_FRAGS64(1, slot, 1);
        DPT_MMA64(0);
        __builtin_amdgcn_sched_barrier(0);
        // every fragment of tile kt is in registers: its slot takes tile kt + 2;
        // tile kt + 1 (issued a K-tile earlier) must have landed
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        barrier_keep_loads();
        if (kt + 2 < ktiles) {
            ld.issue(smem, kt + 2, slot);
            wait_vmcnt<LOADS>();
        } else {
            wait_vmcnt<0>();
        }
        barrier_keep_loads();
        __builtin_amdgcn_sched_barrier(0);
        if (kt + 1 < ktiles) DPT_FRAGS64(0, slot ^ 1, 0);
        DPT_MMA64(1);
        __builtin_amdgcn_sched_barrier(0);
    }
#undef DPT_MMA64
#undef DPT_FRAGS64

    // Epilogue through LDS in two passes of 64 tile rows: the two waves owning
    // the rows store their accumulators (register r of lane l in block (i, j) is
    // C[16 i + 4 r + (l >> 4)][16 j + (l & 15)] of the wave tile) into a 64 x 128
    // tile (row pitch 130 doubles); then every thread updates 16 rows x 2
    // columns with 16-byte accesses (a wave covers one whole 1 KiB output row).
    double *tile = reinterpret_cast<double *>(smem);
    constexpr int TP = EPI_PITCH;
    const double lam = a.lambda;
    const int64_t ldd = a.ld;
    const int c2 = 2 * (tid & 63);
    const int64_t m0 = col0 + c2;
    const double th0 = a.theta[m0], th1 = a.theta[m0 + 1];
    double dmax = 0.0, wmax = 0.0;
    bool bad = false;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        __syncthreads();
        if (wr == p) {
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        tile[(16 * i + 4 * r + (lane >> 4)) * TP + wc * WTN + 16 * j + (lane & 15)] = acc[i][j][r];
        }
        __syncthreads();
#pragma unroll 4
        for (int k = 0; k < 16; ++k) {
            const int row = wave + 4 * k;
            int64_t n = row0 + 64 * p + row;
            if (a.rowmap) {
                n = a.rowmap[n];
                if (n < 0) continue;  // padding of the row list
            }
            const int64_t idx = n * ldd + m0;
            const f64x2 dt = *reinterpret_cast<const f64x2 *>(&deltaT[idx]);
            const f64x2 wo = *reinterpret_cast<const f64x2 *>(&Wold[idx]);
            const f64x2 cv = *reinterpret_cast<const f64x2 *>(&tile[row * TP + c2]);
            const double th_n = a.theta[n], dn = a.d[n];
            f64x2 w;
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int64_t m = m0 + e;
                w[e] = 0.0;
                if (n < a.n && m < a.n && n != m) w[e] = lam * ((cv[e] + dt[e]) - dn * wo[e]) / (th_n - (e ? th1 : th0));
                const double dv = fabs(w[e] - wo[e]), av = fabs(w[e]);
                dmax = fmax(dmax, dv);
                wmax = fmax(wmax, av);
                bad |= !(dv <= DBL_MAX) || !(av <= DBL_MAX);
            }
            *reinterpret_cast<f64x2 *>(&Wnew[idx]) = w;
        }
    }
    publish_stats(a.stat, dmax, wmax, bad);
}

}  // namespace

bool step_f64_large_supported(int64_t ld) { return ld % BM == 0 && ld % BN == 0 && ld >= 2048; }

// Measured against the general kernels: faster from ld 4096 on (N = 16384:
// 128 ms against 140), and below where its tiles make whole waves at one
// workgroup per CU (ld 2048: 0.33 ms against 0.38); slower or level at
// 1024-1536 and at 3072-3584, whose last wave is mostly empty.
bool step_f64_large_preferred(int64_t ld) {
    if (!step_f64_large_supported(ld)) return false;
    return ld >= 4096 || ((ld / BM) * (ld / BN)) % 256 == 0;
}

// With a row map (a.rows entries, a multiple of BM) the tile rows run over the
// listed W rows only.
hipError_t launch_step_f64_large(const StepArgs &a, const double *W, const double *Delta, const double *deltaT,
                                 double *Wn, hipStream_t s) {
    if (!step_f64_large_supported(a.ld) || (a.rowmap && (a.rows < BM || a.rows % BM != 0 || a.rows > a.ld)))
        return hipErrorInvalidValue;
    const int tiles_m = (int)((a.rowmap ? a.rows : a.ld) / BM), tiles_n = (int)(a.ld / BN);
    hipLaunchKernelGGL(k_step_f64_large, dim3((unsigned int)(tiles_m * tiles_n)), dim3(NT), 0, s, W, Delta, deltaT,
                       W, Wn, a, tiles_m, tiles_n);
    return hipGetLastError();
}

}  // namespace dpt
