// Internal launch interface between the host runtime and the HIP kernels.
// Not part of the public ABI (include/dpt.h).
//
// Device state layout (dense path): all N x N matrices are stored padded to
// ld x ld (ld a multiple of 64), row-major, zero outside the leading N x N
// block.  The eigenvector state is W = Z - I (zero diagonal): row n of Z is the
// candidate eigenvector z_n in the chart z_n[n] = 1 (Sec. II.B of the paper).
// Sparse path: the state is stored transposed, WT[m * ld + n] = W[n][m], so that
// one CSR non-zero of Delta touches a contiguous run of eigenvectors.
#pragma once

#include <stddef.h>

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dpt.h"

namespace dpt {

// stats slot layout: two u64 per step, holding the bit patterns of non-negative
// doubles so that unsigned max equals numeric max (NaN sorts above +inf):
//   slot[0] = delta_k = max |W_k - W_{k-1}|,  slot[1] = max |W_k|.
constexpr int kStatRing = 4096;

enum Phase { PH_BF16 = 0, PH_FP32 = 1, PH_FP64 = 2 };

// Optional timing hook: begin/end bracket one kernel launch of a class
// (DPT_PROF_* in dpt.h) on a stream.
struct ProfHook {
    virtual void begin(int kind, hipStream_t s) = 0;
    virtual void end(hipStream_t s) = 0;
    virtual ~ProfHook() {}
};

struct StepArgs {
    int64_t n;                 // valid order N
    int64_t ld;                // padded leading dimension
    double lambda;
    const double *theta;       // ld entries (pad entries arbitrary but finite)
    const double *d;           // ld entries: d_n = (Delta z_n)[n] of the current state
    unsigned long long *stat;  // 2 u64 for this step (zeroed before the step)
    // Per-row retirement: when rowmap is set, the step covers only the rows
    // rowmap[0 .. rows) (rows a multiple of the product tile; -1 marks padding
    // entries, which are neither read as rows nor written).  NULL: all ld rows.
    const int32_t *rowmap = nullptr;
    int64_t rows = 0;
};

// ---- dense kernels (kernels_dense.hip) -----------------------------------
hipError_t launch_zero_u64(unsigned long long *p, int64_t count, hipStream_t s);
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s);
// Clears count (<= kZeroMany) buffers of bytes[i] (multiples of 4) in one launch.
constexpr int kZeroMany = 8;
hipError_t launch_zero_many(void *const *ptrs, const size_t *bytes, int count, hipStream_t s);

// dst (ld x ld, Tdst) <- src (n x n row-major, Tsrc) with zero padding.
hipError_t launch_pad_copy_f32_from_f32(float *dst, const float *src, int64_t n, int64_t ld, hipStream_t s);
hipError_t launch_pad_copy_f32_from_f64(float *dst, const double *src, int64_t n, int64_t ld, hipStream_t s);
hipError_t launch_pad_copy_f64_from_f64(double *dst, const double *src, int64_t n, int64_t ld, hipStream_t s);
hipError_t launch_pad_copy_f64_from_f32(double *dst, const float *src, int64_t n, int64_t ld, hipStream_t s);
// Start state from a caller-given Z (n x n): W = Z - I with the diagonal forced to 0.
hipError_t launch_load_state_f32(float *W, const void *z0, int z0_is_f64, int64_t n, int64_t ld, hipStream_t s);
hipError_t launch_load_state_f64(double *W, const void *z0, int z0_is_f64, int64_t n, int64_t ld, hipStream_t s);

hipError_t launch_cvt_f32_to_bf16(__bf16 *dst, const float *src, int64_t count, hipStream_t s);
hipError_t launch_cvt_f32_to_f64(double *dst, const float *src, int64_t count, hipStream_t s);
hipError_t launch_transpose_f32(float *dst, const float *src, int64_t ld, hipStream_t s);
hipError_t launch_transpose_f64(double *dst, const double *src, int64_t ld, hipStream_t s);
// Per-row retirement helpers: out[i] = max_m |Wn[r][m] - Wo[r][m]| for the
// mapped rows r = rowmap[i] (i < rows; padding entries give -1), and a copy of
// the listed rows from src to dst.
hipError_t launch_row_delta_f32(const float *Wn, const float *Wo, const int32_t *rowmap, int64_t rows, int64_t ld,
                                double *out, hipStream_t s);
hipError_t launch_row_delta_f64(const double *Wn, const double *Wo, const int32_t *rowmap, int64_t rows, int64_t ld,
                                double *out, hipStream_t s);
hipError_t launch_copy_rows_f32(float *dst, const float *src, const int32_t *rows, int64_t count, int64_t ld,
                                hipStream_t s);
hipError_t launch_copy_rows_f64(double *dst, const double *src, const int32_t *rows, int64_t count, int64_t ld,
                                hipStream_t s);
// Tile height of the products when a row map is in use: the row list is
// padded to a multiple of it (at most ld).
inline int64_t row_tile(int64_t ld) { return ld % 128 == 0 ? 128 : 64; }
// Large-tile FP64 step (kernels_gemm_f64.hip): ld a multiple of 128, ld >= 2048;
// preferred: where it is measured faster than the general kernels.
bool step_f64_large_supported(int64_t ld);
bool step_f64_large_preferred(int64_t ld);
hipError_t launch_step_f64_large(const StepArgs &a, const double *W, const double *Delta, const double *deltaT,
                                 double *Wn, hipStream_t s);
// C[i][j] = sum_k A[i][k] B[j][k] for ld x ld FP64 operands (ld a multiple of 64).
hipError_t launch_gemm_nt_f64(const double *A, const double *B, double *C, int64_t ld, hipStream_t s);
// *flag |= 1 when src != src^T anywhere (bitwise).  flag must be zeroed first.
// Exact symmetry test of the padded ld x ld matrix (sets *flag on a difference);
// when bf is not null the same pass writes bf16(src) into bf (ld x ld).
hipError_t launch_symmetry_check_f32(const float *src, int64_t ld, unsigned int *flag, __bf16 *bf, hipStream_t s);
hipError_t launch_symmetry_check_f64(const double *src, int64_t ld, unsigned int *flag, hipStream_t s);

// First application of F from A = I: W_1[n][m] = lambda Delta[m][n] / (theta_n - theta_m).
// Up to nsteps steps of a dense problem with ld = 64 in one workgroup: iterate
// s + 1 into hist + s * 64 * 64, its statistics into ring slot (k0 + s) mod
// kStatRing (first step in closed form when at_identity).  The batch ends after
// a step with delta < stop_below, a non-finite delta or max|W| > blowup; the
// last iterate computed is also written over Wcur.
hipError_t launch_small_steps_f32(float *Wcur, float *hist, const float *D, const float *DT, const StepArgs &a,
                                  unsigned long long *stats, int64_t k0, int nsteps, int at_identity, double *d,
                                  double stop_below, double blowup, hipStream_t s);
hipError_t launch_small_steps_f64(double *Wcur, double *hist, const double *D, const double *DT,
                                  const StepArgs &a, unsigned long long *stats, int64_t k0, int nsteps,
                                  int at_identity, double *d, double stop_below, double blowup, hipStream_t s);
hipError_t launch_first_iterate_f32(const StepArgs &a, const float *deltaT, float *W, __bf16 *Wb, hipStream_t s);
hipError_t launch_first_iterate_f64(const StepArgs &a, const double *deltaT, double *W, hipStream_t s);

// d_n = Delta[n][n] + sum_k W[n][k] Delta[n][k] (FP64 accumulation); E_n = theta_n + lambda d_n
// when E != NULL.  stat_clear (may be NULL) is zeroed (2 u64).
hipError_t launch_prepass_f32_f32(const float *W, const float *D, const StepArgs &a, double *d, double *E,
                                  unsigned long long *stat_clear, hipStream_t s);
hipError_t launch_prepass_f32_f64(const float *W, const double *D, const StepArgs &a, double *d, double *E,
                                  unsigned long long *stat_clear, hipStream_t s);
hipError_t launch_prepass_f64_f64(const double *W, const double *D, const StepArgs &a, double *d, double *E,
                                  unsigned long long *stat_clear, hipStream_t s);

// One fused step: C = W Delta^T on MFMA, then
//   W'[n][m] = lambda (Delta[m][n] + C[n][m] - d_n W[n][m]) / (theta_n - theta_m)   (m != n)
// and the stats.  BF16: A = Wb, B = Deltab, epilogue in FP32 with W (FP32) and
// deltaT (FP32); writes W' (FP32) and Wb' (BF16).
hipError_t launch_step_bf16(const StepArgs &a, const __bf16 *Wb, const __bf16 *Deltab, const float *deltaT,
                            const float *W, float *Wn, __bf16 *Wbn, hipStream_t s);
// Large-problem BF16 and FP32 steps (kernels_gemm_large.hip): 256 x 256 tiles,
// 4 waves of 128 x 128, K-tiles of 128 bytes per row through a 2-stage direct
// global->LDS ring.  Require ld % 256 == 0 and ld >= 1024; the BF16 one also
// writes the BF16 shadow (Wbn != NULL).
bool step_large_supported(int64_t ld);
// Whether the 256 x 256 tiles fill the chip at this order (ld >= 4096).
bool step_large_preferred(int64_t ld);
hipError_t launch_step_bf16_large(const StepArgs &a, const __bf16 *Wb, const __bf16 *Deltab, const float *deltaT,
                                  const float *W, float *Wn, __bf16 *Wbn, hipStream_t s);
// Split BF16 form (DPT_BF16_X3): operands ld x 2ld, A = [Wh | Wl], B = [Dh | Dl],
// product Wh Dh^T + Wl Dh^T + Wh Dl^T; writes W' (FP32) and its split form in
// the layout of A.
hipError_t launch_step_x3_large(const StepArgs &a, const __bf16 *Wx3, const __bf16 *Dx3, const float *deltaT,
                                const float *W, float *Wn, __bf16 *Wx3n, hipStream_t s);
// ld x ld FP32 -> ld x 2ld BF16 [h | l], h = bf16(x), l = bf16(x - h).
hipError_t launch_split_x3(const float *src, int64_t ld, __bf16 *dst, hipStream_t s);
hipError_t launch_step_f32_large(const StepArgs &a, const float *W, const float *Delta, const float *deltaT,
                                 float *Wn, hipStream_t s);
// FP8 step (large problems only): A = block-scaled FP8 copy of W (Wq values,
// Ws E8M0 scales per 32 values of a row), B = the same of Delta; epilogue in
// FP32 with W; writes W' (FP32) and its FP8 copy (Wqn, Wsn).
hipError_t launch_step_fp8_large(const StepArgs &a, const unsigned char *Wq, const unsigned char *Ws,
                                 const unsigned char *Dq, const unsigned char *Ds, const float *deltaT, const float *W,
                                 float *Wn, unsigned char *Wqn, unsigned char *Wsn, hipStream_t s);
// Block-scaled FP8 copy (E4M3 values, E8M0 scale per 32 values) of an FP32
// ld x ld matrix; ld a multiple of 32.
hipError_t launch_quant_fp8(const float *src, int64_t ld, unsigned char *q, unsigned char *sc, hipStream_t s);
hipError_t launch_step_f32(const StepArgs &a, const float *W, const float *Delta, const float *deltaT,
                           float *Wn, __bf16 *Wbn, hipStream_t s);
hipError_t launch_step_f64(const StepArgs &a, const double *W, const double *Delta, const double *deltaT,
                           double *Wn, hipStream_t s);

// Z export: out[i*n + j] = (i == j) ? 1 : W[i*ld + j], as float or double.
hipError_t launch_export_f32(const float *W, int64_t n, int64_t ld, void *out, int out_f64, hipStream_t s);
hipError_t launch_export_f64(const double *W, int64_t n, int64_t ld, void *out, int out_f64, hipStream_t s);

// Residual check (FP64): for each of nrows eigenvector rows r, partial sums of
// |(M z)_m - E z_m|^2 over m-chunks into part[r * nchunks + c].
int residual_chunks(int64_t ld);
hipError_t launch_residual_f32(const float *W, const void *D, int d_is_f64, const StepArgs &a,
                               const int64_t *rows, int64_t nrows, const double *E, double *part, hipStream_t s);
hipError_t launch_residual_f64(const double *W, const void *D, int d_is_f64, const StepArgs &a,
                               const int64_t *rows, int64_t nrows, const double *E, double *part, hipStream_t s);

// ---- serving: grouped persistent kernels (kernels_dense.hip) ---------------
// One in-flight request as the grouped kernels see it (dense, padded to ld, a
// multiple of 64; state W = Z - I in FP32 with a BF16 shadow in the BF16 phase).
struct GroupReq {
    const __bf16 *Wb;           // current BF16 state (BF16 phase)
    const __bf16 *Db;           // BF16 Delta
    const float *W;             // current FP32 state
    const float *D;             // FP32 Delta, row-major
    const float *DT;            // FP32 Delta^T (== D when symmetric)
    float *Wn;                  // next FP32 state
    __bf16 *Wbn;                // next BF16 state (BF16 phase), else null
    const double *theta;        // ld entries
    double *d;                  // ld entries, d_n of the current state
    unsigned long long *stat;   // 2 u64: delta, max|W|
    int64_t n, ld;
    double lambda;
};

constexpr int kServeMaxSlots = 1024;

// Work lists of one serving step, rewritten by the host before every step.
// Output tile shapes of the grouped fused step (rows x columns): shape 0 is
// 64 x 64, 1 is 128 x 64, 2 is 128 x 128 (shapes 1 and 2 need ld % 128 == 0).
// The fused-step work is split into kGroupLists lists by (phase, shape): list
// kGroupShapes * (phase == PH_FP32) + shape.  counts[0] = requests,
// counts[1 + L] = requests in list L; prefix arrays hold running sums of rows
// (pre-pass) and of output tiles (step kernels).
constexpr int kGroupShapes = 3;
constexpr int group_shape_rows(int shape) { return shape == 0 ? 64 : 128; }
constexpr int group_shape_cols(int shape) { return shape == 2 ? 128 : 64; }
constexpr int kGroupLists = 2 * kGroupShapes;
inline int group_list(int phase, int shape) { return kGroupShapes * (phase == PH_FP32 ? 1 : 0) + shape; }

struct GroupTable {
    int32_t counts[1 + kGroupLists];
    int32_t pre_prefix[kServeMaxSlots + 1];
    int32_t idx[kGroupLists][kServeMaxSlots];
    int32_t prefix[kGroupLists][kServeMaxSlots + 1];
    GroupReq reqs[kServeMaxSlots];
};

// Admission of newly placed requests, one launch for all of them: the padded
// FP32 Delta (and its BF16 copy, and its transpose unless DT is null: symmetric
// problems alias DT to D), theta padded with zeros (when theta_src is not the
// padded copy itself), and the closed-form first iterate F(I) with its BF16
// shadow and statistics (skipped when W1 is null).  src is the n x n row-major
// Delta (row stride n) in FP32 or FP64; theta_src has n entries; stat must be
// zero.  Work items are the 64 x 64 tiles of each request's padded order.
struct AdmitReq {
    const void *src;
    const double *theta_src;
    double *theta;              // ld entries
    float *D, *DT;              // DT null: symmetric (DT == D)
    __bf16 *Db;                 // null: FP32 request
    float *W1;                  // first iterate, or null
    __bf16 *Wb1;                // its BF16 shadow, or null
    unsigned long long *stat;   // 2 u64 (delta, max|W|), zero on entry
    int64_t n, ld;
    double lambda;
    int32_t src_f64, pad_;
};
struct AdmitTable {
    int32_t count, pad_;
    int32_t prefix[kServeMaxSlots + 1];  // running sums of 64 x 64 tiles
    AdmitReq reqs[kServeMaxSlots];
};
// Retirement, one launch for all finishing requests: E_n = theta_n + lambda d_n
// of the current state into E (n entries per request) and the request's stats
// cleared for the slot's next user.  One wave per (request, row).
struct RetireReq {
    const float *W, *D;
    const double *theta;
    double *E;
    unsigned long long *stat;
    int64_t n, ld;
    double lambda;
};
struct RetireTable {
    int32_t count, pad_;
    int32_t prefix[kServeMaxSlots + 1];  // running sums of rows
    RetireReq reqs[kServeMaxSlots];
};
hipError_t launch_group_admit(const AdmitTable *t, int grid, hipStream_t s);
// Input checks shared with the single-problem entry points (dpt_api.cpp): theta
// finite and pairwise distinct (host array); theta and Delta of a DPT_MEM_DEVICE
// dense problem are device allocations.
bool host_theta_ok(const double *theta, int64_t n);
// Pinned host blocks of at least 64 KiB, recycled across calls (dpt_api.cpp):
// read-back destinations that make device-to-host copies plain DMAs.  take()
// returns null when none can be allocated; give back only after the stream
// that used the block has drained.
void *pinned_block_take();
void pinned_block_give(void *p);
// Device buffers from the library's pool (dpt_api.cpp): blocks up to 4 MiB are
// recycled instead of going through hipMalloc / hipFree (several microseconds
// each); larger ones are plain allocations.  Free only after the stream that
// used the block has drained.
hipError_t pooled_malloc(void **p, size_t bytes);
void pooled_free(void *p);
bool inputs_on_device(const dpt_problem *p);
hipError_t launch_group_retire(const RetireTable *t, int grid, hipStream_t s);
// bytes (a multiple of 8) of a table in coherent pinned host memory, read by a
// kernel through src (the allocation's device pointer), into dst on the device.
hipError_t launch_fetch_table(const void *src, void *dst, size_t bytes, hipStream_t s);
static_assert(offsetof(GroupTable, reqs) % 8 == 0 && sizeof(GroupReq) % 8 == 0, "tables move in 8-byte words");
static_assert(offsetof(AdmitTable, reqs) % 8 == 0 && sizeof(AdmitReq) % 8 == 0, "tables move in 8-byte words");
static_assert(offsetof(RetireTable, reqs) % 8 == 0 && sizeof(RetireReq) % 8 == 0, "tables move in 8-byte words");

// Persistent grouped launches with a fixed grid (graph-capturable): the
// pre-pass (also clears each request's stats) and the fused step for the
// requests of one phase (PH_BF16 or PH_FP32) with one tile shape.
hipError_t launch_group_prepass(const GroupTable *t, int grid, hipStream_t s);
hipError_t launch_group_step(const GroupTable *t, int phase, int shape, int grid, hipStream_t s);

}  // namespace dpt
