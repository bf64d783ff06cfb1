// Internal interface of the CSR (sparse Delta) path and of the single-vector
// dominant-eigenvector mode.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dpt.h"
#include "dpt_internal.h"

namespace dpt {

struct SparseState;

// Padded order of the transposed sparse-path state (a multiple of 64).
int64_t sparse_pad_order(int64_t n);

// Stage the CSR Delta of p and allocate the transposed state ZT (Z[n][m] at
// panel-major offset, unit diagonal included; two buffers, FP32 or FP64, both
// starting as the identity).  Device CSR arrays are checked on the device and
// borrowed (values too when their dtype matches the state); host arrays are
// checked on the host and copied.  Returns DPT_OK, DPT_EINVAL for a malformed
// CSR, DPT_ENOMEM or DPT_EDEVICE; *out is NULL on failure.
int sparse_create(SparseState **out, const dpt_problem *p, bool fp64, int64_t ld, hipStream_t s);
void sparse_destroy(SparseState *sp);

// One application of eq. (dyn) with the CSR product; stats go to ring slot *k
// of `stats` (2 u64 per slot), then *k is incremented.
int sparse_step(SparseState *sp, double lambda, const double *theta, unsigned long long *stats, int64_t *k,
                hipStream_t s, ProfHook *prof);

// E_n = theta_n + lambda (Delta z_n)[n] of the current iterate, into evec (device).
hipError_t sparse_eigenvalues(SparseState *sp, double lambda, const double *theta, double *evec, hipStream_t s);

// out[i * n + j] = Z[i][j] (eigenvector i), float or double, device memory.
hipError_t sparse_export(SparseState *sp, int64_t n, void *out, int out_f64, hipStream_t s);

// Warm start: make z0 (device, n*n in the eigenvector layout of dpt.h, float or
// double) the current iterate; its diagonal is taken as 1.
hipError_t sparse_load_state(SparseState *sp, const void *z0, int z0_f64, hipStream_t s);

// ||M z_j - E_j z_j||_2 for the host-given rows; res on the host.
hipError_t sparse_residuals(SparseState *sp, double lambda, const double *theta, const double *evec,
                            const int64_t *rows, int64_t nrows, double *res, hipStream_t s);

// Dominant-eigenvector mode: iterate the single-line map F_index from e_index.
// theta_host: the host copy of theta for host inputs (uploaded), NULL for device
// inputs (p->theta is used in place); theta_index = theta[index].
int dominant_solve(const dpt_problem *p, const dpt_options *o, const double *theta_host, double theta_index,
                   int64_t index, double *eigval, void *eigvec, dpt_result *r);

// Limits of the dominant mode without allocation (dpt_dominant_noalloc): at most
// kNoallocMaxIter iterations, and two iterates of n values (each rounded up to
// 256 bytes) within kNoallocVectorBytes, i.e. n <= 8 Mi in FP32, 4 Mi in FP64.
constexpr int kNoallocMaxIter = 4096;
constexpr size_t kNoallocVectorBytes = (size_t)64 << 20;

// Dominant mode on device-resident inputs with every work buffer in the
// library's fixed per-device array (no device allocation).  p->mem must be
// DPT_MEM_DEVICE, p->dtype the state's dtype, eigvec device memory of that
// dtype.  Returns the numerical status, DPT_EINVAL (also for sizes beyond the
// limits above) or DPT_EDEVICE.  Calls on one device share the array: they must
// not overlap.
int dominant_solve_noalloc(const dpt_problem *p, const dpt_options *o, int64_t index, double *eigval, void *eigvec,
                           dpt_result *r);

// The dominant mode for device-resident inputs: theta is checked on the device
// (all values finite, theta[index] occurring once; index < 0 selects the first
// index of the largest value) together with the CSR structure, read back with
// one synchronisation, then the solve as dominant_solve.  Returns what
// dominant_solve returns, or DPT_EINVAL for a bad theta or structure.
int dominant_solve_device(const dpt_problem *p, const dpt_options *o, int64_t index, double *eigval, void *eigvec,
                          dpt_result *r);

}  // namespace dpt
