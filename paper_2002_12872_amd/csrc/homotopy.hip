// Homotopy continuation of the D-PT iteration (Kenmoe, Smerlak, Zadorin,
// arXiv:2002.12872, Sec. III): when lambda lies outside the domain where the
// iteration converges, split it into Q equal parts.  Stage q diagonalises
// M_q = D + (q lambda / Q) Delta by D-PT written in the eigenbasis of M_{q-1}:
//
//     B^-1 M_q B = diag(E_{q-1}) + (lambda / Q) B^-1 Delta B,
//
// so each stage is a perturbation of size lambda/Q of the diagonal matrix the
// previous stage produced.  Rows of V are the eigenvectors of the current M_q
// in the original coordinates (B = V^T), rows of X the matching left
// eigenvectors normalised so that X V^T = I (B^-1 = X):
//   * symmetric Delta: the rows of V are kept orthonormal, so X = V and the
//     stage perturbation V Delta V^T is symmetric;
//   * otherwise the left eigenvectors come from the same iteration on the
//     transposed stage perturbation (rows u_n with u_n^T M' = E_n u_n^T), scaled
//     by 1 / (u_n . y_n).
// Each stage is a full FP64 D-PT solve through the library's own entry points;
// the basis changes are FP64 matrix-core products (launch_gemm_nt_f64).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "dpt.h"
#include "dpt_internal.h"

namespace dpt {
namespace {

// out[i * n + j] = src[i * ld + j] for i, j < n.
__global__ void k_unpad_f64(const double *__restrict__ src, int64_t n, int64_t ld, double *__restrict__ out) {
    const int64_t total = n * n;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x)
        out[t] = src[(t / n) * ld + t % n];
}

// Identity in the leading n x n block of an ld x ld matrix, zeros elsewhere.
__global__ void k_eye_f64(double *__restrict__ A, int64_t n, int64_t ld) {
    const int64_t total = ld * ld;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / ld, j = t % ld;
        A[t] = (i == j && i < n) ? 1.0 : 0.0;
    }
}

// Row i of A (first n entries) scaled by 1 / ||row||_2 (one block per row).
__global__ __launch_bounds__(256) void k_row_normalize(double *__restrict__ A, int64_t n, int64_t ld) {
    __shared__ double red[4];
    double *row = A + blockIdx.x * ld;
    double s = 0.0;
    for (int64_t j = threadIdx.x; j < n; j += 256) s += row[j] * row[j];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    const double inv = 1.0 / sqrt((red[0] + red[1]) + (red[2] + red[3]));
    for (int64_t j = threadIdx.x; j < n; j += 256) row[j] *= inv;
}

// Row i of U scaled by 1 / (U[i] . Y[i]) (biorthonormal left rows; one block per row).
__global__ __launch_bounds__(256) void k_row_scale_dot(double *__restrict__ U, const double *__restrict__ Y,
                                                       int64_t n, int64_t ld) {
    __shared__ double red[4];
    double *u = U + blockIdx.x * ld;
    const double *y = Y + blockIdx.x * ld;
    double s = 0.0;
    for (int64_t j = threadIdx.x; j < n; j += 256) s += u[j] * y[j];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    const double inv = 1.0 / ((red[0] + red[1]) + (red[2] + red[3]));
    for (int64_t j = threadIdx.x; j < n; j += 256) u[j] *= inv;
}

// Z[k][m] = V[k][m] / V[k][k] (chart z_k[k] = 1), n x n output of type TO.
template <typename TO>
__global__ void k_chart_rows(const double *__restrict__ V, int64_t n, int64_t ld, TO *__restrict__ Z) {
    const int64_t total = n * n;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = t / n, m = t % n;
        Z[t] = k == m ? (TO)1 : (TO)(V[k * ld + m] / V[k * ld + k]);
    }
}

unsigned int grid_for(int64_t items) { return (unsigned int)std::max<int64_t>(1, std::min<int64_t>((items + 255) / 256, 1 << 16)); }

int err_of(hipError_t e) {
    if (e == hipSuccess) return DPT_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return DPT_ENOMEM;
    return DPT_EDEVICE;
}

bool is_dev(const void *p) {
    if (!p) return false;
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

struct Buffers {
    std::vector<void *> owned;
    ~Buffers() {
        for (void *p : owned) (void)hipFree(p);
    }
    template <typename T>
    hipError_t get(T **p, size_t count) {
        *p = nullptr;
        hipError_t e = hipMalloc((void **)p, std::max<size_t>(count, 1) * sizeof(T));
        if (e == hipSuccess) owned.push_back(*p);
        return e;
    }
};

#define HT_TRY(expr)                              \
    do {                                          \
        hipError_t e_ = (expr);                   \
        if (e_ != hipSuccess) return err_of(e_);  \
    } while (0)

// One stage solve: D-PT in FP64 on (theta_q, perturbation Dn (n x n, device), lam);
// eigenvectors into Yn (n x n, device), eigenvalues into E_next (device) when
// non-NULL.  Accumulates iterations; *status gets the stage's status.
int stage_solve(int64_t n, const double *theta_q, const double *Dn, double lam, const dpt_options *o, hipStream_t s,
                double *Yn, double *E_next, int *iters, int *status) {
    dpt_problem sp{};
    sp.n = n;
    sp.theta = theta_q;
    sp.delta = Dn;
    sp.lambda = lam;
    sp.stream = s;
    sp.format = DPT_DENSE;
    sp.dtype = DPT_DTYPE_F64;
    sp.mem = DPT_MEM_DEVICE;
    dpt_handle h = nullptr;
    int rc = dpt_init(&h, &sp, o, nullptr);
    if (rc != DPT_OK) return rc;
    dpt_result r{};
    rc = dpt_solve(h, &r);
    if (rc >= 0) {
        *iters += r.iters;
        *status = r.status;
        rc = dpt_eigenvectors(h, Yn, DPT_DTYPE_F64, DPT_MEM_DEVICE);
        if (rc == DPT_OK && E_next) rc = dpt_eigenvalues(h, E_next, DPT_MEM_DEVICE);
    }
    dpt_destroy(h);
    return rc;
}

}  // namespace
}  // namespace dpt

using namespace dpt;

extern "C" int dpt_homotopy(const dpt_problem *p, const dpt_options *o, int32_t stages, double *E, void *Z,
                            int z_dtype, dpt_result *r) {
    if (!p || !o || !E || !Z || stages < 1 || stages > 100000) return DPT_EINVAL;
    if (dpt_validate(p, o) != DPT_OK || p->format != DPT_DENSE || o->precision != DPT_FP64) return DPT_EINVAL;
    if (z_dtype != DPT_DTYPE_F64 && z_dtype != DPT_DTYPE_F32) return DPT_EINVAL;
    const bool dev = p->mem == DPT_MEM_DEVICE;
    if (dev && (!is_dev(p->theta) || !is_dev(p->delta) || !is_dev(E) || !is_dev(Z))) return DPT_EINVAL;
    const int64_t n = p->n;
    const int64_t ld = n >= 1024 ? (n + 255) / 256 * 256 : (n + 63) / 64 * 64;
    hipStream_t s = (hipStream_t)p->stream;
    const size_t l2 = (size_t)(ld * ld), n2 = (size_t)(n * n);
    Buffers buf;
    double *D = nullptr, *V = nullptr, *X = nullptr, *T = nullptr, *Dq = nullptr, *Yp = nullptr, *Up = nullptr;
    double *Wk = nullptr, *Yn = nullptr, *Un = nullptr, *Dn = nullptr, *th = nullptr, *th_next = nullptr;
    unsigned int *flag = nullptr;
    HT_TRY(buf.get(&D, l2));
    HT_TRY(buf.get(&V, l2));
    HT_TRY(buf.get(&T, l2));
    HT_TRY(buf.get(&Dq, l2));
    HT_TRY(buf.get(&Yp, l2));
    HT_TRY(buf.get(&Wk, l2));
    HT_TRY(buf.get(&Yn, n2));
    HT_TRY(buf.get(&Dn, n2));
    HT_TRY(buf.get(&th, (size_t)n));
    HT_TRY(buf.get(&th_next, (size_t)n));
    HT_TRY(buf.get(&flag, 1));
    // padded FP64 copy of Delta, theta on the device
    const size_t in_bytes = n2 * (p->dtype == DPT_DTYPE_F64 ? 8 : 4);
    const void *src = p->delta;
    if (!dev) {
        void *tmp = nullptr;
        HT_TRY(buf.get((unsigned char **)&tmp, in_bytes));
        HT_TRY(hipMemcpyAsync(tmp, p->delta, in_bytes, hipMemcpyHostToDevice, s));
        src = tmp;
    }
    HT_TRY(p->dtype == DPT_DTYPE_F64 ? launch_pad_copy_f64_from_f64(D, (const double *)src, n, ld, s)
                                     : launch_pad_copy_f64_from_f32(D, (const float *)src, n, ld, s));
    HT_TRY(hipMemcpyAsync(th, p->theta, sizeof(double) * n, dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    // exact symmetry of Delta decides the form of the basis inverse
    unsigned int hflag = 0;
    HT_TRY(launch_fill_zero(flag, 4, s));
    HT_TRY(launch_symmetry_check_f64(D, ld, flag, s));
    HT_TRY(hipMemcpyAsync(&hflag, flag, 4, hipMemcpyDeviceToHost, s));
    HT_TRY(hipStreamSynchronize(s));
    const bool sym = hflag == 0;
    if (!sym) {
        HT_TRY(buf.get(&X, l2));
        HT_TRY(buf.get(&Up, l2));
        HT_TRY(buf.get(&Un, n2));
        hipLaunchKernelGGL(k_eye_f64, dim3(grid_for((int64_t)l2)), dim3(256), 0, s, X, n, ld);
    }
    hipLaunchKernelGGL(k_eye_f64, dim3(grid_for((int64_t)l2)), dim3(256), 0, s, V, n, ld);
    HT_TRY(hipGetLastError());

    dpt_options so = *o;
    so.ramp_alpha = 0.0;
    // Stages far from the end of the continuation can contract slowly (rates of
    // 0.6 for the 2x2 at lambda = 3): with the default stall ratio 0.5 such a
    // stage would be taken for a rounding floor once delta enters the floor zone.
    so.stall_ratio = std::max(so.stall_ratio, 0.9);
    const double lam = p->lambda / stages;
    int iters = 0, status = DPT_OK;
    for (int q = 0; q < stages; ++q) {
        // stage perturbation X Delta V^T (Delta itself at the first stage)
        const double *stage = D;
        if (q > 0) {
            HT_TRY(launch_gemm_nt_f64(V, D, T, ld, s));            // T[j][a] = (V Delta^T)[j][a]
            HT_TRY(launch_gemm_nt_f64(sym ? V : X, T, Dq, ld, s));  // Dq[i][j] = (X Delta V^T)[i][j]
            stage = Dq;
        }
        hipLaunchKernelGGL(k_unpad_f64, dim3(grid_for((int64_t)n2)), dim3(256), 0, s, stage, n, ld, Dn);
        HT_TRY(hipGetLastError());
        int st = DPT_OK;
        int rc = stage_solve(n, th, Dn, lam, &so, s, Yn, th_next, &iters, &st);
        if (rc != DPT_OK) return rc;
        status = std::max(status, st);
        if (st != DPT_OK) break;  // the continuation needs every stage's eigenbasis
        const bool need_left = !sym && q + 1 < stages;  // the last stage's inverse basis is never used
        if (need_left) {  // left eigenvectors: the same iteration on the transposed stage perturbation
            HT_TRY(launch_transpose_f64(T, stage, ld, s));
            hipLaunchKernelGGL(k_unpad_f64, dim3(grid_for((int64_t)n2)), dim3(256), 0, s, T, n, ld, Dn);
            HT_TRY(hipGetLastError());
            rc = stage_solve(n, th, Dn, lam, &so, s, Un, nullptr, &iters, &st);
            if (rc != DPT_OK) return rc;
            status = std::max(status, st);
            if (st != DPT_OK) break;
        }
        // V <- Y V (rows of Y: this stage's eigenvectors in the current basis)
        HT_TRY(launch_pad_copy_f64_from_f64(Yp, Yn, n, ld, s));
        HT_TRY(launch_transpose_f64(T, V, ld, s));
        HT_TRY(launch_gemm_nt_f64(Yp, T, Wk, ld, s));
        std::swap(V, Wk);
        if (sym) {
            hipLaunchKernelGGL(k_row_normalize, dim3((unsigned int)n), dim3(256), 0, s, V, n, ld);
        } else if (need_left) {  // X <- diag(1 / (u_n . y_n)) U X
            HT_TRY(launch_pad_copy_f64_from_f64(Up, Un, n, ld, s));
            hipLaunchKernelGGL(k_row_scale_dot, dim3((unsigned int)n), dim3(256), 0, s, Up, Yp, n, ld);
            HT_TRY(launch_transpose_f64(T, X, ld, s));
            HT_TRY(launch_gemm_nt_f64(Up, T, Wk, ld, s));
            std::swap(X, Wk);
        }
        HT_TRY(hipGetLastError());
        std::swap(th, th_next);
    }
    // outputs: chart-normalised rows of V and the last stage's eigenvalues
    void *zdst = Z;
    const size_t zbytes = n2 * (z_dtype == DPT_DTYPE_F64 ? 8 : 4);
    if (!dev) HT_TRY(buf.get((unsigned char **)&zdst, zbytes));
    if (z_dtype == DPT_DTYPE_F64)
        hipLaunchKernelGGL((k_chart_rows<double>), dim3(grid_for((int64_t)n2)), dim3(256), 0, s, V, n, ld,
                           (double *)zdst);
    else
        hipLaunchKernelGGL((k_chart_rows<float>), dim3(grid_for((int64_t)n2)), dim3(256), 0, s, V, n, ld,
                           (float *)zdst);
    HT_TRY(hipGetLastError());
    if (!dev) HT_TRY(hipMemcpyAsync(Z, zdst, zbytes, hipMemcpyDeviceToHost, s));
    HT_TRY(hipMemcpyAsync(E, th, sizeof(double) * n, dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    HT_TRY(hipStreamSynchronize(s));
    if (r) {
        r->status = status;
        r->iters = iters;
        r->iters_bf16 = 0;
        r->iters_fp32 = 0;
        r->iters_fp64 = iters;
        r->last_delta = std::nan("");
    }
    return status;
}
