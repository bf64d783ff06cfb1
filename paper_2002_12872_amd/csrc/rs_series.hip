// Rayleigh-Schroedinger (RS) perturbation series on the GPU, the comparator of
// Sec. II.D-F (Kenmoe, Smerlak, Zadorin, arXiv:2002.12872; recursion eq.
// ARS-alpha, matrix form of Supplement B):
//
//     a^(0) = I,
//     a^(l) = theta (.) ( a^(l-1) Delta'  -  sum_{s=0}^{l-1} (a^(s) Delta') |> a^(l-1-s) ),
//
// with (A |> B)[n][m] = A[n][n] B[n][m], theta[n][m] = 1/(theta_n - theta_m) off the
// diagonal and 0 on it.  Eigenvalue coefficients eps^(l) = diag(a^(l-1) Delta')
// (eps^(1) = diag(Delta)).  Each order is one FP64 matrix-core product
// P_{l-1} = a^(l-1) Delta' (launch_gemm_nt_f64) and one fused pass forming
// a^(l) from P_{l-1}, the stored diagonals eps^(s+1) and the earlier
// coefficients, which also adds lambda^l a^(l) to the partial sum and reduces
// max |a^(l)|.  The ▷ terms need only the diagonals of the earlier products.
#include <hip/hip_runtime.h>
#include <float.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "dpt.h"
#include "dpt_internal.h"

namespace dpt {
namespace {

__device__ __forceinline__ unsigned long long f64_bits(double x) {
    return (unsigned long long)__double_as_longlong(x);
}

// eps[k] = P[k][k] for k < n.
__global__ void k_rs_diag(const double *__restrict__ P, int64_t n, int64_t ld, double *__restrict__ eps) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        eps[k] = P[k * ld + k];
}

// Order l >= 1 of the recursion.  coef[s] points to a^(s) (s < l; a^(0) = I is
// never read: its term eps^(l) |> I is diagonal and the gap factor removes it);
// eps holds eps^(1) .. eps^(l) at eps + (s) * ld for s = 0 .. l-1 (eps^(s+1) =
// diag(P_s)).  Writes a^(l) (zero diagonal and padding), adds lam_l a^(l) to
// Zsum, publishes max |a^(l)| (non-negative double bits, atomicMax).
__global__ __launch_bounds__(256) void k_rs_order(const double *__restrict__ P, const double *const *__restrict__ coef,
                                                  const double *__restrict__ eps, const double *__restrict__ theta,
                                                  int l, int64_t n, int64_t ld, double lam_l,
                                                  double *__restrict__ out, double *__restrict__ Zsum,
                                                  unsigned long long *__restrict__ amax) {
    double m_abs = 0.0;
    const int64_t total = ld * ld;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / ld, j = t % ld;
        double v = 0.0;
        if (i < n && j < n && i != j) {
            double acc = P[t];
            // the term of coefficient a^(u) carries eps^(l-u) = diag(P_{l-1-u})
            for (int u = 1; u < l; ++u) acc -= eps[(int64_t)(l - 1 - u) * ld + i] * coef[u][t];
            v = acc / (theta[i] - theta[j]);
        }
        out[t] = v;
        Zsum[t] += lam_l * v;
        m_abs = fmax(m_abs, fabs(v));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m_abs = fmax(m_abs, __shfl_xor(m_abs, o));
    if ((threadIdx.x & 63) == 0) atomicMax(amax, f64_bits(m_abs));
}

__global__ void k_rs_init(double *__restrict__ I0, double *__restrict__ Zsum, int64_t n, int64_t ld) {
    const int64_t total = ld * ld;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / ld, j = t % ld;
        const double v = (i == j && i < n) ? 1.0 : 0.0;
        I0[t] = v;
        Zsum[t] = v;
    }
}

template <typename TO>
__global__ void k_rs_export(const double *__restrict__ Zsum, int64_t n, int64_t ld, TO *__restrict__ out) {
    const int64_t total = n * n;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x)
        out[t] = (TO)Zsum[(t / n) * ld + t % n];
}

unsigned int grid_of(int64_t items) {
    return (unsigned int)std::max<int64_t>(1, std::min<int64_t>((items + 255) / 256, 1 << 14));
}

int err_rs(hipError_t e) {
    if (e == hipSuccess) return DPT_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return DPT_ENOMEM;
    return DPT_EDEVICE;
}

bool dev_ptr(const void *p) {
    if (!p) return false;
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

struct Owned {
    std::vector<void *> ps;
    ~Owned() {
        for (void *p : ps) (void)hipFree(p);
    }
    template <typename T>
    hipError_t get(T **p, size_t count) {
        *p = nullptr;
        hipError_t e = hipMalloc((void **)p, std::max<size_t>(count, 1) * sizeof(T));
        if (e == hipSuccess) ps.push_back(*p);
        return e;
    }
};

#define RS_TRY(expr)                              \
    do {                                          \
        hipError_t e_ = (expr);                   \
        if (e_ != hipSuccess) return err_rs(e_);  \
    } while (0)

}  // namespace
}  // namespace dpt

using namespace dpt;

extern "C" int dpt_rs_series(const dpt_problem *p, int32_t order, double *eps, double *coef_max, void *Z,
                             int z_dtype) {
    if (!p || order < 1 || order > 4096 || !eps) return DPT_EINVAL;
    if (dpt_validate(p, nullptr) != DPT_OK || p->format != DPT_DENSE) return DPT_EINVAL;
    if (Z && z_dtype != DPT_DTYPE_F64 && z_dtype != DPT_DTYPE_F32) return DPT_EINVAL;
    const bool dev = p->mem == DPT_MEM_DEVICE;
    if (dev && (!dev_ptr(p->theta) || !dev_ptr(p->delta) || (Z && !dev_ptr(Z)))) return DPT_EINVAL;
    const int64_t n = p->n;
    const int64_t ld = n >= 1024 ? (n + 255) / 256 * 256 : (n + 63) / 64 * 64;
    const size_t l2 = (size_t)(ld * ld);
    hipStream_t s = (hipStream_t)p->stream;
    Owned own;
    double *D = nullptr, *P = nullptr, *Zsum = nullptr, *th = nullptr, *epsd = nullptr;
    unsigned long long *amax = nullptr;
    const double **coef_dev = nullptr;
    RS_TRY(own.get(&D, l2));
    RS_TRY(own.get(&P, l2));
    RS_TRY(own.get(&Zsum, l2));
    RS_TRY(own.get(&th, (size_t)ld));
    RS_TRY(own.get(&epsd, (size_t)order * ld));
    RS_TRY(own.get(&amax, (size_t)order));
    RS_TRY(own.get(&coef_dev, (size_t)order + 1));
    std::vector<double *> coef((size_t)order + 1, nullptr);  // a^(0) .. a^(order)
    for (int l = 0; l <= order; ++l) RS_TRY(own.get(&coef[l], l2));
    // padded FP64 Delta; theta zero-padded (entries past n are never read)
    const size_t in_bytes = (size_t)(n * n) * (p->dtype == DPT_DTYPE_F64 ? 8 : 4);
    const void *src = p->delta;
    if (!dev) {
        void *tmp = nullptr;
        RS_TRY(own.get((unsigned char **)&tmp, in_bytes));
        RS_TRY(hipMemcpyAsync(tmp, p->delta, in_bytes, hipMemcpyHostToDevice, s));
        src = tmp;
    }
    RS_TRY(p->dtype == DPT_DTYPE_F64 ? launch_pad_copy_f64_from_f64(D, (const double *)src, n, ld, s)
                                     : launch_pad_copy_f64_from_f32(D, (const float *)src, n, ld, s));
    RS_TRY(launch_fill_zero(th, sizeof(double) * ld, s));
    RS_TRY(hipMemcpyAsync(th, p->theta, sizeof(double) * n, dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    RS_TRY(launch_zero_u64(amax, order, s));
    RS_TRY(hipMemcpyAsync(coef_dev, coef.data(), sizeof(double *) * (order + 1), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_rs_init, dim3(grid_of((int64_t)l2)), dim3(256), 0, s, coef[0], Zsum, n, ld);
    RS_TRY(hipGetLastError());
    double lam_l = 1.0;
    for (int l = 1; l <= order; ++l) {
        lam_l *= p->lambda;
        RS_TRY(launch_gemm_nt_f64(coef[l - 1], D, P, ld, s));  // P_{l-1} = a^(l-1) Delta'
        hipLaunchKernelGGL(k_rs_diag, dim3(grid_of(n)), dim3(256), 0, s, P, n, ld, epsd + (size_t)(l - 1) * ld);
        hipLaunchKernelGGL(k_rs_order, dim3(grid_of((int64_t)l2)), dim3(256), 0, s, P, coef_dev, epsd, th, l, n, ld,
                           lam_l, coef[l], Zsum, amax + (l - 1));
        RS_TRY(hipGetLastError());
    }
    // eps^(l) rows to the caller (host), coefficient maxima, partial sum
    std::vector<double> he((size_t)order * ld);
    std::vector<unsigned long long> hm((size_t)order);
    RS_TRY(hipMemcpyAsync(he.data(), epsd, sizeof(double) * he.size(), hipMemcpyDeviceToHost, s));
    RS_TRY(hipMemcpyAsync(hm.data(), amax, sizeof(unsigned long long) * order, hipMemcpyDeviceToHost, s));
    if (Z) {
        void *zdst = Z;
        const size_t zb = (size_t)(n * n) * (z_dtype == DPT_DTYPE_F64 ? 8 : 4);
        if (!dev) RS_TRY(own.get((unsigned char **)&zdst, zb));
        if (z_dtype == DPT_DTYPE_F64)
            hipLaunchKernelGGL((k_rs_export<double>), dim3(grid_of(n * n)), dim3(256), 0, s, Zsum, n, ld,
                               (double *)zdst);
        else
            hipLaunchKernelGGL((k_rs_export<float>), dim3(grid_of(n * n)), dim3(256), 0, s, Zsum, n, ld,
                               (float *)zdst);
        RS_TRY(hipGetLastError());
        if (!dev) RS_TRY(hipMemcpyAsync(Z, zdst, zb, hipMemcpyDeviceToHost, s));
    }
    RS_TRY(hipStreamSynchronize(s));
    for (int l = 0; l < order; ++l) {
        std::memcpy(eps + (size_t)l * n, he.data() + (size_t)l * ld, sizeof(double) * n);
        if (coef_max) {
            double v;
            std::memcpy(&v, &hm[l], sizeof(v));
            coef_max[l] = v;
        }
    }
    return DPT_OK;
}
