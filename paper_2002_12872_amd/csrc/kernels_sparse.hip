// CSR path and dominant-eigenvector mode for gfx950 (MI355X).
//
// Paper: Kenmoe, Smerlak, Zadorin, arXiv:2002.12872.
//  * Full sparse solve: eq. (dyn) with a CSR Delta.  The state is stored
//    transposed, WT[m][n] = W[n][m] (W = A - I), so that
//        (A Delta')[n][m] = (Delta z_n)[m] = Delta[m][n] + sum_l Delta[m][l] WT[l][n]
//    reads, for every non-zero Delta[m][l], one contiguous run WT[l][n0 .. n0+P)
//    covering P eigenvectors at once (coalesced gathers; the random sparsity
//    offers no other reuse).
//  * Dominant mode (Sec. II.H): the single-line map F_{n*} of eq.
//    (single_line_dyn) on one vector, z' = e + lambda g * (Delta z - (Delta z)[n*] z),
//    one SpMV (or GEMV) per iteration; every block recomputes the scalar
//    (Delta z)[n*] from row n* so that one launch performs one iteration.
#include <float.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <vector>

#include "device_common.h"
#include "dpt_internal.h"
#include "dpt_sparse.h"

namespace dpt {

namespace {

constexpr int kPanel = 256;  // eigenvectors per SpMM wave (4 per lane)
inline unsigned int blocks_for(int64_t items, int per_block, int64_t cap = 1 << 20) {
    int64_t b = (items + per_block - 1) / per_block;
    return (unsigned int)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

// ------------------------------------------------------------------ kernels
template <typename T>
__global__ void k_sp_diag(const int *__restrict__ rowptr, const int *__restrict__ col, const T *__restrict__ val,
                          int64_t n, double *__restrict__ diag) {
    for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < n; m += (int64_t)gridDim.x * blockDim.x) {
        double dv = 0.0;
        for (int e = rowptr[m]; e < rowptr[m + 1]; ++e)
            if (col[e] == m) dv = (double)val[e];
        diag[m] = dv;
    }
}

template <typename T>
__global__ void k_zero(T *__restrict__ p, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (T)0;
}

// F(I): WT_1[m][n] = lambda Delta[m][n] / (theta_n - theta_m) on the pattern of Delta.
template <typename T>
__global__ __launch_bounds__(256) void k_sp_first_iterate(const int *__restrict__ rowptr, const int *__restrict__ col,
                                                          const T *__restrict__ val, int64_t n, int64_t ld,
                                                          double lambda, const double *__restrict__ theta,
                                                          T *__restrict__ WT, unsigned long long *stat) {
    double dmax = 0.0;
    bool bad = false;
    for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < n; m += (int64_t)gridDim.x * blockDim.x) {
        const double tm = theta[m];
        for (int e = rowptr[m]; e < rowptr[m + 1]; ++e) {
            const int64_t c = col[e];
            if (c == m) continue;
            const T w = (T)(lambda * (double)val[e] / (theta[c] - tm));
            WT[m * ld + c] = w;
            const double v = fabs((double)w);
            dmax = fmax(dmax, v);
            bad |= !(v <= DBL_MAX);
        }
    }
    publish_stats(stat, dmax, dmax, bad);
}

// d_n = Delta[n][n] + sum_{l in row n} Delta[n][l] WT[l][n]  (FP64 accumulation).
template <typename T>
__global__ void k_sp_prepass(const int *__restrict__ rowptr, const int *__restrict__ col, const T *__restrict__ val,
                             const double *__restrict__ diag, int64_t n, int64_t ld, const T *__restrict__ WT,
                             double lambda, const double *__restrict__ theta, double *__restrict__ d,
                             double *__restrict__ E, unsigned long long *stat_clear) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i == 0 && stat_clear) {
        stat_clear[0] = 0ull;
        stat_clear[1] = 0ull;
    }
    if (i >= n) return;
    double s = 0.0;
    for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) s += (double)val[e] * (double)WT[(int64_t)col[e] * ld + i];
    const double dn = diag[i] + s;
    d[i] = dn;
    if (E) E[i] = theta[i] + lambda * dn;
}

template <typename T>
struct Vec4;
template <>
struct Vec4<float> {
    __device__ static void load(const float *p, double o[4]) {
        const float4 v = *reinterpret_cast<const float4 *>(p);
        o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
    }
    __device__ static void store(float *p, const double o[4]) {
        *reinterpret_cast<float4 *>(p) = make_float4((float)o[0], (float)o[1], (float)o[2], (float)o[3]);
    }
};
template <>
struct Vec4<double> {
    __device__ static void load(const double *p, double o[4]) {
        const double2 a = *reinterpret_cast<const double2 *>(p), b = *reinterpret_cast<const double2 *>(p + 2);
        o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
    }
    __device__ static void store(double *p, const double o[4]) {
        *reinterpret_cast<double2 *>(p) = make_double2(o[0], o[1]);
        *reinterpret_cast<double2 *>(p + 2) = make_double2(o[2], o[3]);
    }
};

// One wave per (row m of Delta, panel of kPanel eigenvectors); 4 rows per block.
// Blocks are dispatched round-robin over the 8 XCDs; the remap gives every XCD
// a contiguous run of panels so its L2 holds the panel being gathered.
template <typename T>
__global__ __launch_bounds__(256) void k_sp_spmm(const int *__restrict__ rowptr, const int *__restrict__ col,
                                                 const T *__restrict__ val, int64_t n, int64_t ld, double lambda,
                                                 const double *__restrict__ theta, const double *__restrict__ d,
                                                 const T *__restrict__ WT, T *__restrict__ WTn,
                                                 unsigned long long *stat) {
    const int64_t nb = gridDim.x;
    int64_t t = blockIdx.x;
    if ((nb & 7) == 0) t = (t & 7) * (nb >> 3) + (t >> 3);
    const int64_t row_blocks = ld / 4;
    const int64_t panel = t / row_blocks;
    const int64_t m = (t - panel * row_blocks) * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t n0 = panel * kPanel + lane * 4;
    const T *base = WT + n0;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int e0 = m < n ? rowptr[m] : 0, e1 = m < n ? rowptr[m + 1] : 0;  // padded rows have no entries
    for (int e = e0; e < e1; ++e) {
        const int64_t l = col[e];
        const double v = (double)val[e];
        double w[4];
        Vec4<T>::load(base + l * ld, w);
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] += v * w[q];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (l == n0 + q) acc[q] += v;  // identity part of Z = I + W
    }
    double wo[4], wn[4];
    Vec4<T>::load(WT + m * ld + n0, wo);
    const double tm = theta[m];
    double dmax = 0.0, wmax = 0.0;
    bool bad = false;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t nn = n0 + q;
        double w = 0.0;
        if (m < n && nn < n && nn != m) {
            const T num = (T)acc[q] - (T)d[nn] * (T)wo[q];
            w = (double)((T)lambda * num / (T)(theta[nn] - tm));
        }
        wn[q] = w;
        const double dv = fabs(w - wo[q]);
        dmax = fmax(dmax, dv);
        wmax = fmax(wmax, fabs(w));
        bad |= !(dv <= DBL_MAX);
    }
    Vec4<T>::store(WTn + m * ld + n0, wn);
    publish_stats(stat, dmax, wmax, bad);
}

// out[i][j] = Z[i][j] = (i == j) + WT[j][i]; 64x64 tiles through LDS.
template <typename T, typename TO>
__global__ __launch_bounds__(256) void k_sp_export(const T *__restrict__ WT, int64_t n, int64_t ld, TO *__restrict__ out) {
    __shared__ T tile[64][65];
    const int64_t bx = blockIdx.x, by = blockIdx.y;  // tile of WT: rows by*64, cols bx*64
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4) tile[r][tx] = WT[(by * 64 + r) * ld + bx * 64 + tx];
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int64_t i = bx * 64 + r, j = by * 64 + tx;  // out[i][j] = WT[j][i]
        if (i < n && j < n) out[i * n + j] = (i == j) ? (TO)1 : (TO)tile[tx][r];
    }
}

// Residual of eigenvector j = rows[blockIdx.x]; partial sum of squares per block.
template <typename T>
__global__ __launch_bounds__(256) void k_sp_residual(const int *__restrict__ rowptr, const int *__restrict__ col,
                                                     const T *__restrict__ val, int64_t n, int64_t ld, double lambda,
                                                     const double *__restrict__ theta, const double *__restrict__ E,
                                                     const T *__restrict__ WT, const int64_t *__restrict__ rows,
                                                     double *__restrict__ out) {
    const int64_t j = rows[blockIdx.x];
    const double ej = E[j];
    double acc = 0.0;
    for (int64_t m = threadIdx.x; m < n; m += 256) {
        double c = 0.0;
        for (int e = rowptr[m]; e < rowptr[m + 1]; ++e) {
            const int64_t l = col[e];
            c += (double)val[e] * ((l == j ? 1.0 : 0.0) + (double)WT[l * ld + j]);
        }
        const double zm = (m == j ? 1.0 : 0.0) + (double)WT[m * ld + j];
        const double r = theta[m] * zm + lambda * c - ej * zm;
        acc += r * r;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// ---------------------------------------------------------- dominant mode
// s = (Delta z)[nstar] for a CSR row, by one wave; result in *s_out (device).
template <typename T>
__device__ double csr_row_dot_wave(const int *rowptr, const int *col, const T *val, int64_t row, const T *z) {
    const int lane = threadIdx.x & 63;
    double s = 0.0;
    for (int e = rowptr[row] + lane; e < rowptr[row + 1]; e += 64) s += (double)val[e] * (double)z[col[e]];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    return s;
}

template <typename T>
__global__ void k_csr_row_dot(const int *rowptr, const int *col, const T *val, int64_t row, const T *z, double *s_out) {
    const double s = csr_row_dot_wave(rowptr, col, val, row, z);
    if (threadIdx.x == 0) *s_out = s;
}

// One iteration of F_{nstar}: 8 lanes per row, 32 rows per block.
template <typename T>
__global__ __launch_bounds__(256) void k_dom_csr(const int *__restrict__ rowptr, const int *__restrict__ col,
                                                 const T *__restrict__ val, int64_t n, int64_t nstar, double lambda,
                                                 const double *__restrict__ theta, const T *__restrict__ z,
                                                 T *__restrict__ zn, unsigned long long *stat) {
    __shared__ double s_sh;
    if (threadIdx.x < 64) {
        const double s = csr_row_dot_wave(rowptr, col, val, nstar, z);
        if (threadIdx.x == 0) s_sh = s;
    }
    __syncthreads();
    const T s = (T)s_sh;
    const int sub = threadIdx.x & 7;
    const int64_t m = (int64_t)blockIdx.x * 32 + (threadIdx.x >> 3);
    T c = (T)0;
    if (m < n)
        for (int e = rowptr[m] + sub; e < rowptr[m + 1]; e += 8) c += val[e] * z[col[e]];
    c += __shfl_xor(c, 4);
    c += __shfl_xor(c, 2);
    c += __shfl_xor(c, 1);
    double dmax = 0.0, wmax = 0.0;
    bool bad = false;
    if (m < n && sub == 0) {
        T w = (T)1;
        if (m != nstar) w = (T)lambda * (c - s * z[m]) / (T)(theta[nstar] - theta[m]);
        zn[m] = w;
        const double dv = fabs((double)w - (double)z[m]);
        dmax = dv;
        wmax = fabs((double)w - (m == nstar ? 1.0 : 0.0));
        bad = !(dv <= DBL_MAX);
    }
    publish_stats(stat, dmax, wmax, bad);
}

// Dense dominant mode: s computed first by k_dense_row_dot, then one wave per row.
template <typename T>
__global__ void k_dense_row_dot(const T *__restrict__ D, int64_t n, int64_t row, const T *__restrict__ z,
                                double *s_out) {
    __shared__ double red[4];
    double s = 0.0;
    for (int64_t l = threadIdx.x; l < n; l += 256) s += (double)D[row * n + l] * (double)z[l];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) *s_out = (red[0] + red[1]) + (red[2] + red[3]);
}

template <typename T>
__global__ __launch_bounds__(256) void k_dom_dense(const T *__restrict__ D, int64_t n, int64_t nstar, double lambda,
                                                   const double *__restrict__ theta, const double *__restrict__ s_in,
                                                   const T *__restrict__ z, T *__restrict__ zn,
                                                   unsigned long long *stat) {
    const int lane = threadIdx.x & 63;
    const int64_t m = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    double dmax = 0.0, wmax = 0.0;
    bool bad = false;
    if (m < n) {
        T c = (T)0;
        for (int64_t l = lane; l < n; l += 64) c += D[m * n + l] * z[l];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
        if (lane == 0) {
            T w = (T)1;
            if (m != nstar) w = (T)lambda * (c - (T)(*s_in) * z[m]) / (T)(theta[nstar] - theta[m]);
            zn[m] = w;
            const double dv = fabs((double)w - (double)z[m]);
            dmax = dv;
            wmax = fabs((double)w - (m == nstar ? 1.0 : 0.0));
            bad = !(dv <= DBL_MAX);
        }
    }
    publish_stats(stat, dmax, wmax, bad);
}

template <typename TS, typename TD>
__global__ void k_convert(const TS *__restrict__ src, TD *__restrict__ dst, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (TD)src[i];
}

__global__ void k_set_one(float *zf, double *zd, int64_t idx) {
    if (zf) zf[idx] = 1.0f;
    if (zd) zd[idx] = 1.0;
}

double bits_to_double(unsigned long long b) {
    double x;
    std::memcpy(&x, &b, sizeof(x));
    return x;
}

int err_code(hipError_t e) {
    if (e == hipSuccess) return DPT_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return DPT_ENOMEM;
    return DPT_EDEVICE;
}

// Host copy of a CSR matrix given in either memory kind, validated, int32 row pointers.
struct HostCsr {
    std::vector<int> rowptr, col;
    std::vector<double> val;
};

bool fetch_csr(const dpt_problem *p, HostCsr *h) {
    const int64_t n = p->n, nnz = p->nnz;
    std::vector<int64_t> ip((size_t)n + 1);
    h->col.resize((size_t)nnz);
    h->val.resize((size_t)nnz);
    const hipMemcpyKind kind = p->mem == DPT_MEM_DEVICE ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
    if (hipMemcpy(ip.data(), p->indptr, sizeof(int64_t) * (n + 1), kind) != hipSuccess) return false;
    if (nnz > 0 && hipMemcpy(h->col.data(), p->indices, sizeof(int32_t) * nnz, kind) != hipSuccess) return false;
    if (ip[0] != 0 || ip[n] != nnz) return false;
    h->rowptr.resize((size_t)n + 1);
    for (int64_t m = 0; m <= n; ++m) h->rowptr[m] = (int)ip[m];
    for (int64_t m = 0; m < n; ++m) {
        if (ip[m + 1] < ip[m]) return false;
        for (int64_t e = ip[m]; e < ip[m + 1]; ++e) {
            if (h->col[e] < 0 || h->col[e] >= n) return false;
            if (e > ip[m] && h->col[e] <= h->col[e - 1]) return false;
        }
    }
    if (nnz > 0) {
        if (p->dtype == DPT_DTYPE_F64) {
            if (hipMemcpy(h->val.data(), p->delta, sizeof(double) * nnz, kind) != hipSuccess) return false;
        } else {
            std::vector<float> tmp((size_t)nnz);
            if (hipMemcpy(tmp.data(), p->delta, sizeof(float) * nnz, kind) != hipSuccess) return false;
            for (int64_t e = 0; e < nnz; ++e) h->val[e] = tmp[e];
        }
    }
    return true;
}

template <typename T>
hipError_t upload_csr(const HostCsr &h, int **rowptr, int **col, T **val) {
    hipError_t e = hipMalloc((void **)rowptr, sizeof(int) * h.rowptr.size());
    if (e == hipSuccess) e = hipMalloc((void **)col, sizeof(int) * std::max<size_t>(1, h.col.size()));
    if (e == hipSuccess) e = hipMalloc((void **)val, sizeof(T) * std::max<size_t>(1, h.val.size()));
    if (e != hipSuccess) return e;
    std::vector<T> v(h.val.begin(), h.val.end());
    e = hipMemcpy(*rowptr, h.rowptr.data(), sizeof(int) * h.rowptr.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !h.col.empty())
        e = hipMemcpy(*col, h.col.data(), sizeof(int) * h.col.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !v.empty()) e = hipMemcpy(*val, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice);
    return e;
}

}  // namespace

// ============================================================ sparse solve
struct SparseState {
    int64_t n = 0, ld = 0, nnz = 0;
    bool fp64 = false;
    int *rowptr = nullptr, *col = nullptr;
    float *val32 = nullptr;
    double *val64 = nullptr;
    double *diag = nullptr;
    float *WT32[2] = {nullptr, nullptr};
    double *WT64[2] = {nullptr, nullptr};
    double *dvec = nullptr;
    int cur = 0;
    bool at_identity = true;
};

int64_t sparse_pad_order(int64_t n) { return (n + kPanel - 1) / kPanel * kPanel; }

void sparse_destroy(SparseState *sp) {
    if (!sp) return;
    void *ps[] = {sp->rowptr, sp->col, sp->val32, sp->val64, sp->diag, sp->WT32[0], sp->WT32[1],
                  sp->WT64[0], sp->WT64[1], sp->dvec};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    delete sp;
}

hipError_t sparse_create(SparseState **out, const dpt_problem *p, bool fp64, int64_t ld, hipStream_t s) {
    *out = nullptr;
    HostCsr h;
    if (!fetch_csr(p, &h)) return hipErrorInvalidValue;
    SparseState *sp = new SparseState();
    sp->n = p->n;
    sp->ld = ld;
    sp->nnz = p->nnz;
    sp->fp64 = fp64;
    hipError_t e = fp64 ? upload_csr(h, &sp->rowptr, &sp->col, &sp->val64)
                        : upload_csr(h, &sp->rowptr, &sp->col, &sp->val32);
    if (e == hipSuccess) e = hipMalloc((void **)&sp->diag, sizeof(double) * ld);
    if (e == hipSuccess) e = hipMalloc((void **)&sp->dvec, sizeof(double) * ld);
    const size_t elems = (size_t)(ld * ld);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        if (fp64)
            e = hipMalloc((void **)&sp->WT64[i], sizeof(double) * elems);
        else
            e = hipMalloc((void **)&sp->WT32[i], sizeof(float) * elems);
    }
    if (e != hipSuccess) {
        sparse_destroy(sp);
        return e;
    }
    const unsigned int g = blocks_for((int64_t)elems, 256);
    for (int i = 0; i < 2; ++i) {
        if (fp64)
            hipLaunchKernelGGL((k_zero<double>), dim3(g), dim3(256), 0, s, sp->WT64[i], (int64_t)elems);
        else
            hipLaunchKernelGGL((k_zero<float>), dim3(g), dim3(256), 0, s, sp->WT32[i], (int64_t)elems);
    }
    hipLaunchKernelGGL((k_zero<double>), dim3(blocks_for(ld, 256)), dim3(256), 0, s, sp->dvec, ld);
    hipLaunchKernelGGL((k_zero<double>), dim3(blocks_for(ld, 256)), dim3(256), 0, s, sp->diag, ld);
    if (fp64)
        hipLaunchKernelGGL((k_sp_diag<double>), dim3(blocks_for(sp->n, 256)), dim3(256), 0, s, sp->rowptr, sp->col,
                           sp->val64, sp->n, sp->diag);
    else
        hipLaunchKernelGGL((k_sp_diag<float>), dim3(blocks_for(sp->n, 256)), dim3(256), 0, s, sp->rowptr, sp->col,
                           sp->val32, sp->n, sp->diag);
    e = hipGetLastError();
    if (e != hipSuccess) {
        sparse_destroy(sp);
        return e;
    }
    *out = sp;
    return hipSuccess;
}

namespace {
struct NoProf : ProfHook {
    void begin(int, hipStream_t) override {}
    void end(hipStream_t) override {}
};

template <typename T>
hipError_t sparse_step_t(SparseState *sp, const T *val, T *const WT[2], double lambda, const double *theta,
                         unsigned long long *st, hipStream_t s, ProfHook *prof) {
    const int nx = sp->cur ^ 1;
    const int64_t n = sp->n, ld = sp->ld;
    if (sp->at_identity) {
        hipLaunchKernelGGL((k_zero<unsigned long long>), dim3(1), dim3(64), 0, s, st, (int64_t)2);
        prof->begin(DPT_PROF_FIRST, s);
        hipLaunchKernelGGL((k_sp_first_iterate<T>), dim3(blocks_for(n, 256, 4096)), dim3(256), 0, s, sp->rowptr,
                           sp->col, val, n, ld, lambda, theta, WT[nx], st);
        prof->end(s);
        return hipGetLastError();
    }
    prof->begin(DPT_PROF_PREPASS, s);
    hipLaunchKernelGGL((k_sp_prepass<T>), dim3(blocks_for(n, 256)), dim3(256), 0, s, sp->rowptr, sp->col, val,
                       sp->diag, n, ld, (const T *)WT[sp->cur], lambda, theta, sp->dvec, (double *)nullptr, st);
    prof->end(s);
    const int64_t blocks = (ld / kPanel) * (ld / 4);
    prof->begin(DPT_PROF_SPMM, s);
    hipLaunchKernelGGL((k_sp_spmm<T>), dim3((unsigned int)blocks), dim3(256), 0, s, sp->rowptr, sp->col, val, n, ld,
                       lambda, theta, (const double *)sp->dvec, (const T *)WT[sp->cur], WT[nx], st);
    prof->end(s);
    return hipGetLastError();
}
}  // namespace

int sparse_step(SparseState *sp, double lambda, const double *theta, unsigned long long *stats, int64_t *k,
                hipStream_t s, ProfHook *prof) {
    unsigned long long *st = stats + 2 * (int)(*k % kStatRing);
    const int nx = sp->cur ^ 1;
    const bool first = sp->at_identity;
    NoProf none;
    if (!prof) prof = &none;
    hipError_t e = sp->fp64 ? sparse_step_t<double>(sp, sp->val64, sp->WT64, lambda, theta, st, s, prof)
                            : sparse_step_t<float>(sp, sp->val32, sp->WT32, lambda, theta, st, s, prof);
    if (e != hipSuccess) return err_code(e);
    (void)first;  // the first iterate writes only the pattern of Delta into a zeroed buffer
    sp->cur = nx;
    sp->at_identity = false;
    *k += 1;
    return DPT_OK;
}

hipError_t sparse_eigenvalues(SparseState *sp, double lambda, const double *theta, double *evec, hipStream_t s) {
    if (sp->fp64)
        hipLaunchKernelGGL((k_sp_prepass<double>), dim3(blocks_for(sp->n, 256)), dim3(256), 0, s, sp->rowptr, sp->col,
                           sp->val64, sp->diag, sp->n, sp->ld, (const double *)sp->WT64[sp->cur], lambda, theta,
                           sp->dvec, evec, (unsigned long long *)nullptr);
    else
        hipLaunchKernelGGL((k_sp_prepass<float>), dim3(blocks_for(sp->n, 256)), dim3(256), 0, s, sp->rowptr, sp->col,
                           sp->val32, sp->diag, sp->n, sp->ld, (const float *)sp->WT32[sp->cur], lambda, theta,
                           sp->dvec, evec, (unsigned long long *)nullptr);
    return hipGetLastError();
}

hipError_t sparse_export(SparseState *sp, int64_t n, void *out, int out_f64, hipStream_t s) {
    const dim3 grid((unsigned int)(sp->ld / 64), (unsigned int)(sp->ld / 64));
    if (sp->fp64) {
        if (out_f64)
            hipLaunchKernelGGL((k_sp_export<double, double>), grid, dim3(256), 0, s, sp->WT64[sp->cur], n, sp->ld,
                               (double *)out);
        else
            hipLaunchKernelGGL((k_sp_export<double, float>), grid, dim3(256), 0, s, sp->WT64[sp->cur], n, sp->ld,
                               (float *)out);
    } else {
        if (out_f64)
            hipLaunchKernelGGL((k_sp_export<float, double>), grid, dim3(256), 0, s, sp->WT32[sp->cur], n, sp->ld,
                               (double *)out);
        else
            hipLaunchKernelGGL((k_sp_export<float, float>), grid, dim3(256), 0, s, sp->WT32[sp->cur], n, sp->ld,
                               (float *)out);
    }
    return hipGetLastError();
}

hipError_t sparse_residuals(SparseState *sp, double lambda, const double *theta, const double *evec,
                            const int64_t *rows, int64_t nrows, double *res, hipStream_t s) {
    int64_t *drows = nullptr;
    double *part = nullptr;
    hipError_t e = hipMalloc((void **)&drows, sizeof(int64_t) * nrows);
    if (e == hipSuccess) e = hipMalloc((void **)&part, sizeof(double) * nrows);
    if (e == hipSuccess) e = hipMemcpyAsync(drows, rows, sizeof(int64_t) * nrows, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        if (sp->fp64)
            hipLaunchKernelGGL((k_sp_residual<double>), dim3((unsigned int)nrows), dim3(256), 0, s, sp->rowptr, sp->col,
                               sp->val64, sp->n, sp->ld, lambda, theta, evec, (const double *)sp->WT64[sp->cur], drows,
                               part);
        else
            hipLaunchKernelGGL((k_sp_residual<float>), dim3((unsigned int)nrows), dim3(256), 0, s, sp->rowptr, sp->col,
                               sp->val32, sp->n, sp->ld, lambda, theta, evec, (const float *)sp->WT32[sp->cur], drows,
                               part);
        e = hipGetLastError();
    }
    std::vector<double> h((size_t)nrows);
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), part, sizeof(double) * nrows, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (drows) (void)hipFree(drows);
    if (part) (void)hipFree(part);
    if (e == hipSuccess)
        for (int64_t i = 0; i < nrows; ++i) res[i] = std::sqrt(h[i]);
    return e;
}

// ========================================================== dominant mode
namespace {

template <typename T>
int dominant_t(const dpt_problem *p, const dpt_options *o, const double *theta_host, int64_t nstar, double *eigval,
               void *eigvec, dpt_result *r) {
    const int64_t n = p->n;
    hipStream_t s = (hipStream_t)p->stream;
    int rc = DPT_OK;
    int *rowptr = nullptr, *col = nullptr;
    T *val = nullptr, *dense = nullptr;
    T *z[2] = {nullptr, nullptr};
    double *theta = nullptr, *s_dev = nullptr;
    unsigned long long *stats = nullptr;
    void *out_tmp = nullptr;
    const int cap = std::max(1, o->max_iter);
    std::vector<unsigned long long> hs(2);
    int status = DPT_NOT_CONVERGED, iters = 0;
    double last = std::numeric_limits<double>::quiet_NaN();
    auto run = [&]() -> hipError_t {
        hipError_t e;
        if (p->format == DPT_CSR) {
            HostCsr h;
            if (!fetch_csr(p, &h)) {
                rc = DPT_EINVAL;
                return hipSuccess;
            }
            e = upload_csr(h, &rowptr, &col, &val);
            if (e != hipSuccess) return e;
        } else {
            const size_t nn = (size_t)(n * n);
            const bool same = (sizeof(T) == 8) == (p->dtype == DPT_DTYPE_F64);
            if (same && p->mem == DPT_MEM_DEVICE) {
                dense = (T *)p->delta;  // borrowed
            } else {
                e = hipMalloc((void **)&val, sizeof(T) * nn);  // owned dense copy lives in `val`
                if (e != hipSuccess) return e;
                dense = val;
                const hipMemcpyKind kind = p->mem == DPT_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
                const size_t in_b = nn * (p->dtype == DPT_DTYPE_F64 ? 8 : 4);
                void *tmp = nullptr;
                e = hipMalloc(&tmp, in_b);
                if (e == hipSuccess) e = hipMemcpyAsync(tmp, p->delta, in_b, kind, s);
                if (e == hipSuccess) {
                    if (p->dtype == DPT_DTYPE_F64)
                        hipLaunchKernelGGL((k_convert<double, T>), dim3(blocks_for((int64_t)nn, 256)), dim3(256), 0, s,
                                           (const double *)tmp, dense, (int64_t)nn);
                    else
                        hipLaunchKernelGGL((k_convert<float, T>), dim3(blocks_for((int64_t)nn, 256)), dim3(256), 0, s,
                                           (const float *)tmp, dense, (int64_t)nn);
                    e = hipGetLastError();
                }
                if (e == hipSuccess) e = hipStreamSynchronize(s);
                if (tmp) (void)hipFree(tmp);
                if (e != hipSuccess) return e;
            }
        }
        e = hipMalloc((void **)&theta, sizeof(double) * n);
        if (e == hipSuccess) e = hipMalloc((void **)&s_dev, sizeof(double));
        if (e == hipSuccess) e = hipMalloc((void **)&stats, sizeof(unsigned long long) * 2 * (cap + 1));
        for (int i = 0; i < 2 && e == hipSuccess; ++i) e = hipMalloc((void **)&z[i], sizeof(T) * n);
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(theta, theta_host, sizeof(double) * n, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_zero<unsigned long long>), dim3(blocks_for(2 * (cap + 1), 256)), dim3(256), 0, s, stats,
                           (int64_t)2 * (cap + 1));
        hipLaunchKernelGGL((k_zero<T>), dim3(blocks_for(n, 256)), dim3(256), 0, s, z[0], n);
        hipLaunchKernelGGL(k_set_one, dim3(1), dim3(1), 0, s, sizeof(T) == 4 ? (float *)z[0] : nullptr,
                           sizeof(T) == 8 ? (double *)z[0] : nullptr, nstar);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        int cur = 0;
        while (iters < o->max_iter) {
            unsigned long long *st = stats + 2 * iters;
            if (p->format == DPT_CSR) {
                hipLaunchKernelGGL((k_dom_csr<T>), dim3(blocks_for(n, 32)), dim3(256), 0, s, rowptr, col,
                                   (const T *)val, n, nstar, p->lambda, (const double *)theta, (const T *)z[cur],
                                   z[cur ^ 1], st);
            } else {
                hipLaunchKernelGGL((k_dense_row_dot<T>), dim3(1), dim3(256), 0, s, (const T *)dense, n, nstar,
                                   (const T *)z[cur], s_dev);
                hipLaunchKernelGGL((k_dom_dense<T>), dim3(blocks_for(n, 4)), dim3(256), 0, s, (const T *)dense, n,
                                   nstar, p->lambda, (const double *)theta, (const double *)s_dev, (const T *)z[cur],
                                   z[cur ^ 1], st);
            }
            e = hipGetLastError();
            if (e == hipSuccess) e = hipMemcpyAsync(hs.data(), st, 16, hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) return e;
            cur ^= 1;
            ++iters;
            const double dl = bits_to_double(hs[0]), wm = bits_to_double(hs[1]);
            last = dl;
            if (r && r->delta_history && iters - 1 < r->history_cap) r->delta_history[iters - 1] = dl;
            if (!std::isfinite(dl) || !(wm <= o->blowup)) {
                status = DPT_DIVERGED;
                break;
            }
            if (dl < o->tol) {
                status = DPT_OK;
                break;
            }
        }
        // eigenvalue readout from the returned iterate
        if (p->format == DPT_CSR)
            hipLaunchKernelGGL((k_csr_row_dot<T>), dim3(1), dim3(64), 0, s, rowptr, col, (const T *)val, nstar,
                               (const T *)z[cur], s_dev);
        else
            hipLaunchKernelGGL((k_dense_row_dot<T>), dim3(1), dim3(256), 0, s, (const T *)dense, n, nstar,
                               (const T *)z[cur], s_dev);
        double sv = 0.0;
        e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(&sv, s_dev, sizeof(double), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        *eigval = theta_host[nstar] + p->lambda * sv;
        // eigenvector in the problem's dtype and memory kind
        const bool out64 = p->dtype == DPT_DTYPE_F64;
        const size_t ob = (size_t)n * (out64 ? 8 : 4);
        void *dst = eigvec;
        if (p->mem == DPT_MEM_HOST) {
            e = hipMalloc(&out_tmp, ob);
            if (e != hipSuccess) return e;
            dst = out_tmp;
        }
        if (out64)
            hipLaunchKernelGGL((k_convert<T, double>), dim3(blocks_for(n, 256)), dim3(256), 0, s, (const T *)z[cur],
                               (double *)dst, n);
        else
            hipLaunchKernelGGL((k_convert<T, float>), dim3(blocks_for(n, 256)), dim3(256), 0, s, (const T *)z[cur],
                               (float *)dst, n);
        e = hipGetLastError();
        if (e == hipSuccess && out_tmp) e = hipMemcpyAsync(eigvec, out_tmp, ob, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        return e;
    };
    hipError_t e = run();
    (void)hipStreamSynchronize(s);
    if (rowptr) (void)hipFree(rowptr);
    if (col) (void)hipFree(col);
    if (val) (void)hipFree(val);
    for (int i = 0; i < 2; ++i)
        if (z[i]) (void)hipFree(z[i]);
    if (theta) (void)hipFree(theta);
    if (s_dev) (void)hipFree(s_dev);
    if (stats) (void)hipFree(stats);
    if (out_tmp) (void)hipFree(out_tmp);
    if (rc != DPT_OK) return rc;
    if (e != hipSuccess) return err_code(e);
    if (r) {
        r->status = status;
        r->iters = iters;
        r->iters_bf16 = 0;
        r->iters_fp32 = sizeof(T) == 4 ? iters : 0;
        r->iters_fp64 = sizeof(T) == 8 ? iters : 0;
        r->last_delta = last;
    }
    return status;
}

}  // namespace

int dominant_solve(const dpt_problem *p, const dpt_options *o, const double *theta_host, int64_t index,
                   double *eigval, void *eigvec, dpt_result *r) {
    if (o->precision == DPT_FP64) return dominant_t<double>(p, o, theta_host, index, eigval, eigvec, r);
    return dominant_t<float>(p, o, theta_host, index, eigval, eigvec, r);
}

}  // namespace dpt
