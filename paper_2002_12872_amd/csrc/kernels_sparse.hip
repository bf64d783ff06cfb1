// CSR path and dominant-eigenvector mode for gfx950 (MI355X).
//
// Paper: Kenmoe, Smerlak, Zadorin, arXiv:2002.12872.
//  * Full sparse solve: eq. (dyn) with a CSR Delta.  The state is stored
//    transposed and with its unit diagonal, ZT[m][n] = Z[n][m] = z_n[m], so that
//        (A Delta')[n][m] = (Delta z_n)[m] = sum_l Delta[m][l] ZT[l][n]
//    reads, for every non-zero Delta[m][l], one contiguous run ZT[l][n0 .. n0+P)
//    covering P eigenvectors at once (coalesced gathers; the random sparsity
//    offers no other reuse).  Off-diagonal entries of Z equal those of
//    W = Z - I exactly, so storing Z loses nothing.
//    Layout: panel-major.  The columns n of ZT are cut into panels of P, and each
//    panel is one contiguous ld x P block (element (l, n) at
//    (n / P) * ld * P + l * P + n % P), so the gathers of one panel stay inside a
//    few MiB of address space (a handful of TLB pages) instead of striding
//    through the whole ld x ld array.
//  * Dominant mode (Sec. II.H): the single-line map F_{n*} of eq.
//    (single_line_dyn) on one vector, z' = e + lambda g * (Delta z - (Delta z)[n*] z),
//    one SpMV (or GEMV) per iteration, preceded by a one-wave kernel that
//    forms the scalar (Delta z)[n*] from row n* once.
#include <float.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <mutex>
#include <vector>

#include "device_common.h"
#include "dpt_internal.h"
#include "dpt_sparse.h"

namespace dpt {

namespace {

// SpMM lane-group size: LANES lanes x 16 bytes form one gathered run, so the
// panel width is P = LANES * 16 / sizeof(T) values.
#ifndef DPT_SPMM_LANES
#define DPT_SPMM_LANES 32
#endif
constexpr int kSpmmLanes = DPT_SPMM_LANES;
static_assert(kSpmmLanes >= 1 && 64 % kSpmmLanes == 0, "lane groups tile a wave");

// Padding of the sparse-path state: a multiple of the rows per SpMM block and of
// the export tiles (64) and of the widest panel (FP32).
constexpr int kPad = 4 * kSpmmLanes > 64 ? 4 * kSpmmLanes : 64;

template <typename T>
struct Panel {
    static constexpr int64_t P = kSpmmLanes * 16 / (int64_t)sizeof(T);
    static_assert(kPad % P == 0, "panels tile the padded order");
    // offset of element (l, n) of the ld x ld state
    __host__ __device__ static int64_t at(int64_t l, int64_t n, int64_t ld) { return (n / P) * (ld * P) + l * P + n % P; }
};
// Persistent grid of the dominant-mode SpMV: 8 blocks of 256 threads per CU.
constexpr int64_t kDomGrid = 256 * 8;

inline unsigned int blocks_for(int64_t items, int per_block, int64_t cap = 1 << 20) {
    int64_t b = (items + per_block - 1) / per_block;
    return (unsigned int)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

// ------------------------------------------------------------------ kernels
template <typename T>
__global__ void k_zero(T *__restrict__ p, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (T)0;
}

// Structural check of a CSR matrix in device memory (the host-side rules of
// dpt_validate): rowptr[0] = 0, rowptr[n] = nnz, non-decreasing row pointers,
// column indices in [0, n) and strictly increasing within a row.  Any violation
// sets *bad.  Column indices of a row are read only once its pointers are known
// to lie inside [0, nnz].  8 lanes per row (32 rows per block, grid-stride over
// row groups), so the column indices are read in coalesced runs; each lane
// compares its entries with their predecessors in the row.
__global__ __launch_bounds__(256) void k_csr_validate(const int64_t *__restrict__ rowptr,
                                                      const int *__restrict__ col, int64_t n, int64_t nnz,
                                                      unsigned int *bad) {
    const int sub = threadIdx.x & 7;
    bool err = false;
    if (blockIdx.x == 0 && threadIdx.x == 0) err = rowptr[0] != 0 || rowptr[n] != nnz;
    for (int64_t m = (int64_t)blockIdx.x * 32 + (threadIdx.x >> 3); m < n; m += (int64_t)gridDim.x * 32) {
        const int64_t a = rowptr[m], b = rowptr[m + 1];
        if (a < 0 || b > nnz || b < a) {
            err = true;
        } else {
            for (int64_t e = a + sub; e < b; e += 8) {
                const int c = col[e];
                err |= c < 0 || c >= n;
                if (e > a) err |= c <= col[e - 1];
            }
        }
    }
    if (__any(err ? 1 : 0) && (threadIdx.x & 63) == 0) atomicOr(bad, 1u);
}

// ZT[m][m] = 1 for m < n (the buffers start as the identity; the steps keep it).
template <typename T>
__global__ void k_set_unit_diag(T *__restrict__ ZT, int64_t n, int64_t ld) {
    for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < n; m += (int64_t)gridDim.x * blockDim.x)
        ZT[Panel<T>::at(m, m, ld)] = (T)1;
}

// F(I): ZT_1[m][n] = lambda Delta[m][n] / (theta_n - theta_m) on the off-diagonal
// pattern of Delta, written into a buffer that holds the identity.
template <typename T>
__global__ __launch_bounds__(256) void k_sp_first_iterate(const int64_t *__restrict__ rowptr, const int *__restrict__ col,
                                                          const T *__restrict__ val, int64_t n, int64_t ld,
                                                          double lambda, const double *__restrict__ theta,
                                                          T *__restrict__ ZT, unsigned long long *stat) {
    double dmax = 0.0;
    bool bad = false;
    for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < n; m += (int64_t)gridDim.x * blockDim.x) {
        const double tm = theta[m];
        for (int64_t e = rowptr[m]; e < rowptr[m + 1]; ++e) {
            const int64_t c = col[e];
            if (c == m) continue;
            const T w = (T)(lambda * (double)val[e] / (theta[c] - tm));
            ZT[Panel<T>::at(m, c, ld)] = w;
            const double v = fabs((double)w);
            dmax = fmax(dmax, v);
            bad |= !(v <= DBL_MAX);
        }
    }
    publish_stats_block(stat, dmax, dmax, bad);
}

// d_n = sum_{l in row n} Delta[n][l] ZT[l][n] = (Delta z_n)[n]  (FP64 accumulation).
template <typename T>
__global__ void k_sp_prepass(const int64_t *__restrict__ rowptr, const int *__restrict__ col, const T *__restrict__ val,
                             int64_t n, int64_t ld, const T *__restrict__ ZT, double lambda,
                             const double *__restrict__ theta, double *__restrict__ d, double *__restrict__ E,
                             unsigned long long *stat_clear) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i == 0 && stat_clear) {
        stat_clear[0] = 0ull;
        stat_clear[1] = 0ull;
    }
    if (i >= n) return;
    double s = 0.0;
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) s += (double)val[e] * (double)ZT[Panel<T>::at(col[e], i, ld)];
    d[i] = s;
    if (E) E[i] = theta[i] + lambda * s;
}

// One 16-byte vector of T (4 floats or 2 doubles).
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
    typedef float4 type;
    static constexpr int count = 4;
    __device__ static float get(const float4 &v, int i) { return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w; }
    __device__ static float4 make(const float *o) { return make_float4(o[0], o[1], o[2], o[3]); }
};
template <>
struct Vec16<double> {
    typedef double2 type;
    static constexpr int count = 2;
    __device__ static double get(const double2 &v, int i) { return i == 0 ? v.x : v.y; }
    __device__ static double2 make(const double *o) { return make_double2(o[0], o[1]); }
};

// CSR product + update.  Lanes form groups of LANES; each group owns one row m
// of Delta and each lane a 16-byte run of the panel of P = LANES * VEC
// eigenvectors (VEC = values per 16 bytes).  A lane walks the non-zeros of its
// own row, so a wave load instruction gathers 64 / LANES different rows l of the
// panel and no cross-lane reduction is needed; groups whose rows are shorter
// idle for the difference.  Blocks are dispatched round-robin over the 8 XCDs;
// the remap gives each XCD a contiguous run of panels, so the blocks resident on
// one XCD share one panel in its L2.  Accumulation is in T, as the dense steps
// accumulate in their own precision.
#ifndef DPT_SPMM_UNROLL
#define DPT_SPMM_UNROLL 8
#endif
constexpr int kSpmmUnroll = DPT_SPMM_UNROLL;  // gathers in flight per lane
constexpr int kSpmmRowsPerBlock = 64;  // 4 waves x (64 / LANES) rows x passes

template <typename T>
__global__ __launch_bounds__(256) void k_sp_spmm(const int64_t *__restrict__ rowptr, const int *__restrict__ col,
                                                 const T *__restrict__ val, int64_t n, int64_t ld, double lambda,
                                                 const double *__restrict__ theta, const double *__restrict__ d,
                                                 const T *__restrict__ ZT, T *__restrict__ ZTn,
                                                 unsigned long long *stat) {
    typedef typename Vec16<T>::type V;
    constexpr int VEC = Vec16<T>::count, LANES = kSpmmLanes, G = 64 / LANES;
    constexpr int64_t P = Panel<T>::P;
    static_assert(P == LANES * VEC, "panel width");
    constexpr int PASSES = kSpmmRowsPerBlock / (4 * G), U = kSpmmUnroll;
    static_assert(PASSES * 4 * G == kSpmmRowsPerBlock, "rows per block");
    const int64_t nb = gridDim.x;
    int64_t t = blockIdx.x;
    if ((nb & 7) == 0) t = (t & 7) * (nb >> 3) + (t >> 3);
    const int64_t row_blocks = ld / kSpmmRowsPerBlock;
    const int64_t panel = t / row_blocks;
    const int64_t rb = t - panel * row_blocks;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int group = lane / LANES, chunk = lane % LANES;
    const int64_t n0 = panel * P + chunk * VEC;           // first eigenvector of this lane
    const int64_t pbase = panel * (ld * P) + chunk * VEC;  // its offset in row 0 of the panel
    const T *base = ZT + pbase;
    const T lam = (T)lambda;
    double dmax = 0.0, wmax = 0.0;
    bool bad = false;
#pragma unroll 1
    for (int pass = 0; pass < PASSES; ++pass) {
        int64_t m = rb * kSpmmRowsPerBlock + (pass * 4 + wave) * G + group;
        // one row per wave: make it visibly wave-uniform so that the row's CSR
        // entries come through scalar loads and the addresses through SALU
        if constexpr (G == 1) m = __builtin_amdgcn_readfirstlane((int)m);
        const int64_t e0 = m < n ? rowptr[m] : 0, e1 = m < n ? rowptr[m + 1] : 0;  // padded rows: no entries
        T acc[VEC];
#pragma unroll
        for (int q = 0; q < VEC; ++q) acc[q] = (T)0;
        // U gathers in flight per lane; the last batch repeats the row's last
        // entry with weight 0 instead of branching on the remainder
        for (int64_t e = e0; e < e1; e += U) {
            const T *ps[U];
            T vs[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool in = e + u < e1;
                const int64_t idx = in ? e + u : e1 - 1;
                ps[u] = base + (int64_t)col[idx] * P;
                vs[u] = in ? val[idx] : (T)0;
            }
            V w[U];
#pragma unroll
            for (int u = 0; u < U; ++u) w[u] = *reinterpret_cast<const V *>(ps[u]);
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int q = 0; q < VEC; ++q) acc[q] += vs[u] * Vec16<T>::get(w[u], q);
        }
        const V zo = *reinterpret_cast<const V *>(ZT + pbase + m * P);
        const double tm = theta[m];
        T wn[VEC];
#pragma unroll
        for (int q = 0; q < VEC; ++q) {
            const int64_t nn = n0 + q;
            const T old = Vec16<T>::get(zo, q);
            T w = (T)0;
            if (m < n && nn < n) {
                if (nn == m) {
                    w = (T)1;
                } else {
                    const T num = acc[q] - (T)d[nn] * old;
                    w = lam * num / (T)(theta[nn] - tm);
                }
            }
            wn[q] = w;
            const double dv = fabs((double)w - (double)old);
            dmax = fmax(dmax, dv);
            if (nn != m) wmax = fmax(wmax, fabs((double)w));
            bad |= !(dv <= DBL_MAX);
        }
        *reinterpret_cast<V *>(ZTn + pbase + m * P) = Vec16<T>::make(wn);
    }
    publish_stats(stat, dmax, wmax, bad);
}

// out[i][j] = Z[i][j] = ZT[j][i]; 64x64 tiles through LDS.
template <typename T, typename TO>
__global__ __launch_bounds__(256) void k_sp_export(const T *__restrict__ ZT, int64_t n, int64_t ld, TO *__restrict__ out) {
    __shared__ T tile[64][65];
    const int64_t bx = blockIdx.x, by = blockIdx.y;  // tile of ZT: rows by*64, cols bx*64
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4) tile[r][tx] = ZT[Panel<T>::at(by * 64 + r, bx * 64 + tx, ld)];
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int64_t i = bx * 64 + r, j = by * 64 + tx;  // out[i][j] = ZT[j][i]
        if (i < n && j < n) out[i * n + j] = (TO)tile[tx][r];
    }
}

// Warm start: eigenvectors z0[k * n + m] = z_k[m] (device, TS) into the
// transposed panel-major state, ZT[m][k] = z_k[m], unit diagonal, zeros in the
// padding; 64 x 64 tiles transposed through LDS (row k read along m, panel row
// m written along k).
template <typename TS, typename T>
__global__ __launch_bounds__(256) void k_sp_load(const TS *__restrict__ z0, int64_t n, int64_t ld,
                                                 T *__restrict__ ZT) {
    __shared__ T tile[64][65];
    const int64_t bx = blockIdx.x, by = blockIdx.y;  // eigenvectors bx*64.., components by*64..
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4) {
        const int64_t k = bx * 64 + r, m = by * 64 + tx;
        T v = (T)0;
        if (k < n && m < n) v = k == m ? (T)1 : (T)z0[k * n + m];
        tile[r][tx] = v;
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int64_t m = by * 64 + r, k = bx * 64 + tx;
        ZT[Panel<T>::at(m, k, ld)] = tile[tx][r];
    }
}

// Residual of eigenvector j = rows[blockIdx.x]; partial sum of squares per block.
template <typename T>
__global__ __launch_bounds__(256) void k_sp_residual(const int64_t *__restrict__ rowptr, const int *__restrict__ col,
                                                     const T *__restrict__ val, int64_t n, int64_t ld, double lambda,
                                                     const double *__restrict__ theta, const double *__restrict__ E,
                                                     const T *__restrict__ ZT, const int64_t *__restrict__ rows,
                                                     double *__restrict__ out) {
    const int64_t j = rows[blockIdx.x];
    const double ej = E[j];
    double acc = 0.0;
    for (int64_t m = threadIdx.x; m < n; m += 256) {
        double c = 0.0;
        for (int64_t e = rowptr[m]; e < rowptr[m + 1]; ++e) c += (double)val[e] * (double)ZT[Panel<T>::at(col[e], j, ld)];
        const double zm = (double)ZT[Panel<T>::at(m, j, ld)];
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
__device__ double csr_row_dot_wave(const int64_t *rowptr, const int *col, const T *val, int64_t row, const T *z) {
    const int lane = threadIdx.x & 63;
    double s = 0.0;
    for (int64_t e = rowptr[row] + lane; e < rowptr[row + 1]; e += 64) s += (double)val[e] * (double)z[col[e]];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    return s;
}

// Stopping test of the dominant iteration on the device, by the kernel that
// follows an iteration in stream order (its statistics are complete): raise
// the stop flag when delta or max|z - e| is not finite, or max|z - e| exceeds
// blowup, or (may_stop) delta < tol -- the host's rule, so that the iterations
// enqueued after it in the same batch return at once.  st null: no test.
__device__ __forceinline__ void dom_stop_test(unsigned int *stop, const unsigned long long *st, double tol,
                                              double blowup, int may_stop) {
    if (!st) return;
    const double dl = __longlong_as_double((long long)st[0]), wm = __longlong_as_double((long long)st[1]);
    if (!(dl <= DBL_MAX) || !(wm <= blowup) || (may_stop && dl < tol)) *stop = 1u;
}

// s = (Delta z)[row] (the next iteration's scalar, or the eigenvalue's), then
// the stopping test of the iteration that produced z; nothing when stop is set.
template <typename T>
__global__ void k_csr_row_dot(const int64_t *rowptr, const int *col, const T *val, int64_t row, const T *z, double *s_out,
                              unsigned int *stop, const unsigned long long *st, double tol, double blowup,
                              int may_stop) {
    if (stop && *stop) return;
    const double s = csr_row_dot_wave(rowptr, col, val, row, z);
    if (threadIdx.x == 0) {
        *s_out = s;
        dom_stop_test(stop, st, tol, blowup, may_stop);
    }
}

// One iteration of F_{nstar}: 8 lanes per row, 32 rows per block pass; a
// persistent grid (a few blocks per CU) strides over groups of 32 rows.
// s = (Delta z)[nstar] comes from k_csr_row_dot, launched before it on the
// same stream, so each iteration computes s once.
template <typename T>
__global__ __launch_bounds__(256) void k_dom_csr(const int64_t *__restrict__ rowptr, const int *__restrict__ col,
                                                 const T *__restrict__ val, int64_t n, int64_t nstar, double lambda,
                                                 const double *__restrict__ theta, const double *__restrict__ s_in,
                                                 const T *__restrict__ z, T *__restrict__ zn,
                                                 unsigned long long *stat, const unsigned int *__restrict__ stop) {
    if (*stop) return;  // an earlier iteration of the batch met the stopping rule (uniform)
    const T s = (T)(*s_in);
    const int sub = threadIdx.x & 7;
    double dmax = 0.0, wmax = 0.0;
    bool bad = false;
    for (int64_t g = (int64_t)blockIdx.x * 32; g < n; g += (int64_t)gridDim.x * 32) {
        const int64_t m = g + (threadIdx.x >> 3);
        T c = (T)0;
        if (m < n) {
            // four entries per lane at a time: their four gathers are in flight together
            const int64_t e1 = rowptr[m + 1];
            for (int64_t e = rowptr[m] + sub; e < e1; e += 32) {
                int cc[4];
                T vv[4];
                bool in[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    in[u] = e + 8 * u < e1;
                    cc[u] = in[u] ? col[e + 8 * u] : 0;
                    vv[u] = in[u] ? val[e + 8 * u] : (T)0;
                }
                T zz[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) zz[u] = z[cc[u]];
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (in[u]) c += vv[u] * zz[u];
            }
        }
        c += __shfl_xor(c, 4);
        c += __shfl_xor(c, 2);
        c += __shfl_xor(c, 1);
        if (m < n && sub == 0) {
            T w = (T)1;
            if (m != nstar) w = (T)lambda * (c - s * z[m]) / (T)(theta[nstar] - theta[m]);
            zn[m] = w;
            const double dv = fabs((double)w - (double)z[m]);
            dmax = fmax(dmax, dv);
            wmax = fmax(wmax, fabs((double)w - (m == nstar ? 1.0 : 0.0)));
            bad |= !(dv <= DBL_MAX);
        }
    }
    publish_stats_block(stat, dmax, wmax, bad);
}

// The first iteration, from z = e_nstar, in closed form (the single-line
// analogue of F(I)): (Delta z)[m] = Delta[m][nstar] and s = Delta[nstar][nstar],
// so z1[m] = lambda (Delta[m][nstar] - s 0) / (theta_nstar - theta_m) for m !=
// nstar, with the arithmetic of k_dom_csr / k_dom_dense on e_nstar but without
// reading the whole matrix.  CSR entries are found by binary search in the
// row's sorted column indices (absent: 0).  One thread per row, grid-stride.
template <typename T>
__device__ __forceinline__ T csr_entry(const int64_t *__restrict__ rowptr, const int *__restrict__ col,
                                       const T *__restrict__ val, int64_t m, int64_t c) {
    const int64_t end = rowptr[m + 1];
    int64_t lo = rowptr[m], hi = end;
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (col[mid] < c)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo < end && col[lo] == c ? val[lo] : (T)0;
}

template <typename T, bool CSR>
__global__ __launch_bounds__(256) void k_dom_first(const int64_t *__restrict__ rowptr, const int *__restrict__ col,
                                                   const T *__restrict__ val, int64_t n, int64_t nstar,
                                                   double lambda, const double *__restrict__ theta,
                                                   T *__restrict__ zn, unsigned long long *stat) {
    // dense: val is the n x n row-major matrix
    const T s = CSR ? csr_entry(rowptr, col, val, nstar, nstar) : val[nstar * n + nstar];
    double dmax = 0.0, wmax = 0.0;
    bool bad = false;
    for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < n; m += (int64_t)gridDim.x * blockDim.x) {
        const T z = m == nstar ? (T)1 : (T)0;
        T w = (T)1;
        if (m != nstar) {
            const T c = CSR ? csr_entry(rowptr, col, val, m, nstar) : val[m * n + nstar];
            w = (T)lambda * (c - s * z) / (T)(theta[nstar] - theta[m]);
        }
        zn[m] = w;
        const double dv = fabs((double)w - (double)z);
        dmax = fmax(dmax, dv);
        wmax = fmax(wmax, fabs((double)w - (m == nstar ? 1.0 : 0.0)));
        bad |= !(dv <= DBL_MAX);
    }
    publish_stats_block(stat, dmax, wmax, bad);
}

// Dense dominant mode: s computed first by k_dense_row_dot, then one wave per row.
template <typename T>
__global__ void k_dense_row_dot(const T *__restrict__ D, int64_t n, int64_t row, const T *__restrict__ z,
                                double *s_out, unsigned int *stop, const unsigned long long *st, double tol,
                                double blowup, int may_stop) {
    if (stop && *stop) return;
    __shared__ double red[4];
    double s = 0.0;
    for (int64_t l = threadIdx.x; l < n; l += 256) s += (double)D[row * n + l] * (double)z[l];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        *s_out = (red[0] + red[1]) + (red[2] + red[3]);
        dom_stop_test(stop, st, tol, blowup, may_stop);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_dom_dense(const T *__restrict__ D, int64_t n, int64_t nstar, double lambda,
                                                   const double *__restrict__ theta, const double *__restrict__ s_in,
                                                   const T *__restrict__ z, T *__restrict__ zn,
                                                   unsigned long long *stat, const unsigned int *__restrict__ stop) {
    if (*stop) return;  // an earlier iteration of the batch met the stopping rule (uniform)
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
    publish_stats_block(stat, dmax, wmax, bad);
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

// Device-side theta checks of the dominant mode (device inputs, no copy of
// theta to the host): finiteness, the index of the largest value when none is
// given, and how often theta_index occurs.  Keys order doubles like integers.
struct ThetaScan {
    unsigned long long maxkey, index, count, bad, value_bits;
};

__device__ __forceinline__ unsigned long long order_key(double x) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    return (b >> 63) ? ~b : (b | (1ull << 63));
}

__global__ void k_theta_scan_init(ThetaScan *sc, int64_t n, int64_t index) {
    if (threadIdx.x == 0) {
        sc->maxkey = 0ull;
        sc->index = index >= 0 ? (unsigned long long)index : (unsigned long long)n;  // n: not found yet
        sc->count = 0ull;
        sc->bad = 0ull;
        sc->value_bits = 0ull;
    }
}

__global__ __launch_bounds__(256) void k_theta_max(const double *__restrict__ theta, int64_t n, ThetaScan *sc) {
    unsigned long long key = 0ull;
    bool bad = false;
    for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < n; m += (int64_t)gridDim.x * blockDim.x) {
        const double t = theta[m];
        bad |= !isfinite(t);
        key = max(key, order_key(t));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) key = max(key, (unsigned long long)__shfl_xor((long long)key, o));
    bad = __any(bad);
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&sc->maxkey, key);
        if (bad) atomicOr(&sc->bad, 1ull);
    }
}

// First index holding the maximum (only when no index was given).
__global__ __launch_bounds__(256) void k_theta_argmax(const double *__restrict__ theta, int64_t n, ThetaScan *sc,
                                                      int64_t index) {
    if (index >= 0) return;
    const unsigned long long target = sc->maxkey;
    for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < n; m += (int64_t)gridDim.x * blockDim.x)
        if (order_key(theta[m]) == target) atomicMin(&sc->index, (unsigned long long)m);
}

// Occurrences of theta_index (bitwise-equal values), and theta_index itself.
__global__ __launch_bounds__(256) void k_theta_count(const double *__restrict__ theta, int64_t n, ThetaScan *sc) {
    const unsigned long long idx = sc->index;
    if (idx >= (unsigned long long)n) return;
    const double t = theta[idx];
    unsigned long long c = 0ull;
    for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < n; m += (int64_t)gridDim.x * blockDim.x)
        c += theta[m] == t ? 1ull : 0ull;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += (unsigned long long)__shfl_xor((long long)c, o);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(&sc->count, c);
    if (blockIdx.x == 0 && threadIdx.x == 0) sc->value_bits = (unsigned long long)__double_as_longlong(t);
}

// The whole scan in one workgroup of 1024 threads, for theta of at most
// kThetaSmall values: one launch and no atomics between workgroups (the general
// form takes four launches and one atomic per wave on the same word), with the
// same results: the largest key, the non-finite flag, the first index holding
// the maximum when no index is given, and the occurrences of theta_index.
constexpr int64_t kThetaSmall = 65536;
__global__ __launch_bounds__(1024) void k_theta_scan_small(const double *__restrict__ theta, int64_t n,
                                                           int64_t index, ThetaScan *sc) {
    __shared__ unsigned long long red[16];
    __shared__ int red_bad[16];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    unsigned long long key = 0ull;
    bool bad = false;
    for (int64_t m = t; m < n; m += 1024) {
        const double x = theta[m];
        bad |= !isfinite(x);
        key = max(key, order_key(x));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) key = max(key, (unsigned long long)__shfl_xor((long long)key, o));
    const bool wave_bad = __any(bad);
    if (lane == 0) {
        red[w] = key;
        red_bad[w] = wave_bad ? 1 : 0;
    }
    __syncthreads();
    unsigned long long maxkey = red[0];
    int any_bad = red_bad[0];
    for (int i = 1; i < 16; ++i) {
        maxkey = max(maxkey, red[i]);
        any_bad |= red_bad[i];
    }
    __syncthreads();  // red is reused below
    unsigned long long idx = index >= 0 ? (unsigned long long)index : (unsigned long long)n;
    if (index < 0) {
        unsigned long long first = (unsigned long long)n;
        for (int64_t m = t; m < n; m += 1024)
            if (order_key(theta[m]) == maxkey) {
                first = (unsigned long long)m;  // this thread's indices increase
                break;
            }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) first = min(first, (unsigned long long)__shfl_xor((long long)first, o));
        if (lane == 0) red[w] = first;
        __syncthreads();
        idx = red[0];
        for (int i = 1; i < 16; ++i) idx = min(idx, red[i]);
        __syncthreads();
    }
    unsigned long long count = 0ull;
    double tv = 0.0;
    if (idx < (unsigned long long)n) {  // uniform
        tv = theta[idx];
        for (int64_t m = t; m < n; m += 1024) count += theta[m] == tv ? 1ull : 0ull;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) count += (unsigned long long)__shfl_xor((long long)count, o);
        if (lane == 0) red[w] = count;
        __syncthreads();
        count = 0ull;
        for (int i = 0; i < 16; ++i) count += red[i];
    }
    if (t == 0) {
        sc->maxkey = maxkey;
        sc->index = idx;
        sc->count = count;
        sc->bad = any_bad ? 1ull : 0ull;
        sc->value_bits = idx < (unsigned long long)n ? (unsigned long long)__double_as_longlong(tv) : 0ull;
    }
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

// CSR Delta on the device with values in T.  Device inputs are borrowed (row
// pointers and indices always; values when their dtype is T) after a structural
// check on the device; host inputs are checked on the host and uploaded.
template <typename T>
struct DevCsr {
    const int64_t *rowptr = nullptr;
    const int *col = nullptr;
    const T *val = nullptr;
    void *owned[3] = {nullptr, nullptr, nullptr};
    void release() {
        for (void *&q : owned)
            if (q) {
                (void)hipFree(q);
                q = nullptr;
            }
    }
};

bool host_csr_ok(const int64_t *ip, const int *col, int64_t n, int64_t nnz) {
    if (ip[0] != 0 || ip[n] != nnz) return false;
    for (int64_t m = 0; m < n; ++m) {
        if (ip[m + 1] < ip[m] || ip[m] < 0 || ip[m + 1] > nnz) return false;
        for (int64_t e = ip[m]; e < ip[m + 1]; ++e) {
            if (col[e] < 0 || col[e] >= n) return false;
            if (e > ip[m] && col[e] <= col[e - 1]) return false;
        }
    }
    return true;
}

// Structural check of a device CSR (same rules as the host check) with the
// caller's one-word device flag; synchronises the stream.  Returns DPT_OK,
// DPT_EINVAL or a device error code.
int validate_device_csr(const dpt_problem *p, unsigned int *flag, hipStream_t s) {
    unsigned int hflag = 0;
    hipLaunchKernelGGL((k_zero<unsigned int>), dim3(1), dim3(64), 0, s, flag, (int64_t)1);
    hipLaunchKernelGGL(k_csr_validate, dim3(blocks_for(p->n, 32)), dim3(256), 0, s, p->indptr, p->indices, p->n,
                       p->nnz, flag);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&hflag, flag, sizeof(hflag), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return err_code(e);
    return hflag ? DPT_EINVAL : DPT_OK;
}

// Returns DPT_OK, DPT_EINVAL (bad structure) or a device error code; on
// failure nothing stays allocated.
template <typename T>
int stage_csr(const dpt_problem *p, DevCsr<T> *c, hipStream_t s, bool validated = false) {
    const int64_t n = p->n, nnz = p->nnz;
    const bool vals64 = p->dtype == DPT_DTYPE_F64;
    const size_t in_b = (size_t)std::max<int64_t>(1, nnz) * (vals64 ? 8 : 4);
    hipError_t e = hipSuccess;
    if (p->mem == DPT_MEM_HOST) {
        const int64_t *ip = p->indptr;
        if (!host_csr_ok(ip, p->indices, n, nnz)) return DPT_EINVAL;
        e = hipMalloc(&c->owned[0], sizeof(int64_t) * (n + 1));
        if (e == hipSuccess) e = hipMalloc(&c->owned[1], sizeof(int) * std::max<int64_t>(1, nnz));
        if (e == hipSuccess) e = hipMalloc(&c->owned[2], in_b);
        if (e == hipSuccess) e = hipMemcpyAsync(c->owned[0], ip, sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, s);
        if (e == hipSuccess && nnz > 0)
            e = hipMemcpyAsync(c->owned[1], p->indices, sizeof(int) * nnz, hipMemcpyHostToDevice, s);
        if (e == hipSuccess && nnz > 0)
            e = hipMemcpyAsync(c->owned[2], p->delta, (size_t)nnz * (vals64 ? 8 : 4), hipMemcpyHostToDevice, s);
        c->rowptr = (const int64_t *)c->owned[0];
        c->col = (const int *)c->owned[1];
    } else {
        c->rowptr = p->indptr;
        c->col = p->indices;
        if (!validated) {
            unsigned int *flag = nullptr;
            e = hipMalloc((void **)&flag, sizeof(unsigned int));
            if (e == hipSuccess) {
                const int rc = validate_device_csr(p, flag, s);
                (void)hipFree(flag);
                if (rc != DPT_OK) return rc;
            }
        }
        if (e == hipSuccess && vals64 == (sizeof(T) == 8)) {
            c->val = (const T *)p->delta;  // borrowed
            return DPT_OK;
        }
    }
    // values of the other width: convert (from the staged copy or the caller's array)
    if (e == hipSuccess && vals64 != (sizeof(T) == 8)) {
        const void *src = p->mem == DPT_MEM_HOST ? c->owned[2] : p->delta;
        void *conv = nullptr;
        e = hipMalloc(&conv, sizeof(T) * std::max<int64_t>(1, nnz));
        if (e == hipSuccess && nnz > 0) {
            if (vals64)
                hipLaunchKernelGGL((k_convert<double, T>), dim3(blocks_for(nnz, 256)), dim3(256), 0, s,
                                   (const double *)src, (T *)conv, nnz);
            else
                hipLaunchKernelGGL((k_convert<float, T>), dim3(blocks_for(nnz, 256)), dim3(256), 0, s,
                                   (const float *)src, (T *)conv, nnz);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (c->owned[2]) (void)hipFree(c->owned[2]);
        c->owned[2] = conv;
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // host sources may be freed on return
    c->val = (const T *)c->owned[2];
    if (e != hipSuccess) {
        c->release();
        return err_code(e);
    }
    return DPT_OK;
}

}  // namespace

// ============================================================ sparse solve
struct SparseState {
    int64_t n = 0, ld = 0, nnz = 0;
    bool fp64 = false;
    DevCsr<float> csr32;   // FP32 state
    DevCsr<double> csr64;  // FP64 state
    const int64_t *rowptr = nullptr;
    const int *col = nullptr;
    const float *val32 = nullptr;
    const double *val64 = nullptr;
    float *ZT32[2] = {nullptr, nullptr};
    double *ZT64[2] = {nullptr, nullptr};
    double *dvec = nullptr;
    int cur = 0;
    bool at_identity = true;
};

int64_t sparse_pad_order(int64_t n) { return (n + kPad - 1) / kPad * kPad; }

void sparse_destroy(SparseState *sp) {
    if (!sp) return;
    sp->csr32.release();
    sp->csr64.release();
    void *ps[] = {sp->ZT32[0], sp->ZT32[1], sp->ZT64[0], sp->ZT64[1], sp->dvec};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    delete sp;
}

int sparse_create(SparseState **out, const dpt_problem *p, bool fp64, int64_t ld, hipStream_t s) {
    *out = nullptr;
    SparseState *sp = new SparseState();
    sp->n = p->n;
    sp->ld = ld;
    sp->nnz = p->nnz;
    sp->fp64 = fp64;
    const int rc = fp64 ? stage_csr(p, &sp->csr64, s) : stage_csr(p, &sp->csr32, s);
    if (rc != DPT_OK) {
        delete sp;
        return rc;
    }
    sp->rowptr = fp64 ? sp->csr64.rowptr : sp->csr32.rowptr;
    sp->col = fp64 ? sp->csr64.col : sp->csr32.col;
    sp->val32 = sp->csr32.val;
    sp->val64 = sp->csr64.val;
    hipError_t e = hipMalloc((void **)&sp->dvec, sizeof(double) * ld);
    const size_t elems = (size_t)(ld * ld);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        if (fp64)
            e = hipMalloc((void **)&sp->ZT64[i], sizeof(double) * elems);
        else
            e = hipMalloc((void **)&sp->ZT32[i], sizeof(float) * elems);
    }
    if (e != hipSuccess) {
        sparse_destroy(sp);
        return err_code(e);
    }
    const unsigned int g = blocks_for((int64_t)elems, 256);
    for (int i = 0; i < 2; ++i) {  // both buffers start as the identity
        if (fp64) {
            hipLaunchKernelGGL((k_zero<double>), dim3(g), dim3(256), 0, s, sp->ZT64[i], (int64_t)elems);
            hipLaunchKernelGGL((k_set_unit_diag<double>), dim3(blocks_for(sp->n, 256)), dim3(256), 0, s, sp->ZT64[i],
                               sp->n, ld);
        } else {
            hipLaunchKernelGGL((k_zero<float>), dim3(g), dim3(256), 0, s, sp->ZT32[i], (int64_t)elems);
            hipLaunchKernelGGL((k_set_unit_diag<float>), dim3(blocks_for(sp->n, 256)), dim3(256), 0, s, sp->ZT32[i],
                               sp->n, ld);
        }
    }
    hipLaunchKernelGGL((k_zero<double>), dim3(blocks_for(ld, 256)), dim3(256), 0, s, sp->dvec, ld);
    e = hipGetLastError();
    if (e != hipSuccess) {
        sparse_destroy(sp);
        return err_code(e);
    }
    *out = sp;
    return DPT_OK;
}

namespace {
struct NoProf : ProfHook {
    void begin(int, hipStream_t) override {}
    void end(hipStream_t) override {}
};

template <typename T>
hipError_t sparse_step_t(SparseState *sp, const T *val, T *const ZT[2], double lambda, const double *theta,
                         unsigned long long *st, hipStream_t s, ProfHook *prof) {
    const int nx = sp->cur ^ 1;
    const int64_t n = sp->n, ld = sp->ld;
    if (sp->at_identity) {
        hipLaunchKernelGGL((k_zero<unsigned long long>), dim3(1), dim3(64), 0, s, st, (int64_t)2);
        prof->begin(DPT_PROF_FIRST, s);
        hipLaunchKernelGGL((k_sp_first_iterate<T>), dim3(blocks_for(n, 256, 4096)), dim3(256), 0, s, sp->rowptr,
                           sp->col, val, n, ld, lambda, theta, ZT[nx], st);
        prof->end(s);
        return hipGetLastError();
    }
    prof->begin(DPT_PROF_PREPASS, s);
    hipLaunchKernelGGL((k_sp_prepass<T>), dim3(blocks_for(n, 256)), dim3(256), 0, s, sp->rowptr, sp->col, val,
                       n, ld, (const T *)ZT[sp->cur], lambda, theta, sp->dvec, (double *)nullptr, st);
    prof->end(s);
    const int64_t blocks = (ld / Panel<T>::P) * (ld / kSpmmRowsPerBlock);
    prof->begin(DPT_PROF_SPMM, s);
    hipLaunchKernelGGL((k_sp_spmm<T>), dim3((unsigned int)blocks), dim3(256), 0, s, sp->rowptr, sp->col, val, n, ld,
                       lambda, theta, (const double *)sp->dvec, (const T *)ZT[sp->cur], ZT[nx], st);
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
    hipError_t e = sp->fp64 ? sparse_step_t<double>(sp, sp->val64, sp->ZT64, lambda, theta, st, s, prof)
                            : sparse_step_t<float>(sp, sp->val32, sp->ZT32, lambda, theta, st, s, prof);
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
                           sp->val64, sp->n, sp->ld, (const double *)sp->ZT64[sp->cur], lambda, theta,
                           sp->dvec, evec, (unsigned long long *)nullptr);
    else
        hipLaunchKernelGGL((k_sp_prepass<float>), dim3(blocks_for(sp->n, 256)), dim3(256), 0, s, sp->rowptr, sp->col,
                           sp->val32, sp->n, sp->ld, (const float *)sp->ZT32[sp->cur], lambda, theta,
                           sp->dvec, evec, (unsigned long long *)nullptr);
    return hipGetLastError();
}

hipError_t sparse_export(SparseState *sp, int64_t n, void *out, int out_f64, hipStream_t s) {
    const dim3 grid((unsigned int)(sp->ld / 64), (unsigned int)(sp->ld / 64));
    if (sp->fp64) {
        if (out_f64)
            hipLaunchKernelGGL((k_sp_export<double, double>), grid, dim3(256), 0, s, sp->ZT64[sp->cur], n, sp->ld,
                               (double *)out);
        else
            hipLaunchKernelGGL((k_sp_export<double, float>), grid, dim3(256), 0, s, sp->ZT64[sp->cur], n, sp->ld,
                               (float *)out);
    } else {
        if (out_f64)
            hipLaunchKernelGGL((k_sp_export<float, double>), grid, dim3(256), 0, s, sp->ZT32[sp->cur], n, sp->ld,
                               (double *)out);
        else
            hipLaunchKernelGGL((k_sp_export<float, float>), grid, dim3(256), 0, s, sp->ZT32[sp->cur], n, sp->ld,
                               (float *)out);
    }
    return hipGetLastError();
}

hipError_t sparse_load_state(SparseState *sp, const void *z0, int z0_f64, hipStream_t s) {
    const dim3 grid((unsigned int)(sp->ld / 64), (unsigned int)(sp->ld / 64));
    if (sp->fp64) {
        if (z0_f64)
            hipLaunchKernelGGL((k_sp_load<double, double>), grid, dim3(256), 0, s, (const double *)z0, sp->n, sp->ld,
                               sp->ZT64[0]);
        else
            hipLaunchKernelGGL((k_sp_load<float, double>), grid, dim3(256), 0, s, (const float *)z0, sp->n, sp->ld,
                               sp->ZT64[0]);
    } else {
        if (z0_f64)
            hipLaunchKernelGGL((k_sp_load<double, float>), grid, dim3(256), 0, s, (const double *)z0, sp->n, sp->ld,
                               sp->ZT32[0]);
        else
            hipLaunchKernelGGL((k_sp_load<float, float>), grid, dim3(256), 0, s, (const float *)z0, sp->n, sp->ld,
                               sp->ZT32[0]);
    }
    sp->cur = 0;
    sp->at_identity = false;
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
                               sp->val64, sp->n, sp->ld, lambda, theta, evec, (const double *)sp->ZT64[sp->cur], drows,
                               part);
        else
            hipLaunchKernelGGL((k_sp_residual<float>), dim3((unsigned int)nrows), dim3(256), 0, s, sp->rowptr, sp->col,
                               sp->val32, sp->n, sp->ld, lambda, theta, evec, (const float *)sp->ZT32[sp->cur], drows,
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

// Device buffers of one dominant-mode solve: the iterate and its successor,
// the scalar (Delta z)[n*], and the per-iteration statistics (2 u64 per
// iteration, iterations 0 .. cap-1).
template <typename T>
struct DomBuffers {
    T *z[2] = {nullptr, nullptr};
    double *s = nullptr;
    unsigned long long *stats = nullptr;
    unsigned int *stop = nullptr;  // set on the device when an iteration meets the stopping rule
};

struct DomOutcome {
    int status = DPT_NOT_CONVERGED, iters = 0;
    double last = std::numeric_limits<double>::quiet_NaN();
};

// The iteration of F_nstar from e_nstar and the readout, on device buffers the
// caller provides (allocates nothing).  `val` holds the CSR values, or the
// n x n row-major matrix when rowptr is NULL.  The eigenvector goes to the
// device array dst (dtype out64 ? double : float); *eigval gets
// theta_star + lambda (Delta z)[nstar] of the returned iterate.  Iterations are
// enqueued in batches (2, then up to kDomBatch) with one synchronisation per
// batch: each ends with (Delta z)[nstar] of its new iterate (the next
// iteration's scalar, or the eigenvalue's) and the stopping test on the device
// (the host's rule), after which the rest of the batch returns at once; the
// batch's statistics and the last scalar come back together into host_words
// (2 kDomBatch + 1 words, pinned) or a local array when it is null, and the
// host applies the same rule to them in order, so it ends on the iteration the
// device ended on.  The iterates are those of one synchronisation per
// iteration.
constexpr int kDomBatch = 4;

template <typename T>
hipError_t dominant_iterate(const dpt_problem *p, const dpt_options *o, const int64_t *rowptr, const int *col,
                            const T *val, const double *theta, double theta_star, int64_t nstar,
                            const DomBuffers<T> &b, int cap, void *dst, bool out64, double *eigval,
                            DomOutcome *out, dpt_result *r, hipStream_t s,
                            unsigned long long *host_words = nullptr) {
    const int64_t n = p->n;
    const bool csr = rowptr != nullptr;
    unsigned long long local[2 * kDomBatch + 1] = {};
    unsigned long long *hs = host_words ? host_words : local;
    // (Delta z)[nstar] into b.s; with st, then the stopping test of z's iteration
    auto row_dot = [&](const T *z, const unsigned long long *st, int may_stop) {
        if (csr)
            hipLaunchKernelGGL((k_csr_row_dot<T>), dim3(1), dim3(64), 0, s, rowptr, col, val, nstar, z, b.s,
                               st ? b.stop : (unsigned int *)nullptr, st, o->tol, o->blowup, may_stop);
        else
            hipLaunchKernelGGL((k_dense_row_dot<T>), dim3(1), dim3(256), 0, s, val, n, nstar, z, b.s,
                               st ? b.stop : (unsigned int *)nullptr, st, o->tol, o->blowup, may_stop);
    };
    hipLaunchKernelGGL((k_zero<unsigned long long>), dim3(blocks_for(2 * (int64_t)cap, 256)), dim3(256), 0, s,
                       b.stats, (int64_t)2 * cap);
    hipLaunchKernelGGL((k_zero<unsigned int>), dim3(1), dim3(64), 0, s, b.stop, (int64_t)1);
    hipLaunchKernelGGL((k_zero<T>), dim3(blocks_for(n, 256)), dim3(256), 0, s, b.z[0], n);
    hipLaunchKernelGGL(k_set_one, dim3(1), dim3(1), 0, s, sizeof(T) == 4 ? (float *)b.z[0] : nullptr,
                       sizeof(T) == 8 ? (double *)b.z[0] : nullptr, nstar);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int cur = 0;
    double ak = 1.0;  // ramp_alpha^k (Supplement E's coupling ramp)
    bool done = false;
    while (!done && out->iters < o->max_iter) {
        const int batch = std::min(out->iters == 0 ? 2 : kDomBatch, o->max_iter - out->iters);
        bool ramping[kDomBatch] = {};
        for (int j = 0; j < batch; ++j) {
            const int it = out->iters + j;
            unsigned long long *st = b.stats + 2 * it;
            double lam = p->lambda;
            if (o->ramp_alpha > 0.0) {
                ak *= o->ramp_alpha;
                if (ak >= 0x1p-53) {
                    lam = p->lambda * (1.0 - ak);
                    ramping[j] = true;
                }
            }
            const T *zin = b.z[(cur + j) & 1];
            T *zout = b.z[(cur + j + 1) & 1];
            if (it == 0) {  // z = e_nstar: closed form
                if (csr)
                    hipLaunchKernelGGL((k_dom_first<T, true>), dim3(blocks_for(n, 256, 8192)), dim3(256), 0, s,
                                       rowptr, col, val, n, nstar, lam, theta, zout, st);
                else
                    hipLaunchKernelGGL((k_dom_first<T, false>), dim3(blocks_for(n, 256, 8192)), dim3(256), 0, s,
                                       (const int64_t *)nullptr, (const int *)nullptr, val, n, nstar, lam, theta,
                                       zout, st);
            } else if (csr) {  // b.s = (Delta z)[nstar] of zin, from the end of the previous iteration
                hipLaunchKernelGGL((k_dom_csr<T>), dim3(blocks_for(n, 32, kDomGrid)), dim3(256), 0, s, rowptr, col,
                                   val, n, nstar, lam, theta, (const double *)b.s, zin, zout, st,
                                   (const unsigned int *)b.stop);
            } else {
                hipLaunchKernelGGL((k_dom_dense<T>), dim3(blocks_for(n, 4)), dim3(256), 0, s, val, n, nstar, lam,
                                   theta, (const double *)b.s, zin, zout, st, (const unsigned int *)b.stop);
            }
            row_dot(zout, st, ramping[j] ? 0 : 1);
        }
        e = hipGetLastError();
        if (e == hipSuccess)
            e = hipMemcpyAsync(hs, b.stats + 2 * out->iters, 16 * (size_t)batch, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(hs + 2 * batch, b.s, 8, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        int taken = 0;
        for (int j = 0; j < batch && !done; ++j) {
            taken = j + 1;
            out->iters += 1;
            const double dl = bits_to_double(hs[2 * j]), wm = bits_to_double(hs[2 * j + 1]);
            out->last = dl;
            if (r && r->delta_history && out->iters - 1 < r->history_cap) r->delta_history[out->iters - 1] = dl;
            if (!std::isfinite(dl) || !(wm <= o->blowup)) {
                out->status = DPT_DIVERGED;
                done = true;
            } else if (!ramping[j] && dl < o->tol) {
                out->status = DPT_OK;
                done = true;
            }
        }
        cur = (cur + taken) & 1;
        hs[2] = hs[2 * batch];  // the scalar of the returned iterate
    }
    // eigenvalue readout from the returned iterate: read back with the last
    // batch, or (no iteration) from e_nstar
    if (out->iters == 0) {
        row_dot((const T *)b.z[cur], nullptr, 0);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(hs + 2, b.s, 8, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
    }
    *eigval = theta_star + p->lambda * bits_to_double(hs[2]);
    if (out64)
        hipLaunchKernelGGL((k_convert<T, double>), dim3(blocks_for(n, 256)), dim3(256), 0, s, (const T *)b.z[cur],
                           (double *)dst, n);
    else
        hipLaunchKernelGGL((k_convert<T, float>), dim3(blocks_for(n, 256)), dim3(256), 0, s, (const T *)b.z[cur],
                           (float *)dst, n);
    return hipGetLastError();
}

void fill_dom_result(dpt_result *r, const DomOutcome &out, bool fp64) {
    if (!r) return;
    r->status = out.status;
    r->iters = out.iters;
    r->iters_bf16 = 0;
    r->iters_fp32 = fp64 ? 0 : out.iters;
    r->iters_fp64 = fp64 ? out.iters : 0;
    r->last_delta = out.last;
}

template <typename T>
int dominant_t(const dpt_problem *p, const dpt_options *o, const double *theta_host, double theta_star,
               int64_t nstar, double *eigval, void *eigvec, dpt_result *r, bool csr_validated = false) {
    const int64_t n = p->n;
    hipStream_t s = (hipStream_t)p->stream;
    int rc = DPT_OK;
    DevCsr<T> csr;
    T *val = nullptr, *dense = nullptr;
    DomBuffers<T> b;
    const double *theta = nullptr;
    double *theta_own = nullptr;
    void *out_tmp = nullptr;
    const int cap = std::max(1, o->max_iter);
    DomOutcome out;
    unsigned long long *words = (unsigned long long *)pinned_block_take();  // read-backs (null: pageable)
    auto run = [&]() -> hipError_t {
        hipError_t e;
        if (p->format == DPT_CSR) {
            rc = stage_csr(p, &csr, s, csr_validated);
            if (rc != DPT_OK) return hipSuccess;
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
        // work buffers from the library's pool (no hipMalloc / hipFree per call
        // for problems up to 4 MiB per iterate)
        e = pooled_malloc((void **)&b.s, sizeof(double));
        if (e == hipSuccess) e = pooled_malloc((void **)&b.stop, sizeof(unsigned int));
        if (e == hipSuccess) e = pooled_malloc((void **)&b.stats, sizeof(unsigned long long) * 2 * cap);
        for (int i = 0; i < 2 && e == hipSuccess; ++i) e = pooled_malloc((void **)&b.z[i], sizeof(T) * n);
        if (e != hipSuccess) return e;
        if (theta_host) {  // host inputs: upload theta; device inputs: borrow it
            e = pooled_malloc((void **)&theta_own, sizeof(double) * n);
            if (e == hipSuccess)
                e = hipMemcpyAsync(theta_own, theta_host, sizeof(double) * n, hipMemcpyHostToDevice, s);
            if (e != hipSuccess) return e;
            theta = theta_own;
        } else {
            theta = p->theta;
        }
        // eigenvector in the problem's dtype and memory kind
        const bool out64 = p->dtype == DPT_DTYPE_F64;
        const size_t ob = (size_t)n * (out64 ? 8 : 4);
        void *dst = eigvec;
        if (p->mem == DPT_MEM_HOST) {
            e = pooled_malloc(&out_tmp, ob);
            if (e != hipSuccess) return e;
            dst = out_tmp;
        }
        const bool is_csr = p->format == DPT_CSR;
        e = dominant_iterate<T>(p, o, is_csr ? csr.rowptr : nullptr, is_csr ? csr.col : nullptr,
                                is_csr ? csr.val : (const T *)dense, theta, theta_star, nstar, b, cap, dst, out64,
                                eigval, &out, r, s, words);
        if (e == hipSuccess && out_tmp) e = hipMemcpyAsync(eigvec, out_tmp, ob, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        return e;
    };
    hipError_t e = run();
    const hipError_t es = hipStreamSynchronize(s);
    if (es == hipSuccess) pinned_block_give(words);  // drained; after a device error the block is not reused
    csr.release();
    if (val) (void)hipFree(val);
    // the stream has drained (or failed: then the blocks are not reused)
    if (es == hipSuccess) {
        for (int i = 0; i < 2; ++i) pooled_free(b.z[i]);
        pooled_free(theta_own);
        pooled_free(b.s);
        pooled_free(b.stop);
        pooled_free(b.stats);
        pooled_free(out_tmp);
    }
    if (rc != DPT_OK) return rc;
    if (e != hipSuccess) return err_code(e);
    fill_dom_result(r, out, sizeof(T) == 8);
    return out.status;
}

// Device-side theta checks into the caller's ThetaScan: the launches, then the
// verdict on the scan read back.
void theta_check_enqueue(const double *theta, int64_t n, int64_t index, ThetaScan *sc, hipStream_t s) {
    if (n <= kThetaSmall) {
        hipLaunchKernelGGL(k_theta_scan_small, dim3(1), dim3(1024), 0, s, theta, n, index, sc);
        return;
    }
    const unsigned int g = blocks_for(n, 256, 1024);
    hipLaunchKernelGGL(k_theta_scan_init, dim3(1), dim3(64), 0, s, sc, n, index);
    hipLaunchKernelGGL(k_theta_max, dim3(g), dim3(256), 0, s, theta, n, sc);
    hipLaunchKernelGGL(k_theta_argmax, dim3(g), dim3(256), 0, s, theta, n, sc, index);
    hipLaunchKernelGGL(k_theta_count, dim3(g), dim3(256), 0, s, theta, n, sc);
}

int theta_check_verdict(const ThetaScan &h, int64_t n, int64_t *index, double *theta_index) {
    if (h.bad || h.index >= (unsigned long long)n || h.count != 1) return DPT_EINVAL;
    *index = (int64_t)h.index;
    *theta_index = bits_to_double(h.value_bits);
    return DPT_OK;
}

// The checks with their own synchronisation (allocates nothing).
int theta_check_into(const double *theta, int64_t n, int64_t *index, double *theta_index, ThetaScan *sc,
                     hipStream_t s) {
    ThetaScan h{};
    theta_check_enqueue(theta, n, *index, sc, s);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&h, sc, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return err_code(e);
    return theta_check_verdict(h, n, index, theta_index);
}

}  // namespace

int dominant_solve(const dpt_problem *p, const dpt_options *o, const double *theta_host, double theta_index,
                   int64_t index, double *eigval, void *eigvec, dpt_result *r) {
    if (o->precision == DPT_FP64) return dominant_t<double>(p, o, theta_host, theta_index, index, eigval, eigvec, r);
    return dominant_t<float>(p, o, theta_host, theta_index, index, eigval, eigvec, r);
}

// Device inputs: the theta checks and (CSR) the structure check run together
// and are read back with one synchronisation, then the solve.
int dominant_solve_device(const dpt_problem *p, const dpt_options *o, int64_t index, double *eigval, void *eigvec,
                          dpt_result *r) {
    hipStream_t s = (hipStream_t)p->stream;
    unsigned char *dev = nullptr;  // ThetaScan at 0, the CSR flag at 256
    hipError_t e = pooled_malloc((void **)&dev, 512);
    if (e != hipSuccess) return err_code(e);
    ThetaScan *sc = (ThetaScan *)dev;
    unsigned int *flag = (unsigned int *)(dev + 256);
    const bool csr = p->format == DPT_CSR;
    theta_check_enqueue(p->theta, p->n, index, sc, s);
    if (csr) {
        hipLaunchKernelGGL((k_zero<unsigned int>), dim3(1), dim3(64), 0, s, flag, (int64_t)1);
        hipLaunchKernelGGL(k_csr_validate, dim3(blocks_for(p->n, 32)), dim3(256), 0, s, p->indptr, p->indices, p->n,
                           p->nnz, flag);
    }
    unsigned char *hw = (unsigned char *)pinned_block_take();
    unsigned char local[sizeof(ThetaScan) + sizeof(unsigned int)];
    unsigned char *hb = hw ? hw : local;
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(hb, sc, sizeof(ThetaScan), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && csr)
        e = hipMemcpyAsync(hb + sizeof(ThetaScan), flag, sizeof(unsigned int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    ThetaScan h{};
    unsigned int hflag = 0;
    if (e == hipSuccess) {
        std::memcpy(&h, hb, sizeof(ThetaScan));
        if (csr) std::memcpy(&hflag, hb + sizeof(ThetaScan), sizeof(unsigned int));
        pinned_block_give(hw);
        pooled_free(dev);  // drained
    }
    if (e != hipSuccess) return err_code(e);
    double theta_index = 0.0;
    int rc = theta_check_verdict(h, p->n, &index, &theta_index);
    if (rc != DPT_OK) return rc;
    if (hflag) return DPT_EINVAL;
    if (o->precision == DPT_FP64)
        return dominant_t<double>(p, o, nullptr, theta_index, index, eigval, eigvec, r, csr);
    return dominant_t<float>(p, o, nullptr, theta_index, index, eigval, eigvec, r, csr);
}

// ------------------------------------------------- dominant mode, no allocation
// Work memory of dpt_dominant_noalloc: one fixed array per GPU, for callers that
// cannot allocate (HIP graph capture, serving loops).  Layout: a 4 KiB header
// (the scalar s at 0, the theta scan at 256, the CSR check flag at 512, the
// iteration's stop flag at 768), the statistics of up to
// kNoallocMaxIter iterations, then the two iterates.  Host code must use the
// device address from hipGetSymbolAddress (per device), never `scratch` itself.
constexpr size_t kScratchHeader = 4096;
constexpr size_t kScratchStats = (size_t)2 * kNoallocMaxIter * sizeof(unsigned long long);
constexpr size_t kScratchBytes = kScratchHeader + kScratchStats + kNoallocVectorBytes;
static_assert(kScratchStats % 256 == 0, "iterates stay 256-byte aligned");
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// Device address of `scratch` on the current device, looked up once per device.
int scratch_address(unsigned char **out) {
    static std::mutex mu;
    static unsigned char *addr[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return DPT_EDEVICE;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return DPT_EDEVICE;
        }
        addr[dev] = (unsigned char *)ptr;
    }
    *out = addr[dev];
    return DPT_OK;
}

template <typename T>
int dominant_noalloc_t(const dpt_problem *p, const dpt_options *o, int64_t index, double *eigval, void *eigvec,
                       dpt_result *r, unsigned char *base) {
    const int64_t n = p->n;
    hipStream_t s = (hipStream_t)p->stream;
    double *s_dev = (double *)base;
    ThetaScan *scan = (ThetaScan *)(base + 256);
    unsigned int *flag = (unsigned int *)(base + 512);
    DomBuffers<T> b;
    b.s = s_dev;
    b.stop = (unsigned int *)(base + 768);
    b.stats = (unsigned long long *)(base + kScratchHeader);
    const size_t zb = ((size_t)n * sizeof(T) + 255) / 256 * 256;
    b.z[0] = (T *)(base + kScratchHeader + kScratchStats);
    b.z[1] = (T *)(base + kScratchHeader + kScratchStats + zb);
    double theta_index = 0.0;
    int rc = theta_check_into(p->theta, n, &index, &theta_index, scan, s);
    if (rc != DPT_OK) return rc;
    const bool csr = p->format == DPT_CSR;
    if (csr) {
        rc = validate_device_csr(p, flag, s);
        if (rc != DPT_OK) return rc;
    }
    DomOutcome out;
    hipError_t e = dominant_iterate<T>(p, o, csr ? p->indptr : nullptr, csr ? p->indices : nullptr,
                                       (const T *)p->delta, p->theta, theta_index, index, b,
                                       std::max(1, o->max_iter), eigvec, sizeof(T) == 8, eigval, &out, r, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return err_code(e);
    fill_dom_result(r, out, sizeof(T) == 8);
    return out.status;
}

}  // namespace

int dominant_solve_noalloc(const dpt_problem *p, const dpt_options *o, int64_t index, double *eigval, void *eigvec,
                           dpt_result *r) {
    const bool fp64 = o->precision == DPT_FP64;
    const size_t esz = fp64 ? 8 : 4;
    if (p->dtype != (fp64 ? DPT_DTYPE_F64 : DPT_DTYPE_F32)) return DPT_EINVAL;
    if (o->max_iter > kNoallocMaxIter) return DPT_EINVAL;
    if (2 * (((size_t)p->n * esz + 255) / 256 * 256) > kNoallocVectorBytes) return DPT_EINVAL;
    unsigned char *base = nullptr;
    const int rc = scratch_address(&base);
    if (rc != DPT_OK) return rc;
    return fp64 ? dominant_noalloc_t<double>(p, o, index, eigval, eigvec, r, base)
                : dominant_noalloc_t<float>(p, o, index, eigval, eigvec, r, base);
}

}  // namespace dpt
