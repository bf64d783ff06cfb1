// Measurement probe (not part of the method): the rate at which the GPU serves
// random gathers of fixed-size row runs from a panel, the access pattern of
// the CSR product's state gathers.  Each group of 32 lanes reads `gathers`
// runs of 512 bytes from rows of a panel of `panel_rows` rows chosen by a
// counter-based hash (SplitMix64 finaliser of the gather index), and sums them,
// with 8 runs in flight per lane; only one value per group is written.  The
// figure is the roof the product's gathers are compared with.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "dpt.h"

namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// panel: panel_rows x 128 floats (512-byte rows).  Group g (32 lanes, 16 bytes
// each) handles gathers [g * per_group, (g + 1) * per_group).
__global__ __launch_bounds__(256) void k_probe_gather(const float4 *__restrict__ panel, int64_t panel_rows,
                                                      int64_t per_group, uint64_t seed, float *__restrict__ out) {
    const int lane = threadIdx.x & 31;
    const int64_t g = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 5;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    const int64_t base = g * per_group;
    for (int64_t i = 0; i < per_group; i += 8) {
        float4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t row = (int64_t)(mix64(seed + (uint64_t)(base + i + u)) % (uint64_t)panel_rows);
            v[u] = panel[row * 32 + lane];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            acc.x += v[u].x;
            acc.y += v[u].y;
            acc.z += v[u].z;
            acc.w += v[u].w;
        }
    }
    const float s = (acc.x + acc.y) + (acc.z + acc.w);
    if (lane == 0) out[g] = s;
}

}  // namespace

extern "C" int dpt_probe_gather(int64_t panel_rows, int64_t gathers, int reps, double *ms_per_pass, double *gbs) {
    if (panel_rows < 1 || gathers < 1 || reps < 1 || !gbs || !ms_per_pass) return DPT_EINVAL;
    const int64_t groups = 65536;  // 2048 blocks of 8 groups
    const int64_t per_group = std::max<int64_t>(8, (gathers / groups + 7) / 8 * 8);
    float4 *panel = nullptr;
    float *out = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipMalloc((void **)&panel, (size_t)panel_rows * 512);
    if (e == hipSuccess) e = hipMalloc((void **)&out, sizeof(float) * groups);
    if (e == hipSuccess) e = hipMemset(panel, 0, (size_t)panel_rows * 512);
    if (e == hipSuccess) e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    float ms = 0.f;
    if (e == hipSuccess) {
        const dim3 grid((unsigned int)(groups * 32 / 256));
        hipLaunchKernelGGL(k_probe_gather, grid, dim3(256), 0, nullptr, panel, panel_rows, per_group, 1ull, out);
        (void)hipEventRecord(a, nullptr);
        for (int r = 0; r < reps; ++r)
            hipLaunchKernelGGL(k_probe_gather, grid, dim3(256), 0, nullptr, panel, panel_rows, per_group,
                               (uint64_t)(r + 2) << 40, out);
        (void)hipEventRecord(b, nullptr);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipEventSynchronize(b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (panel) (void)hipFree(panel);
    if (out) (void)hipFree(out);
    if (e != hipSuccess) return DPT_EDEVICE;
    const double per = ms / reps;
    *ms_per_pass = per;
    *gbs = (double)(groups * per_group) * 512.0 / (per * 1e-3) / 1e9;
    return DPT_OK;
}
