// Issue-rate and bandwidth probes: the roofline denominators measured on the device the
// library runs on, beside the ones derived from unit counts and clock.
//   k_probe_trans: the spectrum accumulation's transcendental mix, 1 v_exp_f32 : 3 v_sin_f32 :
//                  3 v_cos_f32, as 8 independent dependency chains per lane (each op feeds the
//                  next of its chain, so no other VALU work is mixed in) at full occupancy.
//   k_probe_fma:   16 independent v_fma_f32 chains per lane.
//   k_probe_copy:  a float4 device-to-device copy (one read + one write per byte).
#include "gws_internal.h"

namespace gws {

constexpr int PROBE_THREADS = 256;

__global__ void __launch_bounds__(PROBE_THREADS) k_probe_trans(float *__restrict__ sink, int iters, float seed)
{
    float a[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = seed * (float)(threadIdx.x + 1) * 1e-4f + 0.01f * (float)j;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            a[j] = __builtin_amdgcn_exp2f(-a[j]);
            a[j] = __builtin_amdgcn_sinf(a[j]);
            a[j] = __builtin_amdgcn_cosf(a[j]);
            a[j] = __builtin_amdgcn_sinf(a[j]);
            a[j] = __builtin_amdgcn_cosf(a[j]);
            a[j] = __builtin_amdgcn_sinf(a[j]);
            a[j] = __builtin_amdgcn_cosf(a[j]);
        }
    }
    float r = 0.0f;
#pragma unroll
    for (int j = 0; j < 8; ++j) r += a[j];
    if (r == 12345.0f) sink[blockIdx.x] = r;  // never true in practice; keeps the chains live
}

__global__ void __launch_bounds__(PROBE_THREADS) k_probe_fma(float *__restrict__ sink, int iters, float seed)
{
    float a[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) a[j] = seed * (float)(threadIdx.x + 1) * 1e-4f + 0.01f * (float)j;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < 16; ++j) a[j] = fmaf(a[j], 0.99991f, 1e-7f);
    }
    float r = 0.0f;
#pragma unroll
    for (int j = 0; j < 16; ++j) r += a[j];
    if (r == 12345.0f) sink[blockIdx.x] = r;
}

__global__ void __launch_bounds__(PROBE_THREADS) k_probe_copy(const float4 *__restrict__ in, float4 *__restrict__ out,
                                                              int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = in[i];
}

// Times each probe with HIP events on `s` (best of three launches) and fills the rates.
hipError_t run_probes(int n_cu, hipStream_t s, double *trans_ops, double *valu_ops, double *hbm_bytes)
{
    const int blocks = n_cu * 16, iters_t = 256, iters_f = 4096;
    const int64_t copy_bytes = (int64_t)1 << 30, n4 = copy_bytes / 16;
    float *sink = nullptr;
    float4 *a = nullptr, *b = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t err = hipMalloc(&sink, sizeof(float) * blocks);
    if (err == hipSuccess) err = hipMalloc(&a, copy_bytes);
    if (err == hipSuccess) err = hipMalloc(&b, copy_bytes);
    if (err == hipSuccess) err = hipEventCreate(&e0);
    if (err == hipSuccess) err = hipEventCreate(&e1);
    double best[3] = {1e30, 1e30, 1e30};
    for (int probe = 0; probe < 3 && err == hipSuccess; ++probe) {
        for (int rep = 0; rep < 3 && err == hipSuccess; ++rep) {
            err = hipEventRecord(e0, s);
            if (err != hipSuccess) break;
            if (probe == 0)
                hipLaunchKernelGGL(k_probe_trans, dim3(blocks), dim3(PROBE_THREADS), 0, s, sink, iters_t, 1.0f);
            else if (probe == 1)
                hipLaunchKernelGGL(k_probe_fma, dim3(blocks), dim3(PROBE_THREADS), 0, s, sink, iters_f, 1.0f);
            else
                hipLaunchKernelGGL(k_probe_copy, dim3(n_cu * 8), dim3(PROBE_THREADS), 0, s, a, b, n4);
            err = hipGetLastError();
            if (err == hipSuccess) err = hipEventRecord(e1, s);
            if (err == hipSuccess) err = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
            if (err == hipSuccess && ms > 0.0f && ms < best[probe]) best[probe] = ms;
        }
    }
    if (err == hipSuccess) {
        const double lanes = (double)blocks * PROBE_THREADS;
        *trans_ops = lanes * iters_t * 8 * 7 / (best[0] * 1e-3);
        *valu_ops = lanes * iters_f * 16 / (best[1] * 1e-3);
        *hbm_bytes = 2.0 * (double)copy_bytes / (best[2] * 1e-3);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(sink);
    (void)hipFree(a);
    (void)hipFree(b);
    return err;
}

}  // namespace gws
