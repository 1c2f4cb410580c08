// Display-side kernels after the hologram: double-phase amplitude coding (DPAC) of the
// complex SLM field into one phase-only pattern (Sec. 5 and the supplement's display
// section, in the standard double-phase form of the works cited there), and the unit-phasor
// field e^{jP} of such a pattern for the focal-stack simulation.
//
// DPAC: a e^{j phi} = a_max (e^{j P-} + e^{j P+}) / 2 with P-/+ = phi -/+ arccos(a / a_max);
// P- is written where n_x + n_y is even, P+ where it is odd.  All elementwise and HBM bound.
#include "gws_internal.h"

namespace gws {

constexpr int DISP_THREADS = 256;

static __device__ __forceinline__ float magnitude(float2 v) { return sqrtf(fmaf(v.x, v.x, v.y * v.y)); }

__global__ void __launch_bounds__(64) k_zero_u32(uint32_t *p, int n)
{
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

// Per-channel max |u|: grid-stride per channel (blockIdx.y = channel), wave and work-group
// maxima, one atomicMax per work-group on the float's bits (non-negative floats order like
// their bit patterns).
__global__ void __launch_bounds__(DISP_THREADS) k_amax(const float2 *__restrict__ u, int64_t m,
                                                       uint32_t *__restrict__ amax_bits)
{
    __shared__ float s_max[DISP_THREADS / 64];
    const int c = blockIdx.y;
    const float2 *src = u + (int64_t)c * m;
    float mx = 0.0f;
    const int64_t stride = (int64_t)gridDim.x * DISP_THREADS;
    for (int64_t i = (int64_t)blockIdx.x * DISP_THREADS + threadIdx.x; i < m; i += 4 * stride) {
        // four independent loads in flight per thread
        float2 v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = i + q * stride < m ? src[i + q * stride] : make_float2(0.0f, 0.0f);
#pragma unroll
        for (int q = 0; q < 4; ++q) mx = fmaxf(mx, magnitude(v[q]));
    }
    for (int d = 32; d >= 1; d >>= 1) mx = fmaxf(mx, __shfl_xor(mx, d));
    if ((threadIdx.x & 63) == 0) s_max[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        float b = s_max[0];
        for (int w = 1; w < DISP_THREADS / 64; ++w) b = fmaxf(b, s_max[w]);
        atomicMax(&amax_bits[c], __float_as_uint(b));
    }
}

hipError_t launch_amax(const float2 *u, int64_t m, int C, uint32_t *amax_bits, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, amax_bits, C);
    if (m <= 0) return hipGetLastError();
    // few work-groups per channel: each ends with one atomic on the channel's word
    const int64_t want = (m + DISP_THREADS * 16 - 1) / (DISP_THREADS * 16);
    const int nb = (int)(want < 128 ? want : 128);
    hipLaunchKernelGGL(k_amax, dim3(nb, C), dim3(DISP_THREADS), 0, s, u, m, amax_bits);
    return hipGetLastError();
}

// One row of one channel per blockIdx.y, DPAC_PER_THREAD pixels of it per thread.
constexpr int DPAC_PER_THREAD = 4;
__global__ void __launch_bounds__(DISP_THREADS) k_dpac(const float2 *__restrict__ u, int nx, int ny,
                                                       const uint32_t *__restrict__ amax_bits, float amax_fixed,
                                                       float *__restrict__ phase)
{
    const int row = blockIdx.y, c = row / ny, y = row - c * ny;
    const float am = amax_bits ? __uint_as_float(amax_bits[c]) : amax_fixed;
    const float2 *src = u + (int64_t)row * nx;
    float *dst = phase + (int64_t)row * nx;
#pragma unroll
    for (int q = 0; q < DPAC_PER_THREAD; ++q) {
        const int x = (blockIdx.x * DPAC_PER_THREAD + q) * DISP_THREADS + threadIdx.x;
        if (x < nx) {
            const float2 v = src[x];
            const float r = am > 0.0f ? fminf(magnitude(v) / am, 1.0f) : 0.0f;
            const float th = acosf(r), phi = atan2f(v.y, v.x);
            dst[x] = ((x + y) & 1) ? phi + th : phi - th;
        }
    }
}

hipError_t launch_dpac(const float2 *u, int nx, int ny, int C, const uint32_t *amax_bits, float amax_fixed,
                       float *phase, hipStream_t s)
{
    if ((int64_t)nx * ny * C <= 0) return hipSuccess;
    if ((int64_t)C * ny > 65535) return hipErrorInvalidValue;  // one grid row per image row
    const int per = DPAC_PER_THREAD * DISP_THREADS;
    hipLaunchKernelGGL(k_dpac, dim3((nx + per - 1) / per, C * ny), dim3(DISP_THREADS), 0, s, u, nx, ny, amax_bits,
                       amax_fixed, phase);
    return hipGetLastError();
}

__global__ void __launch_bounds__(DISP_THREADS) k_phase_field(const float *__restrict__ phase, int64_t n,
                                                              float2 *__restrict__ u)
{
    for (int64_t i = (int64_t)blockIdx.x * DISP_THREADS + threadIdx.x; i < n; i += (int64_t)gridDim.x * DISP_THREADS) {
        float sn, cs;
        sincosf(phase[i], &sn, &cs);
        u[i] = make_float2(cs, sn);
    }
}

hipError_t launch_phase_field(const float *phase, int64_t n, float2 *u, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t want = (n + DISP_THREADS * 4 - 1) / (DISP_THREADS * 4);
    const int nb = (int)(want < 8192 ? want : 8192);
    hipLaunchKernelGGL(k_phase_field, dim3(nb), dim3(DISP_THREADS), 0, s, phase, n, u);
    return hipGetLastError();
}

}  // namespace gws
