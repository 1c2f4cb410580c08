// Field loss used by the training step around the hot path: L = sum |u - t|^2 and its
// gradient in torch's complex convention, G = dL/dRe u + j dL/dIm u = 2 (u - t).
// One pass over u and t; the sum is reduced per block in a fixed order, then the block
// sums are added in a fixed order by one more block (bitwise reproducible).
#include "gws_internal.h"

namespace gws {

constexpr int LOSS_THREADS = 256;
constexpr int LOSS_BLOCKS = 1024;

__global__ void __launch_bounds__(LOSS_THREADS) k_l2_grad(const float2 *__restrict__ u, const float2 *__restrict__ t,
                                                          float2 *__restrict__ g, double *__restrict__ block_sums,
                                                          int64_t n)
{
    __shared__ double red[LOSS_THREADS];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float2 a = u[i], b = t[i];
        const float dx = a.x - b.x, dy = a.y - b.y;
        if (g) g[i] = make_float2(2.0f * dx, 2.0f * dy);
        s += (double)dx * dx + (double)dy * dy;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = LOSS_THREADS / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) block_sums[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(LOSS_THREADS) k_sum_blocks(const double *__restrict__ block_sums, int nb,
                                                             double *__restrict__ out)
{
    __shared__ double red[LOSS_THREADS];
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) s += block_sums[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = LOSS_THREADS / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

size_t l2_workspace_bytes() { return sizeof(double) * (LOSS_BLOCKS + 1); }

hipError_t launch_l2_grad(const float2 *u, const float2 *t, float2 *g, double *loss, void *ws, int64_t n, hipStream_t s)
{
    double *bs = (double *)ws;
    const int64_t want = (n + LOSS_THREADS - 1) / LOSS_THREADS;
    const int nb = (int)(want < LOSS_BLOCKS ? (want > 0 ? want : 1) : LOSS_BLOCKS);
    hipLaunchKernelGGL(k_l2_grad, dim3(nb), dim3(LOSS_THREADS), 0, s, u, t, g, bs, n);
    hipLaunchKernelGGL(k_sum_blocks, dim3(1), dim3(LOSS_THREADS), 0, s, bs, nb, loss);
    return hipGetLastError();
}

}  // namespace gws
