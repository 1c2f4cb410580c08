// Exact alpha wave blending (Sec. 4, Eq. 5-6; supplement Alg. 2) on gfx950.
//
// The Gaussians are taken front to back (descending depth, ties by input index).  Gaussian k
// splats its own wavefront u_k = e^{j phi_k} g_k(x) (its profile on its plane, peak 1),
// masked by the transmittance T_k(x) = prod_{j in front} (1 - alpha_j(x)), into the
// spectrum after propagation by H(nu, -z_k):
//   U_c(nu) += a_{k,c} o_k H_c(nu, -z_k) DFT(T_k u_k)(nu),
// and alpha_k = o_k g_k, dropped where it does not exceed 1/255, updates the map.
//
// The map makes the work sequential in k, so it runs in batches of B Gaussians:
//   k_exact_mask   one work-group per 16 x 16 pixel tile: walks the batch in order, writes
//                  T u_k of every batch Gaussian into its own full-grid image (zero where
//                  the Gaussian's eps-window misses the tile) and updates T in place;
//   (FFT)          the batched forward 2D transform of the B images (k_fft);
//   k_exact_splat  one thread per frequency: H(nu, -z_k) with the phase -z_k sqrt(1/l^2 -
//                  |nu|^2) reduced in FP64, times a_{k,c} o_k, accumulated into the spectrum.
// The spectrum is kept in the library's convention (U (-1)^{m'} / (Nx Ny px py), FFT order),
// so DFT(T u_k)(nu_m) = px py (-1)^{m'} FFT(T u_k)[m] enters as FFT(T u_k)[m] / (Nx Ny).
// The profile is truncated where it falls below eps of its peak (the same eps as the
// order-invariant path's spectral culling).
#include <algorithm>

#include "gws_internal.h"

namespace gws {

constexpr float EXACT_T_EPS = 1.0f / 255.0f;
constexpr int EXACT_TILE = 16;

// Per-Gaussian record of the exact path, in front-to-back order (64 bytes).
struct alignas(16) ERec {
    float cx, cy;           // centre in pixel coordinates: n = x / p + N / 2
    float qa, qb, qc;       // exponent in powers of two: -(qa dx^2 + qb dx dy + qc dy^2), pixel units
    float o;                // opacity (alpha = o g)
    float cphi, sphi;       // e^{j phi}
    float z;                // depth (m)
    int32_t hwx, hwy;       // eps-window half-widths (pixels)
    int32_t valid;
    float amp[4];           // a_c o
};
static_assert(sizeof(ERec) == 64, "ERec is 64 bytes");

static __device__ __forceinline__ bool finite_e(float v) { return (__float_as_uint(v) & 0x7f800000u) != 0x7f800000u; }

// Sort key: descending depth (front to back), as an unsigned order on the float bits.
__global__ void __launch_bounds__(256) k_exact_keys(GView g, uint64_t *__restrict__ keys, uint32_t *__restrict__ vals)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.n) return;
    const float z = g.depth[i];
    uint32_t b = __float_as_uint(finite_e(z) && z != 0.0f ? z : 0.0f);  // one zero, so -0 ties with +0
    b = (b & 0x80000000u) ? ~b : (b | 0x80000000u);  // ascending unsigned order of z
    keys[i] = (uint64_t)(~b);                         // descending z
    vals[i] = (uint32_t)i;
}

__global__ void __launch_bounds__(256) k_exact_records(GView g, Consts k, const uint32_t *__restrict__ order,
                                                       ERec *__restrict__ rec)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.n) return;
    const int64_t j = order[i];
    const float sxx = g.cov_xx[j], sxy = g.cov_xy[j], syy = g.cov_yy[j];
    const float mx = g.mean_x[j], my = g.mean_y[j], z = g.depth[j], o = g.opacity[j], ph = g.phase[j];
    const double det = (double)sxx * syy - (double)sxy * sxy;
    bool ok = finite_e(sxx) && finite_e(sxy) && finite_e(syy) && finite_e(mx) && finite_e(my) && finite_e(z) &&
              finite_e(o) && finite_e(ph) && sxx > 0.0f && syy > 0.0f && det > 0.0 && o >= 0.0f;
    ERec r;
    r.cx = (float)(mx / k.px + 0.5 * k.nx);
    r.cy = (float)(my / k.py + 0.5 * k.ny);
    // Sigma in pixel units and its inverse; exponent -1/2 d^T Sigma^-1 d in powers of two
    const double a = sxx / (k.px * k.px), b = sxy / (k.px * k.py), c = syy / (k.py * k.py);
    const double dpx = a * c - b * b;
    const double h = 0.5 / log(2.0);
    r.qa = ok ? (float)(h * c / dpx) : 0.0f;
    r.qb = ok ? (float)(-2.0 * h * b / dpx) : 0.0f;
    r.qc = ok ? (float)(h * a / dpx) : 0.0f;
    r.o = ok ? o : 0.0f;
    r.cphi = cosf(ph);
    r.sphi = sinf(ph);
    r.z = ok ? z : 0.0f;
    // eps-window: g >= eps  <=>  d^T Sigma^-1 d <= 2 ln(1/eps) = 2 ln 2 tau2
    const double r2 = 2.0 * log(2.0) * k.tau2;
    r.hwx = ok ? (int)min(ceil(sqrt(r2 * a)), (double)(k.nx / 2 - 1)) : -1;
    r.hwy = ok ? (int)min(ceil(sqrt(r2 * c)), (double)(k.ny / 2 - 1)) : -1;
    for (int q = 0; q < 4; ++q) {
        float v = 0.0f;
        if (q < k.C) {
            const float am = g.amplitude[(int64_t)q * g.amp_stride + j];
            ok = ok && finite_e(am);
            v = am * o;
        }
        r.amp[q] = v;
    }
    r.valid = ok ? 1 : 0;
    if (!ok) {
        r.o = 0.0f;
        r.hwx = r.hwy = -1;
        for (int q = 0; q < 4; ++q) r.amp[q] = 0.0f;
    }
    rec[i] = r;
}

// Wrapped displacement of pixel coordinate v from centre c on a periodic axis of length n.
static __device__ __forceinline__ float wrap_d(float d, float n)
{
    return d - n * rintf(d / n);
}

// One work-group per 16 x 16 pixel tile; walks Gaussians [b0, b0 + nb) in order.
__global__ void __launch_bounds__(256) k_exact_mask(const ERec *__restrict__ rec, int b0, int nb, int nx, int ny,
                                                    float *__restrict__ tmap, float2 *__restrict__ imgs)
{
    __shared__ ERec s_rec[64];
    const int tx = blockIdx.x, ty = blockIdx.y;
    const int px = tx * EXACT_TILE + (threadIdx.x & 15), py = ty * EXACT_TILE + (threadIdx.x >> 4);
    const bool in = px < nx && py < ny;
    for (int i = threadIdx.x; i < nb * 4; i += blockDim.x)
        reinterpret_cast<float4 *>(s_rec)[i] = reinterpret_cast<const float4 *>(rec + b0)[i];
    __syncthreads();
    const int64_t M = (int64_t)nx * ny;
    const int64_t pix = (int64_t)py * nx + px;
    float T = in ? tmap[pix] : 1.0f;
    // tile centre, for the work-group-uniform window test
    const float tcx = tx * EXACT_TILE + 7.5f, tcy = ty * EXACT_TILE + 7.5f;
    for (int b = 0; b < nb; ++b) {
        const ERec &r = s_rec[b];
        const float dcx = fabsf(wrap_d(tcx - r.cx, (float)nx)), dcy = fabsf(wrap_d(tcy - r.cy, (float)ny));
        const bool hit = r.hwx >= 0 && dcx <= (float)r.hwx + 8.5f && dcy <= (float)r.hwy + 8.5f;
        float2 v = make_float2(0.0f, 0.0f);
        if (hit) {
            const float dx = wrap_d((float)px - r.cx, (float)nx), dy = wrap_d((float)py - r.cy, (float)ny);
            const float q = fmaf(r.qa * dx, dx, fmaf(r.qb * dx, dy, r.qc * dy * dy));
            const float gk = __builtin_amdgcn_exp2f(-q);
            const float m = T * gk;
            v = make_float2(m * r.cphi, m * r.sphi);
            const float alpha = r.o * gk;
            if (alpha > EXACT_T_EPS) T *= 1.0f - alpha;
        }
        if (in) imgs[(int64_t)b * M + pix] = v;
    }
    if (in) tmap[pix] = T;
}

// One thread per frequency (FFT order): U_c += a_{k,c} o_k H_c(nu, -z_k) FFT(T u_k) / (Nx Ny).
__global__ void __launch_bounds__(256) k_exact_splat(const ERec *__restrict__ rec, int b0, int nb, Consts k,
                                                     const float2 *__restrict__ imgs, float2 *__restrict__ spec)
{
    const int64_t M = (int64_t)k.nx * k.ny;
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const int mx = (int)(m % k.nx), my = (int)(m / k.nx);
    const int mxp = 2 * mx < k.nx ? mx : mx - k.nx, myp = 2 * my < k.ny ? my : my - k.ny;
    const double nux = mxp / (k.nx * k.px), nuy = myp / (k.ny * k.py);
    const double nu2 = nux * nux + nuy * nuy;
    const float scale = (float)(1.0 / ((double)k.nx * k.ny));
    double w[4];
    bool prop[4];
    float2 acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const double w2 = k.inv_lambda[c] * k.inv_lambda[c] - nu2;
        prop[c] = c < k.C && w2 > 0.0;
        w[c] = prop[c] ? sqrt(w2) : 0.0;
        acc[c] = c < k.C ? spec[(int64_t)c * M + m] : make_float2(0.0f, 0.0f);
    }
    for (int b = 0; b < nb; ++b) {
        const ERec &r = rec[b0 + b];
        if (!r.valid) continue;
        const float2 S = imgs[(int64_t)b * M + m];
        const double zd = (double)r.z;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (!prop[c]) continue;
            const double ph = -zd * w[c];  // revolutions of H(nu, -z)
            const float t = (float)(ph - floor(ph));
            const float cs = __builtin_amdgcn_cosf(t), sn = __builtin_amdgcn_sinf(t);
            const float A = r.amp[c] * scale;
            const float hr = A * cs, hi = A * sn;
            acc[c].x = fmaf(hr, S.x, fmaf(-hi, S.y, acc[c].x));
            acc[c].y = fmaf(hr, S.y, fmaf(hi, S.x, acc[c].y));
        }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
        if (c < k.C) spec[(int64_t)c * M + m] = acc[c];
}

__global__ void __launch_bounds__(256) k_exact_fill(float *__restrict__ tmap, float2 *__restrict__ spec, int64_t M,
                                                    int C)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < M) tmap[i] = 1.0f;
    if (i < M * C) spec[i] = make_float2(0.0f, 0.0f);
}

size_t exact_batch(int nx, int ny)
{
    // up to 64 Gaussians per batch, their images within 1 GiB
    const size_t img = (size_t)nx * ny * sizeof(float2);
    size_t b = ((size_t)1 << 30) / img;
    if (b > 64) b = 64;
    if (b < 1) b = 1;
    return b;
}

hipError_t run_exact_forward(const Plan &p, const Consts &k, const GView &g, const ExactBuffers &eb, float2 *spec,
                             hipStream_t s)
{
    ERec *rec = (ERec *)eb.rec;
    const int64_t n = g.n, M = (int64_t)k.nx * k.ny;
    const unsigned gn = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_exact_fill, dim3((unsigned)((M * k.C + 255) / 256)), dim3(256), 0, s, eb.tmap, spec, M,
                       k.C);
    if (n == 0) return hipGetLastError();
    hipLaunchKernelGGL(k_exact_keys, dim3(gn), dim3(256), 0, s, g, eb.keys_a, eb.vals_a);
    uint64_t *keys = nullptr;
    uint32_t *order = nullptr;
    hipError_t e = radix_sort_48(eb.keys_a, eb.vals_a, eb.keys_b, eb.vals_b, eb.sort_hist, n, eb.sort_blocks, s, &keys,
                                 &order);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_exact_records, dim3(gn), dim3(256), 0, s, g, k, order, rec);
    const int B = (int)exact_batch(k.nx, k.ny);
    const dim3 tiles((k.nx + EXACT_TILE - 1) / EXACT_TILE, (k.ny + EXACT_TILE - 1) / EXACT_TILE);
    for (int64_t b0 = 0; b0 < n; b0 += B) {
        const int nb = (int)std::min<int64_t>(B, n - b0);
        hipLaunchKernelGGL(k_exact_mask, tiles, dim3(256), 0, s, rec, (int)b0, nb, k.nx, k.ny, eb.tmap, eb.imgs);
        e = launch_fft2d(p, nb, -1, eb.imgs, eb.imgs, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_exact_splat, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, rec, (int)b0, nb, k,
                           eb.imgs, spec);
    }
    return hipGetLastError();
}

}  // namespace gws
