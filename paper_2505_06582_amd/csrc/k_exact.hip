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
//   k_exact_mask   one work-group per 16 x 16 pixel tile: walks the batch Gaussians whose
//                  window meets the tile in order, writes the real masked profiles T g_k of
//                  Gaussians 2p and 2p + 1 as the real and imaginary parts of image p (inside
//                  the pair's window rectangles only) and updates T in place;
//   (FFT)          the batched forward 2D transform of the B / 2 packed images (k_fft), only
//                  over the windows' columns and rectangles;
//   k_exact_splat  one thread per frequency pair {m, -m}: separates the pair's transforms by
//                  Hermitian symmetry, applies e^{j phi_k} and H(nu, -z_k) (the phase
//                  -z_k sqrt(1/l^2 - |nu|^2) reduced in FP64) times a_{k,c} o_k, and
//                  accumulates into the spectrum.
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

__global__ void k_exact_zero_counters(long long *__restrict__ counters)
{
    if (threadIdx.x < CTR_COUNT) counters[threadIdx.x] = 0;
}

// The record of input Gaussian j.  *culled: skipped as invalid; *clamped: its eps-window was
// cut at half the grid (its profile is truncated there).
static __device__ ERec make_erec(const GView &g, const Consts &k, int64_t j, bool *culled, bool *clamped)
{
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
    // eps-window: g >= eps  <=>  d^T Sigma^-1 d <= 2 ln(1/eps) = 2 ln 2 tau2, cut at N/2 - 1
    const double r2 = 2.0 * log(2.0) * k.tau2;
    const double wx = ceil(sqrt(r2 * a)), wy = ceil(sqrt(r2 * c));
    const double cx = (double)(k.nx / 2 - 1), cy = (double)(k.ny / 2 - 1);
    r.hwx = ok ? (int)min(wx, cx) : -1;
    r.hwy = ok ? (int)min(wy, cy) : -1;
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
    *culled = !ok;
    *clamped = ok && (wx > cx || wy > cy);
    return r;
}

// Records in front-to-back order; counts the culled and the clamped Gaussians (one atomic
// per wavefront and counter).
__global__ void __launch_bounds__(256) k_exact_records(GView g, Consts k, const uint32_t *__restrict__ order,
                                                       ERec *__restrict__ rec, long long *__restrict__ counters)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool culled = false, clamped = false;
    if (i < g.n) rec[i] = make_erec(g, k, order[i], &culled, &clamped);
    const int nc = __popcll(__ballot(culled)), nk = __popcll(__ballot(clamped));
    if ((threadIdx.x & 63) == 0) {
        if (nc) atomicAdd((unsigned long long *)&counters[CTR_NCULLED], (unsigned long long)nc);
        if (nk) atomicAdd((unsigned long long *)&counters[CTR_CLAMPED], (unsigned long long)nk);
    }
}

// The index of the frequency -m (periodic) of m = (mx, my).
static __device__ __forceinline__ int64_t neg_freq(int mx, int my, int nx, int ny)
{
    return (int64_t)(my == 0 ? 0 : ny - my) * nx + (mx == 0 ? 0 : nx - mx);
}

// Wrapped displacement of pixel coordinate v from centre c on a periodic axis of length n.
static __device__ __forceinline__ float wrap_d(float d, float n)
{
    return d - n * rintf(d / n);
}

// The window rectangle of a record on the periodic grid, as (first, count) per axis: the
// columns ceil(cx - hwx) .. floor(cx + hwx) and the rows likewise (count 0 when the record
// contributes nothing).  The transforms of the masked images read exactly this rectangle.
static __device__ __forceinline__ void window_rect(const ERec &r, int nx, int ny, int2 &cw, int2 &rw)
{
    if (r.hwx < 0) {
        cw = rw = make_int2(0, 0);
        return;
    }
    const int x0 = (int)ceilf(r.cx - (float)r.hwx), x1 = (int)floorf(r.cx + (float)r.hwx);
    const int y0 = (int)ceilf(r.cy - (float)r.hwy), y1 = (int)floorf(r.cy + (float)r.hwy);
    cw = make_int2(((x0 % nx) + nx) % nx, min(x1 - x0 + 1, nx));
    rw = make_int2(((y0 % ny) + ny) % ny, min(y1 - y0 + 1, ny));
}

// One work-group per 16 x 16 pixel tile; walks Gaussians [b0, b0 + nb) in order.  Reads the
// map from t_in; writes the map at the batch start to ckpt and at its end to t_out, and the
// masked profiles to imgs (each optional).  The masked wavefront of Gaussian k is
// e^{j phi_k} T g_k with T g_k real, so two Gaussians share one complex image: batch
// Gaussians 2p and 2p + 1 write T g as the real and the imaginary part of image p (the phase
// is applied after the transform, which separates the two by Hermitian symmetry).  Image p
// is written only inside the union of the pair's window rectangles, each part zero outside
// its own rectangle; the rest of an image is never written and never read.
__global__ void __launch_bounds__(256) k_exact_mask(const ERec *__restrict__ rec, int b0, int nb, int nx, int ny,
                                                    const float *t_in, float *t_out, float2 *__restrict__ imgs,
                                                    float *__restrict__ ckpt)
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
    float T = in ? t_in[pix] : 1.0f;
    if (ckpt && in) ckpt[pix] = T;
    // tile centre, for the work-group-uniform window test: lane b of every wavefront tests
    // batch Gaussian b, and only the Gaussians whose window meets the tile are walked
    const float tcx = tx * EXACT_TILE + 7.5f, tcy = ty * EXACT_TILE + 7.5f;
    const int lane = threadIdx.x & 63;
    bool meets = false;
    if (lane < nb) {
        const ERec &r = s_rec[lane];
        const float dcx = fabsf(wrap_d(tcx - r.cx, (float)nx)), dcy = fabsf(wrap_d(tcy - r.cy, (float)ny));
        meets = r.hwx >= 0 && dcx <= (float)r.hwx + 8.5f && dcy <= (float)r.hwy + 8.5f;
    }
    const uint64_t hits = __ballot(meets);
    float pend = 0.0f;     // the value of a pair's first Gaussian, waiting for the second's
    bool pend_in = false;  // is the pixel inside that first Gaussian's rectangle?
    for (uint64_t mk = hits; mk; mk &= mk - 1) {
        const int b = __builtin_ctzll(mk);
        const ERec &r = s_rec[b];
        float v = 0.0f;
        const float dx = wrap_d((float)px - r.cx, (float)nx), dy = wrap_d((float)py - r.cy, (float)ny);
        if (fabsf(dx) <= (float)r.hwx && fabsf(dy) <= (float)r.hwy) {  // the profile's window
            const float q = fmaf(r.qa * dx, dx, fmaf(r.qb * dx, dy, r.qc * dy * dy));
            const float gk = __builtin_amdgcn_exp2f(-q);
            v = T * gk;
            const float alpha = r.o * gk;
            if (alpha > EXACT_T_EPS) T *= 1.0f - alpha;
        }
        if (imgs && in) {
            int2 cw, rw;
            window_rect(r, nx, ny, cw, rw);
            // px, py and the window starts lie in [0, n): one wrap at most
            const int ex = px - cw.x + (px < cw.x ? nx : 0), ey = py - rw.x + (py < rw.x ? ny : 0);
            const bool inb = ex < cw.y && ey < rw.y;
            float2 *dst = imgs + (int64_t)(b >> 1) * M + pix;
            if ((b & 1) == 0) {
                if (b + 1 < nb && ((hits >> (b + 1)) & 1)) {  // its partner meets the tile too
                    pend = v;
                    pend_in = inb;
                } else if (inb) {
                    *dst = make_float2(v, 0.0f);
                }
            } else {
                const bool first = ((hits >> (b - 1)) & 1) && pend_in;
                if (first || inb) *dst = make_float2(first ? pend : 0.0f, inb ? v : 0.0f);
                pend_in = false;
            }
        }
    }
    if (t_out && in) t_out[pix] = T;
}

// U_c += a_{k,c} o_k H_c(nu, -z_k) FFT(T u_k) / (Nx Ny), with FFT(T u_k) = e^{j phi_k} F_k
// separated from the packed transform Z of a pair (a, b): F_a(m) = (Z(m) + conj Z(-m)) / 2,
// F_b(m) = (Z(m) - conj Z(-m)) / 2j.  The profiles are real, so F(-m) = conj F(m), and
// H(nu, -z) depends on |nu| only: one thread takes the frequencies m and -m together, reads
// Z at both once and evaluates H once for the two.  Threads cover rows 0 .. Ny / 2; in the
// rows 0 and Ny / 2 (their own mirror) only columns 0 .. Nx / 2 (the rest are partners).
__global__ void __launch_bounds__(256) k_exact_splat(const ERec *__restrict__ rec, int b0, int nb, Consts k,
                                                     const float2 *__restrict__ imgs, float2 *__restrict__ spec)
{
    const int nx = k.nx, ny = k.ny, hy = ny / 2;
    const int64_t M = (int64_t)nx * ny;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)(hy + 1) * nx) return;
    const int my = (int)(t / nx), mx = (int)(t - (int64_t)my * nx);
    if ((my == 0 || my == hy) && 2 * mx > nx) return;  // its partner's thread takes it
    const int64_t m = (int64_t)my * nx + mx, mn = neg_freq(mx, my, nx, ny);
    const bool pair = mn != m;
    const int mxp = 2 * mx < nx ? mx : mx - nx, myp = 2 * my < ny ? my : my - ny;
    const double nux = mxp / (nx * k.px), nuy = myp / (ny * k.py);
    const double nu2 = nux * nux + nuy * nuy;
    const float scale = (float)(1.0 / ((double)nx * ny));
    double w[4];
    bool prop[4];
    float2 acc[4], accn[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const double w2 = k.inv_lambda[c] * k.inv_lambda[c] - nu2;
        prop[c] = c < k.C && w2 > 0.0;
        w[c] = prop[c] ? sqrt(w2) : 0.0;
        acc[c] = c < k.C ? spec[(int64_t)c * M + m] : make_float2(0.0f, 0.0f);
        accn[c] = (c < k.C && pair) ? spec[(int64_t)c * M + mn] : make_float2(0.0f, 0.0f);
    }
    const int P = (nb + 1) / 2;
    // the next pair's values are fetched while this pair is applied
    float2 Zn = make_float2(0.0f, 0.0f), Zrn = Zn;
    if (P > 0) {
        Zn = imgs[m];
        Zrn = imgs[mn];
    }
    float2 Fa = make_float2(0.0f, 0.0f), Fb = Fa;
    for (int b = 0; b < nb; ++b) {
        if ((b & 1) == 0) {
            const float2 Z = Zn, Zr = Zrn;
            const int p = b >> 1;
            if (p + 1 < P) {
                Zn = imgs[(int64_t)(p + 1) * M + m];
                Zrn = imgs[(int64_t)(p + 1) * M + mn];
            }
            Fa = make_float2(0.5f * (Z.x + Zr.x), 0.5f * (Z.y - Zr.y));
            Fb = make_float2(0.5f * (Z.y + Zr.y), 0.5f * (Zr.x - Z.x));
        }
        const ERec &rr = rec[b0 + b];
        // the fields used below, loaded together
        const int valid = rr.valid;
        const float rz = rr.z, cph = rr.cphi * scale, sph = rr.sphi * scale;
        const float4 ramp = *reinterpret_cast<const float4 *>(rr.amp);
        if (!valid) continue;
        const float2 F = (b & 1) ? Fb : Fa;
        // e^{j phi} F at m and e^{j phi} conj(F) at -m, times 1 / (Nx Ny)
        const float2 S = make_float2(cph * F.x - sph * F.y, cph * F.y + sph * F.x);
        const float2 Sn = make_float2(cph * F.x + sph * F.y, sph * F.x - cph * F.y);
        const float ampc[4] = {ramp.x, ramp.y, ramp.z, ramp.w};
        const double zd = (double)rz;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (!prop[c]) continue;
            const double ph = -zd * w[c];  // revolutions of H(nu, -z)
            const float tt = (float)(ph - floor(ph));
            const float cs = __builtin_amdgcn_cosf(tt), sn = __builtin_amdgcn_sinf(tt);
            const float A = ampc[c];
            const float hr = A * cs, hi = A * sn;
            acc[c].x = fmaf(hr, S.x, fmaf(-hi, S.y, acc[c].x));
            acc[c].y = fmaf(hr, S.y, fmaf(hi, S.x, acc[c].y));
            accn[c].x = fmaf(hr, Sn.x, fmaf(-hi, Sn.y, accn[c].x));
            accn[c].y = fmaf(hr, Sn.y, fmaf(hi, Sn.x, accn[c].y));
        }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
        if (c < k.C) {
            spec[(int64_t)c * M + m] = acc[c];
            if (pair) spec[(int64_t)c * M + mn] = accn[c];
        }
}

// Per batch image: the columns and rows of the profile's window, as (first, count) on the
// periodic axes (count 0 for a Gaussian that contributes nothing).
// Windows of a batch: per Gaussian (colwin, rowwin: one interval, the second empty) and per
// packed image p (pcolwin, prowwin: the rectangles of Gaussians 2p and 2p + 1).
__global__ void __launch_bounds__(64) k_exact_windows(const ERec *__restrict__ rec, int b0, int nb, int nx, int ny,
                                                      int4 *__restrict__ colwin, int4 *__restrict__ rowwin,
                                                      int4 *__restrict__ pcolwin, int4 *__restrict__ prowwin)
{
    const int b = threadIdx.x;
    if (b >= nb) return;
    int2 cw, rw;
    window_rect(rec[b0 + b], nx, ny, cw, rw);
    colwin[b] = make_int4(cw.x, cw.y, 0, 0);
    rowwin[b] = make_int4(rw.x, rw.y, 0, 0);
    if (2 * b < nb) {
        int2 ca, ra, cb = make_int2(0, 0), rb = make_int2(0, 0);
        window_rect(rec[b0 + 2 * b], nx, ny, ca, ra);
        if (2 * b + 1 < nb) window_rect(rec[b0 + 2 * b + 1], nx, ny, cb, rb);
        pcolwin[b] = make_int4(ca.x, ca.y, cb.x, cb.y);
        prowwin[b] = make_int4(ra.x, ra.y, rb.x, rb.y);
    }
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
    // up to 64 Gaussians per batch, their images (two Gaussians each) within 1 GiB
    const size_t img = (size_t)nx * ny * sizeof(float2);
    size_t b = 2 * (((size_t)1 << 30) / img);
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
    hipLaunchKernelGGL(k_exact_zero_counters, dim3(1), dim3(64), 0, s, eb.counters);
    hipLaunchKernelGGL(k_exact_fill, dim3((unsigned)((M * k.C + 255) / 256)), dim3(256), 0, s, eb.tmap, spec, M,
                       k.C);
    if (n == 0) return hipGetLastError();
    hipLaunchKernelGGL(k_exact_keys, dim3(gn), dim3(256), 0, s, g, eb.keys_a, eb.vals_a);
    uint64_t *keys = nullptr;
    uint32_t *order = nullptr;
    hipError_t e = radix_sort_48(eb.keys_a, eb.vals_a, eb.keys_b, eb.vals_b, eb.sort_hist, n, eb.sort_blocks, s, &keys,
                                 &order);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_exact_records, dim3(gn), dim3(256), 0, s, g, k, order, rec, eb.counters);
    const int B = (int)exact_batch(k.nx, k.ny);
    const dim3 tiles((k.nx + EXACT_TILE - 1) / EXACT_TILE, (k.ny + EXACT_TILE - 1) / EXACT_TILE);
    for (int64_t b0 = 0; b0 < n; b0 += B) {
        const int nb = (int)std::min<int64_t>(B, n - b0);
        hipLaunchKernelGGL(k_exact_mask, tiles, dim3(256), 0, s, rec, (int)b0, nb, k.nx, k.ny, eb.tmap, eb.tmap,
                           eb.pimgs, (float *)nullptr);
        hipLaunchKernelGGL(k_exact_windows, dim3(1), dim3(64), 0, s, rec, (int)b0, nb, k.nx, k.ny, eb.colwin,
                           eb.rowwin, eb.pcolwin, eb.prowwin);
        e = launch_fft2d_win(p, (nb + 1) / 2, -1, eb.pimgs, eb.pimgs, eb.pcolwin, eb.prowwin, s);
        if (e != hipSuccess) return e;
        const int64_t half = (int64_t)(k.ny / 2 + 1) * k.nx;  // frequencies m, -m taken together
        hipLaunchKernelGGL(k_exact_splat, dim3((unsigned)((half + 255) / 256)), dim3(256), 0, s, rec, (int)b0, nb, k,
                           eb.pimgs, spec);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Adjoint.  With Gs_c = FFT(dL/du_c) (torch's complex-gradient convention) and F_k = FFT(T_k u_k),
//   dL = Re sum_{c,m} conj(Gs_c) d(A_{k,c} H_{k,c} F_k) / (Nx Ny),
// which splits into
//   * the spectral sums P_{k,c} = sum_m conj(Gs_c) H F_k and Q_{k,c} = sum_m W_c conj(Gs_c) H F_k
//     (W_c = sqrt(1/l^2 - |nu|^2)): dL/da_c = o Re P_c / NxNy, dL/do gains sum_c a_c Re P_c / NxNy,
//     dL/dz = 2 pi sum_c A_c Im Q_c / NxNy (dH/dz = -j 2 pi W H), and, since phi enters only
//     through the factor e^{j phi} of F_k, dL/dphi = -sum_c A_c Im P_c / NxNy;
//   * the spatial part Re sum_x d(T_k g_k) r_k with the real r_k = Re(e^{-j phi} R_k),
//     R_k = IFFT(sum_c A_c Gs_c conj(H_c)) / NxNy.  Through g_k it gives the mean and covariance
//     gradients; through the map, with w_k = g_k r_k, dL/d alpha_j(x) = -T_j(x) D_j(x), where
//     D_j = sum_{k > j} w_k prod_{j < i < k} (1 - alpha_i) is accumulated back to front
//     (D_{j-1} = w_j + (1 - alpha_j) D_j): the map is recomputed from per-batch checkpoints and
//     never divided by (1 - alpha).
// ---------------------------------------------------------------------------------
constexpr int EXACT_BTILE = 8;          // 8 x 8 pixels: one wavefront per work-group
constexpr int EXACT_NSPEC = 16;         // Re/Im P_c, Re/Im Q_c for c < 4
constexpr int EXACT_NSPAT = 8;          // Sx, Sy, Sxx, Sxy, Syy, So, pad, pad

// One thread per frequency pair {m, -m} (as in k_exact_splat; F(-m) = conj F(m), H shared):
// spectral partial sums per (work-group, Gaussian), and the spectra whose inverse transforms
// give r_k.  With V_k = sum_c A_c Gs_c conj(H_c) and V'_k = e^{-j phi_k} V_k, r_k is the
// inverse transform of the Hermitian part Vh_k(m) = (V'_k(m) + conj V'_k(-m)) / 2, which is
// real, so Gaussians 2p and 2p + 1 share one image: Vh_{2p} + j Vh_{2p+1} overwrites the packed
// transform of pair p in pimgs (each thread reads its own two entries of image p before it
// writes them).
__global__ void __launch_bounds__(256) k_exact_gsplat(const ERec *__restrict__ rec, int b0, int nb, Consts k,
                                                      const float2 *__restrict__ gspec, float2 *pimgs,
                                                      float *__restrict__ part)
{
    // per wave and batch Gaussian, the wave's 16 sums: the four waves are summed in a fixed
    // order once, after the batch, so the waves never wait for each other inside it
    __shared__ float s_red[4][64][16];
    const int nx = k.nx, ny = k.ny, hy = ny / 2;
    const int64_t M = (int64_t)nx * ny;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int my = (int)(t / nx), mx = (int)(t - (int64_t)my * nx);
    // rows 0 .. Ny / 2; in the rows 0 and Ny / 2 only columns 0 .. Nx / 2 (the rest are partners)
    const bool live = t < (int64_t)(hy + 1) * nx && !((my == 0 || my == hy) && 2 * mx > nx);
    if (!live) mx = my = 0;
    const int m = my * nx + mx, mn = (int)neg_freq(mx, my, nx, ny);  // M < 2^31
    const bool pair = live && mn != m;
    double w[4];
    bool prop[4];
    float2 gs0[4], gs1[4];  // Gs_c at m and at -m
    {
        const int mxp = 2 * mx < nx ? mx : mx - nx, myp = 2 * my < ny ? my : my - ny;
        const double nux = mxp / (nx * k.px), nuy = myp / (ny * k.py);
        const double nu2 = nux * nux + nuy * nuy;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double w2 = k.inv_lambda[c] * k.inv_lambda[c] - nu2;
            prop[c] = live && c < k.C && w2 > 0.0;
            w[c] = prop[c] ? sqrt(w2) : 0.0;
            gs0[c] = (live && c < k.C) ? gspec[(int64_t)c * M + m] : make_float2(0.0f, 0.0f);
            gs1[c] = (pair && c < k.C) ? gspec[(int64_t)c * M + mn] : make_float2(0.0f, 0.0f);
        }
    }
    float2 Fa = make_float2(0.0f, 0.0f), Fb = Fa;
    float2 Ha = Fa;  // Vh of the pair's first Gaussian at m
    for (int b = 0; b < nb; ++b) {
        const int64_t pb = (int64_t)(b >> 1) * M;
        if ((b & 1) == 0) {
            float2 Z = make_float2(0.0f, 0.0f), Zr = Z;
            if (live) {
                Z = pimgs[pb + m];
                Zr = pimgs[pb + mn];
            }
            Fa = make_float2(0.5f * (Z.x + Zr.x), 0.5f * (Z.y - Zr.y));
            Fb = make_float2(0.5f * (Z.y + Zr.y), 0.5f * (Zr.x - Z.x));
        }
        const ERec &rr = rec[b0 + b];
        // the fields used below, loaded together
        const int valid = rr.valid;
        const float rz = rr.z, cph = rr.cphi, sph = rr.sphi;
        const float4 ramp = *reinterpret_cast<const float4 *>(rr.amp);
        const float ampc[4] = {ramp.x, ramp.y, ramp.z, ramp.w};
        float v[EXACT_NSPEC];
#pragma unroll
        for (int i = 0; i < EXACT_NSPEC; ++i) v[i] = 0.0f;
        const double zd = (double)rz;
        float2 V0 = make_float2(0.0f, 0.0f), V1 = V0;
        if (live && valid) {
            const float2 F = (b & 1) ? Fb : Fa;
            // e^{j phi} F at m and e^{j phi} conj(F) at -m
            const float2 S0 = make_float2(cph * F.x - sph * F.y, cph * F.y + sph * F.x);
            const float2 S1 = make_float2(cph * F.x + sph * F.y, sph * F.x - cph * F.y);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                if (!prop[c]) continue;
                const double ph = -zd * w[c];
                const float tt = (float)(ph - floor(ph));
                const float hc = __builtin_amdgcn_cosf(tt), hs = __builtin_amdgcn_sinf(tt);
                // Y = Gs conj(H) at m and at -m (zero at -m when -m = m: gs1 = 0)
                const float2 Y0 = make_float2(gs0[c].x * hc + gs0[c].y * hs, gs0[c].y * hc - gs0[c].x * hs);
                const float2 Y1 = make_float2(gs1[c].x * hc + gs1[c].y * hs, gs1[c].y * hc - gs1[c].x * hs);
                // X = conj(Gs) H e^{j phi} F = conj(Y) S, summed over the two frequencies
                const float xr = Y0.x * S0.x + Y0.y * S0.y + Y1.x * S1.x + Y1.y * S1.y;
                const float xi = Y0.x * S0.y - Y0.y * S0.x + Y1.x * S1.y - Y1.y * S1.x;
                const float wf = (float)w[c];
                v[4 * c + 0] += xr;
                v[4 * c + 1] += xi;
                v[4 * c + 2] = fmaf(wf, xr, v[4 * c + 2]);
                v[4 * c + 3] = fmaf(wf, xi, v[4 * c + 3]);
                // V += A_c Y
                const float A = ampc[c];
                V0.x = fmaf(A, Y0.x, V0.x);
                V0.y = fmaf(A, Y0.y, V0.y);
                V1.x = fmaf(A, Y1.x, V1.x);
                V1.y = fmaf(A, Y1.y, V1.y);
            }
        }
        // V' = e^{-j phi} V at m and -m, and Vh(m) (at a frequency that is its own mirror, the
        // real part of V'(m))
        const float2 P0 = make_float2(cph * V0.x + sph * V0.y, cph * V0.y - sph * V0.x);
        const float2 P1 = make_float2(cph * V1.x + sph * V1.y, cph * V1.y - sph * V1.x);
        const float2 Hm = pair ? make_float2(0.5f * (P0.x + P1.x), 0.5f * (P0.y - P1.y)) : make_float2(P0.x, 0.0f);
        if ((b & 1) == 0) {
            Ha = Hm;
            if (b + 1 == nb && live) {  // no partner: Vh alone, Hermitian
                pimgs[pb + m] = Ha;
                if (pair) pimgs[pb + mn] = make_float2(Ha.x, -Ha.y);
            }
        } else if (live) {
            // Vh_a + j Vh_b at m, and conj Vh_a + j conj Vh_b at -m
            pimgs[pb + m] = make_float2(Ha.x - Hm.y, Ha.y + Hm.x);
            if (pair) pimgs[pb + mn] = make_float2(Ha.x + Hm.y, Hm.x - Ha.y);
        }
        // one transposed butterfly over the 16 sums: afterwards lane l with
        // bits 0-2 clear holds sums 2 (4 b5 + 2 b4 + b3) and that + 1
        float x[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) x[i] = i < EXACT_NSPEC ? v[i] : 0.0f;
        float unused = 0.0f;
        reduce_transposed<16, false>(x, unused, lane);
        if ((lane & 7) == 0) {
            const int v0 = 2 * (((lane >> 5) & 1) * 4 + ((lane >> 4) & 1) * 2 + ((lane >> 3) & 1));
            s_red[wave][b][v0] = x[0];
            s_red[wave][b][v0 + 1] = x[1];
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nb * EXACT_NSPEC; i += blockDim.x) {
        const int b = i / EXACT_NSPEC, v = i - b * EXACT_NSPEC;
        const float t = s_red[0][b][v] + s_red[1][b][v] + s_red[2][b][v] + s_red[3][b][v];
        part[((int64_t)b * gridDim.x + blockIdx.x) * EXACT_NSPEC + v] = t;  // Gaussian-major
    }
}

// One wavefront per 8 x 8 pixel tile: replays the map over the batch (kept in LDS), then walks
// the batch back to front with the running D, and reduces the spatial sums per Gaussian.
__global__ void __launch_bounds__(64) k_exact_back(const ERec *__restrict__ rec, int b0, int nb, int nx, int ny,
                                                   double px_m, double py_m, float rscale,
                                                   const float *__restrict__ tck, float *__restrict__ dmap,
                                                   const float2 *__restrict__ R, float *__restrict__ part)
{
    // the map before each batch Gaussian, per pixel (each lane touches only its own column);
    // the records are read from memory (uniform indices: scalar loads), which leaves 16 KB of
    // LDS per work-group and ten work-groups per CU
    __shared__ float s_T[64][64];
    const ERec *__restrict__ brec = rec + b0;
    const int lane = threadIdx.x;
    const int tx = blockIdx.x, ty = blockIdx.y;
    const int ntx = gridDim.x;
    const int px = tx * EXACT_BTILE + (lane & 7), py = ty * EXACT_BTILE + (lane >> 3);
    const bool in = px < nx && py < ny;
    const int64_t M = (int64_t)nx * ny;
    const int64_t pix = (int64_t)py * nx + px;
    const float tcx = tx * EXACT_BTILE + 3.5f, tcy = ty * EXACT_BTILE + 3.5f;
    const float fx = (float)px, fy = (float)py;
    // the batch Gaussians whose window meets this tile (lane b tests Gaussian b); the others
    // leave the map, D and their partial sums (zero) unchanged here
    bool meets = false;
    if (lane < nb) {
        const ERec &r = brec[lane];
        const float dcx = fabsf(wrap_d(tcx - r.cx, (float)nx)), dcy = fabsf(wrap_d(tcy - r.cy, (float)ny));
        meets = r.hwx >= 0 && dcx <= (float)r.hwx + 4.5f && dcy <= (float)r.hwy + 4.5f;
    }
    const uint64_t hits = __ballot(meets);
    // partial sums Gaussian-major: part[b][tile][8]
    const int64_t tile = (int64_t)ty * ntx + tx, ntiles = (int64_t)ntx * gridDim.y;
    for (int i = lane; i < nb * EXACT_NSPAT; i += 64) {
        const int b = i / EXACT_NSPAT;
        if (!((hits >> b) & 1)) part[((int64_t)b * ntiles + tile) * EXACT_NSPAT + (i - b * EXACT_NSPAT)] = 0.0f;
    }
    // forward replay of the map over the batch
    float T = in ? tck[pix] : 1.0f;
    for (uint64_t m = hits; m; m &= m - 1) {
        const int b = __builtin_ctzll(m);
        s_T[b][lane] = T;
        const ERec &r = brec[b];
        const float dx = wrap_d(fx - r.cx, (float)nx), dy = wrap_d(fy - r.cy, (float)ny);
        if (fabsf(dx) <= (float)r.hwx && fabsf(dy) <= (float)r.hwy) {
            const float gk = __builtin_amdgcn_exp2f(-fmaf(r.qa * dx, dx, fmaf(r.qb * dx, dy, r.qc * dy * dy)));
            const float alpha = r.o * gk;
            if (alpha > EXACT_T_EPS) T *= 1.0f - alpha;
        }
    }
    // back to front
    const float ln2x2 = 2.0f * 0.69314718055994531f;
    float D = in ? dmap[pix] : 0.0f;
    for (uint64_t m = hits; m; m &= ~(1ull << (63 - __builtin_clzll(m)))) {
        const int b = 63 - __builtin_clzll(m);
        const ERec &r = brec[b];
        float v[EXACT_NSPAT];
#pragma unroll
        for (int i = 0; i < EXACT_NSPAT; ++i) v[i] = 0.0f;
        {
            const float dx = wrap_d(fx - r.cx, (float)nx), dy = wrap_d(fy - r.cy, (float)ny);
            if (in && fabsf(dx) <= (float)r.hwx && fabsf(dy) <= (float)r.hwy) {
                const float Tb = s_T[b][lane];
                const float gk = __builtin_amdgcn_exp2f(-fmaf(r.qa * dx, dx, fmaf(r.qb * dx, dy, r.qc * dy * dy)));
                // Sigma^-1 d in pixel units (natural-log exponent -1/2 d^T Sigma^-1 d), then metres
                const float ex = ln2x2 * (r.qa * dx + 0.5f * r.qb * dy) / (float)px_m;
                const float ey = ln2x2 * (0.5f * r.qb * dx + r.qc * dy) / (float)py_m;
                // r_k: Gaussian 2p in the real part of image p, 2p + 1 in the imaginary part
                const float2 Rv = R[(int64_t)(b >> 1) * M + pix];
                const float zr = ((b & 1) ? Rv.y : Rv.x) * rscale;
                const float alpha = r.o * gk;
                const bool kept = alpha > EXACT_T_EPS;
                const float ga = kept ? -Tb * D : 0.0f;         // dL/d alpha at this pixel
                const float cg = Tb * zr + r.o * ga;           // coefficient on g
                const float cgg = cg * gk;
                v[0] = cgg * ex;
                v[1] = cgg * ey;
                v[2] = cgg * ex * ex;
                v[3] = cgg * ex * ey;
                v[4] = cgg * ey * ey;
                v[5] = ga * gk;                                // opacity through alpha
                D = fmaf(kept ? 1.0f - alpha : 1.0f, D, gk * zr);
            }
            // one transposed butterfly over the 8 sums: afterwards lane l with bits 0-2 clear
            // holds sum 4 b5 + 2 b4 + b3
            float unused = 0.0f;
            reduce_transposed<EXACT_NSPAT, false>(v, unused, lane);
        }
        if ((lane & 7) == 0) {
            const int i = ((lane >> 5) & 1) * 4 + ((lane >> 4) & 1) * 2 + ((lane >> 3) & 1);
            part[((int64_t)b * ntiles + tile) * EXACT_NSPAT + i] = v[0];
        }
    }
    if (in) dmap[pix] = D;
}

// One work-group per batch Gaussian: fixed-order sums of its partials, then the chain rule.
constexpr int EXACT_GF_THREADS = 512;  // one work-group per Gaussian: 8 wavefronts of loads in flight
__global__ void __launch_bounds__(EXACT_GF_THREADS) k_exact_gfinal(const ERec *__restrict__ rec, int b0, GView g, Consts k,
                                                      const uint32_t *__restrict__ order,
                                                      const float *__restrict__ pspec, int nblk_spec,
                                                      const float *__restrict__ pspat, int ntx, int ntile,
                                                      GradView out)
{
    constexpr int NW = EXACT_GF_THREADS / 64;
    __shared__ double s_red[NW][EXACT_NSPEC + EXACT_NSPAT];
    const int b = blockIdx.x, t = threadIdx.x, lane = t & 63, wave = t >> 6;
    double acc[EXACT_NSPEC + EXACT_NSPAT];
#pragma unroll
    for (int i = 0; i < EXACT_NSPEC + EXACT_NSPAT; ++i) acc[i] = 0.0;
    for (int q = t; q < nblk_spec; q += EXACT_GF_THREADS)
#pragma unroll
        for (int i = 0; i < EXACT_NSPEC; ++i) acc[i] += (double)pspec[((int64_t)b * nblk_spec + q) * EXACT_NSPEC + i];
    // spatial partials: only the tiles near the Gaussian's window are read.  The test is the
    // back-to-front kernel's with one pixel more of margin, so it passes every tile that kernel
    // wrote sums for; the tiles skipped hold exact zeros and the sums are unchanged.
    const ERec &rb = rec[b0 + b];
    const bool any = rb.hwx >= 0;
    const float lim_x = (float)rb.hwx + 5.5f, lim_y = (float)rb.hwy + 5.5f;
    for (int q = t; any && q < ntile; q += EXACT_GF_THREADS) {
        const int ty = q / ntx, tx = q - ty * ntx;
        const float dcx = fabsf(wrap_d(tx * EXACT_BTILE + 3.5f - rb.cx, (float)k.nx));
        const float dcy = fabsf(wrap_d(ty * EXACT_BTILE + 3.5f - rb.cy, (float)k.ny));
        if (dcx > lim_x || dcy > lim_y) continue;
#pragma unroll
        for (int i = 0; i < EXACT_NSPAT; ++i) acc[EXACT_NSPEC + i] += (double)pspat[((int64_t)b * ntile + q) * EXACT_NSPAT + i];
    }
#pragma unroll
    for (int i = 0; i < EXACT_NSPEC + EXACT_NSPAT; ++i) {
        double v = acc[i];
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
        if (lane == 0) s_red[wave][i] = v;
    }
    __syncthreads();
    if (t != 0) return;
    double S[EXACT_NSPEC + EXACT_NSPAT];
#pragma unroll
    for (int i = 0; i < EXACT_NSPEC + EXACT_NSPAT; ++i) {
        double v = 0.0;
        for (int w = 0; w < NW; ++w) v += s_red[w][i];  // fixed order
        S[i] = v;
    }
    const ERec &r = rec[b0 + b];
    const int64_t j = order[b0 + b];
    const double inv = 1.0 / ((double)k.nx * k.ny);
    double d_o = S[EXACT_NSPEC + 5], d_z = 0.0, d_phi = 0.0;
    const double o = g.opacity[j];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        if (c >= k.C) break;
        const double a = g.amplitude[(int64_t)c * g.amp_stride + j];
        const double rp = S[4 * c + 0] * inv, iq = S[4 * c + 3] * inv;
        if (out.amplitude) out.amplitude[(int64_t)c * out.amp_stride + j] = r.valid ? (float)(o * rp) : 0.0f;
        d_o += a * rp;
        d_z += 2.0 * M_PI * (double)r.amp[c] * iq;
        d_phi -= (double)r.amp[c] * S[4 * c + 1] * inv;
    }
    const double* P = S + EXACT_NSPEC;
    const bool ok = r.valid != 0;
    if (out.mean_x) out.mean_x[j] = ok ? (float)P[0] : 0.0f;
    if (out.mean_y) out.mean_y[j] = ok ? (float)P[1] : 0.0f;
    if (out.cov_xx) out.cov_xx[j] = ok ? (float)(0.5 * P[2]) : 0.0f;
    if (out.cov_xy) out.cov_xy[j] = ok ? (float)P[3] : 0.0f;
    if (out.cov_yy) out.cov_yy[j] = ok ? (float)(0.5 * P[4]) : 0.0f;
    if (out.phase) out.phase[j] = ok ? (float)d_phi : 0.0f;
    if (out.opacity) out.opacity[j] = ok ? (float)d_o : 0.0f;
    if (out.depth) out.depth[j] = ok ? (float)d_z : 0.0f;
}

__global__ void __launch_bounds__(256) k_exact_fill1(float *__restrict__ p, int64_t n, float v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

int64_t exact_ckpt_count(int64_t n, int nx, int ny)
{
    const int64_t B = (int64_t)exact_batch(nx, ny);
    return std::max<int64_t>(1, (n + B - 1) / B);
}

hipError_t run_exact_backward(const Plan &p, const Consts &k, const GView &g, const ExactBuffers &eb,
                              const ExactBwdBuffers &bb, const float2 *grad_field, const GradView &out, hipStream_t s)
{
    const int64_t n = g.n, M = (int64_t)k.nx * k.ny;
    hipLaunchKernelGGL(k_exact_zero_counters, dim3(1), dim3(64), 0, s, eb.counters);
    if (n == 0) return hipGetLastError();
    ERec *rec = (ERec *)eb.rec;
    const unsigned gn = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_exact_keys, dim3(gn), dim3(256), 0, s, g, eb.keys_a, eb.vals_a);
    uint64_t *keys = nullptr;
    uint32_t *order = nullptr;
    hipError_t e = radix_sort_48(eb.keys_a, eb.vals_a, eb.keys_b, eb.vals_b, eb.sort_hist, n, eb.sort_blocks, s, &keys,
                                 &order);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_exact_records, dim3(gn), dim3(256), 0, s, g, k, order, rec, eb.counters);
    // Gs = FFT(dL/du)
    e = launch_fft2d(p, k.C, -1, grad_field, bb.gspec, s);
    if (e != hipSuccess) return e;
    const int B = (int)exact_batch(k.nx, k.ny);
    const int64_t nbatch = (n + B - 1) / B;
    const dim3 tiles((k.nx + EXACT_TILE - 1) / EXACT_TILE, (k.ny + EXACT_TILE - 1) / EXACT_TILE);
    const dim3 btiles((k.nx + EXACT_BTILE - 1) / EXACT_BTILE, (k.ny + EXACT_BTILE - 1) / EXACT_BTILE);
    const unsigned mblk = (unsigned)((M + 255) / 256);
    const unsigned gsblk = (unsigned)(((int64_t)(k.ny / 2 + 1) * k.nx + 255) / 256);  // pairs {m, -m}
    // forward sweep of the map, checkpointed at every batch start
    hipLaunchKernelGGL(k_exact_fill1, dim3(mblk), dim3(256), 0, s, eb.tmap, M, 1.0f);
    for (int64_t q = 0; q < nbatch; ++q) {
        const int64_t b0 = q * B;
        const int nb = (int)std::min<int64_t>(B, n - b0);
        hipLaunchKernelGGL(k_exact_mask, tiles, dim3(256), 0, s, rec, (int)b0, nb, k.nx, k.ny, eb.tmap, eb.tmap,
                           (float2 *)nullptr, bb.ckpt + q * M);
    }
    hipLaunchKernelGGL(k_exact_fill1, dim3(mblk), dim3(256), 0, s, bb.dmap, M, 0.0f);
    const float rscale = (float)(1.0 / ((double)k.nx * k.ny));
    for (int64_t q = nbatch - 1; q >= 0; --q) {
        const int64_t b0 = q * B;
        const int nb = (int)std::min<int64_t>(B, n - b0);
        hipLaunchKernelGGL(k_exact_mask, tiles, dim3(256), 0, s, rec, (int)b0, nb, k.nx, k.ny, bb.ckpt + q * M,
                           (float *)nullptr, eb.pimgs, (float *)nullptr);
        hipLaunchKernelGGL(k_exact_windows, dim3(1), dim3(64), 0, s, rec, (int)b0, nb, k.nx, k.ny, eb.colwin,
                           eb.rowwin, eb.pcolwin, eb.prowwin);
        e = launch_fft2d_win(p, (nb + 1) / 2, -1, eb.pimgs, eb.pimgs, eb.pcolwin, eb.prowwin, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_exact_gsplat, dim3(gsblk), dim3(256), 0, s, rec, (int)b0, nb, k, bb.gspec, eb.pimgs,
                           bb.pspec);
        // r is read only inside each window: full row pass, columns of the pair's windows only
        e = launch_fft2d_cols_out(p, (nb + 1) / 2, +1, eb.pimgs, eb.pcolwin, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_exact_back, btiles, dim3(64), 0, s, rec, (int)b0, nb, k.nx, k.ny, k.px, k.py, rscale,
                           bb.ckpt + q * M, bb.dmap, eb.pimgs, bb.pspat);
        hipLaunchKernelGGL(k_exact_gfinal, dim3(nb), dim3(EXACT_GF_THREADS), 0, s, rec, (int)b0, g, k, order, bb.pspec,
                           (int)gsblk,
                           bb.pspat, (int)btiles.x, (int)(btiles.x * btiles.y), out);
    }
    return hipGetLastError();
}

}  // namespace gws
