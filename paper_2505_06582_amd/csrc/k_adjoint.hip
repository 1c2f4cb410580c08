// Adjoint of the order-invariant sum (Sec. 4.2, Eq. 12) for gfx950.
//
// Given Gs = dL/dS (the forward DFT of dL/du, torch's complex-gradient convention), the
// gradient with respect to a real parameter t of Gaussian i is
//   dL/dt = Re sum_{c,m} conj(Gs_c[m]) dT_{c,i}[m]/dt,   T = A_c exp2(-q) exp(j 2 pi Theta_c).
// Every derivative of T is T times a factor that is constant, linear or quadratic in the
// frequency, so per Gaussian it suffices to accumulate, with g_c = conj(Gs_c) exp2(-q)
// exp(j 2 pi Theta_c) and rho = sum_c A_c g_c,
//   P_c = sum_m g_c,  W_c = sum_m D_c(m) Im g_c,
//   Sfx = sum_m m_x' Im rho, Sfy = sum_m m_y' Im rho,
//   Qxx = sum_m m_x'^2 Re rho, Qxy = sum_m m_x' m_y' Re rho, Qyy = sum_m m_y'^2 Re rho,
// and apply the chain rule once per Gaussian (k_grad_final).  Terms are recomputed exactly
// as the forward computes them; nothing per (Gaussian, frequency) is stored.
//
// Work: a wavefront owns 64 consecutive sorted Gaussians (one per lane, its record in
// registers) and a range of tiles.  For each 16 x 16 sub-tile, lanes test their own
// Gaussian against it and stage the accepted ones in LDS; then every lane evaluates its 4
// frequencies for each accepted Gaussian and the wave reduces the 3C + 5 sums across
// lanes into that Gaussian's LDS accumulator.  Item partials are summed per Gaussian in a
// fixed order, so results are bitwise reproducible.
#include "gws_internal.h"

namespace gws {

static __device__ __forceinline__ double frac_d(double v) { return v - floor(v); }

static __device__ __forceinline__ bool ellipse_meets_rect_b(float a, float b2, float g, float lim, float x0, float x1,
                                                            float y0, float y1)
{
    return ellipse_meets_rect_r(a, b2, g, 0.5f / a, 0.5f / g, lim, x0, x1, y0, y1);
}

struct alignas(16) BEntry {
    float alpha, beta2, gamma, z;
    float rxf, ryf;
    int32_t owner;   // lane (0..63) that owns this Gaussian
    uint32_t rows;   // row_block_mask of this Gaussian on the sub-tile
    float amp[4];
    float base[4];
};

// Per-frequency FP32 table D_c(nu_m) - D_c(nu_0(sub-tile of m)) in FFT order, and the FP64
// sub-tile centre values D_c(nu_0).  Sub-tiles are the DC-aligned SUBX x SY blocks.
__global__ void __launch_bounds__(256) k_dtable(Consts k, float *__restrict__ dD, double *__restrict__ D0, int nsx,
                                                int nsy, int sx_min, int sy_min, int SY)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t M = (int64_t)k.nx * k.ny;
    const double Wx = k.nx * k.px, Wy = k.ny * k.py;
    if (idx < M) {
        const int mx = (int)(idx % k.nx), my = (int)(idx / k.nx);
        const int mxp = 2 * mx < k.nx ? mx : mx - k.nx, myp = 2 * my < k.ny ? my : my - k.ny;
        const int sx = (int)floor(mxp / (double)SUBX), sy = (int)floor(myp / (double)SY);
        const int cx = sx * SUBX + SUBX / 2, cy = sy * SY + SY / 2;
        const double nux = mxp / Wx, nuy = myp / Wy, ncx = cx / Wx, ncy = cy / Wy;
        const double nu2 = nux * nux + nuy * nuy, nc2 = ncx * ncx + ncy * ncy;
        for (int c = 0; c < k.C; ++c) {
            const double il = k.inv_lambda[c];
            const double w2 = il * il - nu2, wc = il * il - nc2;
            const double d = w2 > 0.0 ? -nu2 / (il + sqrt(w2)) : 0.0;
            const double d0 = wc > 0.0 ? -nc2 / (il + sqrt(wc)) : 0.0;
            dD[(int64_t)c * M + idx] = (float)(d - d0);
        }
    }
    const int64_t ns = (int64_t)nsx * nsy;
    if (idx < ns) {
        const int sx = (int)(idx % nsx) + sx_min, sy = (int)(idx / nsx) + sy_min;
        const double ncx = (sx * SUBX + SUBX / 2) / Wx, ncy = (sy * SY + SY / 2) / Wy;
        const double nc2 = ncx * ncx + ncy * ncy;
        for (int c = 0; c < k.C; ++c) {
            const double il = k.inv_lambda[c];
            const double wc = il * il - nc2;
            D0[(int64_t)c * ns + idx] = wc > 0.0 ? -nc2 / (il + sqrt(wc)) : 0.0;
        }
    }
}

hipError_t launch_dtable(const Consts &k, float *dD, double *D0, int nsx, int nsy, int sx_min, int sy_min, int sy,
                         hipStream_t s)
{
    const int64_t M = (int64_t)k.nx * k.ny;
    const int64_t n = M > (int64_t)nsx * nsy ? M : (int64_t)nsx * nsy;
    hipLaunchKernelGGL(k_dtable, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, k, dD, D0, nsx, nsy, sx_min, sy_min,
                       sy);
    return hipGetLastError();
}

// Gs in polar form, in place: (Re, Im) -> (|Gs|, arg Gs / 2 pi).  The adjoint then forms
// conj(Gs) e^{j 2 pi Theta} as |Gs| e^{j 2 pi (Theta - arg Gs / 2 pi)}: one more phase term,
// two products instead of a complex product.
__global__ void __launch_bounds__(256) k_polar(float2 *__restrict__ g, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float2 v = g[i];
    g[i] = make_float2(hypotf(v.x, v.y), atan2f(v.y, v.x) * 0.15915494309189535f);
}

hipError_t launch_polar(float2 *g, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_polar, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, n);
    return hipGetLastError();
}

template <int C, bool DEPTH, int F>
__global__ void __launch_bounds__(WG, waves_per_simd(F)) k_adjoint(Consts k, const int32_t *__restrict__ tile_xy,
                                                const BwdScene *__restrict__ scenes, const int32_t *__restrict__ prefix,
                                                int n_scenes, long long *__restrict__ queue,
                                                const float *__restrict__ dtab, const double *__restrict__ d0tab,
                                                int nsx, int nsy, int sx_min, int sy_min)
{
    // reduced values: Re P_c, Sfx, Sfy, Qxx, Qxy, Qyy, and with depth Im P_c, W_c; without
    // depth the phase gradient's sum_m Im rho rides along as one extra fully reduced value
    constexpr int NV = (DEPTH ? 3 : 1) * C + 5;
    constexpr int NR = NV <= 8 ? 8 : 16;
    constexpr int EXTRA_SLOT = 8;
    static_assert(NV <= 16, "too many accumulators");
    static_assert(DEPTH || NV <= 8, "without depth the sums must fit 8 transposed values");
    __shared__ BEntry s_w[WAVES][64];
    __shared__ float s_acc[WAVES][64][NACC];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int total_items = prefix[n_scenes];
    const int hx = k.nx / 2, hy = k.ny / 2;
    const int64_t M = (int64_t)k.nx * k.ny;
    const int64_t ns = (int64_t)nsx * nsy;
    const float lim = (float)(k.tau2 * (1.0 + 1e-5)) + 1e-4f;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    constexpr int SY = sub_h(F), TY = 2 * SY;
    const int col = lane & (SUBX - 1), row0 = lane >> 4;
    const float dxf = (float)(col - SUBX / 2);
    for (;;) {
        int q = 0, sc = 0;
        if (lane == 0) {
            q = (int)atomicAdd((unsigned long long *)queue, 1ull);
            if (q < total_items)
                while (sc + 1 < n_scenes && prefix[sc + 1] <= q) ++sc;
        }
        q = __shfl(q, 0);
        sc = __shfl(sc, 0);
        if (q >= total_items) break;
        const BwdScene S = scenes[sc];
        const GRec *__restrict__ rec = S.rec;
        const float2 *__restrict__ gspec = S.gspec;  // polar: (|Gs|, arg Gs / 2 pi)
        const int64_t nvalid = S.n - S.counters[CTR_NCULLED];
        const BItem bi = S.bitems[q - prefix[sc]];
        long long pairs = 0;
        const int64_t gidx = (int64_t)bi.chunk * 64 + lane;
        const bool gvalid = gidx < nvalid;
        // this lane's record as four 16-byte registers (a struct would be kept in scratch):
        // r0 = (alpha, beta2, gamma, z), r1 = (rx, ry, rxf, ryf), r2 = kappa[4], r3 = amp[4]
        float4 r0 = make_float4(1.f, 1.f, 1.f, 0.f), r1 = make_float4(0.f, 0.f, 0.f, 0.f), r2 = r1, r3 = r1;
        if (gvalid) {
            const float4 *src = reinterpret_cast<const float4 *>(rec + gidx);
            r0 = src[0];
            r1 = src[1];
            r2 = src[2];
            r3 = src[3];
        }
        const uint32_t rx = __float_as_uint(r1.x), ry = __float_as_uint(r1.y);
        const float kap[4] = {r2.x, r2.y, r2.z, r2.w};
#pragma unroll
        for (int v = 0; v < NACC; ++v) s_acc[wave][lane][v] = 0.0f;

        for (int kt = bi.k0; kt < bi.k1; ++kt) {
            const int32_t txy = tile_xy[kt];
            const int tx = (int)(int16_t)(txy & 0xffff), ty = txy >> 16;
            for (int st = 0; st < 4; ++st) {
                const int sx0 = tx * TILEX + (st & 1) * SUBX, sy0 = ty * TY + (st >> 1) * SY;
                const float x0 = (float)max(sx0, -hx), x1 = (float)min(sx0 + SUBX - 1, hx - 1);
                const float y0 = (float)max(sy0, -hy), y1 = (float)min(sy0 + SY - 1, hy - 1);
                if (x0 > x1 || y0 > y1) continue;
                const int cx = sx0 + SUBX / 2, cy = sy0 + SY / 2;
                const int64_t sidx = (int64_t)(sy0 / SY - sy_min) * nsx + (sx0 / SUBX - sx_min);
                // stage this sub-tile's accepted Gaussians
                const bool p = gvalid && ellipse_meets_rect_b(r0.x, r0.y, r0.z, lim, x0, x1, y0, y1);
                const uint64_t bal = __ballot(p);
                const int cnt = __popcll(bal);
                if (cnt == 0) continue;
                if (p) {
                    const uint32_t rows = row_block_mask<F>(r0.x, r0.y, r0.z, lim, x0, x1, sy0, hy);
                    pairs += __popc(rows) * (SUBX * 4);
                    const uint32_t ramp = (uint32_t)cx * rx + (uint32_t)cy * ry;
                    const double ramp_rev = (double)ramp * (1.0 / 4294967296.0);
                    float4 b4 = make_float4(0.f, 0.f, 0.f, 0.f);
                    float bs[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int c = 0; c < C; ++c)
                        bs[c] = (float)frac_d((double)kap[c] - ramp_rev - (double)r0.w * d0tab[c * ns + sidx]);
                    b4 = make_float4(bs[0], bs[1], bs[2], bs[3]);
                    float4 *dst = reinterpret_cast<float4 *>(&s_w[wave][__popcll(bal & lt)]);
                    dst[0] = r0;
                    dst[1] = make_float4(r1.z, r1.w, __int_as_float(lane), __uint_as_float(rows));
                    dst[2] = r3;
                    dst[3] = b4;
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                // per-lane frequency data
                const int mxp = sx0 + col;
                const float fmx = (float)mxp;
                const float mxx = fmx * fmx;
                const int mx = mxp < 0 ? mxp + k.nx : mxp;
                const bool xin = mxp >= -hx && mxp < hx;
                float fmy[F], mxy[F], myy[F], dyf[F], dD[F][C], gm[F][C], gp[F][C];
                float D0f[C];
#pragma unroll
                for (int c = 0; c < C; ++c) D0f[c] = (float)d0tab[c * ns + sidx];
#pragma unroll
                for (int f = 0; f < F; ++f) {
                    const int myp = sy0 + row0 + 4 * f;
                    fmy[f] = (float)myp;
                    mxy[f] = fmx * fmy[f];
                    myy[f] = fmy[f] * fmy[f];
                    dyf[f] = (float)(row0 + 4 * f - SY / 2);
                    const bool in = xin && myp >= -hy && myp < hy;
                    const int my = myp < 0 ? myp + k.ny : myp;
                    const int64_t o = (int64_t)my * k.nx + mx;
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        if (in) {
                            const float2 gv = gspec[c * M + o];
                            gm[f][c] = gv.x;
                            gp[f][c] = gv.y;
                            dD[f][c] = dtab[c * M + o];
                        } else {
                            gm[f][c] = gp[f][c] = 0.0f;
                            dD[f][c] = 0.0f;
                        }
                    }
                }
                const float4 *sw = reinterpret_cast<const float4 *>(&s_w[wave][0]);
                for (int ei = 0; ei < cnt; ++ei) {
                    // e0 = (alpha, beta2, gamma, z), e1 = (rxf, ryf, owner, rows), e2 = amp, e3 = base
                    const float4 e0 = sw[4 * ei], e1 = sw[4 * ei + 1], e2 = sw[4 * ei + 2], e3 = sw[4 * ei + 3];
                    const float alpha = e0.x, beta2 = e0.y, gamma = e0.z, z = e0.w, rxf = e1.x, ryf = e1.y;
                    const int owner = __float_as_int(e1.z);
                    const uint32_t rows = __builtin_amdgcn_readfirstlane(__float_as_uint(e1.w));
                    const float ampv[4] = {e2.x, e2.y, e2.z, e2.w}, basev[4] = {e3.x, e3.y, e3.z, e3.w};
                    float amp[C], bx[C];
                    const float ax = alpha * mxx;
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        amp[c] = ampv[c];
                        bx[c] = __builtin_amdgcn_fractf(fmaf(-dxf, rxf, basev[c]));
                    }
                    float Pr[C], Pi[C], Wc[C];
#pragma unroll
                    for (int c = 0; c < C; ++c) Pr[c] = Pi[c] = Wc[c] = 0.0f;
                    // rho = sum_c amp_c E conj(Gs_c) e^{j 2 pi th_c} at one frequency;
                    // R1 = sum m_y' Re rho, R2 = sum m_y'^2 Re rho, I0 = sum Im rho, I1 = sum m_y' Im rho,
                    // and sum Re rho = sum_c amp_c Re P_c is formed once after the loop
                    float R1 = 0.0f, R2 = 0.0f, I0 = 0.0f, I1 = 0.0f;
#pragma unroll
                    for (int f = 0; f < F; ++f) {
                        if (!(rows & (1u << f))) continue;  // the support misses this 4-row block
                        const float q = fmaf(gamma, myy[f], fmaf(beta2, mxy[f], ax));
                        const float E = __builtin_amdgcn_exp2f(-q);
                        float rr = 0.0f, ri = 0.0f;
#pragma unroll
                        for (int c = 0; c < C; ++c) {
                            // E conj(Gs) e^{j 2 pi th} = E |Gs| e^{j 2 pi (th - arg Gs / 2 pi)}
                            const float th = fmaf(-z, dD[f][c], fmaf(-dyf[f], ryf, bx[c]) - gp[f][c]);
                            const float sn = __builtin_amdgcn_sinf(th);
                            const float cs = __builtin_amdgcn_cosf(th);
                            const float eg = E * gm[f][c];
                            Pr[c] = fmaf(eg, cs, Pr[c]);
                            if (DEPTH) Pi[c] = fmaf(eg, sn, Pi[c]);
                            if (DEPTH) Wc[c] = fmaf(dD[f][c] * eg, sn, Wc[c]);
                            const float ae = amp[c] * eg;
                            rr = fmaf(ae, cs, rr);
                            ri = fmaf(ae, sn, ri);
                        }
                        R1 = fmaf(fmy[f], rr, R1);
                        R2 = fmaf(myy[f], rr, R2);
                        I0 += ri;
                        I1 = fmaf(fmy[f], ri, I1);
                    }
                    float R0 = 0.0f;
#pragma unroll
                    for (int c = 0; c < C; ++c) R0 = fmaf(amp[c], Pr[c], R0);
                    // value layout: Re P_c (C), Sfx, Sfy, Qxx, Qxy, Qyy, then with depth Im P_c (C), W_c (C)
                    float x[NR];
#pragma unroll
                    for (int c = 0; c < C; ++c) x[c] = Pr[c];
                    x[C + 0] = fmx * I0;   // Sfx
                    x[C + 1] = I1;         // Sfy
                    x[C + 2] = mxx * R0;   // Qxx
                    x[C + 3] = fmx * R1;   // Qxy
                    x[C + 4] = R2;         // Qyy
                    if (DEPTH) {
#pragma unroll
                        for (int c = 0; c < C; ++c) {
                            x[C + 5 + c] = Pi[c];
                            x[2 * C + 5 + c] = fmaf(D0f[c], Pi[c], Wc[c]);
                        }
                    }
#pragma unroll
                    for (int i = NV; i < NR; ++i) x[i] = 0.0f;
                    // without depth, sum_m Im rho (the phase gradient) rides along as y
                    float sim = I0;
                    reduce_transposed<NR, !DEPTH>(x, sim, lane);
                    if ((lane & 7) == 0) {
                        const int v0 = (NR / 8) * (((lane >> 5) & 1) * 4 + ((lane >> 4) & 1) * 2 + ((lane >> 3) & 1));
#pragma unroll
                        for (int j = 0; j < NR / 8; ++j)
                            if (v0 + j < NV) atomicAdd(&s_acc[wave][owner][v0 + j], x[j]);  // ds_add_f32, no return
                    }
                    if (!DEPTH && lane == 4) atomicAdd(&s_acc[wave][owner][EXTRA_SLOT], sim);
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }
        float *dst = S.bpartials + ((int64_t)bi.slot * 64 + lane) * NACC;
#pragma unroll
        for (int v = 0; v < NACC; ++v) dst[v] = s_acc[wave][lane][v];
        __builtin_amdgcn_wave_barrier();
        pairs = wave_sum_i64(pairs);
        if (lane == 0 && pairs) atomicAdd((unsigned long long *)&S.counters[CTR_PAIRS], (unsigned long long)pairs);
    }
}

template <int C, int F>
static hipError_t launch_adj_cf(const Plan &p, const Consts &k, const BwdScene *scenes, const int32_t *prefix,
                                int n_scenes, long long *queue, const float *dtab, const double *d0tab, int nsx,
                                int nsy, int sx_min, int sy_min, int grid, hipStream_t s)
{
    if (k.depth_grad)
        hipLaunchKernelGGL((k_adjoint<C, true, F>), dim3(grid), dim3(WG), 0, s, k, p.tile_xy, scenes, prefix, n_scenes,
                           queue, dtab, d0tab, nsx, nsy, sx_min, sy_min);
    else
        hipLaunchKernelGGL((k_adjoint<C, false, F>), dim3(grid), dim3(WG), 0, s, k, p.tile_xy, scenes, prefix, n_scenes,
                           queue, dtab, d0tab, nsx, nsy, sx_min, sy_min);
    return hipGetLastError();
}

template <int C>
static hipError_t launch_adj_c(const Plan &p, const Consts &k, const BwdScene *scenes, const int32_t *prefix,
                               int n_scenes, long long *queue, const float *dtab, const double *d0tab, int nsx, int nsy,
                               int sx_min, int sy_min, int grid, hipStream_t s)
{
    switch (p.F) {
    case 2: return launch_adj_cf<C, 2>(p, k, scenes, prefix, n_scenes, queue, dtab, d0tab, nsx, nsy, sx_min, sy_min, grid, s);
    case 8: return launch_adj_cf<C, 8>(p, k, scenes, prefix, n_scenes, queue, dtab, d0tab, nsx, nsy, sx_min, sy_min, grid, s);
    default: return launch_adj_cf<C, 4>(p, k, scenes, prefix, n_scenes, queue, dtab, d0tab, nsx, nsy, sx_min, sy_min, grid, s);
    }
}

hipError_t launch_adjoint(const Plan &p, const Consts &k, const BwdScene *scenes, const int32_t *prefix, int n_scenes,
                          long long *queue, const float *dtab, const double *d0tab, int nsx, int nsy, int sx_min,
                          int sy_min, int grid, hipStream_t s)
{
    switch (k.C) {
    case 1: return launch_adj_c<1>(p, k, scenes, prefix, n_scenes, queue, dtab, d0tab, nsx, nsy, sx_min, sy_min, grid, s);
    case 2: return launch_adj_c<2>(p, k, scenes, prefix, n_scenes, queue, dtab, d0tab, nsx, nsy, sx_min, sy_min, grid, s);
    case 3: return launch_adj_c<3>(p, k, scenes, prefix, n_scenes, queue, dtab, d0tab, nsx, nsy, sx_min, sy_min, grid, s);
    default: return hipErrorInvalidValue;  // 3C + 5 accumulators must fit 16
    }
}

template <int C, bool DEPTH>
static const void *adj_kernel_ptr(int F)
{
    switch (F) {
    case 2: return (const void *)k_adjoint<C, DEPTH, 2>;
    case 8: return (const void *)k_adjoint<C, DEPTH, 8>;
    default: return (const void *)k_adjoint<C, DEPTH, 4>;
    }
}

int adjoint_occupancy(int C, int F, int depth)
{
    const void *kp = nullptr;
    switch (C) {
    case 1: kp = depth ? adj_kernel_ptr<1, true>(F) : adj_kernel_ptr<1, false>(F); break;
    case 2: kp = depth ? adj_kernel_ptr<2, true>(F) : adj_kernel_ptr<2, false>(F); break;
    default: kp = depth ? adj_kernel_ptr<3, true>(F) : adj_kernel_ptr<3, false>(F); break;
    }
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kp, WG, 0) != hipSuccess || nb < 1) nb = 1;
    return nb;
}

// Per Gaussian: sum the item partials of its chunk in order (FP64), then the chain rule.
__global__ void __launch_bounds__(256) k_grad_final(GView g, Consts k, const uint32_t *__restrict__ vals,
                                                    const int2 *__restrict__ chunk_items,
                                                    const int32_t *__restrict__ range_base,
                                                    const float *__restrict__ bpartials, GradView grads, int64_t n,
                                                    const long long *__restrict__ counters)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int64_t nvalid = n - counters[CTR_NCULLED];
    const int64_t i = vals[s];
    const int C = k.C;
    if (s >= nvalid) {
        grads.mean_x[i] = grads.mean_y[i] = 0.0f;
        if (grads.depth) grads.depth[i] = 0.0f;
        grads.cov_xx[i] = grads.cov_xy[i] = grads.cov_yy[i] = 0.0f;
        grads.opacity[i] = grads.phase[i] = 0.0f;
        for (int c = 0; c < C; ++c) grads.amplitude[(int64_t)c * grads.amp_stride + i] = 0.0f;
        return;
    }
    const int64_t b = s / 64;
    const int lane = (int)(s - b * 64);
    const int2 ci = chunk_items[b];
    const long long nbitems = counters[CTR_NBITEMS];
    double acc[NACC];
    for (int v = 0; v < NACC; ++v) acc[v] = 0.0;
    for (int j = 0; j < ci.y; ++j) {
        const int64_t it = (int64_t)range_base[j] + b;  // range j of chunk b
        if (it >= nbitems) break;
        const float *src = bpartials + (it * 64 + lane) * NACC;
        for (int v = 0; v < NACC; ++v) acc[v] += (double)src[v];
    }
    const double PI = 3.14159265358979323846;
    const double sxx = g.cov_xx[i], sxy = g.cov_xy[i], syy = g.cov_yy[i];
    const double det = sxx * syy - sxy * sxy;
    const double o = g.opacity[i];
    const double fx = 1.0 / (k.nx * k.px), fy = 1.0 / (k.ny * k.py);
    const double K = 2.0 * PI * sqrt(det) / (k.px * k.py * (double)k.nx * (double)k.ny);
    double Sre = 0.0, gz = 0.0, go = 0.0;
    for (int c = 0; c < C; ++c) {
        const double a = g.amplitude[(int64_t)c * g.amp_stride + i];
        const double A = a * o * K;
        const double Pr = acc[c];
        const double Pi = k.depth_grad ? acc[C + 5 + c] : 0.0, Wc = k.depth_grad ? acc[2 * C + 5 + c] : 0.0;
        Sre += A * Pr;
        gz += A * (k.inv_lambda[c] * Pi + Wc);
        go += a * K * Pr;
        grads.amplitude[(int64_t)c * grads.amp_stride + i] = (float)(o * K * Pr);
    }
    const double Sfx = acc[C], Sfy = acc[C + 1], Qxx = acc[C + 2], Qxy = acc[C + 3], Qyy = acc[C + 4];
    // sum_c A_c Im P_c (= sum_m Im rho): from Im P_c with depth, else the extra reduced slot
    double Sim = 0.0;
    if (k.depth_grad) {
        for (int c = 0; c < C; ++c) Sim += (double)g.amplitude[(int64_t)c * g.amp_stride + i] * o * K * acc[C + 5 + c];
    } else {
        Sim = acc[8];
    }
    grads.phase[i] = (float)(-Sim);
    grads.mean_x[i] = (float)(2.0 * PI * fx * Sfx);
    grads.mean_y[i] = (float)(2.0 * PI * fy * Sfy);
    grads.opacity[i] = (float)go;
    grads.cov_xx[i] = (float)(syy / (2.0 * det) * Sre - 2.0 * PI * PI * fx * fx * Qxx);
    grads.cov_yy[i] = (float)(sxx / (2.0 * det) * Sre - 2.0 * PI * PI * fy * fy * Qyy);
    grads.cov_xy[i] = (float)(-sxy / det * Sre - 4.0 * PI * PI * fx * fy * Qxy);
    if (grads.depth) grads.depth[i] = (float)(2.0 * PI * gz);
}

hipError_t launch_grad_final(const GView &g, const Consts &k, const uint32_t *vals, const int2 *chunk_items,
                             const int32_t *range_base, const float *bpartials, const GradView &grads, int64_t n,
                             const long long *counters, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_grad_final, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, k, vals, chunk_items,
                       range_base, bpartials, grads, n, counters);
    return hipGetLastError();
}

}  // namespace gws
