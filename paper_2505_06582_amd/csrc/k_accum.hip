// Spectrum accumulation (gfx950): the order-invariant sum of Sec. 4.2, Eq. 12,
//   S_c[m] = sum_i A_{c,i} exp2(-q_i(m)) exp(j 2 pi Theta_{c,i}(m)),
// evaluated only where the Gaussian envelope exceeds eps of its peak.  The paper's own
// kernel (supplement Alg. 4) gives every thread one pixel and loops over all Gaussians;
// here a work-group owns a 32 x 32 tile of frequencies and a chunk of the Gaussians whose
// support reaches it, stages the accepted Gaussians in LDS, and every lane evaluates four
// frequencies per Gaussian with hardware exp2 / sin / cos.
//
// Phase, in revolutions, for Gaussian i, wavelength c, frequency m' = m0' + d (m0' the
// centre of the lane's 16 x 16 sub-tile):
//   Theta = kappa_c - m'.r - z D_c(nu_m)
//         = [kappa_c - m0'.r - z D_c(nu_0)]            exact: fixed point + FP64, per (sub-tile, i)
//           - d.r_f32 - z (D_c(nu_m) - D_c(nu_0))      small: FP32, per lane
// with r = frac(mu / (N p) + 1/2) (the +1/2 folds the SLM centring), kappa_c =
// frac(phi/2pi - z/lambda_c), and D_c(nu) = sqrt(1/lambda_c^2 - |nu|^2) - 1/lambda_c
// written without cancellation as -|nu|^2 / (1/lambda_c + sqrt(1/lambda_c^2 - |nu|^2)).
// v_sin_f32 / v_cos_f32 take revolutions, so no 2 pi scaling is needed.
#include "gws_internal.h"

namespace gws {

static __device__ __forceinline__ double frac_d(double v) { return v - floor(v); }

// D_c(nu) in cycles per metre (negative), or +inf marker when evanescent.
static __device__ __forceinline__ double dprop(double nu2, double inv_l)
{
    const double w2 = inv_l * inv_l - nu2;
    if (!(w2 > 0.0)) return 0.0;
    return -nu2 / (inv_l + sqrt(w2));
}

static __device__ __forceinline__ bool ellipse_meets_rect(float a, float b2, float g, float lim, float x0, float x1,
                                                          float y0, float y1)
{
    return ellipse_meets_rect_r(a, b2, g, 0.5f / a, 0.5f / g, lim, x0, x1, y0, y1);
}

// Compacted per-(sub-tile, Gaussian) entry, 16 floats.
struct alignas(16) WEntry {
    float alpha, beta2, gamma, z;
    float rxf, ryf;
    uint32_t rows;   // row_block_mask of this Gaussian on the sub-tile
    float pad1;
    float amp[4];
    float base[4];
};

// One persistent launch serves every scene of a batch: the queue head walks the
// concatenation of the scenes' work-item lists (prefix[s] = first item of scene s).
template <int C, bool EVAN, int F>
__global__ void __launch_bounds__(WG, waves_per_simd(F)) k_accumulate(Consts k, const int32_t *__restrict__ tile_xy,
                                                   const FwdScene *__restrict__ scenes, const int32_t *__restrict__ prefix,
                                                   int n_scenes, long long *__restrict__ queue)
{
    __shared__ GRec s_rec[WG];
    __shared__ WEntry s_w[WAVES][64];
    __shared__ int s_item, s_scene;
    __shared__ int s_cnt[WAVES];

    constexpr int SY = sub_h(F), TY = 2 * SY;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int total_items = prefix[n_scenes];
    const int hx = k.nx / 2, hy = k.ny / 2;
    const double Wx = k.nx * k.px, Wy = k.ny * k.py;
    const float lim = (float)(k.tau2 * (1.0 + 1e-5)) + 1e-4f;
    // every support is an ellipse centred at m_r (DC unless a reference plane wave tilts the
    // illumination): the support tests and the envelope take frequencies relative to it
    const float mrxf = (float)k.mrx, mryf = (float)k.mry;

    for (;;) {
        if (tid == 0) {
            const int q = (int)atomicAdd((unsigned long long *)queue, 1ull);
            int sc = 0;
            if (q < total_items)
                while (sc + 1 < n_scenes && prefix[sc + 1] <= q) ++sc;
            s_item = q;
            s_scene = sc;
        }
        __syncthreads();
        const int gitem = s_item, scene = s_scene;
        __syncthreads();
        if (gitem >= total_items) break;
        const FwdScene S = scenes[scene];
        const GRec *__restrict__ rec = S.rec;
        const Item it = S.items[gitem - prefix[scene]];
        const int CH = (int)S.counters[CTR_CHUNK];
        const int32_t *__restrict__ tile_L = S.tile_L;
        long long pairs = 0;
        const int32_t txy = tile_xy[it.tile];
        const int tx = (int)(int16_t)(txy & 0xffff), ty = txy >> 16;
        const int L = tile_L[it.tile];
        const int c0 = it.chunk * CH, c1 = min(c0 + CH, L);
        // work-group tile rectangle, clipped to the grid
        const float X0 = (float)max(tx * TILEX, -hx), X1 = (float)min(tx * TILEX + TILEX - 1, hx - 1);
        const float Y0 = (float)max(ty * TY, -hy), Y1 = (float)min(ty * TY + TY - 1, hy - 1);
        // this wave's sub-tile
        const int sx0 = tx * TILEX + (wave & 1) * SUBX, sy0 = ty * TY + (wave >> 1) * SY;
        const int cx = sx0 + SUBX / 2, cy = sy0 + SY / 2;
        const float x0 = (float)max(sx0, -hx), x1 = (float)min(sx0 + SUBX - 1, hx - 1);
        const float y0 = (float)max(sy0, -hy), y1 = (float)min(sy0 + SY - 1, hy - 1);
        const bool wave_live = (x0 <= x1) && (y0 <= y1);
        // per-lane frequency constants
        const int col = lane & (SUBX - 1), row0 = lane >> 4;
        const int mxp = sx0 + col;
        const float fmx = (float)((double)mxp - k.mrx);  // envelope coordinate, relative to m_r
        const float mxx = fmx * fmx, dxf = (float)(col - SUBX / 2);
        float mxy[F], myy[F], dyf[F], dD[F][C], msk[F][C];
        double D0[C];
        {
            const double ncx = cx / Wx, ncy = cy / Wy;
            for (int c = 0; c < C; ++c) D0[c] = dprop(ncx * ncx + ncy * ncy, k.inv_lambda[c]);
        }
#pragma unroll
        for (int f = 0; f < F; ++f) {
            const int myp = sy0 + row0 + 4 * f;
            const float fmy = (float)((double)myp - k.mry);
            mxy[f] = fmx * fmy;
            myy[f] = fmy * fmy;
            dyf[f] = (float)(row0 + 4 * f - SY / 2);
            const double nux = mxp / Wx, nuy = myp / Wy;
            const double nu2 = nux * nux + nuy * nuy;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const double il = k.inv_lambda[c];
                dD[f][c] = (float)(dprop(nu2, il) - D0[c]);
                msk[f][c] = (nu2 < il * il) ? 1.0f : 0.0f;
            }
        }
        float acc_re[F][C], acc_im[F][C];
#pragma unroll
        for (int f = 0; f < F; ++f)
#pragma unroll
            for (int c = 0; c < C; ++c) acc_re[f][c] = acc_im[f][c] = 0.0f;

        for (int base = c0; base < c1; base += WG) {
            const int gi = base + tid;
            bool pred = false;
            // the record as four 16-byte registers (a struct here would be kept in scratch)
            float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0, r2 = r0, r3 = r0;
            if (gi < c1) {
                const float4 *src = reinterpret_cast<const float4 *>(rec + gi);
                r0 = src[0];
                r1 = src[1];
                r2 = src[2];
                r3 = src[3];
                pred = ellipse_meets_rect(r0.x, r0.y, r0.z, lim, X0 - mrxf, X1 - mrxf, Y0 - mryf, Y1 - mryf);
            }
            const uint64_t bal = __ballot(pred);
            const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
            if (lane == 0) s_cnt[wave] = __popcll(bal);
            __syncthreads();
            int off = 0, total = 0;
#pragma unroll
            for (int w = 0; w < WAVES; ++w) {
                const int cw = s_cnt[w];
                off += (w < wave) ? cw : 0;
                total += cw;
            }
            if (pred) {
                float4 *dst = reinterpret_cast<float4 *>(&s_rec[off + __popcll(bal & lt)]);
                dst[0] = r0;
                dst[1] = r1;
                dst[2] = r2;
                dst[3] = r3;
            }
            __syncthreads();
            if (wave_live) {
                for (int j0 = 0; j0 < total; j0 += 64) {
                    const int j = j0 + lane;
                    bool p = false;
                    WEntry e = {};
                    if (j < total) {
                        const GRec q = s_rec[j];
                        p = ellipse_meets_rect(q.alpha, q.beta2, q.gamma, lim, x0 - mrxf, x1 - mrxf, y0 - mryf,
                                               y1 - mryf);
                        if (p) {
                            e.alpha = q.alpha; e.beta2 = q.beta2; e.gamma = q.gamma; e.z = q.z;
                            e.rxf = q.rxf; e.ryf = q.ryf; e.pad1 = 0.0f;
                            e.rows = row_block_mask<F>(q.alpha, q.beta2, q.gamma, lim, x0 - mrxf, x1 - mrxf, sy0, hy,
                                                       mryf);
                            pairs += __popc(e.rows) * (SUBX * 4);
                            // exact ramp at the sub-tile centre: 0.32 fixed point, wraps mod 1
                            const uint32_t ramp = (uint32_t)cx * q.rx + (uint32_t)cy * q.ry;
                            const double ramp_rev = (double)ramp * (1.0 / 4294967296.0);
#pragma unroll
                            for (int c = 0; c < 4; ++c) {
                                e.amp[c] = q.amp[c];
                                if (c < C) {
                                    if (k.phase_mode == 1) {
                                        // plain FP32 phase (precision study only)
                                        const float rr = (float)cx * q.rxf + (float)cy * q.ryf;
                                        const float v = q.kappa[c] - rr - q.z * (float)D0[c];
                                        e.base[c] = v - floorf(v);
                                    } else {
                                        e.base[c] = (float)frac_d((double)q.kappa[c] - ramp_rev - (double)q.z * D0[c]);
                                    }
                                } else {
                                    e.base[c] = 0.0f;
                                }
                            }
                        }
                    }
                    const uint64_t b2 = __ballot(p);
                    const int cnt = __popcll(b2);
                    if (p) s_w[wave][__popcll(b2 & lt)] = e;
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    for (int ei = 0; ei < cnt; ++ei) {
                        const WEntry &w = s_w[wave][ei];
                        const float alpha = w.alpha, beta2 = w.beta2, gamma = w.gamma, z = w.z;
                        const float rxf = w.rxf, ryf = w.ryf;
                        const uint32_t rows = __builtin_amdgcn_readfirstlane(w.rows);
                        float amp[C], bx[C];
                        const float ax = alpha * mxx;
#pragma unroll
                        for (int c = 0; c < C; ++c) {
                            amp[c] = w.amp[c];
                            bx[c] = __builtin_amdgcn_fractf(fmaf(-dxf, rxf, w.base[c]));
                        }
#pragma unroll
                        for (int f = 0; f < F; ++f) {
                            if (!(rows & (1u << f))) continue;  // the support misses this 4-row block
                            const float q = fmaf(gamma, myy[f], fmaf(beta2, mxy[f], ax));
                            const float E = __builtin_amdgcn_exp2f(-q);
#pragma unroll
                            for (int c = 0; c < C; ++c) {
                                const float t = fmaf(-dyf[f], ryf, bx[c]);
                                const float th = fmaf(-z, dD[f][c], t);
                                const float sn = __builtin_amdgcn_sinf(th);
                                const float cs = __builtin_amdgcn_cosf(th);
                                float wgt = amp[c] * E;
                                if (EVAN) wgt *= msk[f][c];
                                acc_re[f][c] = fmaf(wgt, cs, acc_re[f][c]);
                                acc_im[f][c] = fmaf(wgt, sn, acc_im[f][c]);
                            }
                        }
                    }
                    __builtin_amdgcn_wave_barrier();
                }
            }
            __syncthreads();
        }
        // write out
#pragma unroll
        for (int f = 0; f < F; ++f) {
            const int myp = sy0 + row0 + 4 * f;
            const bool valid = mxp >= -hx && mxp < hx && myp >= -hy && myp < hy;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const float2 v = make_float2(acc_re[f][c], acc_im[f][c]);
                if (it.slot < 0) {
                    if (valid) {
                        const int mx = mxp < 0 ? mxp + k.nx : mxp, my = myp < 0 ? myp + k.ny : myp;
                        S.spectrum[((int64_t)c * k.ny + my) * k.nx + mx] = v;
                    }
                } else {
                    S.partials[(((int64_t)it.slot * C + c) * F + f) * WG + tid] = v;
                }
            }
        }
        pairs = wave_sum_i64(pairs);
        if (lane == 0 && pairs) atomicAdd((unsigned long long *)&S.counters[CTR_PAIRS], (unsigned long long)pairs);
    }
}

template <int C, int F>
__global__ void __launch_bounds__(WG) k_reduce_partials(Consts k, const int32_t *__restrict__ tile_xy,
                                                        const FwdScene *__restrict__ scenes)
{
    const int t = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const FwdScene S = scenes[blockIdx.y];
    const float2 *__restrict__ partials = S.partials;
    float2 *__restrict__ spectrum = S.spectrum;
    const int2 ts = S.tile_slots[t];
    if (ts.x == 1) return;  // written directly by the accumulation
    const int32_t txy = tile_xy[t];
    const int tx = (int)(int16_t)(txy & 0xffff), ty = txy >> 16;
    const int hx = k.nx / 2, hy = k.ny / 2;
    constexpr int SY = sub_h(F), TY = 2 * SY;
    const int sx0 = tx * TILEX + (wave & 1) * SUBX, sy0 = ty * TY + (wave >> 1) * SY;
    const int mxp = sx0 + (lane & (SUBX - 1)), row0 = lane >> 4;
#pragma unroll
    for (int f = 0; f < F; ++f) {
        const int myp = sy0 + row0 + 4 * f;
        const bool valid = mxp >= -hx && mxp < hx && myp >= -hy && myp < hy;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            // slots summed in order; eight loads are issued before their adds
            const float2 *src = partials + (((int64_t)ts.y * C + c) * F + f) * WG + tid;
            const int64_t stride = (int64_t)C * F * WG;
            float2 s = make_float2(0.0f, 0.0f);
            int j = 0;
            for (; j + 8 <= ts.x; j += 8) {
                float2 v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = src[(j + u) * stride];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    s.x += v[u].x;
                    s.y += v[u].y;
                }
            }
            for (; j < ts.x; ++j) {
                const float2 v = src[j * stride];
                s.x += v.x;
                s.y += v.y;
            }
            if (valid) {
                const int mx = mxp < 0 ? mxp + k.nx : mxp, my = myp < 0 ? myp + k.ny : myp;
                spectrum[((int64_t)c * k.ny + my) * k.nx + mx] = s;
            }
        }
    }
}

static bool tile_needs_evanescent(const Plan &p, const Consts &k)
{
    // is any grid frequency at or beyond 1/lambda for some channel?
    const double nux = (p.nx / 2) / (p.nx * k.px), nuy = (p.ny / 2) / (p.ny * k.py);
    const double nu2 = nux * nux + nuy * nuy;
    for (int c = 0; c < k.C; ++c)
        if (!(nu2 < k.inv_lambda[c] * k.inv_lambda[c])) return true;
    return false;
}

template <int C, int F>
static hipError_t launch_acc_cf(const Plan &p, const Consts &k, const FwdScene *scenes, const int32_t *prefix,
                                int n_scenes, long long *queue, int grid, hipStream_t s)
{
    if (tile_needs_evanescent(p, k))
        hipLaunchKernelGGL((k_accumulate<C, true, F>), dim3(grid), dim3(WG), 0, s, k, p.tile_xy, scenes, prefix, n_scenes,
                           queue);
    else
        hipLaunchKernelGGL((k_accumulate<C, false, F>), dim3(grid), dim3(WG), 0, s, k, p.tile_xy, scenes, prefix, n_scenes,
                           queue);
    return hipGetLastError();
}

template <int C>
static hipError_t launch_acc_c(const Plan &p, const Consts &k, const FwdScene *scenes, const int32_t *prefix,
                               int n_scenes, long long *queue, int grid, hipStream_t s)
{
    switch (p.F) {
    case 2: return launch_acc_cf<C, 2>(p, k, scenes, prefix, n_scenes, queue, grid, s);
    case 8: return launch_acc_cf<C, 8>(p, k, scenes, prefix, n_scenes, queue, grid, s);
    default: return launch_acc_cf<C, 4>(p, k, scenes, prefix, n_scenes, queue, grid, s);
    }
}

hipError_t launch_accumulate(const Plan &p, const Consts &k, const FwdScene *scenes, const int32_t *prefix, int n_scenes,
                             long long *queue, int grid, hipStream_t s)
{
    switch (k.C) {
    case 1: return launch_acc_c<1>(p, k, scenes, prefix, n_scenes, queue, grid, s);
    case 2: return launch_acc_c<2>(p, k, scenes, prefix, n_scenes, queue, grid, s);
    case 3: return launch_acc_c<3>(p, k, scenes, prefix, n_scenes, queue, grid, s);
    case 4: return launch_acc_c<4>(p, k, scenes, prefix, n_scenes, queue, grid, s);
    default: return hipErrorInvalidValue;
    }
}

template <int C>
static void launch_red_c(const Plan &p, const Consts &k, const FwdScene *scenes, int n_scenes, hipStream_t s)
{
    const dim3 grid(p.ntiles, n_scenes), block(WG);
    switch (p.F) {
    case 2: hipLaunchKernelGGL((k_reduce_partials<C, 2>), grid, block, 0, s, k, p.tile_xy, scenes); break;
    case 8: hipLaunchKernelGGL((k_reduce_partials<C, 8>), grid, block, 0, s, k, p.tile_xy, scenes); break;
    default: hipLaunchKernelGGL((k_reduce_partials<C, 4>), grid, block, 0, s, k, p.tile_xy, scenes); break;
    }
}

hipError_t launch_reduce_partials(const Plan &p, const Consts &k, const FwdScene *scenes, int n_scenes, hipStream_t s)
{
    switch (k.C) {
    case 1: launch_red_c<1>(p, k, scenes, n_scenes, s); break;
    case 2: launch_red_c<2>(p, k, scenes, n_scenes, s); break;
    case 3: launch_red_c<3>(p, k, scenes, n_scenes, s); break;
    case 4: launch_red_c<4>(p, k, scenes, n_scenes, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int C>
static const void *acc_kernel_ptr(int F)
{
    switch (F) {
    case 2: return (const void *)k_accumulate<C, false, 2>;
    case 8: return (const void *)k_accumulate<C, false, 8>;
    default: return (const void *)k_accumulate<C, false, 4>;
    }
}

int accumulate_occupancy(int C, int F)
{
    int nb = 0;
    const void *kp = nullptr;
    switch (C) {
    case 1: kp = acc_kernel_ptr<1>(F); break;
    case 2: kp = acc_kernel_ptr<2>(F); break;
    case 3: kp = acc_kernel_ptr<3>(F); break;
    default: kp = acc_kernel_ptr<4>(F); break;
    }
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kp, WG, 0) != hipSuccess || nb < 1) nb = 1;
    return nb;
}

}  // namespace gws
