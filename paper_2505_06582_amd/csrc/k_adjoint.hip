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
// Work.  A region is a 16-column x 64-row block of the centred frequency plane (one half
// of a 32 x 64 tile of the adjoint's tile list), made of two 16 x 32 sub-tiles, the unit of
// the exact phase base.  Everything the sums need per frequency -- |Gs_c|, arg Gs_c / 2 pi
// and D_c(nu) - D_c(nu_0) -- is packed region-major once per call (k_adj_pack_g,
// k_adj_pack_d), so a work-group of 8 wavefronts copies one region into LDS with
// coalesced loads and every wavefront reads it from there.  The work-group owns 512
// consecutive sorted Gaussians (one per thread) and a range of tiles; for each region,
// every thread tests its own Gaussian (exact ellipse test, 4-row block mask, FP64 phase
// bases of both sub-tiles), then each wavefront walks its accepted Gaussians one at a time:
// the record arrives by scalar loads, lane l evaluates column l % 16 and rows l / 16 + 4 b
// of every 4-row block b the support reaches (up to 16 blocks, 1024 frequencies), and the
// per-lane sums are reduced across the wavefront once per (Gaussian, region) into that
// Gaussian's LDS accumulator.  No per-lane frequency tables are held in registers, so two
// work-groups (four wavefronts per SIMD) share a CU and one's barriers overlap the other's
// work.  Item partials are summed per Gaussian in a fixed order, so results are bitwise
// reproducible.
#include "gws_internal.h"

namespace gws {

static __device__ __forceinline__ double frac_d(double v) { return v - floor(v); }

// D_c(nu) = sqrt(1/lambda^2 - |nu|^2) - 1/lambda written without cancellation; 0 when the
// frequency is evanescent (such frequencies carry no signal, see k_adj_pack_g).
static __device__ __forceinline__ double dprop_b(double nu2, double il)
{
    const double w2 = il * il - nu2;
    return w2 > 0.0 ? -nu2 / (il + sqrt(w2)) : 0.0;
}

// Frequency (signed index units) of element (region r, block b, lane) of the packed layout.
static __device__ __forceinline__ void adj_elem_freq(const AdjGeom &geo, int r, int b, int lane, int *mxp, int *myp)
{
    const int h = r & 1, t = r >> 1;
    const int tx = t % geo.ntx + geo.tx_min, ty = t / geo.ntx + geo.ty_min;
    *mxp = tx * TILEX + h * ADJ_RW + (lane & (ADJ_RW - 1));
    *myp = ty * ADJ_RH + 4 * b + (lane >> 4);
}

// Geometry-only part of the packed table (shared by every scene): dD[r][b][c][lane] =
// D_c(nu) - D_c(nu_0) with nu_0 the centre of the element's sub-tile (0 outside the grid or
// when evanescent), and D0[r][s][c] = D_c(nu_0) of sub-tile s in FP64.
__global__ void __launch_bounds__(256) k_adj_pack_d(Consts k, AdjGeom geo, float *__restrict__ dpack,
                                                   double *__restrict__ d0)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int C = k.C;
    const int64_t per_r = (int64_t)ADJ_NB * C * 64;
    const int64_t total = (int64_t)geo.nreg * per_r;
    if (idx >= total) return;
    const int r = (int)(idx / per_r);
    const int rem = (int)(idx - (int64_t)r * per_r);
    const int b = rem / (C * 64), c = (rem / 64) % C, lane = rem & 63;
    int mxp, myp;
    adj_elem_freq(geo, r, b, lane, &mxp, &myp);
    const double Wx = k.nx * k.px, Wy = k.ny * k.py;
    const int hx = k.nx / 2, hy = k.ny / 2;
    const int mx0 = mxp - (lane & (ADJ_RW - 1));
    const int cx = mx0 + ADJ_RW / 2, cy = myp - (lane >> 4) - 4 * (b & 7) + ADJ_SH / 2;
    const double ncx = cx / Wx, ncy = cy / Wy;
    const double D0 = dprop_b(ncx * ncx + ncy * ncy, k.inv_lambda[c]);
    float v = 0.0f;
    if (mxp >= -hx && mxp < hx && myp >= -hy && myp < hy) {
        const double nux = mxp / Wx, nuy = myp / Wy;
        const double nu2 = nux * nux + nuy * nuy;
        const double il = k.inv_lambda[c];
        if (nu2 < il * il) v = (float)(dprop_b(nu2, il) - D0);
    }
    dpack[idx] = v;
    if (lane == 0 && (b & 7) == 0) d0[((int64_t)r * 2 + (b >> 3)) * C + c] = D0;
}

// Per-scene part: gpack[r][b][c][lane] = (|Gs_c|, arg Gs_c / 2 pi) at the element's
// frequency, zero outside the grid and where the frequency is evanescent for channel c (the
// forward sets H to zero there, so its adjoint has nothing to propagate).  The adjoint then
// forms conj(Gs) e^{j 2 pi Theta} as |Gs| e^{j 2 pi (Theta - arg Gs / 2 pi)}: one more phase
// term, two products instead of a complex product.
__global__ void __launch_bounds__(256) k_adj_pack_g(Consts k, AdjGeom geo, const float2 *__restrict__ gspec,
                                                   float2 *__restrict__ gpack)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int C = k.C;
    const int64_t per_r = (int64_t)ADJ_NB * C * 64;
    const int64_t total = (int64_t)geo.nreg * per_r;
    if (idx >= total) return;
    const int r = (int)(idx / per_r);
    const int rem = (int)(idx - (int64_t)r * per_r);
    const int b = rem / (C * 64), c = (rem / 64) % C, lane = rem & 63;
    int mxp, myp;
    adj_elem_freq(geo, r, b, lane, &mxp, &myp);
    const int hx = k.nx / 2, hy = k.ny / 2;
    float2 v = make_float2(0.0f, 0.0f);
    if (mxp >= -hx && mxp < hx && myp >= -hy && myp < hy) {
        const double nux = mxp / (k.nx * k.px), nuy = myp / (k.ny * k.py);
        const double il = k.inv_lambda[c];
        if (nux * nux + nuy * nuy < il * il) {
            const int mx = mxp < 0 ? mxp + k.nx : mxp, my = myp < 0 ? myp + k.ny : myp;
            const float2 gv = gspec[((int64_t)c * k.ny + my) * k.nx + mx];
            v = make_float2(hypotf(gv.x, gv.y), atan2f(gv.y, gv.x) * 0.15915494309189535f);
        }
    }
    gpack[idx] = v;
}

hipError_t launch_adj_pack(const Consts &k, const AdjGeom &geo, int n_scenes, const float2 *gspecs, float2 *gpack,
                           float *dpack, double *d0, hipStream_t s)
{
    const int64_t per_scene = (int64_t)geo.nreg * ADJ_NB * k.C * 64;
    const unsigned blocks = (unsigned)((per_scene + 255) / 256);
    hipLaunchKernelGGL(k_adj_pack_d, dim3(blocks), dim3(256), 0, s, k, geo, dpack, d0);
    const int64_t M = (int64_t)k.nx * k.ny * k.C;
    for (int i = 0; i < n_scenes; ++i)
        hipLaunchKernelGGL(k_adj_pack_g, dim3(blocks), dim3(256), 0, s, k, geo, gspecs + (int64_t)i * M,
                           gpack + (int64_t)i * per_scene);
    return hipGetLastError();
}

// Reduce NV per-lane values over the wavefront and add the totals to acc[0..NV) (LDS).
// Up to 8 values (+ 1 carried along), 16, or 24 (16 + 8) use the transposed butterfly.
template <int NV>
static __device__ __forceinline__ void reduce_into(float (&x)[NV], float *acc, int lane)
{
    if constexpr (NV <= 9) {
        float v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = i < NV ? x[i] : 0.0f;
        float y = NV == 9 ? x[NV - 1] : 0.0f;
        if constexpr (NV == 9) {
            reduce_transposed<8, true>(v, y, lane);
            if (lane == 4) atomicAdd(&acc[8], y);
        } else {
            reduce_transposed<8, false>(v, y, lane);
        }
        if ((lane & 7) == 0) {
            const int v0 = ((lane >> 5) & 1) * 4 + ((lane >> 4) & 1) * 2 + ((lane >> 3) & 1);
            if (v0 < NV && (NV != 9 || v0 < 8)) atomicAdd(&acc[v0], v[0]);  // ds_add_f32, no return
        }
    } else if constexpr (NV <= 16) {
        float v[16];
        float y = 0.0f;
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = i < NV ? x[i] : 0.0f;
        reduce_transposed<16, false>(v, y, lane);
        if ((lane & 7) == 0) {
            const int v0 = 2 * (((lane >> 5) & 1) * 4 + ((lane >> 4) & 1) * 2 + ((lane >> 3) & 1));
#pragma unroll
            for (int j = 0; j < 2; ++j)
                if (v0 + j < NV) atomicAdd(&acc[v0 + j], v[j]);
        }
    } else {
        static_assert(NV <= 24, "at most 24 reduced values");
        float v[16], w[8];
        float y = 0.0f;
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = x[i];
#pragma unroll
        for (int i = 0; i < 8; ++i) w[i] = 16 + i < NV ? x[16 + i] : 0.0f;
        reduce_transposed<16, false>(v, y, lane);
        reduce_transposed<8, false>(w, y, lane);
        if ((lane & 7) == 0) {
            const int g = ((lane >> 5) & 1) * 4 + ((lane >> 4) & 1) * 2 + ((lane >> 3) & 1);
#pragma unroll
            for (int j = 0; j < 2; ++j) atomicAdd(&acc[2 * g + j], v[j]);
            if (16 + g < NV) atomicAdd(&acc[16 + g], w[0]);
        }
    }
}

// A Gaussian accepted for the current region: its index in the item, its 4-row block mask and
// the phase bases of the region's two sub-tiles.
template <int C>
struct alignas(16) AdjEntry {
    int32_t g;
    uint32_t rows;
    float base[2 * C];
};

// Loads through the constant address space are scalar when the address is uniform.
#define CONST_AS __attribute__((address_space(4)))

template <int C, bool DEPTH>
__global__ void __launch_bounds__(adj_wg(C, DEPTH), adj_waves_per_simd(C, DEPTH))
    k_adjoint(Consts k, const int32_t *__restrict__ tile_xy, const BwdScene *__restrict__ scenes,
              const int32_t *__restrict__ prefix, int n_scenes, long long *__restrict__ queue,
              const float *__restrict__ dpack, const double *__restrict__ d0tab, AdjGeom geo)
{
    constexpr int NV = adj_nv(C, DEPTH);
    constexpr int ADJ_WG = adj_wg(C, DEPTH);
    constexpr int RE = ADJ_NB * C * 64;  // packed elements per region
    __shared__ __attribute__((aligned(16))) float2 s_g[RE];  // [b][c][lane] (|Gs|, arg Gs / 2 pi)
    __shared__ __attribute__((aligned(16))) float s_d[RE];   // [b][c][lane] D_c(nu) - D_c(nu_0)
    __shared__ float s_acc[ADJ_WG * NV]; // [Gaussian of the item][value]
    __shared__ AdjEntry<C> s_ent[ADJ_WG];  // accepted Gaussians of the current region
    __shared__ int s_cnt[2], s_next[2];    // list length and visit counter, by region parity
    __shared__ int s_item, s_scene;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int total_items = prefix[n_scenes];
    const int hx = k.nx / 2, hy = k.ny / 2;
    const float lim = (float)(k.tau2 * (1.0 + 1e-5)) + 1e-4f;
    // every support is an ellipse centred at m_r (DC unless a reference plane wave tilts the
    // illumination): support tests, envelope and the frequency weights of the sums are taken
    // relative to it (the weights are those of nu - nu_r, the argument of the Gaussian's spectrum)
    const float mrxf = (float)k.mrx, mryf = (float)k.mry;
    const int col = lane & (ADJ_RW - 1), row4 = lane >> 4;
    const float dxf = (float)(col - ADJ_RW / 2);   // column offset from the sub-tile centre
    const float dyr = (float)(row4 - ADJ_SH / 2);  // row offset from the sub-tile centre at block 0
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;

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
        // wave-uniform from here on: scalar loads and scalar control flow
        const int q = __builtin_amdgcn_readfirstlane(s_item), sc = __builtin_amdgcn_readfirstlane(s_scene);
        if (q >= total_items) break;
        const BwdScene S = scenes[sc];
        const GRec *__restrict__ rec = S.rec;
        const float2 *__restrict__ gpack = S.gpack;
        const int64_t nvalid = S.n - S.counters[CTR_NCULLED];
        const BItem bi = S.bitems[q - prefix[sc]];
        const int64_t g0 = (int64_t)bi.chunk * ADJ_WG;
        const int64_t gidx = g0 + tid;
        const bool gvalid = gidx < nvalid;
        long long pairs = 0;
        for (int i = tid; i < ADJ_WG * NV; i += ADJ_WG) s_acc[i] = 0.0f;
        if (tid < 2) s_cnt[tid] = s_next[tid] = 0;
        int par = 0;  // parity of the region being processed

        for (int kt = bi.k0; kt < bi.k1; ++kt) {
            const int32_t txy = tile_xy[kt];
            const int tx = (int)(int16_t)(txy & 0xffff), ty = txy >> 16;
            for (int h = 0; h < 2; ++h) {
                const int x0 = tx * TILEX + h * ADJ_RW, y0 = ty * ADJ_RH;
                const float X0 = (float)max(x0, -hx), X1 = (float)min(x0 + ADJ_RW - 1, hx - 1);
                const float Y0 = (float)max(y0, -hy), Y1 = (float)min(y0 + ADJ_RH - 1, hy - 1);
                if (X0 > X1 || Y0 > Y1) continue;  // uniform over the work-group
                const int r = ((ty - geo.ty_min) * geo.ntx + (tx - geo.tx_min)) * 2 + h;
                __syncthreads();  // the previous region's data is no longer read
                {
                    const float4 *sg = reinterpret_cast<const float4 *>(gpack + (int64_t)r * RE);
                    float4 *dg = reinterpret_cast<float4 *>(s_g);
                    for (int i = tid; i < RE / 2; i += ADJ_WG) dg[i] = sg[i];
                    const float4 *sd = reinterpret_cast<const float4 *>(dpack + (int64_t)r * RE);
                    float4 *dd = reinterpret_cast<float4 *>(s_d);
                    for (int i = tid; i < RE / 4; i += ADJ_WG) dd[i] = sd[i];
                }
                // this thread's own Gaussian against the region: accept, row blocks, phase bases,
                // appended to the region's list (a wavefront's entries are contiguous; the list
                // order does not affect any result: each Gaussian is visited once per region)
                bool p = false;
                uint32_t rows = 0;
                float b0[C], b1[C];
#pragma unroll
                for (int c = 0; c < C; ++c) b0[c] = b1[c] = 0.0f;
                if (gvalid) {
                    const float4 *src = reinterpret_cast<const float4 *>(rec + gidx);
                    const float4 r0 = src[0];
                    p = ellipse_meets_rect_r(r0.x, r0.y, r0.z, 0.5f / r0.x, 0.5f / r0.z, lim, X0 - mrxf, X1 - mrxf,
                                             Y0 - mryf, Y1 - mryf);
                    if (p) {
                        rows = row_block_mask<ADJ_NB>(r0.x, r0.y, r0.z, lim, X0 - mrxf, X1 - mrxf, y0, hy, mryf);
                        pairs += (long long)__popc(rows) * 64;
                        const float4 r1 = src[1], r2 = src[2];
                        const uint32_t rx = __float_as_uint(r1.x), ry = __float_as_uint(r1.y);
                        const float kap[4] = {r2.x, r2.y, r2.z, r2.w};
                        const int cx = x0 + ADJ_RW / 2;
#pragma unroll
                        for (int s = 0; s < 2; ++s) {
                            const int cy = y0 + s * ADJ_SH + ADJ_SH / 2;
                            const double *D0 = d0tab + ((int64_t)r * 2 + s) * C;
                            float bs[C];
                            if (k.phase_mode == 1) {
                                // plain FP32 phase (precision study only)
                                const float rr = (float)cx * r1.z + (float)cy * r1.w;
#pragma unroll
                                for (int c = 0; c < C; ++c) {
                                    const float v = kap[c] - rr - r0.w * (float)D0[c];
                                    bs[c] = v - floorf(v);
                                }
                            } else {
                                // exact ramp at the sub-tile centre: 0.32 fixed point, wraps mod 1
                                const uint32_t ramp = (uint32_t)cx * rx + (uint32_t)cy * ry;
                                const double ramp_rev = (double)ramp * (1.0 / 4294967296.0);
#pragma unroll
                                for (int c = 0; c < C; ++c)
                                    bs[c] = (float)frac_d((double)kap[c] - ramp_rev - (double)r0.w * D0[c]);
                            }
#pragma unroll
                            for (int c = 0; c < C; ++c) {
                                if (s == 0) b0[c] = bs[c];
                                else b1[c] = bs[c];
                            }
                        }
                    }
                }
                {
                    const uint64_t bal = __ballot(p);
                    int slot = 0;
                    if (lane == 0 && bal) slot = atomicAdd(&s_cnt[par], __popcll(bal));
                    slot = __builtin_amdgcn_readlane(slot, 0) + __popcll(bal & lt);
                    if (p) {
                        AdjEntry<C> e;
                        e.g = tid;
                        e.rows = rows;
#pragma unroll
                        for (int c = 0; c < C; ++c) {
                            e.base[c] = b0[c];
                            e.base[C + c] = b1[c];
                        }
                        s_ent[slot] = e;
                    }
                }
                __syncthreads();  // region data and the list in LDS
                if (tid == 0) s_cnt[par ^ 1] = s_next[par ^ 1] = 0;  // for the next region
                const int cnt = __builtin_amdgcn_readfirstlane(s_cnt[par]);
                // per-lane frequency of this region: column x0 + col, rows y0 + row4 + 4 b
                const float fmx = (float)((double)(x0 + col) - k.mrx), mxx = fmx * fmx;
                const float fmy0 = (float)((double)(y0 + row4) - k.mry);
                for (;;) {
                    // the next accepted Gaussian of the region, taken by whichever wavefront is free
                    int ei = 0;
                    if (lane == 0) ei = atomicAdd(&s_next[par], 1);
                    ei = __builtin_amdgcn_readlane(ei, 0);
                    if (ei >= cnt) break;
                    const AdjEntry<C> &en = s_ent[ei];
                    const int o = __builtin_amdgcn_readfirstlane(en.g);
                    const uint32_t vrows = __builtin_amdgcn_readfirstlane(en.rows);
                    // the Gaussian's record: uniform address, constant memory (written by an earlier
                    // kernel), so scalar loads
                    const uint64_t ra = (uint64_t)(rec + g0 + o);
                    const uint64_t rau = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(ra >> 32)) << 32) |
                                         (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)ra);
                    const CONST_AS float *rp = (const CONST_AS float *)rau;
                    const float alpha = rp[0], beta2 = rp[1], gamma = rp[2], z = rp[3], rxf = rp[6], ryf = rp[7];
                    const float ampv[4] = {rp[12], rp[13], rp[14], rp[15]};
                    float bs0[C], bs1[C], amp[C];
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        bs0[c] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(en.base[c])));
                        bs1[c] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(en.base[C + c])));
                        amp[c] = ampv[c];
                    }
                    // the lane's row at block 0, opaque to the optimiser so that the sixteen rows are
                    // formed in the block loop rather than held in registers across visits
                    float fmy0v = fmy0;
                    asm volatile("" : "+v"(fmy0v));
                    // exponent q = alpha m_x'^2 + m_y' (beta2 m_x' + gamma m_y'), evaluated at each row
                    // (a quadratic in the block index about a reference row loses accuracy when the
                    // reference lies far outside a narrow support)
                    const float bmx = beta2 * fmx, ax = alpha * mxx;
                    // phase base of the lane's column and first row in the current sub-tile (formed only
                    // for a sub-tile the support reaches; vrows is wave-uniform)
                    float bxr[C];
#pragma unroll
                    for (int c = 0; c < C; ++c) bxr[c] = 0.0f;
                    if (vrows & 0xffu) {
#pragma unroll
                        for (int c = 0; c < C; ++c)
                            bxr[c] = fmaf(-dyr, ryf, __builtin_amdgcn_fractf(fmaf(-dxf, rxf, bs0[c])));
                    }
                    float Pr[C], Pi[C], Wc[C], Pi0[C];
#pragma unroll
                    for (int c = 0; c < C; ++c) Pr[c] = Pi[c] = Wc[c] = Pi0[c] = 0.0f;
                    // R1 = sum m_y' Re rho, R2 = sum m_y'^2 Re rho, I0 = sum Im rho, I1 = sum m_y' Im rho
                    // over this lane's rows, with the exact row index as weight (sum Re rho comes
                    // from the P_c)
                    float R1 = 0.0f, R2 = 0.0f, I0 = 0.0f, I1 = 0.0f;
#pragma unroll
                    for (int b = 0; b < ADJ_NB; ++b) {
                        if (b == ADJ_NB / 2) {
                            // second sub-tile: its own phase base (and D0 for the depth sums)
#pragma unroll
                            for (int c = 0; c < C; ++c)
                                if (DEPTH) Pi0[c] = Pi[c];
                            if (vrows >> (ADJ_NB / 2)) {
#pragma unroll
                                for (int c = 0; c < C; ++c)
                                    bxr[c] = fmaf(-dyr, ryf, __builtin_amdgcn_fractf(fmaf(-dxf, rxf, bs1[c])));
                            }
                        }
                        if (!(vrows & (1u << b))) continue;  // the support misses this 4-row block
                        const float my = fmy0v + (float)(4 * b);
                        const float qq = fmaf(my, fmaf(gamma, my, bmx), ax);
                        const float E = __builtin_amdgcn_exp2f(-qq);
                        const float dyb = (float)(4 * (b & 7));
                        float rr = 0.0f, ri = 0.0f;
#pragma unroll
                        for (int c = 0; c < C; ++c) {
                            const float2 gv = s_g[(b * C + c) * 64 + lane];
                            const float dD = s_d[(b * C + c) * 64 + lane];
                            const float tb = (b & 7) ? fmaf(-dyb, ryf, bxr[c]) : bxr[c];
                            // E conj(Gs) e^{j 2 pi th} = E |Gs| e^{j 2 pi (th - arg Gs / 2 pi)}
                            const float th = fmaf(-z, dD, tb - gv.y);
                            const float sn = __builtin_amdgcn_sinf(th);
                            const float cs = __builtin_amdgcn_cosf(th);
                            const float eg = E * gv.x;
                            Pr[c] = fmaf(eg, cs, Pr[c]);
                            if (DEPTH) {
                                Pi[c] = fmaf(eg, sn, Pi[c]);
                                Wc[c] = fmaf(dD * eg, sn, Wc[c]);
                            }
                            const float ae = amp[c] * eg;
                            rr = fmaf(ae, cs, rr);
                            ri = fmaf(ae, sn, ri);
                        }
                        R1 = fmaf(my, rr, R1);
                        R2 = fmaf(my * my, rr, R2);
                        I0 += ri;
                        I1 = fmaf(my, ri, I1);
                    }
                    float R0 = 0.0f;
#pragma unroll
                    for (int c = 0; c < C; ++c) R0 = fmaf(amp[c], Pr[c], R0);
                    // value layout: Re P_c (C), Sfx, Sfy, Qxx, Qxy, Qyy, then with depth Im P_c (C),
                    // W_c (C), else sum Im rho (the phase gradient)
                    float x[NV];
#pragma unroll
                    for (int c = 0; c < C; ++c) x[c] = Pr[c];
                    x[C + 0] = fmx * I0;
                    x[C + 1] = I1;
                    x[C + 2] = mxx * R0;
                    x[C + 3] = fmx * R1;
                    x[C + 4] = R2;
                    if constexpr (DEPTH) {
                        const double *D0 = d0tab + (int64_t)r * 2 * C;
#pragma unroll
                        for (int c = 0; c < C; ++c) {
                            x[C + 5 + c] = Pi[c];
                            // W_c = sum (dD + D0 of the element's sub-tile) Im g_c
                            x[2 * C + 5 + c] = fmaf((float)D0[C + c], Pi[c] - Pi0[c], fmaf((float)D0[c], Pi0[c], Wc[c]));
                        }
                    } else {
                        x[C + 5] = I0;
                    }
                    reduce_into<NV>(x, s_acc + o * NV, lane);
                }
                par ^= 1;
            }
        }
        __syncthreads();
        float *dst = S.bpartials + (int64_t)bi.slot * ADJ_WG * NV;
        for (int i = tid; i < ADJ_WG * NV; i += ADJ_WG) dst[i] = s_acc[i];
        pairs = wave_sum_i64(pairs);
        if (lane == 0 && pairs) atomicAdd((unsigned long long *)&S.counters[CTR_PAIRS], (unsigned long long)pairs);
    }
}

template <int C, bool DEPTH>
static const void *adj_kernel_ptr() { return (const void *)k_adjoint<C, DEPTH>; }

hipError_t launch_adjoint(const Plan &p, const Consts &k, const BwdScene *scenes, const int32_t *prefix, int n_scenes,
                          long long *queue, const float *dpack, const double *d0, const AdjGeom &geo, int grid,
                          hipStream_t s)
{
#define GWS_ADJ_LAUNCH(CC, DD)                                                                                   \
    hipLaunchKernelGGL((k_adjoint<CC, DD>), dim3(grid), dim3(adj_wg(CC, DD)), 0, s, k, p.tile_xy, scenes, prefix,  \
                       n_scenes, \
                       queue, dpack, d0, geo)
    const bool d = k.depth_grad != 0;
    switch (k.C) {
    case 1: if (d) GWS_ADJ_LAUNCH(1, true); else GWS_ADJ_LAUNCH(1, false); break;
    case 2: if (d) GWS_ADJ_LAUNCH(2, true); else GWS_ADJ_LAUNCH(2, false); break;
    case 3: if (d) GWS_ADJ_LAUNCH(3, true); else GWS_ADJ_LAUNCH(3, false); break;
    case 4: if (d) GWS_ADJ_LAUNCH(4, true); else GWS_ADJ_LAUNCH(4, false); break;
    default: return hipErrorInvalidValue;
    }
#undef GWS_ADJ_LAUNCH
    return hipGetLastError();
}

int adjoint_occupancy(int C, int depth)
{
    const void *kp = nullptr;
    switch (C) {
    case 1: kp = depth ? adj_kernel_ptr<1, true>() : adj_kernel_ptr<1, false>(); break;
    case 2: kp = depth ? adj_kernel_ptr<2, true>() : adj_kernel_ptr<2, false>(); break;
    case 3: kp = depth ? adj_kernel_ptr<3, true>() : adj_kernel_ptr<3, false>(); break;
    default: kp = depth ? adj_kernel_ptr<4, true>() : adj_kernel_ptr<4, false>(); break;
    }
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kp, adj_wg(C, depth != 0), 0) != hipSuccess || nb < 1) nb = 1;
    return nb;
}

// Per Gaussian: sum the item partials of its chunk in order (FP64), then the chain rule.  The
// number of sums is a compile-time constant of the variant, so they stay in registers.
template <int C, bool DEPTH>
__global__ void __launch_bounds__(256) k_grad_final(GView g, Consts k, const uint32_t *__restrict__ vals,
                                                    const int2 *__restrict__ chunk_items,
                                                    const int32_t *__restrict__ range_base,
                                                    const float *__restrict__ bpartials, GradView grads, int64_t n,
                                                    const long long *__restrict__ counters, int chunk)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int64_t nvalid = n - counters[CTR_NCULLED];
    const int64_t i = vals[s];
    if (s >= nvalid) {
        grads.mean_x[i] = grads.mean_y[i] = 0.0f;
        if (grads.depth) grads.depth[i] = 0.0f;
        grads.cov_xx[i] = grads.cov_xy[i] = grads.cov_yy[i] = 0.0f;
        grads.opacity[i] = grads.phase[i] = 0.0f;
#pragma unroll
        for (int c = 0; c < C; ++c) grads.amplitude[(int64_t)c * grads.amp_stride + i] = 0.0f;
        return;
    }
    constexpr int NV = adj_nv(C, DEPTH);
    const int64_t b = s / chunk;
    const int t = (int)(s - b * chunk);
    const int2 ci = chunk_items[b];
    const long long nbitems = counters[CTR_NBITEMS];
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
    for (int j = 0; j < ci.y; ++j) {
        const int64_t it = (int64_t)range_base[j] + b;  // range j of chunk b
        if (it >= nbitems) break;
        const float *src = bpartials + (it * chunk + t) * NV;
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] += (double)src[v];
    }
    const double PI = 3.14159265358979323846;
    const double sxx = g.cov_xx[i], sxy = g.cov_xy[i], syy = g.cov_yy[i];
    const double det = sxx * syy - sxy * sxy;
    const double o = g.opacity[i];
    const double fx = 1.0 / (k.nx * k.px), fy = 1.0 / (k.ny * k.py);
    const double K = 2.0 * PI * sqrt(det) / (k.px * k.py * (double)k.nx * (double)k.ny);
    double Sre = 0.0, gz = 0.0, go = 0.0, Sim = 0.0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const double a = g.amplitude[(int64_t)c * g.amp_stride + i];
        const double A = a * o * K;
        const double Pr = acc[c];
        Sre += A * Pr;
        if constexpr (DEPTH) {
            const double Pi = acc[C + 5 + c], Wc = acc[2 * C + 5 + c];
            gz += A * (k.inv_lambda[c] * Pi + Wc);
            Sim += A * Pi;
        }
        go += a * K * Pr;
        grads.amplitude[(int64_t)c * grads.amp_stride + i] = (float)(o * K * Pr);
    }
    // sum_c A_c Im P_c (= sum_m Im rho): from Im P_c with depth, else the extra reduced value
    if constexpr (!DEPTH) Sim = acc[C + 5];
    const double Sfx = acc[C], Sfy = acc[C + 1], Qxx = acc[C + 2], Qxy = acc[C + 3], Qyy = acc[C + 4];
    grads.phase[i] = (float)(-Sim);
    grads.mean_x[i] = (float)(2.0 * PI * fx * Sfx);
    grads.mean_y[i] = (float)(2.0 * PI * fy * Sfy);
    grads.opacity[i] = (float)go;
    grads.cov_xx[i] = (float)(syy / (2.0 * det) * Sre - 2.0 * PI * PI * fx * fx * Qxx);
    grads.cov_yy[i] = (float)(sxx / (2.0 * det) * Sre - 2.0 * PI * PI * fy * fy * Qyy);
    grads.cov_xy[i] = (float)(-sxy / det * Sre - 4.0 * PI * PI * fx * fy * Qxy);
    if (DEPTH && grads.depth) grads.depth[i] = (float)(2.0 * PI * gz);
}

hipError_t launch_grad_final(const GView &g, const Consts &k, const uint32_t *vals, const int2 *chunk_items,
                             const int32_t *range_base, const float *bpartials, const GradView &grads, int64_t n,
                             const long long *counters, int chunk, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
#define GWS_GF(CC, DD)                                                                                                  \
    hipLaunchKernelGGL((k_grad_final<CC, DD>), grid, block, 0, s, g, k, vals, chunk_items, range_base, bpartials, grads, \
                       n, counters, chunk)
    const bool d = k.depth_grad != 0;
    switch (k.C) {
    case 1: if (d) GWS_GF(1, true); else GWS_GF(1, false); break;
    case 2: if (d) GWS_GF(2, true); else GWS_GF(2, false); break;
    case 3: if (d) GWS_GF(3, true); else GWS_GF(3, false); break;
    case 4: if (d) GWS_GF(4, true); else GWS_GF(4, false); break;
    default: return hipErrorInvalidValue;
    }
#undef GWS_GF
    return hipGetLastError();
}

}  // namespace gws
