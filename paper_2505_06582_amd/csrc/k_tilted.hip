// Tilted 2D Gaussians (Sec. 4.1, Eq. 8-10; the supplement's translation, rotation and scaling
// steps) summed order-invariantly (Sec. 4.2, Eq. 12) on gfx950.
//
// A tilted Gaussian is the canonical Gaussian of the plane z_c = 0 placed by x = R S x_c + mu,
// S = diag(s_u, s_v, 0), R from a unit quaternion.  On the plane through its centre parallel
// to the SLM its spectrum is |det J| G_o(k_ox, k_oy) with k_o = R^T k, k = (nu_x, nu_y, k_z),
// k_z = sqrt(1/lambda^2 - |nu|^2), det J = k_oz / k_z (the magnitude: the disk radiates to
// both sides, and R, R diag(1,-1,-1) describe the same disk), G_o the scaled canonical
// spectrum 2 pi s_u s_v exp(-2 pi^2 (s_u^2 k_ox^2 + s_v^2 k_oy^2)).  The ramp, the carrier and
// the propagation H(nu, -z) are those of an in-plane Gaussian, so the term of Gaussian i at
// wavelength c and frequency m (index units) is
//   A_c |w_c(m)| / k_z,c(m) exp2(-(u_c(m)^2 + v_c(m)^2)) exp(j 2 pi Theta_c(m))
//     = (A_c lambda_c) |w_c(m)| exp2(log2(1 / (k_z,c lambda_c)) - u_c^2 - v_c^2) exp(j 2 pi Theta_c),
//   u_c = U . (m_x, m_y, k_z,c),  v_c = V . (...),  w_c = N . (...)  (= k_oz, 1/m),
// with U = sqrt(2 pi^2 log2 e) s_u (R11 / W, R21 / H, R31), V likewise from column 2 and s_v,
// N = (R13 / W, R23 / H, R33), W = nx px, H = ny py, and Theta_c as in the in-plane kernel.
// Unlike an in-plane Gaussian, the exponent depends on the wavelength (through k_z), so there
// is one exp2 per (Gaussian, frequency, wavelength).
//
// Precision: u, v, w are large sums of nearly cancelling terms (R31 k_z alone reaches
// ~1e2 in exp2 units at a few degrees of tilt), so as the phase they are split into an FP64
// base at the centre of each 16 x 16 sub-tile in the forward (of each 32 x 32 tile in the
// adjoint), formed per Gaussian by one lane, and FP32 deltas per lane:
// u = u0 + U_x dx + U_y dy + U_z (D_c(m) - D_c(m0)), D_c = k_z,c - 1/lambda_c.
//
// Work.  The support of a tilted Gaussian sits near n_xy / lambda_c (n = R e_z, the disk's
// normal), one off-centre patch per wavelength, so the in-plane path's DC-centred binning does
// not apply.  Each Gaussian gets a conservative rectangle of 32 x 32 tiles (the union over
// wavelengths and both sides of the disk of the bounding box of its eps-support on the sphere
// |k| = 1/lambda).  A persistent work-group takes tiles from a queue in rings around DC, scans
// every Gaussian's rectangle in input order (8 bytes each, L2-resident), stages the ones that
// reach the tile, and each wavefront tests them against its 16 x 16 sub-tile and 4-row blocks
// (bounds of u and v over the block), forms the FP64 bases and evaluates.  Every frequency of
// the grid belongs to one tile; from 16384 Gaussians a tile's Gaussians are split into parts
// (one work item each, so the crowded tiles do not hold the launch's tail) whose partial
// spectra are added in part order.  The order of every sum is fixed: results are bitwise
// reproducible.
#include "gws_internal.h"

namespace gws {

constexpr int TT = 32;          // tile side (frequencies)
constexpr int TF = 4;           // 4-row blocks per sub-tile (16 rows)
constexpr int TWG = 256;        // threads per work-group (4 wavefronts, one 16 x 16 sub-tile each)
// A tile's Gaussians are split into up to this many parts (one work item each; one per 8192
// Gaussians) so that the tiles every support crowds do not hold a launch's tail.
constexpr int TILT_PARTS_MAX = 8;

static __device__ __forceinline__ bool finite_t(float v) { return (__float_as_uint(v) & 0x7f800000u) != 0x7f800000u; }
static __device__ __forceinline__ double frac_t(double v) { return v - floor(v); }
static __device__ __forceinline__ int floor_div_t(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// D_c(nu) = k_z - 1/lambda (negative, no cancellation); -1/lambda (k_z = 0) when evanescent.
static __device__ __forceinline__ double dprop_t(double nu2, double il)
{
    const double w2 = il * il - nu2;
    return w2 > 0.0 ? -nu2 / (il + sqrt(w2)) : -il;
}

__global__ void k_tilt_zero(long long *__restrict__ counters)
{
    if (threadIdx.x < CTR_COUNT) counters[threadIdx.x] = 0;
}

__global__ void k_tilt_zero64(int64_t *__restrict__ p, int n)
{
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

// One thread per Gaussian (input order): validity, record, tile rectangle.
__global__ void __launch_bounds__(256) k_tilt_records(TView g, Consts k, TRec *__restrict__ rec,
                                                       int2 *__restrict__ rect, long long *__restrict__ counters)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.n) return;
    const float mx = g.mean_x[i], my = g.mean_y[i], z = g.depth[i], o = g.opacity[i], ph = g.phase[i];
    const float qw = g.quat_w[i], qx = g.quat_x[i], qy = g.quat_y[i], qz = g.quat_z[i];
    const float su = g.scale_u[i], sv = g.scale_v[i];
    bool ok = finite_t(mx) && finite_t(my) && finite_t(z) && finite_t(o) && finite_t(ph) && finite_t(qw) &&
              finite_t(qx) && finite_t(qy) && finite_t(qz) && finite_t(su) && finite_t(sv) && su > 0.0f && sv > 0.0f;
    bool any_amp = false;
    for (int c = 0; c < k.C; ++c) {
        const float a = g.amplitude[(int64_t)c * g.n + i];
        ok = ok && finite_t(a);
        any_amp = any_amp || (a != 0.0f);
    }
    const double qn = (double)qw * qw + (double)qx * qx + (double)qy * qy + (double)qz * qz;
    // the forward also skips Gaussians that add nothing; the adjoint keeps them (their opacity and
    // amplitude gradients are not zero)
    ok = ok && qn > 0.0 && (!k.forward || (o != 0.0f && any_amp));
    TRec r = {};
    int2 box = make_int2(1, 0);  // empty: tx0 > tx1
    if (ok) {
        // rotation of the normalised quaternion
        const double s = 1.0 / sqrt(qn);
        const double w = qw * s, x = qx * s, y = qy * s, zq = qz * s;
        const double R[3][3] = {{1 - 2 * (y * y + zq * zq), 2 * (x * y - w * zq), 2 * (x * zq + w * y)},
                                {2 * (x * y + w * zq), 1 - 2 * (x * x + zq * zq), 2 * (y * zq - w * x)},
                                {2 * (x * zq - w * y), 2 * (y * zq + w * x), 1 - 2 * (x * x + y * y)}};
        const double Wx = k.nx * k.px, Wy = k.ny * k.py;
        const double sk = sqrt(k.K2);
        const double su_d = su, sv_d = sv;
        r.U[0] = (float)(sk * su_d * R[0][0] / Wx);
        r.U[1] = (float)(sk * su_d * R[1][0] / Wy);
        r.U[2] = (float)(sk * su_d * R[2][0]);
        r.V[0] = (float)(sk * sv_d * R[0][1] / Wx);
        r.V[1] = (float)(sk * sv_d * R[1][1] / Wy);
        r.V[2] = (float)(sk * sv_d * R[2][1]);
        r.N[0] = (float)(R[0][2] / Wx);
        r.N[1] = (float)(R[1][2] / Wy);
        r.N[2] = (float)R[2][2];
        r.z = z;
        const double fx = frac_t((double)mx / Wx + 0.5), fy = frac_t((double)my / Wy + 0.5);
        r.rx = (uint32_t)(uint64_t)llrint(fx * 4294967296.0);
        r.ry = (uint32_t)(uint64_t)llrint(fy * 4294967296.0);
        r.rxf = (float)((double)(int32_t)r.rx * (1.0 / 4294967296.0));
        r.ryf = (float)((double)(int32_t)r.ry * (1.0 / 4294967296.0));
        const double norm = 6.283185307179586 * su_d * sv_d / (k.px * k.py * (double)k.nx * (double)k.ny);
        const double phi_rev = frac_t((double)ph * 0.15915494309189535);
        for (int c = 0; c < 4; ++c) {
            r.kappa[c] = c < k.C ? (float)frac_t(phi_rev - (double)z * k.inv_lambda[c]) : 0.0f;
            r.amp[c] = c < k.C ? (float)((double)g.amplitude[(int64_t)c * g.n + i] * (double)o * norm * k.lambda[c])
                               : 0.0f;
        }
        // Bounding box of the eps-support u^2 + v^2 <= tau2: in the disk frame an ellipse of
        // semi-axes A = sqrt(tau2 / K2) / s_u, B = .../ s_v in (k_ox, k_oy); on the sphere
        // k_o = (a, b, +-w), w in [w_min, 1/lambda].  nu = R k_o, so each transverse component
        // is bounded by the ellipse's support function plus the range of R_j3 (+-w); a side
        // whose waves cannot reach k_z > 0 is skipped.  Union over wavelengths and sides,
        // clipped to the propagating disk and the grid.
        const double t = sqrt(k.tau2 / k.K2);
        const double A = t / su_d, B = t / sv_d, rho2 = fmax(A, B) * fmax(A, B);
        const double hxx = t * sqrt(R[0][0] * R[0][0] / (su_d * su_d) + R[0][1] * R[0][1] / (sv_d * sv_d));
        const double hyy = t * sqrt(R[1][0] * R[1][0] / (su_d * su_d) + R[1][1] * R[1][1] / (sv_d * sv_d));
        const double gz = t * sqrt(R[2][0] * R[2][0] / (su_d * su_d) + R[2][1] * R[2][1] / (sv_d * sv_d));
        double lox = 1e300, hix = -1e300, loy = 1e300, hiy = -1e300;
        for (int c = 0; c < k.C; ++c) {
            const double il = k.inv_lambda[c];
            const double wmin = sqrt(fmax(0.0, il * il - rho2));
            for (int sd = -1; sd <= 1; sd += 2) {
                const double z0 = sd * R[2][2] * wmin, z1 = sd * R[2][2] * il;
                if (fmax(z0, z1) + gz <= 0.0) continue;  // no wave of this side heads for the SLM
                const double x0 = sd * R[0][2] * wmin, x1 = sd * R[0][2] * il;
                const double y0 = sd * R[1][2] * wmin, y1 = sd * R[1][2] * il;
                lox = fmin(lox, fmax(fmin(x0, x1) - hxx, -il));
                hix = fmax(hix, fmin(fmax(x0, x1) + hxx, il));
                loy = fmin(loy, fmax(fmin(y0, y1) - hyy, -il));
                hiy = fmax(hiy, fmin(fmax(y0, y1) + hyy, il));
            }
        }
        if (lox <= hix && loy <= hiy) {
            const int hx = k.nx / 2, hy = k.ny / 2;
            const int mx0 = (int)fmax(floor(lox * Wx) - 1.0, (double)-hx), mx1 = (int)fmin(ceil(hix * Wx) + 1.0, (double)(hx - 1));
            const int my0 = (int)fmax(floor(loy * Wy) - 1.0, (double)-hy), my1 = (int)fmin(ceil(hiy * Wy) + 1.0, (double)(hy - 1));
            if (mx0 <= mx1 && my0 <= my1) {
                const int tx0 = floor_div_t(mx0, TT), tx1 = floor_div_t(mx1, TT);
                const int ty0 = floor_div_t(my0, TT), ty1 = floor_div_t(my1, TT);
                box = make_int2((int)(((uint32_t)tx0 & 0xffffu) | ((uint32_t)tx1 << 16)),
                                (int)(((uint32_t)ty0 & 0xffffu) | ((uint32_t)ty1 << 16)));
            }
        }
    } else {
        atomicAdd((unsigned long long *)&counters[CTR_NCULLED], 1ull);
    }
    rec[i] = r;
    rect[i] = box;
}

// Tile of queue index q: rings of tiles around DC (ring r is the square [-r-1, r]^2 minus
// [-r, r-1]^2), each walked along its top, right, bottom and left edges.
static __device__ __forceinline__ void ring_tile(int q, int *tx, int *ty)
{
    int r = (int)(sqrtf((float)q) * 0.5f);
    while (4 * (r + 1) * (r + 1) <= q) ++r;
    while (4 * r * r > q) --r;
    int p = q - 4 * r * r;
    const int side = 2 * r + 2;
    if (p < side) { *tx = -r - 1 + p; *ty = -r - 1; return; }
    p -= side;
    if (p < side - 1) { *tx = r; *ty = -r + p; return; }
    p -= side - 1;
    if (p < side - 1) { *tx = r - 1 - p; *ty = r; return; }
    p -= side - 1;
    *tx = -r - 1;
    *ty = r - 1 - p;
}

// The terms of one staged Gaussian at a lane's frequencies (bit c * 4 + f of `rows`: wavelength c
// reaches 4-row block f).  Phase
// delta z (D_c(m) - D_c(m0)) in revolutions: one FP32 product while it stays below 16
// revolutions (error <= 16 x 2^-24); WIDE (sub-tiles where D_c changes fast, towards the
// evanescent edge or at fine pitch): z times the double-float delta, its integer part removed
// inside one fused product so that the fraction keeps full precision.
template <int C, bool WIDE>
static __device__ __forceinline__ void tilt_eval(uint32_t rows, float U1, float U2, float V1, float V2, float N1,
                                                 float N2, float z, float ryf, const float (&u0)[C],
                                                 const float (&v0)[C], const float (&w0)[C], const float (&bx)[C],
                                                 const float (&amp)[C], const float (&dyf)[TF],
                                                 const float (&dD)[TF][C], const float (&dlo)[TF][C][64], int lane,
                                                 const float (&lkz)[TF][C], float (&acc_re)[TF][C],
                                                 float (&acc_im)[TF][C])
{
#pragma unroll
    for (int f = 0; f < TF; ++f) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            if (!(rows & (1u << (c * TF + f)))) continue;   // this wavelength's support misses the block
            const float u = fmaf(U2, dD[f][c], fmaf(U1, dyf[f], u0[c]));
            const float v = fmaf(V2, dD[f][c], fmaf(V1, dyf[f], v0[c]));
            const float kw = fmaf(N2, dD[f][c], fmaf(N1, dyf[f], w0[c]));
            // exp2(log2(1 / (k_z lambda)) - u^2 - v^2): 1/k_z folded into the exponent, lambda into amp
            const float E = __builtin_amdgcn_exp2f(-fmaf(u, u, fmaf(v, v, -lkz[f][c])));
            const float wgt = amp[c] * fabsf(kw) * E;
            const float t = fmaf(-dyf[f], ryf, bx[c]);
            float th;
            if (!WIDE) {
                th = fmaf(-z, dD[f][c], t);
            } else {
                // an integer near the product (any rounding of it will do), then the product
                // minus that integer in one fused operation: |result| <= 1/2, one rounding
                const float r = rintf(z * dD[f][c]);
                const float pr = fmaf(z, dD[f][c], -r);
                th = fmaf(-z, dlo[f][c][lane], t - pr);
            }
            const float sn = __builtin_amdgcn_sinf(th);
            const float cs = __builtin_amdgcn_cosf(th);
            acc_re[f][c] = fmaf(wgt, cs, acc_re[f][c]);
            acc_im[f][c] = fmaf(wgt, sn, acc_im[f][c]);
        }
    }
}

// Per-(sub-tile, Gaussian) entry in LDS: the record's linear forms, then per wavelength the
// FP64-formed bases.  Layout (floats): U[3] V[3] N[3] z rxf ryf rows | u0[C] v0[C] w0[C] base[C] amp[C].
__host__ __device__ constexpr int te_floats(int c) { return (13 + 5 * c + 3) & ~3; }

// Wavefronts per SIMD the accumulation is compiled for: 4 (128 VGPRs) for one wavelength, 3
// (168) for two or three, 2 for four: the per-lane tables (2 x 4 x C) and accumulators
// (2 x 4 x C) grow with the wavelengths.
__host__ __device__ constexpr int tilt_waves(int c) { return c <= 1 ? 4 : (c <= 3 ? 3 : 2); }

template <int C>
__global__ void __launch_bounds__(TWG, tilt_waves(C)) k_tilt_accumulate(Consts k, const TRec *__restrict__ rec,
                                                           const int2 *__restrict__ rect, int64_t n,
                                                           float2 *__restrict__ spectrum,
                                                           float2 *__restrict__ partial, int n_queue, int nparts,
                                                           long long *__restrict__ counters)
{
    constexpr int TE = te_floats(C);
    __shared__ int s_idx[TWG];
    __shared__ int s_cnt[4];
    __shared__ int s_tile;
    __shared__ __align__(16) float s_w[4][64][TE];
    __shared__ float s_lo[4][TF][C][64];   // low part of each lane's D_c(m) - D_c(m0) (read only near the evanescent edge)

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int hx = k.nx / 2, hy = k.ny / 2;
    const double Wx = k.nx * k.px, Wy = k.ny * k.py;
    const float lim = (float)(k.tau2 * (1.0 + 1e-5)) + 1e-4f;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    const int col = lane & 15, row0 = lane >> 4;
    const float dxf = (float)(col - 8);
    float dyf[TF];
#pragma unroll
    for (int f = 0; f < TF; ++f) dyf[f] = (float)(row0 + 4 * f - 8);
    long long pairs = 0, cand = 0;

    for (;;) {
        if (tid == 0) s_tile = (int)atomicAdd((unsigned long long *)&counters[CTR_WORK], 1ull);
        __syncthreads();
        const int q = s_tile;
        __syncthreads();
        if (q >= n_queue) break;
        // item q: part q % nparts of the Gaussians (input order) on tile q / nparts of the ring;
        // with several parts each writes its own partial spectrum of the tile
        const int qt = q / nparts, qp = q - qt * nparts;
        int tx, ty;
        ring_tile(qt, &tx, &ty);
        if (tx * TT >= hx || (tx + 1) * TT <= -hx || ty * TT >= hy || (ty + 1) * TT <= -hy) continue;
        const int64_t g_lo = n * qp / nparts, g_hi = n * (qp + 1) / nparts;
        float2 *__restrict__ dst =
            nparts > 1 ? partial + (int64_t)qp * C * k.ny * k.nx : spectrum;
        // this wavefront's 16 x 16 sub-tile and its per-lane tables
        const int sx0 = tx * TT + (wave & 1) * 16, sy0 = ty * TT + (wave >> 1) * 16;
        const int cx = sx0 + 8, cy = sy0 + 8;
        const int mxp = sx0 + col;
        double D0[C];
        float dD[TF][C], lkz[TF][C], dmax[C];
        {
            const double ncx = cx / Wx, ncy = cy / Wy;
            for (int c = 0; c < C; ++c) D0[c] = dprop_t(ncx * ncx + ncy * ncy, k.inv_lambda[c]);
        }
#pragma unroll
        for (int c = 0; c < C; ++c) dmax[c] = 0.0f;
#pragma unroll
        for (int f = 0; f < TF; ++f) {
            const int myp = sy0 + row0 + 4 * f;
            const double nux = mxp / Wx, nuy = myp / Wy;
            const double nu2 = nux * nux + nuy * nuy;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const double il = k.inv_lambda[c];
                const double w2 = il * il - nu2;
                if (w2 > 0.0) {
                    const double kz = sqrt(w2);
                    const double d = -nu2 / (il + kz) - D0[c];
                    dD[f][c] = (float)d;
                    s_lo[wave][f][c][lane] = (float)(d - (double)dD[f][c]);
                    lkz[f][c] = (float)log2(il / kz);
                } else {
                    dD[f][c] = 0.0f;   // evanescent: the term vanishes (1/k_z taken as 0)
                    s_lo[wave][f][c][lane] = 0.0f;
                    lkz[f][c] = -1000.0f;   // exp2 underflows to 0
                }
                dmax[c] = fmaxf(dmax[c], fabsf(dD[f][c]));
            }
        }
#pragma unroll
        for (int c = 0; c < C; ++c)
            for (int o = 32; o >= 1; o >>= 1) dmax[c] = fmaxf(dmax[c], __shfl_xor(dmax[c], o));
        float dmax_all = 0.0f;
#pragma unroll
        for (int c = 0; c < C; ++c) dmax_all = fmaxf(dmax_all, dmax[c]);
        float acc_re[TF][C], acc_im[TF][C];
#pragma unroll
        for (int f = 0; f < TF; ++f)
#pragma unroll
            for (int c = 0; c < C; ++c) acc_re[f][c] = acc_im[f][c] = 0.0f;
        // grid clipping of the sub-tile's rows (for the block masks)
        const int rlo = max(sy0, -hy), rhi = min(sy0 + 15, hy - 1);
        const bool wave_live = (max(sx0, -hx) <= min(sx0 + 15, hx - 1)) && (rlo <= rhi);

        for (int64_t base = g_lo; base < g_hi; base += TWG) {
            const int64_t gi = base + tid;
            bool pred = false;
            if (gi < g_hi) {
                const int2 b = rect[gi];
                const int tx0 = (int)(int16_t)(b.x & 0xffff), tx1 = b.x >> 16;
                const int ty0 = (int)(int16_t)(b.y & 0xffff), ty1 = b.y >> 16;
                pred = tx >= tx0 && tx <= tx1 && ty >= ty0 && ty <= ty1;
            }
            const uint64_t bal = __ballot(pred);
            if (lane == 0) s_cnt[wave] = __popcll(bal);
            __syncthreads();
            int off = 0, total = 0;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const int cw = s_cnt[w];
                off += (w < wave) ? cw : 0;
                total += cw;
            }
            if (pred) s_idx[off + __popcll(bal & lt)] = (int)gi;
            __syncthreads();
            if (tid == 0) cand += total;
            if (wave_live) {
                for (int j0 = 0; j0 < total; j0 += 64) {
                    // each lane forms the entry of one staged Gaussian in its own slot
                    const int j = j0 + lane;
                    uint32_t rows = 0;
                    if (j < total) {
                        const TRec &r = rec[s_idx[j]];
                        const float4 *src = reinterpret_cast<const float4 *>(&r);
                        const float4 a0 = src[0], a1 = src[1], a2 = src[2];
                        const float U0 = a0.x, U1 = a0.y, U2 = a0.z, V0 = a0.w, V1 = a1.x, V2 = a1.y;
                        const float N0 = a1.z, N1 = a1.w, N2 = a2.x, z = a2.y;
                        float *e = &s_w[wave][lane][0];
                        // per wavelength: bases at the sub-tile centre (FP64), then the bounds of
                        // u, v over each 4-row block of the sub-tile
                        const double ramp_rev =
                            (double)((uint32_t)cx * __float_as_uint(a2.z) + (uint32_t)cy * __float_as_uint(a2.w)) *
                            (1.0 / 4294967296.0);
                        const float ez0 = fabsf(U0) * 8.0f + fabsf(U1) * 1.5f, fz0 = fabsf(V0) * 8.0f + fabsf(V1) * 1.5f;
#pragma unroll
                        for (int c = 0; c < C; ++c) {
                            const double kz0 = k.inv_lambda[c] + D0[c];
                            const float u0 = (float)((double)U0 * cx + (double)U1 * cy + (double)U2 * kz0);
                            const float v0 = (float)((double)V0 * cx + (double)V1 * cy + (double)V2 * kz0);
                            const float kap = r.kappa[c];
                            float bs;
                            if (k.phase_mode == 1) {
                                const float v = kap - ((float)cx * r.rxf + (float)cy * r.ryf) - z * (float)D0[c];
                                bs = v - floorf(v);
                            } else {
                                bs = (float)frac_t((double)kap - ramp_rev - (double)z * D0[c]);
                            }
                            e[13 + c] = u0;
                            e[13 + C + c] = v0;
                            e[13 + 2 * C + c] = (float)((double)N0 * cx + (double)N1 * cy + (double)N2 * kz0);
                            e[13 + 3 * C + c] = bs;
                            e[13 + 4 * C + c] = r.amp[c];
                            const float eu = fmaf(fabsf(U2), dmax[c], ez0), ev = fmaf(fabsf(V2), dmax[c], fz0);
#pragma unroll
                            for (int f = 0; f < TF; ++f) {
                                const int b0 = sy0 + 4 * f;
                                if (b0 + 3 < rlo || b0 > rhi) continue;   // block outside the grid
                                const float dyc = (float)(4 * f) - 6.5f;
                                const float mu = fmaxf(fabsf(fmaf(U1, dyc, u0)) - eu, 0.0f);
                                const float mv = fmaxf(fabsf(fmaf(V1, dyc, v0)) - ev, 0.0f);
                                if (fmaf(mu, mu, mv * mv) <= lim) rows |= 1u << (c * TF + f);
                            }
                        }
                        if (rows) {
                            reinterpret_cast<float4 *>(e)[0] = a0;
                            reinterpret_cast<float4 *>(e)[1] = a1;
                            reinterpret_cast<float4 *>(e)[2] = make_float4(N2, z, r.rxf, r.ryf);
                            e[12] = __uint_as_float(rows);
                            pairs += __popc(rows) * 64;   // (Gaussian, frequency, wavelength) triples
                        }
                    }
                    uint64_t live = __ballot(rows != 0);
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    while (live) {
                        const int ei = __builtin_ctzll(live);
                        live &= live - 1;
                        const float *w = &s_w[wave][ei][0];
                        const float U0 = w[0], U1 = w[1], U2 = w[2], V0 = w[3], V1 = w[4], V2 = w[5];
                        const float N0 = w[6], N1 = w[7], N2 = w[8], z = w[9], rxf = w[10], ryf = w[11];
                        const uint32_t rows = __builtin_amdgcn_readfirstlane(__float_as_uint(w[12]));
                        const float lux = U0 * dxf, lvx = V0 * dxf, lwx = N0 * dxf;
                        float u0[C], v0[C], w0[C], bx[C], amp[C];
#pragma unroll
                        for (int c = 0; c < C; ++c) {
                            u0[c] = w[13 + c] + lux;
                            v0[c] = w[13 + C + c] + lvx;
                            w0[c] = w[13 + 2 * C + c] + lwx;
                            bx[c] = __builtin_amdgcn_fractf(fmaf(-dxf, rxf, w[13 + 3 * C + c]));
                            amp[c] = w[13 + 4 * C + c];
                        }
                        const bool wide = fabsf(z) * dmax_all > 16.0f;
                        if (!wide)
                            tilt_eval<C, false>(rows, U1, U2, V1, V2, N1, N2, z, ryf, u0, v0, w0, bx, amp, dyf, dD, s_lo[wave], lane,
                                                lkz, acc_re, acc_im);
                        else
                            tilt_eval<C, true>(rows, U1, U2, V1, V2, N1, N2, z, ryf, u0, v0, w0, bx, amp, dyf, dD, s_lo[wave], lane,
                                               lkz, acc_re, acc_im);
                    }
                    __builtin_amdgcn_wave_barrier();
                }
            }
            __syncthreads();
        }
        // every frequency of the tile is written once per part (zeros where no Gaussian reaches)
#pragma unroll
        for (int f = 0; f < TF; ++f) {
            const int myp = sy0 + row0 + 4 * f;
            if (mxp >= -hx && mxp < hx && myp >= -hy && myp < hy) {
                const int mx = mxp < 0 ? mxp + k.nx : mxp, my = myp < 0 ? myp + k.ny : myp;
#pragma unroll
                for (int c = 0; c < C; ++c)
                    dst[((int64_t)c * k.ny + my) * k.nx + mx] = make_float2(acc_re[f][c], acc_im[f][c]);
            }
        }
    }
    pairs = wave_sum_i64(pairs);
    if (lane == 0 && pairs) atomicAdd((unsigned long long *)&counters[CTR_PAIRS], (unsigned long long)pairs);
    if (tid == 0 && cand) atomicAdd((unsigned long long *)&counters[CTR_CAND], (unsigned long long)cand);
}

// ---------------------------------------------------------------------------------
// Adjoint.  For a real loss L with Gs = dL/dS (the forward DFT of dL/du), the gradient of a
// parameter t of Gaussian i is Re sum_{c,m} conj(Gs_c[m]) dS_ic[m]/dt, where S_ic = A_c g_c with
// g_c = |w| exp2(L - u^2 - v^2) e^{j 2 pi Theta} (A_c, u, v, w, L as in the forward).  With
// rho_c = conj(Gs_c) S_ic, every derivative is rho times a factor, so per Gaussian the sums
//   P_c = Re sum_m conj(Gs_c) g_c,     I0 = sum Im rho,   Sx = sum m_x Im rho,  Sy = sum m_y Im rho,
//   Z = sum k_z Im rho,                SU_j = sum u x_j Re rho,  SV_j = sum v x_j Re rho,
//   SN_j = sum x_j Re rho / w,         x = (m_x, m_y, k_z)
// carry the whole gradient (chain rule in k_tilt_grad_final).
//
// The kernel walks the forward's (tile, part of the Gaussians) items with the work split the
// other way: the work-group builds the tile's per-frequency tables in LDS (per wavelength D_c(m) - D_c(m0), log2 of
// |Gs_c| 2^-e_t / (k_z lambda_c) with 2^e_t the tile's scale of |Gs|, arg Gs_c / 2 pi and k_z),
// and each wavefront takes whole staged
// Gaussians over the 32 x 32 tile (lane l: column l % 32 and rows l / 32 + 2 f, f < 16), so a
// Gaussian's sums over the tile come out of one transposed cross-lane reduction and go straight
// to its slot for the tile -- off[i] + the tile's place in Gaussian i's rectangle.  Every slot is
// written once and the per-Gaussian sums over slots run in a fixed order: results are bitwise
// reproducible.  The ramp m . r (0.32 fixed point) is formed exactly per lane and row in integer
// arithmetic; the carrier's FP64 base is taken at the tile centre.
// ---------------------------------------------------------------------------------
__host__ __device__ constexpr int tilt_nv(int c) { return c + 13; }
__host__ __device__ constexpr int tilt_nvp(int c) { return tilt_nv(c) <= 16 ? 16 : 24; }
constexpr int TA_F = 16;   // row pairs of a tile: lane l holds rows l / 32 + 2 f
// Wavefronts per SIMD: three up to three wavelengths (the tables take 16 KB per wavelength, so
// three work-groups share a CU), two for four.
__host__ __device__ constexpr int tilt_adj_waves(int c) { return c <= 3 ? 3 : 2; }

// One staged Gaussian's sums at a lane's frequencies (bit f * C + c of `rows`: wavelength c
// reaches row pair f).  The weights m_x (the lane's column) and m_y (one per row pair) are
// applied once per lane and once per row pair: per term only the unweighted and the
// k_z-weighted sums run.  x on return: P_c, I0, Sx, Sy, Z, SU(x,y,z), SV(x,y,z), SN(x,y,z).
// WIDE (tiles where |z| (D_c(m) - D_c(m0)) can exceed 16 revolutions): that product reduced in
// FP64.
template <int C, bool WIDE>
static __device__ __forceinline__ void tilt_adj_eval(uint64_t rows, const float4 (&tab)[TA_F][C][64], int lane,
                                                     float U1, float U2, float V1, float V2, float N1, float N2,
                                                     float z, float dy0, float my0, float mx, uint32_t r0, uint32_t r2,
                                                     const float (&u0)[C], const float (&v0)[C], const float (&w0)[C],
                                                     const float (&kc)[C], const float (&amp)[C],
                                                     const double (&D0)[C], const double (&il)[C], double iwx,
                                                     double iwy, float (&x)[tilt_nvp(C)])
{
    float aI = 0.0f, aU = 0.0f, aV = 0.0f, aS = 0.0f;   // unweighted: times m_x at the end
    // the row pairs from the first to the last one the support reaches
    const int f0 = __builtin_ctzll(rows) / C, f1 = (63 - __builtin_clzll(rows)) / C;
    uint32_t rm = r0 + (uint32_t)f0 * r2;   // the lane's ramp m . r in 0.32 fixed point (exact, wraps mod 1)
    float dy = dy0 + (float)(2 * f0), my = my0 + (float)(2 * f0);   // row offset from the tile centre, row index
#pragma unroll 2
    for (int f = f0; f <= f1; ++f, rm += r2, dy += 2.0f, my += 2.0f) {
        const uint32_t fb = (uint32_t)(rows >> (f * C)) & ((1u << C) - 1u);
        if (fb == 0) continue;
        const float rf = (float)(int32_t)rm * 0x1p-32f;   // in revolutions, one rounding
        float tI = 0.0f, tU = 0.0f, tV = 0.0f, tS = 0.0f;   // this row pair's sums over the wavelengths
#pragma unroll
        for (int c = 0; c < C; ++c) {
            if (!(fb & (1u << c))) continue;
            const float4 tv = tab[f][c][lane];   // D_c(m) - D_c(m0), log2(|Gs| 2^-e_t / (k_z lambda)), arg Gs / 2 pi, k_z
            const float d = tv.x;
            const float u = fmaf(U2, d, fmaf(U1, dy, u0[c]));
            const float v = fmaf(V2, d, fmaf(V1, dy, v0[c]));
            const float kw = fmaf(N2, d, fmaf(N1, dy, w0[c]));
            const float eg = __builtin_amdgcn_exp2f(-fmaf(u, u, fmaf(v, v, -tv.y)));
            const float t = (kc[c] - rf) - tv.z;
            float th;
            if (!WIDE) {
                th = fmaf(-z, d, t);
            } else {
                const double nux = mx * iwx, nuy = my * iwy, nu2 = nux * nux + nuy * nuy;
                const double w2 = il[c] * il[c] - nu2;
                const double dd = w2 > 0.0 ? -nu2 / (il[c] + sqrt(w2)) - D0[c] : 0.0;
                const double p = (double)z * dd;
                th = (float)((double)t - (p - rint(p)));
            }
            const float sn = __builtin_amdgcn_sinf(th);
            const float cs = __builtin_amdgcn_cosf(th);
            const float gr = eg * cs, gi = eg * sn;
            const float aw = fabsf(kw);
            x[c] = fmaf(aw, gr, x[c]);               // P_c
            const float kz = tv.w;
            const float ak = amp[c] * aw, kak = kz * ak;
            const float rr = ak * gr, kr = kak * gr;
            const float sa = copysignf(amp[c], kw);   // Re rho / w = sa gr
            tI = fmaf(ak, gi, tI);
            x[C + 3] = fmaf(kak, gi, x[C + 3]);      // Z
            tU = fmaf(u, rr, tU);
            x[C + 6] = fmaf(u, kr, x[C + 6]);        // SUz
            tV = fmaf(v, rr, tV);
            x[C + 9] = fmaf(v, kr, x[C + 9]);        // SVz
            tS = fmaf(sa, gr, tS);
            x[C + 12] = fmaf(kz * sa, gr, x[C + 12]);   // SNz
        }
        x[C + 2] = fmaf(my, tI, x[C + 2]);           // Sy
        x[C + 5] = fmaf(my, tU, x[C + 5]);           // SUy
        x[C + 8] = fmaf(my, tV, x[C + 8]);           // SVy
        x[C + 11] = fmaf(my, tS, x[C + 11]);         // SNy
        aI += tI;
        aU += tU;
        aV += tV;
        aS += tS;
    }
    x[C + 0] = aI;
    x[C + 1] = mx * aI;                              // Sx
    x[C + 4] = mx * aU;                              // SUx
    x[C + 7] = mx * aV;                              // SVx
    x[C + 10] = mx * aS;                             // SNx
}

static __device__ __forceinline__ float rl_f(float v, int l) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l)); }
static __device__ __forceinline__ uint32_t rl_u(uint32_t v, int l) { return (uint32_t)__builtin_amdgcn_readlane((int)v, l); }

template <int C>
__global__ void __launch_bounds__(TWG, tilt_adj_waves(C)) k_tilt_adjoint(Consts k, const TRec *__restrict__ rec,
                                                                          const int2 *__restrict__ rect, int64_t n,
                                                                          const float2 *__restrict__ gspec,
                                                                          const int64_t *__restrict__ off,
                                                                          float *__restrict__ part, int n_queue,
                                                                          int nparts, long long *__restrict__ counters)
{
    constexpr int NV = tilt_nv(C), NVP = tilt_nvp(C);
    __shared__ int s_idx[TWG];
    __shared__ int s_cnt[4];
    __shared__ int s_tile;
    __shared__ int s_e[4];
    __shared__ float s_dm[4][C];
    __shared__ float4 s_t[TA_F][C][64];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int hx = k.nx / 2, hy = k.ny / 2;
    const double Wx = k.nx * k.px, Wy = k.ny * k.py;
    double ilam[C];
#pragma unroll
    for (int c = 0; c < C; ++c) ilam[c] = k.inv_lambda[c];
    const float lim = (float)(k.tau2 * (1.0 + 1e-5)) + 1e-4f;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    const int col = lane & 31, row0 = lane >> 5;
    const float dxf = (float)(col - 16);
    long long pairs = 0;

    for (;;) {
        if (tid == 0) s_tile = (int)atomicAdd((unsigned long long *)&counters[CTR_WORK], 1ull);
        __syncthreads();
        const int q = s_tile;
        __syncthreads();
        if (q >= n_queue) break;
        // item q: part q % nparts of the Gaussians (input order) on tile q / nparts of the ring
        const int qt = q / nparts, qp = q - qt * nparts;
        int tx, ty;
        ring_tile(qt, &tx, &ty);
        if (tx * TT >= hx || (tx + 1) * TT <= -hx || ty * TT >= hy || (ty + 1) * TT <= -hy) continue;
        const int64_t g_lo = n * qp / nparts, g_hi = n * (qp + 1) / nparts;
        const int mx0 = tx * TT, my0 = ty * TT, cx = mx0 + 16, cy = my0 + 16;
        double D0[C];
        {
            const double ncx = cx / Wx, ncy = cy / Wy;
#pragma unroll
            for (int c = 0; c < C; ++c) D0[c] = dprop_t(ncx * ncx + ncy * ncy, ilam[c]);
        }
        // The tile's tables: |Gs| first (its largest finite binary exponent e_t over the tile is
        // taken out of the logarithm, and the tile's sums are scaled by 2^e_t when written; an
        // infinite |Gs| still reaches the sums as one).
        float dm[C];
        int emax = -1000;
#pragma unroll
        for (int c = 0; c < C; ++c) dm[c] = 0.0f;
        for (int p = tid; p < TA_F * 64; p += TWG) {
            const int l = p & 63, f = p >> 6;
            const int mxp = mx0 + (l & 31), myp = my0 + (l >> 5) + 2 * f;
            const double nux = mxp / Wx, nuy = myp / Wy, nu2 = nux * nux + nuy * nuy;
            const bool in_grid = mxp >= -hx && mxp < hx && myp >= -hy && myp < hy;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const double il = ilam[c];
                const double w2 = il * il - nu2;
                float4 tv = make_float4(0.0f, 0.0f, 0.0f, 0.0f);   // evanescent: no contribution
                if (w2 > 0.0) {
                    const double kz = sqrt(w2);
                    tv.x = (float)(-nu2 / (il + kz) - D0[c]);
                    tv.w = (float)kz;
                    if (in_grid) {
                        const int gx = mxp < 0 ? mxp + k.nx : mxp, gy = myp < 0 ? myp + k.ny : myp;
                        const float2 g = gspec[((int64_t)c * k.ny + gy) * k.nx + gx];
                        tv.y = hypotf(g.x, g.y);
                        tv.z = atan2f(g.y, g.x) * 0.15915494309189535f;
                        if (tv.y > 0.0f && tv.y <= 3.4028234663852886e38f) emax = max(emax, ilogbf(tv.y));
                    }
                }
                dm[c] = fmaxf(dm[c], fabsf(tv.x));
                s_t[f][c][l] = tv;
            }
        }
#pragma unroll
        for (int c = 0; c < C; ++c)
            for (int o = 32; o >= 1; o >>= 1) dm[c] = fmaxf(dm[c], __shfl_xor(dm[c], o));
        for (int o = 32; o >= 1; o >>= 1) emax = max(emax, __shfl_xor(emax, o));
        if (lane == 0) {
            s_e[wave] = emax;
#pragma unroll
            for (int c = 0; c < C; ++c) s_dm[wave][c] = dm[c];
        }
        __syncthreads();
        const int et = max(max(s_e[0], s_e[1]), max(s_e[2], s_e[3]));
        const int es = et > -1000 ? et : 0;
        float dmax[C], dmax_all = 0.0f;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            dmax[c] = fmaxf(fmaxf(s_dm[0][c], s_dm[1][c]), fmaxf(s_dm[2][c], s_dm[3][c]));
            dmax_all = fmaxf(dmax_all, dmax[c]);
        }
        // the same entries, by the same threads: |Gs| -> log2(|Gs| 2^-e_t / (k_z lambda))
        for (int p = tid; p < TA_F * 64; p += TWG) {
            const int l = p & 63, f = p >> 6;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                float4 tv = s_t[f][c][l];
                tv.y = (tv.y > 0.0f && tv.w > 0.0f)
                           ? fmaxf((float)(log2(ilam[c] / (double)tv.w) + (double)log2f(ldexpf(tv.y, -es))), -1000.0f)
                           : -1000.0f;
                s_t[f][c][l] = tv;
            }
        }
        __syncthreads();
        const int rlo = max(my0, -hy), rhi = min(my0 + TT - 1, hy - 1);
        const int mxp = mx0 + col, myl = my0 + row0;

        for (int64_t base = g_lo; base < g_hi; base += TWG) {
            const int64_t gi = base + tid;
            bool pred = false;
            if (gi < g_hi) {
                const int2 b = rect[gi];
                const int tx0 = (int)(int16_t)(b.x & 0xffff), tx1 = b.x >> 16;
                const int ty0 = (int)(int16_t)(b.y & 0xffff), ty1 = b.y >> 16;
                pred = tx >= tx0 && tx <= tx1 && ty >= ty0 && ty <= ty1;
            }
            const uint64_t bal = __ballot(pred);
            if (lane == 0) s_cnt[wave] = __popcll(bal);
            __syncthreads();
            int offs = 0, total = 0;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const int cw = s_cnt[w];
                offs += (w < wave) ? cw : 0;
                total += cw;
            }
            if (pred) s_idx[offs + __popcll(bal & lt)] = (int)gi;
            __syncthreads();
            // staging: lane l of wavefront w holds staged Gaussian 4 l + w at the tile centre
            const int j = 4 * lane + wave;
            uint64_t rows = 0;
            int64_t slot = 0;
            float eU0 = 0, eU1 = 0, eU2 = 0, eV0 = 0, eV1 = 0, eV2 = 0, eN0 = 0, eN1 = 0, eN2 = 0, ez = 0;
            float eu0[C], ev0[C], ew0[C], ekc[C], eamp[C];
            uint32_t erx = 0, ery = 0;
#pragma unroll
            for (int c = 0; c < C; ++c) eu0[c] = ev0[c] = ew0[c] = ekc[c] = eamp[c] = 0.0f;
            if (j < total) {
                const int gidx = s_idx[j];
                const TRec &r = rec[gidx];
                const float4 *src = reinterpret_cast<const float4 *>(&r);
                const float4 a0 = src[0], a1 = src[1], a2 = src[2];
                eU0 = a0.x; eU1 = a0.y; eU2 = a0.z; eV0 = a0.w; eV1 = a1.x; eV2 = a1.y;
                eN0 = a1.z; eN1 = a1.w; eN2 = a2.x; ez = a2.y;
                erx = __float_as_uint(a2.z);
                ery = __float_as_uint(a2.w);
                const float ez0 = fabsf(eU0) * 16.0f + fabsf(eU1) * 0.5f, fz0 = fabsf(eV0) * 16.0f + fabsf(eV1) * 0.5f;
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const double kzc = ilam[c] + D0[c];
                    eu0[c] = (float)((double)eU0 * cx + (double)eU1 * cy + (double)eU2 * kzc);
                    ev0[c] = (float)((double)eV0 * cx + (double)eV1 * cy + (double)eV2 * kzc);
                    ew0[c] = (float)((double)eN0 * cx + (double)eN1 * cy + (double)eN2 * kzc);
                    const float kap = r.kappa[c];
                    if (k.phase_mode == 1) {
                        const float vv = kap - ez * (float)D0[c];
                        ekc[c] = vv - floorf(vv);
                    } else {
                        ekc[c] = (float)frac_t((double)kap - (double)ez * D0[c]);
                    }
                    eamp[c] = r.amp[c];
                    // row pairs the support can reach: bounds of u and v over the pair
                    const float eu = fmaf(fabsf(eU2), dmax[c], ez0), ev = fmaf(fabsf(eV2), dmax[c], fz0);
#pragma unroll
                    for (int f = 0; f < TA_F; ++f) {
                        const int b0 = my0 + 2 * f;
                        if (b0 + 1 < rlo || b0 > rhi) continue;
                        const float dyc = (float)(2 * f) - 15.5f;
                        const float mu = fmaxf(fabsf(fmaf(eU1, dyc, eu0[c])) - eu, 0.0f);
                        const float mv = fmaxf(fabsf(fmaf(eV1, dyc, ev0[c])) - ev, 0.0f);
                        if (fmaf(mu, mu, mv * mv) <= lim) rows |= 1ull << (f * C + c);
                    }
                }
                const int2 b = rect[gidx];
                const int tx0 = (int)(int16_t)(b.x & 0xffff), tx1 = b.x >> 16;
                const int ty0 = (int)(int16_t)(b.y & 0xffff);
                slot = off[gidx] + (int64_t)(ty - ty0) * (tx1 - tx0 + 1) + (tx - tx0);
                pairs += (long long)__popcll(rows) * 64;
                if (!rows) {   // the rectangle reaches the tile, the support does not: its slot holds zeros
#pragma unroll
                    for (int v = 0; v < NV; ++v) part[slot * NV + v] = 0.0f;
                }
            }
            uint64_t live = __ballot(rows != 0);
            while (live) {
                const int ei = __builtin_ctzll(live);
                live &= live - 1;
                const float U0 = rl_f(eU0, ei), U1 = rl_f(eU1, ei), U2 = rl_f(eU2, ei);
                const float V0 = rl_f(eV0, ei), V1 = rl_f(eV1, ei), V2 = rl_f(eV2, ei);
                const float N0 = rl_f(eN0, ei), N1 = rl_f(eN1, ei), N2 = rl_f(eN2, ei), z = rl_f(ez, ei);
                const uint64_t erows = ((uint64_t)rl_u((uint32_t)(rows >> 32), ei) << 32) | rl_u((uint32_t)rows, ei);
                const int64_t eslot = (int64_t)(((uint64_t)rl_u((uint32_t)((uint64_t)slot >> 32), ei) << 32) |
                                                rl_u((uint32_t)slot, ei));
                float u0[C], v0[C], w0[C], kc[C], amp[C];
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    u0[c] = fmaf(U0, dxf, rl_f(eu0[c], ei));
                    v0[c] = fmaf(V0, dxf, rl_f(ev0[c], ei));
                    w0[c] = fmaf(N0, dxf, rl_f(ew0[c], ei));
                    kc[c] = rl_f(ekc[c], ei);
                    amp[c] = rl_f(eamp[c], ei);
                }
                // the ramp at the lane's first frequency (m_x, m_y0) and its step over two rows
                const uint32_t rx = rl_u(erx, ei), ry = rl_u(ery, ei);
                uint32_t r0;
                if (k.phase_mode == 1) {
                    // FP32 ramp (the record's rounded r): m_x r_x + m_y r_y, its fraction
                    const float vv = (float)mxp * ((float)(int32_t)rx * 0x1p-32f) + (float)myl * ((float)(int32_t)ry * 0x1p-32f);
                    r0 = (uint32_t)(int64_t)((vv - floorf(vv)) * 4294967296.0f);
                } else {
                    r0 = (uint32_t)mxp * rx + (uint32_t)myl * ry;
                }
                const uint32_t r2 = 2u * ry;
                float x[NVP];
#pragma unroll
                for (int v = 0; v < NVP; ++v) x[v] = 0.0f;
                const float dy0 = (float)(row0 - 16), myf0 = (float)myl, mxw = (float)mxp;
                if (fabsf(z) * dmax_all > 16.0f)
                    tilt_adj_eval<C, true>(erows, s_t, lane, U1, U2, V1, V2, N1, N2, z, dy0, myf0, mxw, r0, r2, u0, v0,
                                           w0, kc, amp, D0, ilam, 1.0 / Wx, 1.0 / Wy, x);
                else
                    tilt_adj_eval<C, false>(erows, s_t, lane, U1, U2, V1, V2, N1, N2, z, dy0, myf0, mxw, r0, r2, u0, v0,
                                            w0, kc, amp, D0, ilam, 1.0 / Wx, 1.0 / Wy, x);
                // sums over the wavefront: after the transposed butterfly register j of lane l
                // holds value 2 (4 b5 + 2 b4 + b3) + j (and + 16 for the second block)
                float y0 = 0.0f;
                float xa[16];
#pragma unroll
                for (int v = 0; v < 16; ++v) xa[v] = x[v];
                reduce_transposed<16, false>(xa, y0, lane);
                const int g8 = ((lane >> 5) & 1) * 4 + ((lane >> 4) & 1) * 2 + ((lane >> 3) & 1);
                float *dst = part + eslot * NV;
                if ((lane & 7) == 0) {
#pragma unroll
                    for (int jj = 0; jj < 2; ++jj)
                        if (2 * g8 + jj < NV) dst[2 * g8 + jj] = ldexpf(xa[jj], es);
                }
                if constexpr (NVP > 16) {
                    float xb[8];
#pragma unroll
                    for (int v = 0; v < 8; ++v) xb[v] = x[16 + v];
                    reduce_transposed<8, false>(xb, y0, lane);
                    if ((lane & 7) == 0 && 16 + g8 < NV) dst[16 + g8] = ldexpf(xb[0], es);
                }
            }
            __syncthreads();   // before the next chunk overwrites the staged indices
        }
    }
    pairs = wave_sum_i64(pairs);
    if (lane == 0 && pairs) atomicAdd((unsigned long long *)&counters[CTR_PAIRS], (unsigned long long)pairs);
}

// Rectangle areas (tiles per Gaussian) and their exclusive prefix: off[i] = first slot of
// Gaussian i, off[n] = all slots.  Three passes: per 1024-block scans, a scan of the block
// totals in one work-group, the block offsets added.
__global__ void __launch_bounds__(1024) k_tilt_scan1(const int2 *__restrict__ rect, int64_t n, int64_t *__restrict__ off,
                                                    int64_t *__restrict__ bsum)
{
    __shared__ int64_t sh[1024];
    const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    int64_t a = 0;
    if (i < n) {
        const int2 b = rect[i];
        const int tx0 = (int)(int16_t)(b.x & 0xffff), tx1 = b.x >> 16;
        const int ty0 = (int)(int16_t)(b.y & 0xffff), ty1 = b.y >> 16;
        a = (tx1 >= tx0 && ty1 >= ty0) ? (int64_t)(tx1 - tx0 + 1) * (ty1 - ty0 + 1) : 0;
    }
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const int64_t v = threadIdx.x >= (unsigned)d ? sh[threadIdx.x - d] : 0;
        __syncthreads();
        sh[threadIdx.x] += v;
        __syncthreads();
    }
    if (i < n) off[i] = sh[threadIdx.x] - a;
    if (threadIdx.x == 1023) bsum[blockIdx.x] = sh[1023];
}

__global__ void __launch_bounds__(1024) k_tilt_scan2(int64_t *__restrict__ bsum, int nb, int64_t *__restrict__ total)
{
    __shared__ int64_t sh[1024];
    const int per = (nb + 1023) / 1024, b0 = threadIdx.x * per;
    int64_t s = 0;
    for (int j = 0; j < per && b0 + j < nb; ++j) s += bsum[b0 + j];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const int64_t v = threadIdx.x >= (unsigned)d ? sh[threadIdx.x - d] : 0;
        __syncthreads();
        sh[threadIdx.x] += v;
        __syncthreads();
    }
    int64_t run = sh[threadIdx.x] - s;
    for (int j = 0; j < per && b0 + j < nb; ++j) {
        const int64_t v = bsum[b0 + j];
        bsum[b0 + j] = run;
        run += v;
    }
    if (threadIdx.x == 1023) *total = sh[1023];
}

__global__ void __launch_bounds__(1024) k_tilt_scan3(int64_t *__restrict__ off, int64_t n, const int64_t *__restrict__ bsum)
{
    const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    if (i < n) off[i] += bsum[blockIdx.x];
}

hipError_t launch_tilt_offsets(const int2 *rect, int64_t n, int64_t *off, int64_t *bsum, hipStream_t s)
{
    const int nb = (int)std::max<int64_t>(1, (n + 1023) / 1024);
    if (n > 0) hipLaunchKernelGGL(k_tilt_scan1, dim3(nb), dim3(1024), 0, s, rect, n, off, bsum);
    else hipLaunchKernelGGL(k_tilt_zero64, dim3(1), dim3(64), 0, s, bsum, 1);
    hipLaunchKernelGGL(k_tilt_scan2, dim3(1), dim3(1024), 0, s, bsum, nb, off + n);
    if (n > 0) hipLaunchKernelGGL(k_tilt_scan3, dim3(nb), dim3(1024), 0, s, off, n, bsum);
    return hipGetLastError();
}

// Per Gaussian (one wavefront): its slots summed in a fixed order (FP64), then the chain rule to
// the parameters.  A Gaussian with no slots (culled, or its support outside the band) gets zeros.
template <int C>
__global__ void __launch_bounds__(256) k_tilt_grad_final(TView g, Consts k, const int2 *__restrict__ rect,
                                                         const int64_t *__restrict__ off,
                                                         const float *__restrict__ part, TGrads gr)
{
    constexpr int NV = tilt_nv(C);
    const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (i >= g.n) return;
    const int64_t s0 = off[i], ns = off[i + 1] - s0;
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
    for (int64_t t = lane; t < ns; t += 64) {
        const float *src = part + (s0 + t) * NV;
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] += (double)src[v];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v)
        for (int o = 32; o >= 1; o >>= 1) acc[v] += __shfl_xor(acc[v], o);
    if (lane != 0) return;
    if (ns == 0) {
        gr.mean_x[i] = gr.mean_y[i] = gr.depth[i] = 0.0f;
        gr.quat_w[i] = gr.quat_x[i] = gr.quat_y[i] = gr.quat_z[i] = 0.0f;
        gr.scale_u[i] = gr.scale_v[i] = gr.opacity[i] = gr.phase[i] = 0.0f;
#pragma unroll
        for (int c = 0; c < C; ++c) gr.amplitude[(int64_t)c * g.n + i] = 0.0f;
        return;
    }
    const double PI = 3.14159265358979323846, LN2 = 0.69314718055994530942;
    const double qw0 = g.quat_w[i], qx0 = g.quat_x[i], qy0 = g.quat_y[i], qz0 = g.quat_z[i];
    const double qn = sqrt(qw0 * qw0 + qx0 * qx0 + qy0 * qy0 + qz0 * qz0);
    const double w = qw0 / qn, x = qx0 / qn, y = qy0 / qn, z = qz0 / qn;
    const double R[3][3] = {{1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
                            {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
                            {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
    const double Wx = k.nx * k.px, Wy = k.ny * k.py, sk = sqrt(k.K2);
    const double su = g.scale_u[i], sv = g.scale_v[i], o = g.opacity[i];
    const double K = 2.0 * PI * su * sv / (k.px * k.py * (double)k.nx * (double)k.ny);
    const double cs[3] = {1.0 / Wx, 1.0 / Wy, 1.0};
    // amplitude, opacity and the part of the scale gradient through A_c = a_c o K lambda_c
    double R0 = 0.0, go = 0.0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const double a = g.amplitude[(int64_t)c * g.n + i];
        const double P = acc[c];
        gr.amplitude[(int64_t)c * g.n + i] = (float)(o * K * k.lambda[c] * P);
        go += a * K * k.lambda[c] * P;
        R0 += a * o * K * k.lambda[c] * P;
    }
    const double I0 = acc[C], Sx = acc[C + 1], Sy = acc[C + 2], Zs = acc[C + 3];
    gr.opacity[i] = (float)go;
    gr.phase[i] = (float)(-I0);
    gr.mean_x[i] = (float)(2.0 * PI / Wx * Sx);
    gr.mean_y[i] = (float)(2.0 * PI / Wy * Sy);
    gr.depth[i] = (float)(2.0 * PI * Zs);
    // u = U.x, v = V.x, w = N.x: dL/dU_j = -2 ln2 SU_j, dL/dV_j = -2 ln2 SV_j, dL/dN_j = SN_j
    double gU[3], gV[3], gN[3], GR[3][3];
    for (int j = 0; j < 3; ++j) {
        gU[j] = -2.0 * LN2 * acc[C + 4 + j];
        gV[j] = -2.0 * LN2 * acc[C + 7 + j];
        gN[j] = acc[C + 10 + j];
        GR[j][0] = gU[j] * sk * su * cs[j];
        GR[j][1] = gV[j] * sk * sv * cs[j];
        GR[j][2] = gN[j] * cs[j];
    }
    double dsu = R0 / su, dsv = R0 / sv;
    for (int j = 0; j < 3; ++j) {
        dsu += gU[j] * sk * R[j][0] * cs[j];
        dsv += gV[j] * sk * R[j][1] * cs[j];
    }
    gr.scale_u[i] = (float)dsu;
    gr.scale_v[i] = (float)dsv;
    // R of the unit quaternion (w, x, y, z): dR/dw, dR/dx, dR/dy, dR/dz, then the normalisation
    const double dW[3][3] = {{0, -2 * z, 2 * y}, {2 * z, 0, -2 * x}, {-2 * y, 2 * x, 0}};
    const double dX[3][3] = {{0, 2 * y, 2 * z}, {2 * y, -4 * x, -2 * w}, {2 * z, 2 * w, -4 * x}};
    const double dY[3][3] = {{-4 * y, 2 * x, 2 * w}, {2 * x, 0, 2 * z}, {-2 * w, 2 * z, -4 * y}};
    const double dZ[3][3] = {{-4 * z, -2 * w, 2 * x}, {2 * w, -4 * z, 2 * y}, {2 * x, 2 * y, 0}};
    double gq[4] = {0, 0, 0, 0};
    for (int r = 0; r < 3; ++r)
        for (int cc = 0; cc < 3; ++cc) {
            gq[0] += GR[r][cc] * dW[r][cc];
            gq[1] += GR[r][cc] * dX[r][cc];
            gq[2] += GR[r][cc] * dY[r][cc];
            gq[3] += GR[r][cc] * dZ[r][cc];
        }
    const double qh[4] = {w, x, y, z};
    const double dotp = qh[0] * gq[0] + qh[1] * gq[1] + qh[2] * gq[2] + qh[3] * gq[3];
    gr.quat_w[i] = (float)((gq[0] - qh[0] * dotp) / qn);
    gr.quat_x[i] = (float)((gq[1] - qh[1] * dotp) / qn);
    gr.quat_y[i] = (float)((gq[2] - qh[2] * dotp) / qn);
    gr.quat_z[i] = (float)((gq[3] - qh[3] * dotp) / qn);
}

static int tilt_queue_len(int nx, int ny);

template <int C>
static hipError_t launch_tilt_adjoint_c(const Consts &k, const TRec *rec, const int2 *rect, int64_t n,
                                        const float2 *gspec, const int64_t *off, float *part, long long *counters,
                                        int n_cu, hipStream_t s)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void *)k_tilt_adjoint<C>, TWG, 0) != hipSuccess ||
        nb < 1)
        nb = 1;
    // each tile's Gaussians split into parts taken as separate items (each (Gaussian, tile) slot
    // is still written once), so the tiles every support crowds do not hold the launch's tail
    const int nparts = tilt_parts(n);
    const int nq = tilt_queue_len(k.nx, k.ny) * nparts;
    const int grid = std::max(1, std::min(n_cu * nb, nq));
    hipLaunchKernelGGL(k_tilt_adjoint<C>, dim3(grid), dim3(TWG), 0, s, k, rec, rect, n, gspec, off, part, nq, nparts,
                       counters);
    return hipGetLastError();
}

hipError_t launch_tilt_adjoint(const Consts &k, const TRec *rec, const int2 *rect, int64_t n, const float2 *gspec,
                               const int64_t *off, float *part, long long *counters, int n_cu, hipStream_t s)
{
    switch (k.C) {
    case 1: return launch_tilt_adjoint_c<1>(k, rec, rect, n, gspec, off, part, counters, n_cu, s);
    case 2: return launch_tilt_adjoint_c<2>(k, rec, rect, n, gspec, off, part, counters, n_cu, s);
    case 3: return launch_tilt_adjoint_c<3>(k, rec, rect, n, gspec, off, part, counters, n_cu, s);
    case 4: return launch_tilt_adjoint_c<4>(k, rec, rect, n, gspec, off, part, counters, n_cu, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_tilt_grad_final(const TView &g, const Consts &k, const int2 *rect, const int64_t *off,
                                  const float *part, const TGrads &gr, hipStream_t s)
{
    if (g.n == 0) return hipSuccess;
    const dim3 grid((unsigned)((g.n * 64 + 255) / 256)), block(256);
    switch (k.C) {
    case 1: hipLaunchKernelGGL(k_tilt_grad_final<1>, grid, block, 0, s, g, k, rect, off, part, gr); break;
    case 2: hipLaunchKernelGGL(k_tilt_grad_final<2>, grid, block, 0, s, g, k, rect, off, part, gr); break;
    case 3: hipLaunchKernelGGL(k_tilt_grad_final<3>, grid, block, 0, s, g, k, rect, off, part, gr); break;
    case 4: hipLaunchKernelGGL(k_tilt_grad_final<4>, grid, block, 0, s, g, k, rect, off, part, gr); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int tilt_slot_floats(int C) { return tilt_nv(C); }

hipError_t launch_tilt_records(const TView &g, const Consts &k, TRec *rec, int2 *rect, long long *counters,
                               hipStream_t s)
{
    hipLaunchKernelGGL(k_tilt_zero, dim3(1), dim3(64), 0, s, counters);
    if (g.n > 0)
        hipLaunchKernelGGL(k_tilt_records, dim3((unsigned)((g.n + 255) / 256)), dim3(256), 0, s, g, k, rec, rect,
                           counters);
    return hipGetLastError();
}

// Queue length: the rings around DC that cover the grid's tiles.
static int tilt_queue_len(int nx, int ny)
{
    const int hx = nx / 2, hy = ny / 2;
    const int txmax = (hx - 1) / TT, txmin = -((hx + TT - 1) / TT), tymax = (hy - 1) / TT, tymin = -((hy + TT - 1) / TT);
    const int r = std::max(std::max(txmax, -1 - txmin), std::max(tymax, -1 - tymin));
    return 4 * (r + 1) * (r + 1);
}

template <int C>
static const void *tilt_kernel() { return (const void *)k_tilt_accumulate<C>; }

// The parts' partial spectra added in part order (fixed, so the result is reproducible).
__global__ void __launch_bounds__(256) k_tilt_sum_parts(const float2 *__restrict__ partial, int nparts, int64_t m,
                                                        float2 *__restrict__ spectrum)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        float2 a = partial[i];
        for (int p = 1; p < nparts; ++p) {
            const float2 b = partial[(int64_t)p * m + i];
            a.x += b.x;
            a.y += b.y;
        }
        spectrum[i] = a;
    }
}

int tilt_parts(int64_t n) { return (int)std::min<int64_t>(TILT_PARTS_MAX, std::max<int64_t>(1, n / 8192)); }

hipError_t launch_tilt_accumulate(const Consts &k, const TRec *rec, const int2 *rect, int64_t n, float2 *spectrum,
                                  float2 *partial, long long *counters, int n_cu, hipStream_t s)
{
    const void *kp = nullptr;
    switch (k.C) {
    case 1: kp = tilt_kernel<1>(); break;
    case 2: kp = tilt_kernel<2>(); break;
    case 3: kp = tilt_kernel<3>(); break;
    case 4: kp = tilt_kernel<4>(); break;
    default: return hipErrorInvalidValue;
    }
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kp, TWG, 0) != hipSuccess || nb < 1) nb = 1;
    const int np = tilt_parts(n);
    if (np > 1 && !partial) return hipErrorInvalidValue;
    const int nq = tilt_queue_len(k.nx, k.ny) * np;
    const int grid = std::max(1, std::min(n_cu * nb, nq));
    switch (k.C) {
    case 1: hipLaunchKernelGGL(k_tilt_accumulate<1>, dim3(grid), dim3(TWG), 0, s, k, rec, rect, n, spectrum, partial, nq, np, counters); break;
    case 2: hipLaunchKernelGGL(k_tilt_accumulate<2>, dim3(grid), dim3(TWG), 0, s, k, rec, rect, n, spectrum, partial, nq, np, counters); break;
    case 3: hipLaunchKernelGGL(k_tilt_accumulate<3>, dim3(grid), dim3(TWG), 0, s, k, rec, rect, n, spectrum, partial, nq, np, counters); break;
    default: hipLaunchKernelGGL(k_tilt_accumulate<4>, dim3(grid), dim3(TWG), 0, s, k, rec, rect, n, spectrum, partial, nq, np, counters); break;
    }
    if (np > 1) {
        const int64_t m = (int64_t)k.C * k.ny * k.nx;
        const int blocks = (int)std::min<int64_t>((m + 255) / 256, 8192);
        hipLaunchKernelGGL(k_tilt_sum_parts, dim3(blocks), dim3(256), 0, s, (const float2 *)partial, np, m, spectrum);
    }
    return hipGetLastError();
}

}  // namespace gws
