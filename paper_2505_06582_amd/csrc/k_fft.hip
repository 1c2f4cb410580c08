// Mixed-radix (2, 3, 4, 5, 8, 9, 15, 16) Stockham FFT in LDS for gfx950: the one inverse 2D transform
// that brings the accumulated spectrum to the SLM plane (supplement Alg. 1 and Alg. 4, last
// step), and the forward transform the adjoint needs.  Unnormalised:
//   direction +1:  out[n] = sum_m in[m] exp(+j 2 pi m n / N)
//   direction -1:  out[n] = sum_m in[m] exp(-j 2 pi m n / N)
// Pass 1 transforms rows (one row per work-group); pass 2 transforms columns, a slab of
// B adjacent columns per work-group, read and written as contiguous row segments.
// Twiddles come from per-size FP32 tables computed on the host in FP64.
#include "gws_internal.h"

namespace gws {

constexpr int FFT_THREADS = 256;
constexpr int FFT_MAX_RAD = 16;

// sh[b]: the LDS layout of a row between pass b - 1 and pass b (b = 0: as loaded, b = nrad:
// as stored), element i at i + (i >> sh[b]); 31 is the plain layout.
struct RadixPlan {
    int n;
    int nrad;
    int r[FFT_MAX_RAD];
    int sh[FFT_MAX_RAD + 1];
};

static __device__ __forceinline__ float2 cmul(float2 a, float2 b) { return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
static __device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
static __device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// multiply by -j*s (s = +1 forward kernel e^{-j..}, s = -1 inverse)
template <int S>
static __device__ __forceinline__ float2 mul_mj(float2 a) { return S > 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x); }

// In-register DFT of size R with kernel exp(-S j 2 pi r q / R), S = +1 forward, -1 inverse.
template <int S>
static __device__ __forceinline__ void dft2(float2 *v)
{
    const float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}
template <int S>
static __device__ __forceinline__ void dft4(float2 *v)
{
    const float2 a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
    const float2 b0 = cadd(v[1], v[3]), b1 = mul_mj<S>(csub(v[1], v[3]));
    v[0] = cadd(a0, b0);
    v[2] = csub(a0, b0);
    v[1] = cadd(a1, b1);
    v[3] = csub(a1, b1);
}
template <int S>
static __device__ __forceinline__ void dft3(float2 *v)
{
    const float c1 = -0.5f, s1 = 0.86602540378443864676f * (float)S;  // sin(2pi/3), sign by direction
    const float2 t = cadd(v[1], v[2]);
    const float2 d = csub(v[1], v[2]);
    const float2 m = make_float2(v[0].x + c1 * t.x, v[0].y + c1 * t.y);
    // X1 = v0 + w v1 + w^2 v2, w = exp(-S j 2pi/3): X1 = m - j s1 d, X2 = m + j s1 d
    const float2 jd = make_float2(-s1 * d.y, s1 * d.x);
    v[0] = cadd(v[0], t);
    v[1] = csub(m, jd);
    v[2] = cadd(m, jd);
}
template <int S>
static __device__ __forceinline__ void dft5(float2 *v)
{
    const float c1 = 0.30901699437494742410f, c2 = -0.80901699437494742410f;   // cos(2pi/5), cos(4pi/5)
    const float s1 = 0.95105651629515357212f * (float)S, s2 = 0.58778525229247312917f * (float)S;  // sin(2pi/5), sin(4pi/5)
    const float2 t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    const float2 d1 = csub(v[1], v[4]), d2 = csub(v[2], v[3]);
    const float2 m1 = make_float2(v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y);
    const float2 m2 = make_float2(v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y);
    // j-rotated odd parts
    const float2 n1 = make_float2(s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y);
    const float2 n2 = make_float2(s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y);
    v[0] = cadd(v[0], cadd(t1, t2));
    // X_q = m_q - j n_q for q = 1, 2 ; X_{5-q} = m_q + j n_q
    v[1] = make_float2(m1.x + n1.y, m1.y - n1.x);
    v[4] = make_float2(m1.x - n1.y, m1.y + n1.x);
    v[2] = make_float2(m2.x + n2.y, m2.y - n2.x);
    v[3] = make_float2(m2.x - n2.y, m2.y + n2.x);
}
template <int S>
static __device__ __forceinline__ void dft8(float2 *v)
{
    const float h = 0.70710678118654752440f;
    // radix-2 first stage over pairs (r, r+4)
    float2 a[4], b[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        a[r] = cadd(v[r], v[r + 4]);
        b[r] = csub(v[r], v[r + 4]);
    }
    // twiddles exp(-S j 2 pi r / 8) on b
    b[1] = make_float2(h * (b[1].x + (float)S * b[1].y), h * (b[1].y - (float)S * b[1].x));
    b[2] = mul_mj<S>(b[2]);
    b[3] = make_float2(h * (-b[3].x + (float)S * b[3].y), h * (-b[3].y - (float)S * b[3].x));
    dft4<S>(a);
    dft4<S>(b);
    v[0] = a[0]; v[2] = a[1]; v[4] = a[2]; v[6] = a[3];
    v[1] = b[0]; v[3] = b[1]; v[5] = b[2]; v[7] = b[3];
}

// Composite radices 9 = 3 x 3, 15 = 3 x 5 and 16 = 4 x 4, one Cooley-Tukey step in registers:
// with n = R2 n1 + n2 and k = k1 + R1 k2, X[k] = DFT_R2 over n2 of W^(n2 k1) DFT_R1 over n1 of
// x[R2 n1 + n2], W = exp(-S j 2 pi / R).  TwR<R> holds cos and sin of 2 pi m / R.
template <int R> struct TwR;
template <> struct TwR<9> {
    static constexpr float c[9] = {1.0f, 0.76604444311897801f, 0.17364817766693041f, -0.5f, -0.93969262078590832f,
                                   -0.93969262078590843f, -0.5f, 0.17364817766692997f, 0.76604444311897779f};
    static constexpr float s[9] = {0.0f, 0.64278760968653925f, 0.98480775301220802f, 0.86602540378443871f,
                                   0.34202014332566888f, -0.34202014332566866f, -0.86602540378443837f,
                                   -0.98480775301220813f, -0.64278760968653958f};
};
template <> struct TwR<15> {
    static constexpr float c[15] = {1.0f, 0.91354545764260087f, 0.66913060635885824f, 0.30901699437494745f,
                                    -0.10452846326765333f, -0.5f, -0.80901699437494734f, -0.97814760073380569f,
                                    -0.97814760073380569f, -0.80901699437494756f, -0.5f, -0.10452846326765423f,
                                    0.30901699437494723f, 0.66913060635885846f, 0.91354545764260098f};
    static constexpr float s[15] = {0.0f, 0.40673664307580015f, 0.74314482547739413f, 0.95105651629515353f,
                                    0.9945218953682734f, 0.86602540378443871f, 0.58778525229247325f,
                                    0.20791169081775931f, -0.20791169081775907f, -0.58778525229247303f,
                                    -0.86602540378443837f, -0.99452189536827329f, -0.95105651629515364f,
                                    -0.74314482547739402f, -0.40673664307580015f};
};
template <> struct TwR<16> {
    static constexpr float c[16] = {1.0f, 0.92387953251128674f, 0.70710678118654757f, 0.38268343236508984f, 0.0f,
                                    -0.38268343236508973f, -0.70710678118654746f, -0.92387953251128674f, -1.0f,
                                    -0.92387953251128685f, -0.70710678118654768f, -0.38268343236509034f, 0.0f,
                                    0.38268343236509f, 0.70710678118654735f, 0.92387953251128652f};
    static constexpr float s[16] = {0.0f, 0.38268343236508978f, 0.70710678118654746f, 0.92387953251128674f, 1.0f,
                                    0.92387953251128674f, 0.70710678118654757f, 0.38268343236508989f, 0.0f,
                                    -0.38268343236508967f, -0.70710678118654746f, -0.92387953251128652f, -1.0f,
                                    -0.92387953251128663f, -0.70710678118654768f, -0.38268343236509039f};
};

template <int S, int R> static __device__ __forceinline__ void dftR(float2 *v);

template <int S, int R1, int R2>
static __device__ __forceinline__ void dft_ct(float2 *v)
{
    constexpr int R = R1 * R2;
    float2 a[R2][R1];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1) a[n2][n1] = v[R2 * n1 + n2];
        dftR<S, R1>(a[n2]);
    }
#pragma unroll
    for (int n2 = 1; n2 < R2; ++n2)
#pragma unroll
        for (int k1 = 1; k1 < R1; ++k1) {
            const int m = n2 * k1;
            a[n2][k1] = cmul(a[n2][k1], make_float2(TwR<R>::c[m], -(float)S * TwR<R>::s[m]));
        }
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
        float2 t[R2];
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) t[n2] = a[n2][k1];
        dftR<S, R2>(t);
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = t[k2];
    }
}

template <int S, int R>
static __device__ __forceinline__ void dftR(float2 *v)
{
    if constexpr (R == 2) dft2<S>(v);
    else if constexpr (R == 3) dft3<S>(v);
    else if constexpr (R == 4) dft4<S>(v);
    else if constexpr (R == 5) dft5<S>(v);
    else if constexpr (R == 8) dft8<S>(v);
    else if constexpr (R == 9) dft_ct<S, 3, 3>(v);
    else if constexpr (R == 15) dft_ct<S, 3, 5>(v);
    else if constexpr (R == 16) dft_ct<S, 4, 4>(v);
}

// j / d for j < 2^16 and 2 <= d <= 2^14: with m = floor((2^32 - 1) / d) + 1, umulhi(j, m) = j / d
// exactly (the error j (m - 2^32/d) / 2^32 < 2^-16 is below the smallest non-zero fraction 1/d).
// (d = 1 would need m = 2^32; callers handle it.)
static __device__ __forceinline__ int div_small(int j, uint32_t m) { return (int)__umulhi((uint32_t)j, m); }

// Row transforms keep one row in ONE LDS buffer and run each Stockham pass in place: every
// thread reads the inputs of its butterflies into registers, the work-group synchronises,
// then every thread writes its outputs.  NPT bounds the row elements per thread
// (n <= NPT * FFT_THREADS), so a radix-R pass holds at most ceil(NPT / R) butterflies per
// thread; one buffer and few registers let eight work-groups share a CU.
//
// Layouts.  Between two passes element i sits at i + (i >> s): one element of padding every
// 2^s spreads the early passes' strided stores over the banks.  The host picks s per pass
// boundary (make_radix) so that a butterfly's R inputs j + r nb, and its R outputs
// o + r Ns, stay evenly spaced in LDS: each element then costs one add of a uniform offset
// instead of a shift, an add and a multiply.
static __device__ __forceinline__ int lds_at(int i, int s) { return i + (i >> s); }
constexpr int FFT_MIN_PAD_SHIFT = 3;  // padding at most every 8 elements
static __host__ __device__ constexpr int lds_padded_len(int n) { return n + (n >> FFT_MIN_PAD_SHIFT) + 1; }

// tw + off bytes: a 32-bit offset from the table's uniform base
static __device__ __forceinline__ float2 tw_at(const float2 *tw, uint32_t off)
{
    return *reinterpret_cast<const float2 *>(reinterpret_cast<const char *>(tw) + off);
}

// Twiddles of a butterfly: only W^1, W^2, W^4, W^8 (those below R) are fetched, before the
// barrier; W^r for other r is the product of the fetched powers in r's binary expansion (at
// most three complex products, a few ulp).  Fewer registers held across the barrier let more
// rows share a CU (59 VGPRs instead of 71 with all R - 1 fetched: eight rows per CU, not seven).
template <int R> struct TwPow {
    static constexpr int NP = R <= 2 ? 1 : (R <= 4 ? 2 : (R <= 8 ? 3 : 4));
};
template <int R>
static __device__ __forceinline__ void twiddle_powers(const float2 *wp, float2 *wr)
{
#pragma unroll
    for (int r = 1; r < R; ++r) {
        const int hb = 1 << (31 - __builtin_clz(r));
        if (hb == r) wr[r] = wp[__builtin_ctz(r)];
        else wr[r] = cmul(wr[hb], wr[r - hb]);
    }
}

template <int R, int S, int NPT>
static __device__ __forceinline__ void row_pass_inplace(float2 *buf, int n, int Ns, const float2 *__restrict__ tw,
                                                        int tid, int sr, int sw)
{
    constexpr int KB = (NPT + R - 1) / R;
    constexpr int NW = TwPow<R>::NP;
    asm volatile("" : "+v"(tid));  // addresses formed per pass, not hoisted out of the pass loop
    const int nb = n / R, tstep = n / (Ns * R);
    const int rstr = nb + (nb >> sr), wstr = Ns + (Ns >> sw);
    const uint32_t mNs = Ns > 1 ? 0xffffffffu / (uint32_t)Ns + 1u : 0u;  // Ns = 1: quotient is j itself
    float2 v[KB][R], w[KB][NW];
    int o[KB];
    // the twiddles are fetched from memory before the barrier, so their latency overlaps it
#pragma unroll
    for (int q = 0; q < KB; ++q) {
        const int j = tid + q * FFT_THREADS;
        o[q] = 0;
        if (j < nb) {
            const int jq = Ns > 1 ? div_small(j, mNs) : j, k = j - jq * Ns;
            o[q] = jq * Ns * R + k;
            const uint32_t kt8 = (uint32_t)(k * tstep) * 8u;  // < 8 n / R: 24 bits
#pragma unroll
            for (int i = 0; i < NW; ++i)
                w[q][i] = tw_at(tw, __umul24(1u << i, kt8));
            const int a = lds_at(j, sr);
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = buf[a + r * rstr];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < KB; ++q) {
        const int j = tid + q * FFT_THREADS;
        if (j < nb) {
            float2 wr[R];
            twiddle_powers<R>(w[q], wr);
#pragma unroll
            for (int r = 1; r < R; ++r) {
                float2 t = wr[r];
                if (S < 0) t.y = -t.y;
                v[q][r] = cmul(v[q][r], t);
            }
            dftR<S, R>(v[q]);
            const int a = lds_at(o[q], sw);
#pragma unroll
            for (int r = 0; r < R; ++r) buf[a + r * wstr] = v[q][r];
        }
    }
    __syncthreads();
}

template <int S, int NPT>
static __device__ void fft_row_lds(float2 *buf, const RadixPlan &pl, const float2 *__restrict__ tw)
{
    int Ns = 1;
    for (int p = 0; p < pl.nrad; ++p) {
        const int R = pl.r[p], sr = pl.sh[p], sw = pl.sh[p + 1];
        switch (R) {
        case 2: row_pass_inplace<2, S, NPT>(buf, pl.n, Ns, tw, threadIdx.x, sr, sw); break;
        case 3: row_pass_inplace<3, S, NPT>(buf, pl.n, Ns, tw, threadIdx.x, sr, sw); break;
        case 4: row_pass_inplace<4, S, NPT>(buf, pl.n, Ns, tw, threadIdx.x, sr, sw); break;
        case 5: row_pass_inplace<5, S, NPT>(buf, pl.n, Ns, tw, threadIdx.x, sr, sw); break;
        case 9: row_pass_inplace<9, S, NPT>(buf, pl.n, Ns, tw, threadIdx.x, sr, sw); break;
        case 15: row_pass_inplace<15, S, NPT>(buf, pl.n, Ns, tw, threadIdx.x, sr, sw); break;
        case 16: row_pass_inplace<16, S, NPT>(buf, pl.n, Ns, tw, threadIdx.x, sr, sw); break;
        default: row_pass_inplace<8, S, NPT>(buf, pl.n, Ns, tw, threadIdx.x, sr, sw); break;
        }
        Ns *= R;
    }
}

// Position d of index v inside the periodic window w = (start, len) of an axis of length n;
// inside when d < len.  Both v and the start lie in [0, n).
static __device__ __forceinline__ int win_pos(int v, int2 w, int n)
{
    const int d = v - w.x;
    return d < 0 ? d + n : d;
}
// A window is one or two periodic intervals (x, y) and (z, w) as (start, length); an unused
// second interval has length 0.  v lies in [0, n).
static __device__ __forceinline__ bool in_win(int v, int4 w, int n)
{
    return win_pos(v, make_int2(w.x, w.y), n) < w.y || win_pos(v, make_int2(w.z, w.w), n) < w.w;
}
// Does any of the b indexes v0 .. v0 + b - 1 lie in the interval (start, len)?
static __device__ __forceinline__ bool interval_meets(int v0, int b, int start, int len, int n)
{
    const int d = win_pos(v0, make_int2(start, len), n);
    return len > 0 && (d < len || d + b > n);
}

// Row transforms: one row per work-group.  in/out: [rows][n].  With colin, each image's
// input is nonzero only in its window of columns: the others are read as zero, not loaded.
// With colout, only each image's window of columns is stored.
template <int S, int NPT>
__global__ void __launch_bounds__(FFT_THREADS) k_fft_rows(const float2 *__restrict__ in, float2 *__restrict__ out,
                                                          RadixPlan pl, const float2 *__restrict__ tw,
                                                          const int4 *__restrict__ colin,
                                                          const int4 *__restrict__ colout, int rows_per_img)
{
    extern __shared__ float2 lds[];
    const int64_t row = blockIdx.x;
    const int n = pl.n;
    const float2 *src = in + row * n;
    float2 *dst = out + row * n;
    const int s0 = pl.sh[0], s1 = pl.sh[pl.nrad];
    const int4 wi = colin ? colin[row / rows_per_img] : make_int4(0, n, 0, 0);
    const int4 wo = colout ? colout[row / rows_per_img] : make_int4(0, n, 0, 0);
    // Rows are moved two elements (16 bytes) per access when both ends are 16-byte aligned
    // (n is even): elements i and i + 1 of an even i are adjacent in every layout (padding
    // comes at most every 8 elements).
    if ((((uintptr_t)in | (uintptr_t)out) & 15) == 0) {
        const float4 *src4 = reinterpret_cast<const float4 *>(src);
        for (int i = 2 * threadIdx.x; i < n; i += 2 * FFT_THREADS) {
            const bool l0 = in_win(i, wi, n), l1 = in_win(i + 1, wi, n);
            float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (l0 || l1) v = src4[i >> 1];
            const int a = lds_at(i, s0);
            lds[a] = l0 ? make_float2(v.x, v.y) : make_float2(0.0f, 0.0f);
            lds[a + 1] = l1 ? make_float2(v.z, v.w) : make_float2(0.0f, 0.0f);
        }
        __syncthreads();
        fft_row_lds<S, NPT>(lds, pl, tw);
        float4 *dst4 = reinterpret_cast<float4 *>(dst);
        for (int i = 2 * threadIdx.x; i < n; i += 2 * FFT_THREADS) {
            const int a = lds_at(i, s1);
            const float2 v0 = lds[a], v1 = lds[a + 1];
            const bool l0 = in_win(i, wo, n), l1 = in_win(i + 1, wo, n);
            if (l0 && l1) dst4[i >> 1] = make_float4(v0.x, v0.y, v1.x, v1.y);
            else if (l0) dst[i] = v0;
            else if (l1) dst[i + 1] = v1;
        }
    } else {
        for (int i = threadIdx.x; i < n; i += FFT_THREADS)
            lds[lds_at(i, s0)] = in_win(i, wi, n) ? src[i] : make_float2(0.0f, 0.0f);
        __syncthreads();
        fft_row_lds<S, NPT>(lds, pl, tw);
        for (int i = threadIdx.x; i < n; i += FFT_THREADS)
            if (in_win(i, wo, n)) dst[i] = lds[lds_at(i, s1)];
    }
}

// Column transforms.  A work-group of FFT_COL_THREADS owns columns [c0, c0 + B) of one image
// [n][width] and keeps them in ONE LDS buffer laid out [n][B], so the global reads and writes
// are contiguous row segments and a butterfly's R inputs of column c sit B apart (consecutive
// threads take consecutive columns: no bank conflicts).  Each Stockham pass runs in place:
// every thread first reads the inputs of its (at most KMAX) butterflies into registers, the
// work-group synchronises, then every thread writes its outputs.  The twiddle table sits in
// LDS after the data.  Two LDS budgets: 80 KB (B <= 8 columns, two work-groups per CU, so
// one's loads and stores overlap the other's passes) where B >= 4 fits, else 160 KB.
constexpr int FFT_COL_THREADS = 512;
constexpr int FFT_COL_LDS_SMALL = 80 * 1024, FFT_COL_LDS_BIG = 160 * 1024;

template <int R, int LDSB>
struct ColK {
    static constexpr int KMAX = (LDSB / 8 / R + FFT_COL_THREADS - 1) / FFT_COL_THREADS;
};


template <int R, int S, int LDSB>
static __device__ __forceinline__ void stockham_pass_inplace(float2 *buf, int n, int lb, int Ns, const float2 *tw,
                                                             int tid)
{
    constexpr int KMAX = ColK<R, LDSB>::KMAX;
    // an opaque copy of the thread index: the addresses below are then formed in each pass
    // instead of being hoisted out of the pass loop for every radix (which spills them)
    asm volatile("" : "+v"(tid));
    const int B = 1 << lb, nb = n / R, total = nb << lb, tstep = n / (Ns * R);
    const int rstr = nb << lb, wstr = Ns << lb;  // a butterfly's elements are evenly spaced
    const uint32_t mNs = Ns > 1 ? 0xffffffffu / (uint32_t)Ns + 1u : 0u;  // Ns = 1: quotient is j itself
    float2 v[KMAX][R];
#pragma unroll
    for (int q = 0; q < KMAX; ++q) {
        const int idx = tid + q * FFT_COL_THREADS;
        if (idx < total) {
            const int a = idx;  // (j << lb) + c with j = idx >> lb, c = idx & (B - 1)
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = buf[a + r * rstr];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < KMAX; ++q) {
        const int idx = tid + q * FFT_COL_THREADS;
        if (idx < total) {
            const int j = idx >> lb, c = idx & (B - 1);
            const int jq = Ns > 1 ? div_small(j, mNs) : j, k = j - jq * Ns;
            const uint32_t kt8 = (uint32_t)(k * tstep) * 8u;  // < 8 n / R: 24 bits
#pragma unroll
            for (int r = 1; r < R; ++r) {
                float2 w = tw_at(tw, __umul24((uint32_t)r, kt8));
                if (S < 0) w.y = -w.y;
                v[q][r] = cmul(v[q][r], w);
            }
            dftR<S, R>(v[q]);
            const int a = ((jq * Ns * R + k) << lb) + c;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[a + r * wstr] = v[q][r];
        }
    }
    __syncthreads();
}

// Work-groups are dispatched to the 8 XCDs round robin (block i to XCD i mod 8).  Renumber them
// so that each XCD takes one contiguous range of slabs: neighbouring slabs, which share cache
// lines when B < 16, then meet in the same L2.
static __device__ __forceinline__ int xcd_contiguous(int i, int G)
{
    const int x = i & 7, j = i >> 3, q = G >> 3, r = G & 7;
    return x * q + min(x, r) + j;
}

// With INTENSITY the results are not stored: |x|^2 goes to outf (float, same indexing).
template <int S, bool INTENSITY, int LDSB>
__global__ void __launch_bounds__(FFT_COL_THREADS, LDSB == FFT_COL_LDS_SMALL ? 4 : 2) k_fft_cols(const float2 *__restrict__ in, float2 *__restrict__ out,
                                                              RadixPlan pl, const float2 *__restrict__ tw, int width,
                                                              int lb, const int4 *__restrict__ colwin,
                                                              float *__restrict__ outf,
                                                              const int4 *__restrict__ rowin)
{
    extern __shared__ float2 lds[];
    const int n = pl.n, B = 1 << lb;
    const int blk = xcd_contiguous(blockIdx.x, gridDim.x);
    const int nslab = (width + B - 1) / B;
    const int64_t img = blk / nslab;
    const int c0 = (blk - (int)(img * nslab)) * B;
    // colwin: only the slabs meeting each image's window of columns are transformed, and only
    // the window's columns are loaded (the others are read as zero) and stored.  rowin (input
    // support): the image is zero outside the rectangles colwin.xy x rowin.xy and
    // colwin.zw x rowin.zw, whose outside is not loaded.
    if (colwin) {
        const int4 w = colwin[img];
        if (!interval_meets(c0, B, w.x, w.y, width) && !interval_meets(c0, B, w.z, w.w, width)) return;
    }
    float2 *tw_s = lds + n * B;  // the twiddle table, read by every pass
    for (int i = threadIdx.x; i < n; i += FFT_COL_THREADS) tw_s[i] = tw[i];
    const int bw = min(B, width - c0);
    const float2 *src = in + img * (int64_t)n * width;
    float2 *dst = out + img * (int64_t)n * width;
    const int4 wc = colwin ? colwin[img] : make_int4(0, width, 0, 0);
    if (colwin) {
        const int4 wr = rowin ? rowin[img] : make_int4(0, n, 0, n);
        for (int i = threadIdx.x; i < n * B; i += FFT_COL_THREADS) {
            const int r = i >> lb, c = i & (B - 1), v = c0 + c;
            const bool live = c < bw && ((win_pos(v, make_int2(wc.x, wc.y), width) < wc.y &&
                                          win_pos(r, make_int2(wr.x, wr.y), n) < wr.y) ||
                                         (win_pos(v, make_int2(wc.z, wc.w), width) < wc.w &&
                                          win_pos(r, make_int2(wr.z, wr.w), n) < wr.w));
            lds[i] = live ? src[(int64_t)r * width + c0 + c] : make_float2(0.0f, 0.0f);
        }
    } else {
        for (int i = threadIdx.x; i < n * B; i += FFT_COL_THREADS) {
            const int r = i >> lb, c = i & (B - 1);
            lds[i] = c < bw ? src[(int64_t)r * width + c0 + c] : make_float2(0.0f, 0.0f);
        }
    }
    __syncthreads();
    int Ns = 1;
    for (int p = 0; p < pl.nrad; ++p) {
        const int R = pl.r[p];
        switch (R) {
        case 2: stockham_pass_inplace<2, S, LDSB>(lds, n, lb, Ns, tw_s, threadIdx.x); break;
        case 3: stockham_pass_inplace<3, S, LDSB>(lds, n, lb, Ns, tw_s, threadIdx.x); break;
        case 4: stockham_pass_inplace<4, S, LDSB>(lds, n, lb, Ns, tw_s, threadIdx.x); break;
        case 5: stockham_pass_inplace<5, S, LDSB>(lds, n, lb, Ns, tw_s, threadIdx.x); break;
        case 9: stockham_pass_inplace<9, S, LDSB>(lds, n, lb, Ns, tw_s, threadIdx.x); break;
        case 15: stockham_pass_inplace<15, S, LDSB>(lds, n, lb, Ns, tw_s, threadIdx.x); break;
        case 16: stockham_pass_inplace<16, S, LDSB>(lds, n, lb, Ns, tw_s, threadIdx.x); break;
        default: stockham_pass_inplace<8, S, LDSB>(lds, n, lb, Ns, tw_s, threadIdx.x); break;
        }
        Ns *= R;
    }
    if (INTENSITY) {
        float *dstf = outf + img * (int64_t)n * width;
        for (int i = threadIdx.x; i < n * B; i += FFT_COL_THREADS) {
            const int r = i >> lb, c = i & (B - 1);
            const float2 v = lds[i];
            if (c < bw && in_win(c0 + c, wc, width)) dstf[(int64_t)r * width + c0 + c] = fmaf(v.x, v.x, v.y * v.y);
        }
    } else {
        for (int i = threadIdx.x; i < n * B; i += FFT_COL_THREADS) {
            const int r = i >> lb, c = i & (B - 1);
            if (c < bw && in_win(c0 + c, wc, width)) dst[(int64_t)r * width + c0 + c] = lds[i];
        }
    }
}

// Focal stack, row pass.  One work-group per (wavelength c, spectrum row y) reads the row of
// the forward spectrum DFT(u) once, forms per element the angular-spectrum phase
// d_c(nu) = sqrt(1/lambda_c^2 - |nu|^2) - 1/lambda_c = -|nu|^2 / (1/lambda_c + sqrt(...))
// in FP64 (Eq. 4 without cancellation), and then for every plane k multiplies the row by
// H(nu, z_k) = exp(j 2 pi (frac(z_k / lambda_c) + z_k d_c(nu))) (zero outside the propagating
// band and, with the half-band filter, outside |m'_x| < N_x / 4, |m'_y| < N_y / 4), times the
// 1 / (N_x N_y) of the inverse, transforms it and stores it to plane k.
constexpr int STACK_MAXPT = 16;  // row elements per thread: N_x <= 16 * FFT_THREADS
template <int S, int NPT>
__global__ void __launch_bounds__(FFT_THREADS) k_fft_rows_stack(const float2 *__restrict__ spec,
                                                                float2 *__restrict__ planes, RadixPlan pl,
                                                                const float2 *__restrict__ tw, StackArgs sa)
{
    extern __shared__ float2 lds[];
    const int nx = pl.n, ny = sa.ny;
    const int row = blockIdx.x, c = row / ny, y = row - c * ny;
    const int myp = y < ny / 2 ? y : y - ny;
    const double nuy = (double)myp * sa.dnuy, il = sa.inv_l[c];
    const bool yin = !sa.half_band || 4 * abs(myp) < ny;
    float2 sv[NPT];
    double dv[NPT];
    bool keep[NPT];
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
        const int i = threadIdx.x + j * FFT_THREADS;
        sv[j] = make_float2(0.0f, 0.0f);
        dv[j] = 0.0;
        keep[j] = false;
        if (i < nx) {
            const int mxp = i < nx / 2 ? i : i - nx;
            const double nux = (double)mxp * sa.dnux;
            const double nu2 = fma(nux, nux, nuy * nuy);
            const double w2 = fma(il, il, -nu2);
            keep[j] = w2 > 0.0 && yin && (!sa.half_band || 4 * abs(mxp) < nx);
            if (keep[j]) {
                dv[j] = -nu2 / (il + sqrt(w2));
                sv[j] = spec[(int64_t)row * nx + i];
            }
        }
    }
    for (int k = 0; k < sa.K; ++k) {
        const double zk = sa.z[k], pk = sa.piston[k * STACK_MAXC + c];
#pragma unroll
        for (int j = 0; j < NPT; ++j) {
            const int i = threadIdx.x + j * FFT_THREADS;
            if (i < nx) {
                float2 v = make_float2(0.0f, 0.0f);
                if (keep[j]) {
                    double t = fma(zk, dv[j], pk);
                    t -= floor(t);
                    const float th = (float)t;
                    const float cs = __builtin_amdgcn_cosf(th) * sa.scale, sn = __builtin_amdgcn_sinf(th) * sa.scale;
                    v = make_float2(sv[j].x * cs - sv[j].y * sn, sv[j].x * sn + sv[j].y * cs);
                }
                lds[lds_at(i, pl.sh[0])] = v;
            }
        }
        __syncthreads();
        fft_row_lds<S, NPT>(lds, pl, tw);
        float2 *dst = planes + ((int64_t)(k * sa.C + c) * ny + y) * nx;
        for (int i = threadIdx.x; i < nx; i += FFT_THREADS) dst[i] = lds[lds_at(i, pl.sh[pl.nrad])];
        __syncthreads();
    }
}

// The layout shift of each pass boundary b: the padding period P = 2^s must keep the outputs
// of pass b - 1 evenly spaced (Ns a multiple of P, or the whole span Ns R of a butterfly
// inside one period) and the inputs of pass b (n / R a multiple of P).  P = 16 is preferred
// (it spreads a stride-16 store over the banks), then 8, else the plain layout.
static RadixPlan make_radix(int n, const int32_t *r, int nrad)
{
    RadixPlan p;
    p.n = n;
    p.nrad = nrad;
    for (int i = 0; i < FFT_MAX_RAD; ++i) p.r[i] = i < nrad ? r[i] : 0;
    int Ns = 1;  // at boundary b >= 1: Ns of pass b - 1, the product r[0] ... r[b - 2]
    for (int b = 0; b <= nrad; ++b) {
        p.sh[b] = 31;
        for (const int s : {4, FFT_MIN_PAD_SHIFT}) {
            const int P = 1 << s;
            const bool wr_ok = b == 0 || Ns % P == 0 || P % (Ns * r[b - 1]) == 0;
            const bool rd_ok = b == nrad || (n / r[b]) % P == 0;
            if (wr_ok && rd_ok) {
                p.sh[b] = s;
                break;
            }
        }
        if (b >= 1) Ns *= r[b - 1];
    }
    for (int b = nrad + 1; b <= FFT_MAX_RAD; ++b) p.sh[b] = 31;
    return p;
}

// Columns per work-group and LDS budget for columns of length n: the largest B <= 8 with the
// B n data and the n twiddles in 80 KB if that B is at least 4, else the largest B <= 16 in
// 160 KB (B = 1 fits up to n = 8192).
struct ColCfg {
    int B, lb, ldsb;
};
static ColCfg col_config(int n)
{
    ColCfg c{8, 0, FFT_COL_LDS_SMALL};
    while (c.B > 1 && (int64_t)(c.B + 1) * n * 8 > FFT_COL_LDS_SMALL) c.B >>= 1;
    if (c.B < 4) {
        c.B = 16;
        c.ldsb = FFT_COL_LDS_BIG;
        while (c.B > 1 && (int64_t)(c.B + 1) * n * 8 > FFT_COL_LDS_BIG) c.B >>= 1;
    }
    while ((1 << c.lb) < c.B) ++c.lb;
    return c;
}

int fft_col_batch(int n) { return col_config(n).B; }

template <int S, bool INTENSITY>
static void set_col_lds()
{
    hipFuncSetAttribute((const void *)k_fft_cols<S, INTENSITY, FFT_COL_LDS_SMALL>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, FFT_COL_LDS_SMALL);
    hipFuncSetAttribute((const void *)k_fft_cols<S, INTENSITY, FFT_COL_LDS_BIG>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, FFT_COL_LDS_BIG);
}

static void allow_big_lds()
{
    static bool done = false;
    if (done) return;
    const int lim = 160 * 1024;
    set_col_lds<1, false>();
    set_col_lds<-1, false>();
    set_col_lds<-1, true>();
    hipFuncSetAttribute((const void *)k_fft_rows<1, 32>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    hipFuncSetAttribute((const void *)k_fft_rows<-1, 32>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    done = true;
}

// Row passes: the smallest elements-per-thread bound that covers n.
template <int S>
static void rows_launch(const Plan &p, const RadixPlan &px, int rows, const float2 *src, float2 *dst,
                        const int4 *colin, hipStream_t s, const int4 *colout = nullptr)
{
    const size_t lds = (size_t)lds_padded_len(p.nx) * sizeof(float2);
    const int npt = (p.nx + FFT_THREADS - 1) / FFT_THREADS;
    const dim3 g(rows), b(FFT_THREADS);
    if (npt <= 2)
        hipLaunchKernelGGL((k_fft_rows<S, 2>), g, b, lds, s, src, dst, px, p.tw_x, colin, colout, p.ny);
    else if (npt <= 4)
        hipLaunchKernelGGL((k_fft_rows<S, 4>), g, b, lds, s, src, dst, px, p.tw_x, colin, colout, p.ny);
    else if (npt <= 8)
        hipLaunchKernelGGL((k_fft_rows<S, 8>), g, b, lds, s, src, dst, px, p.tw_x, colin, colout, p.ny);
    else if (npt <= 16)
        hipLaunchKernelGGL((k_fft_rows<S, 16>), g, b, lds, s, src, dst, px, p.tw_x, colin, colout, p.ny);
    else
        hipLaunchKernelGGL((k_fft_rows<S, 32>), g, b, lds, s, src, dst, px, p.tw_x, colin, colout, p.ny);
}

// One column pass over nimg images [ny][nx] in place (or, with intensity, |x|^2 to it).
template <int S, bool INTENSITY>
static void cols_launch(const Plan &p, const RadixPlan &py, int nimg, float2 *buf, const int4 *colwin, float *outf,
                        hipStream_t s, const int4 *rowin = nullptr)
{
    const ColCfg c = col_config(p.ny);
    const size_t lds = (size_t)(c.B + 1) * p.ny * sizeof(float2);
    const int nslab = (p.nx + c.B - 1) / c.B;
    const dim3 grid(nimg * nslab), block(FFT_COL_THREADS);
    if (c.ldsb == FFT_COL_LDS_SMALL)
        hipLaunchKernelGGL((k_fft_cols<S, INTENSITY, FFT_COL_LDS_SMALL>), grid, block, lds, s, buf, buf, py, p.tw_y,
                           p.nx, c.lb, colwin, outf, rowin);
    else
        hipLaunchKernelGGL((k_fft_cols<S, INTENSITY, FFT_COL_LDS_BIG>), grid, block, lds, s, buf, buf, py, p.tw_y,
                           p.nx, c.lb, colwin, outf, rowin);
}

hipError_t launch_fft2d(const Plan &p, int batch, int direction, const float2 *in, float2 *out, hipStream_t s)
{
    return launch_fft2d_win(p, batch, direction, in, out, nullptr, nullptr, s);
}

// Rows then columns.  With windows, the input of each image is nonzero only inside its
// rectangles colwin.xy x rowwin.xy and colwin.zw x rowwin.zw (rowwin may be NULL: all rows):
// columns first, only colwin's columns, loading only the rectangles; then every row, loading
// only colwin's columns (what lies outside the rectangles is never read, so it need not be
// zero).  In place.
hipError_t launch_fft2d_win(const Plan &p, int batch, int direction, const float2 *in, float2 *out,
                            const int4 *colwin, const int4 *rowwin, hipStream_t s)
{
    allow_big_lds();
    const RadixPlan px = make_radix(p.nx, p.radix_x, p.nrad_x);
    const RadixPlan py = make_radix(p.ny, p.radix_y, p.nrad_y);
    const int rows = batch * p.ny;
    if (!colwin && rowwin) return hipErrorInvalidValue;
    if (colwin && in != out) return hipErrorInvalidValue;  // the windowed form works in place
    if (colwin) {
        if (direction > 0) {
            cols_launch<-1, false>(p, py, batch, out, colwin, nullptr, s, rowwin);
            rows_launch<-1>(p, px, rows, out, out, colwin, s);
        } else {
            cols_launch<1, false>(p, py, batch, out, colwin, nullptr, s, rowwin);
            rows_launch<1>(p, px, rows, out, out, colwin, s);
        }
    } else if (direction > 0) {
        rows_launch<-1>(p, px, rows, in, out, nullptr, s);
        cols_launch<-1, false>(p, py, batch, out, nullptr, nullptr, s);
    } else {
        rows_launch<1>(p, px, rows, in, out, nullptr, s);
        cols_launch<1, false>(p, py, batch, out, nullptr, nullptr, s);
    }
    return hipGetLastError();
}

// Rows first over every row, storing only colwin's columns, then only those columns (the
// output is wanted only there; the others are left unfinished).  In place.
hipError_t launch_fft2d_cols_out(const Plan &p, int batch, int direction, float2 *buf, const int4 *colwin,
                                 hipStream_t s)
{
    allow_big_lds();
    const RadixPlan px = make_radix(p.nx, p.radix_x, p.nrad_x);
    const RadixPlan py = make_radix(p.ny, p.radix_y, p.nrad_y);
    if (direction > 0) {
        rows_launch<-1>(p, px, batch * p.ny, buf, buf, nullptr, s, colwin);
        cols_launch<-1, false>(p, py, batch, buf, colwin, nullptr, s);
    } else {
        rows_launch<1>(p, px, batch * p.ny, buf, buf, nullptr, s, colwin);
        cols_launch<1, false>(p, py, batch, buf, colwin, nullptr, s);
    }
    return hipGetLastError();
}

bool focal_stack_fits(int nx) { return nx <= STACK_MAXPT * FFT_THREADS; }

// The inverse transforms of sa.K planes: the row pass forms and transforms every plane from
// the spectrum, then the column pass either finishes them in place (intensity == nullptr)
// or writes |u|^2 of each to `intensity`.
hipError_t launch_focal_stack(const Plan &p, const float2 *spec, float2 *planes, float *intensity,
                              const StackArgs &sa, hipStream_t s)
{
    if (sa.K <= 0) return hipSuccess;
    if (!focal_stack_fits(p.nx) || sa.K > STACK_MAXK || sa.C > STACK_MAXC) return hipErrorInvalidValue;
    allow_big_lds();
    const RadixPlan px = make_radix(p.nx, p.radix_x, p.nrad_x);
    const RadixPlan py = make_radix(p.ny, p.radix_y, p.nrad_y);
    const size_t row_lds = (size_t)lds_padded_len(p.nx) * sizeof(float2);
    const int npt = (p.nx + FFT_THREADS - 1) / FFT_THREADS;
    const dim3 g(sa.C * p.ny), b(FFT_THREADS);
    if (npt <= 2)
        hipLaunchKernelGGL((k_fft_rows_stack<-1, 2>), g, b, row_lds, s, spec, planes, px, p.tw_x, sa);
    else if (npt <= 4)
        hipLaunchKernelGGL((k_fft_rows_stack<-1, 4>), g, b, row_lds, s, spec, planes, px, p.tw_x, sa);
    else if (npt <= 8)
        hipLaunchKernelGGL((k_fft_rows_stack<-1, 8>), g, b, row_lds, s, spec, planes, px, p.tw_x, sa);
    else
        hipLaunchKernelGGL((k_fft_rows_stack<-1, STACK_MAXPT>), g, b, row_lds, s, spec, planes, px, p.tw_x, sa);
    if (intensity)
        cols_launch<-1, true>(p, py, sa.K * sa.C, planes, nullptr, intensity, s);
    else
        cols_launch<-1, false>(p, py, sa.K * sa.C, planes, nullptr, nullptr, s);
    return hipGetLastError();
}

}  // namespace gws
