// Mixed-radix (2, 3, 4, 5, 8) Stockham FFT in LDS for gfx950: the one inverse 2D transform
// that brings the accumulated spectrum to the SLM plane (supplement Alg. 1 and Alg. 4, last
// step), and the forward transform the adjoint needs.  Unnormalised:
//   direction +1:  out[n] = sum_m in[m] exp(+j 2 pi m n / N)
//   direction -1:  out[n] = sum_m in[m] exp(-j 2 pi m n / N)
// Pass 1 transforms rows (one row per work-group); pass 2 transforms columns, a slab of
// B adjacent columns per work-group, read and written as whole-cache-line row segments.
// Twiddles come from per-size FP32 tables computed on the host in FP64.
#include "gws_internal.h"

namespace gws {

constexpr int FFT_THREADS = 256;
constexpr int FFT_MAX_RAD = 16;

struct RadixPlan {
    int n;
    int nrad;
    int r[FFT_MAX_RAD];
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

// One Stockham pass of radix R over `nb = n/R` butterflies for each of `batch` transforms
// stored contiguously (stride n) in src; result into dst.
template <int R, int S>
static __device__ __forceinline__ void stockham_pass(const float2 *src, float2 *dst, int n, int batch, int Ns,
                                                     const float2 *__restrict__ tw, int tid, int nthr)
{
    const int nb = n / R;
    const int total = nb * batch;
    const int tstep = n / (Ns * R);
    for (int idx = tid; idx < total; idx += nthr) {
        const int b = idx / nb, j = idx - b * nb;
        const float2 *s = src + b * n;
        float2 *d = dst + b * n;
        const int k = j % Ns;
        float2 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = s[j + r * nb];
#pragma unroll
        for (int r = 1; r < R; ++r) {
            float2 w = tw[r * k * tstep];
            if (S < 0) w.y = -w.y;
            v[r] = cmul(v[r], w);
        }
        if (R == 2) dft2<S>(v);
        if (R == 3) dft3<S>(v);
        if (R == 4) dft4<S>(v);
        if (R == 5) dft5<S>(v);
        if (R == 8) dft8<S>(v);
        const int o = (j / Ns) * Ns * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) d[o + r * Ns] = v[r];
    }
}

// Runs all passes; returns which buffer (0: a, 1: b) holds the result.
template <int S>
static __device__ int fft_lds(float2 *a, float2 *b, const RadixPlan &pl, int batch, const float2 *__restrict__ tw)
{
    int Ns = 1, cur = 0;
    for (int p = 0; p < pl.nrad; ++p) {
        const int R = pl.r[p];
        float2 *src = cur ? b : a, *dst = cur ? a : b;
        switch (R) {
        case 2: stockham_pass<2, S>(src, dst, pl.n, batch, Ns, tw, threadIdx.x, blockDim.x); break;
        case 3: stockham_pass<3, S>(src, dst, pl.n, batch, Ns, tw, threadIdx.x, blockDim.x); break;
        case 4: stockham_pass<4, S>(src, dst, pl.n, batch, Ns, tw, threadIdx.x, blockDim.x); break;
        case 5: stockham_pass<5, S>(src, dst, pl.n, batch, Ns, tw, threadIdx.x, blockDim.x); break;
        default: stockham_pass<8, S>(src, dst, pl.n, batch, Ns, tw, threadIdx.x, blockDim.x); break;
        }
        __syncthreads();
        Ns *= R;
        cur ^= 1;
    }
    return cur;
}

// Row transforms: one row per work-group.  in/out: [rows][n].
template <int S>
__global__ void __launch_bounds__(FFT_THREADS) k_fft_rows(const float2 *__restrict__ in, float2 *__restrict__ out,
                                                          RadixPlan pl, const float2 *__restrict__ tw,
                                                          const int2 *__restrict__ rowwin, int rows_per_img)
{
    extern __shared__ float2 lds[];
    float2 *a = lds, *b = lds + pl.n;
    const int64_t row = blockIdx.x;
    if (rowwin) {  // only rows (start + i) mod rows_per_img, i < len, of each image are wanted
        const int img = (int)(row / rows_per_img), r = (int)(row - (int64_t)img * rows_per_img);
        const int2 w = rowwin[img];
        const int d = ((r - w.x) % rows_per_img + rows_per_img) % rows_per_img;
        if (d >= w.y) return;
    }
    const float2 *src = in + row * pl.n;
    for (int i = threadIdx.x; i < pl.n; i += blockDim.x) a[i] = src[i];
    __syncthreads();
    const int cur = fft_lds<S>(a, b, pl, 1, tw);
    const float2 *res = cur ? b : a;
    float2 *dst = out + row * pl.n;
    for (int i = threadIdx.x; i < pl.n; i += blockDim.x) dst[i] = res[i];
}

// Column transforms.  A work-group of FFT_COL_THREADS owns columns [c0, c0 + B) of one image
// [n][width] (B = 16: 128-byte row segments, whole cache lines) and keeps them in ONE LDS
// buffer laid out [n][B], so the global reads and writes are contiguous row segments and a
// butterfly's R inputs of column c sit B apart (consecutive threads take consecutive columns:
// no bank conflicts).  Each Stockham pass runs in place: every thread first reads the inputs
// of its (at most KMAX) butterflies into registers, the work-group synchronises, then every
// thread writes its outputs.  The twiddle table sits in LDS after the data.
constexpr int FFT_COL_THREADS = 1024;
constexpr int FFT_COL_MAXELEM = 150 * 1024 / 8;  // complex64 elements of data in LDS (n * B)
constexpr int FFT_COL_LDSELEM = 160 * 1024 / 8;  // data + twiddle table (n * (B + 1))

template <int R>
struct ColK {
    static constexpr int KMAX = (FFT_COL_MAXELEM / R + FFT_COL_THREADS - 1) / FFT_COL_THREADS;
};

// j / d for j < 2^16 and 2 <= d <= 2^14: with m = floor((2^32 - 1) / d) + 1, umulhi(j, m) = j / d
// exactly (the error j (m - 2^32/d) / 2^32 < 2^-16 is below the smallest non-zero fraction 1/d).
// (d = 1 would need m = 2^32; callers handle it.)
static __device__ __forceinline__ int div_small(int j, uint32_t m) { return (int)__umulhi((uint32_t)j, m); }

template <int R, int S>
static __device__ __forceinline__ void stockham_pass_inplace(float2 *buf, int n, int lb, int Ns, const float2 *tw,
                                                             int tid)
{
    constexpr int KMAX = ColK<R>::KMAX;
    const int B = 1 << lb, nb = n / R, total = nb << lb, tstep = n / (Ns * R);
    const uint32_t mNs = Ns > 1 ? 0xffffffffu / (uint32_t)Ns + 1u : 0u;  // Ns = 1: quotient is j itself
    float2 v[KMAX][R];
#pragma unroll
    for (int q = 0; q < KMAX; ++q) {
        const int idx = tid + q * FFT_COL_THREADS;
        if (idx < total) {
            const int j = idx >> lb, c = idx & (B - 1);
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = buf[((j + r * nb) << lb) + c];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < KMAX; ++q) {
        const int idx = tid + q * FFT_COL_THREADS;
        if (idx < total) {
            const int j = idx >> lb, c = idx & (B - 1);
            const int jq = Ns > 1 ? div_small(j, mNs) : j, k = j - jq * Ns;
#pragma unroll
            for (int r = 1; r < R; ++r) {
                float2 w = tw[r * k * tstep];
                if (S < 0) w.y = -w.y;
                v[q][r] = cmul(v[q][r], w);
            }
            if (R == 2) dft2<S>(v[q]);
            if (R == 3) dft3<S>(v[q]);
            if (R == 4) dft4<S>(v[q]);
            if (R == 5) dft5<S>(v[q]);
            if (R == 8) dft8<S>(v[q]);
            const int o = jq * Ns * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[((o + r * Ns) << lb) + c] = v[q][r];
        }
    }
    __syncthreads();
}

template <int S>
__global__ void __launch_bounds__(FFT_COL_THREADS) k_fft_cols(const float2 *__restrict__ in, float2 *__restrict__ out,
                                                              RadixPlan pl, const float2 *__restrict__ tw, int width,
                                                              int lb, const int2 *__restrict__ colwin)
{
    extern __shared__ float2 lds[];
    const int n = pl.n, B = 1 << lb;
    if (colwin) {  // only columns (start + i) mod width, i < len, of each image are nonzero
        const int ns = (width + B - 1) / B;
        const int im = blockIdx.x / ns, c0s = (blockIdx.x - im * ns) * B;
        const int2 w = colwin[im];
        const int d = ((c0s - w.x) % width + width) % width;
        if (!(d < w.y || d + B > width)) return;
    }
    float2 *tw_s = lds + n * B;  // the twiddle table, read by every pass
    for (int i = threadIdx.x; i < n; i += FFT_COL_THREADS) tw_s[i] = tw[i];
    const int nslab = (width + B - 1) / B;
    const int64_t img = blockIdx.x / nslab;
    const int c0 = (blockIdx.x - (int)(img * nslab)) * B;
    const int bw = min(B, width - c0);
    const float2 *src = in + img * (int64_t)n * width;
    float2 *dst = out + img * (int64_t)n * width;
    for (int i = threadIdx.x; i < n * B; i += FFT_COL_THREADS) {
        const int r = i >> lb, c = i & (B - 1);
        lds[i] = c < bw ? src[(int64_t)r * width + c0 + c] : make_float2(0.0f, 0.0f);
    }
    __syncthreads();
    int Ns = 1;
    for (int p = 0; p < pl.nrad; ++p) {
        const int R = pl.r[p];
        switch (R) {
        case 2: stockham_pass_inplace<2, S>(lds, n, lb, Ns, tw_s, threadIdx.x); break;
        case 3: stockham_pass_inplace<3, S>(lds, n, lb, Ns, tw_s, threadIdx.x); break;
        case 4: stockham_pass_inplace<4, S>(lds, n, lb, Ns, tw_s, threadIdx.x); break;
        case 5: stockham_pass_inplace<5, S>(lds, n, lb, Ns, tw_s, threadIdx.x); break;
        default: stockham_pass_inplace<8, S>(lds, n, lb, Ns, tw_s, threadIdx.x); break;
        }
        Ns *= R;
    }
    for (int i = threadIdx.x; i < n * B; i += FFT_COL_THREADS) {
        const int r = i >> lb, c = i & (B - 1);
        if (c < bw) dst[(int64_t)r * width + c0 + c] = lds[i];
    }
}

static RadixPlan make_radix(int n, const int32_t *r, int nrad)
{
    RadixPlan p;
    p.n = n;
    p.nrad = nrad;
    for (int i = 0; i < FFT_MAX_RAD; ++i) p.r[i] = i < nrad ? r[i] : 0;
    return p;
}

int fft_col_batch(int n)
{
    // largest B (power of two, <= 16) with B n complex64 of data and the n twiddles in LDS
    int B = 16;
    while (B > 1 && ((int64_t)B * n > FFT_COL_MAXELEM || (int64_t)(B + 1) * n > FFT_COL_LDSELEM)) B >>= 1;
    return B;
}

static void allow_big_lds()
{
    static bool done = false;
    if (done) return;
    const int lim = 160 * 1024;
    hipFuncSetAttribute((const void *)k_fft_cols<1>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    hipFuncSetAttribute((const void *)k_fft_cols<-1>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    hipFuncSetAttribute((const void *)k_fft_rows<1>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    hipFuncSetAttribute((const void *)k_fft_rows<-1>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    done = true;
}

hipError_t launch_fft2d(const Plan &p, int batch, int direction, const float2 *in, float2 *out, hipStream_t s)
{
    return launch_fft2d_win(p, batch, direction, in, out, nullptr, nullptr, s);
}

// Rows then columns; with windows, columns first (only the slabs meeting colwin, the rest
// being zero) and then the rows (only those in rowwin; the others are left unfinished).
hipError_t launch_fft2d_win(const Plan &p, int batch, int direction, const float2 *in, float2 *out,
                            const int2 *colwin, const int2 *rowwin, hipStream_t s)
{
    allow_big_lds();
    const RadixPlan px = make_radix(p.nx, p.radix_x, p.nrad_x);
    const RadixPlan py = make_radix(p.ny, p.radix_y, p.nrad_y);
    const size_t row_lds = 2 * (size_t)p.nx * sizeof(float2);
    const int rows = batch * p.ny;
    const int B = fft_col_batch(p.ny);
    int lb = 0;
    while ((1 << lb) < B) ++lb;
    const size_t col_lds = (size_t)(B + 1) * p.ny * sizeof(float2);
    const int nslab = (p.nx + B - 1) / B;
    const bool cols_first = colwin != nullptr || rowwin != nullptr;
    if (cols_first && in != out) return hipErrorInvalidValue;  // the windowed form works in place
    auto rows_pass = [&](const float2 *src, float2 *dst) {
        if (direction > 0)
            hipLaunchKernelGGL(k_fft_rows<-1>, dim3(rows), dim3(FFT_THREADS), row_lds, s, src, dst, px, p.tw_x, rowwin,
                               p.ny);
        else
            hipLaunchKernelGGL(k_fft_rows<1>, dim3(rows), dim3(FFT_THREADS), row_lds, s, src, dst, px, p.tw_x, rowwin,
                               p.ny);
    };
    auto cols_pass = [&](float2 *buf) {
        if (direction > 0)
            hipLaunchKernelGGL(k_fft_cols<-1>, dim3(batch * nslab), dim3(FFT_COL_THREADS), col_lds, s, buf, buf, py,
                               p.tw_y, p.nx, lb, colwin);
        else
            hipLaunchKernelGGL(k_fft_cols<1>, dim3(batch * nslab), dim3(FFT_COL_THREADS), col_lds, s, buf, buf, py,
                               p.tw_y, p.nx, lb, colwin);
    };
    if (cols_first) {
        cols_pass(out);
        rows_pass(out, out);
    } else {
        rows_pass(in, out);
        cols_pass(out);
    }
    return hipGetLastError();
}

}  // namespace gws
