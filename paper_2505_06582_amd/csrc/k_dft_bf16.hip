// The 2D DFT as two dense complex GEMMs on the gfx950 matrix cores, with every FP32
// operand split into a bf16 high part and a bf16 residual and three products per real
// product (hi*hi + hi*lo + lo*hi), accumulated in FP32 by v_mfma_f32_16x16x32_bf16.
//
// One kernel computes Yt = (X F)^T for X [M][K] complex64 and the DFT matrix
// F[m][n] = exp(+-j 2 pi m n / N) (K = N), writing the result transposed.  Applied twice
// -- first to the rows of the image, then to the rows of the transposed intermediate --
// it gives the 2D transform in natural layout:  (S F_x)^T = T^T, (T^T F_y)^T = F_y S F_x.
//
// The DFT matrices are built once per size on the host from exactly reduced phases
// (m n mod N) in FP64 and stored pre-split as four bf16 planes (Re hi, Re lo, Im hi,
// Im lo), transposed ([n][k]) and zero-padded to the block tile.  The data operand is
// split on the fly when its tile is staged in LDS.
#include <math.h>
#include <string.h>

#include <vector>

#include "gws_internal.h"

namespace gws {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

constexpr int DBM = 64, DBN = 64, DBK = 32;
constexpr int DSTR = DBK + 8;  // padded LDS row stride (bf16 elements): conflict-free 16-byte fragment reads

struct DftMats {
    int n, npad, kpad;
    uint16_t *planes;  // [4][npad][kpad]
};

static __device__ __forceinline__ uint16_t f32_to_bf16_rne(float x)
{
    const uint32_t b = __float_as_uint(x);
    return (uint16_t)((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);
}
static __device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

template <int DIR>
__global__ void __launch_bounds__(256) k_dft_gemm(const float2 *__restrict__ X, const uint16_t *__restrict__ Bt,
                                                  float2 *__restrict__ Yt, int M, int N, int K, int npad, int kpad)
{
    __shared__ __attribute__((aligned(16))) uint16_t As[4][DBM * DSTR];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[4][DBN * DSTR];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n0 = blockIdx.x * DBN, m0 = blockIdx.y * DBM;
    const int64_t img = blockIdx.z;
    const float2 *Xi = X + img * (int64_t)M * K;
    float2 *Yi = Yt + img * (int64_t)M * N;
    const int wm = wave & 1, wn = wave >> 1;
    f32x4 accR[2][2], accI[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            accR[a][b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            accI[a][b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        }
    const size_t plane = (size_t)npad * kpad;
    for (int kc = 0; kc < kpad; kc += DBK) {
        // stage A: 64 rows x 32 k complex, split into (Re hi, Re lo, Im hi, Im lo)
        {
            const int row = tid >> 2, k0 = (tid & 3) * 8;
            const int gr = m0 + row;
            u16x8 rh, rl, ih, il;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int gk = kc + k0 + i;
                float2 v = make_float2(0.0f, 0.0f);
                if (gr < M && gk < K) v = Xi[(int64_t)gr * K + gk];
                const uint16_t hr = f32_to_bf16_rne(v.x), hi_ = f32_to_bf16_rne(v.y);
                rh[i] = hr;
                rl[i] = f32_to_bf16_rne(v.x - bf16_to_f32(hr));
                ih[i] = hi_;
                il[i] = f32_to_bf16_rne(v.y - bf16_to_f32(hi_));
            }
            *(u16x8 *)&As[0][row * DSTR + k0] = rh;
            *(u16x8 *)&As[1][row * DSTR + k0] = rl;
            *(u16x8 *)&As[2][row * DSTR + k0] = ih;
            *(u16x8 *)&As[3][row * DSTR + k0] = il;
        }
        // stage B: 64 n x 32 k per plane, already split and padded
        {
            const int p = tid >> 6, n = tid & 63;
            const uint16_t *src = Bt + p * plane + (size_t)(n0 + n) * kpad + kc;
#pragma unroll
            for (int q = 0; q < 4; ++q) *(u16x8 *)&Bs[p][n * DSTR + q * 8] = *(const u16x8 *)(src + q * 8);
        }
        __syncthreads();
        const int kk = (lane >> 4) * 8;
        bf16x8 a[2][4], b[2][4];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int r = wm * 32 + t * 16 + (lane & 15);
            const int c = wn * 32 + t * 16 + (lane & 15);
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                a[t][p] = *(const bf16x8 *)&As[p][r * DSTR + kk];
                b[t][p] = *(const bf16x8 *)&Bs[p][c * DSTR + kk];
            }
        }
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            // -Im parts of the data for the real output; DIR = -1 conjugates the matrix
            const bf16x8 nih = -a[t][2], nil = -a[t][3];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                bf16x8 bih = b[u][2], bil = b[u][3];
                if (DIR < 0) {
                    bih = -bih;
                    bil = -bil;
                }
                f32x4 cr = accR[t][u], ci = accI[t][u];
                // Re: Xr Fr - Xi Fi
                cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[t][0], b[u][0], cr, 0, 0, 0);
                cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[t][0], b[u][1], cr, 0, 0, 0);
                cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[t][1], b[u][0], cr, 0, 0, 0);
                cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nih, bih, cr, 0, 0, 0);
                cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nih, bil, cr, 0, 0, 0);
                cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nil, bih, cr, 0, 0, 0);
                // Im: Xr Fi + Xi Fr
                ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[t][0], bih, ci, 0, 0, 0);
                ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[t][0], bil, ci, 0, 0, 0);
                ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[t][1], bih, ci, 0, 0, 0);
                ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[t][2], b[u][0], ci, 0, 0, 0);
                ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[t][2], b[u][1], ci, 0, 0, 0);
                ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[t][3], b[u][0], ci, 0, 0, 0);
                accR[t][u] = cr;
                accI[t][u] = ci;
            }
        }
        __syncthreads();
    }
    // D[row][col]: row = (lane / 16) * 4 + i of the 16 x 16 tile, col = lane % 16; write transposed
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int col = n0 + wn * 32 + u * 16 + (lane & 15);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = m0 + wm * 32 + t * 16 + (lane >> 4) * 4 + i;
                if (row < M && col < N) Yi[(int64_t)col * M + row] = make_float2(accR[t][u][i], accI[t][u][i]);
            }
        }
}

static uint16_t host_bf16(float x)
{
    uint32_t b;
    memcpy(&b, &x, 4);
    return (uint16_t)((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);
}
static float host_bf16_f(uint16_t h)
{
    const uint32_t b = (uint32_t)h << 16;
    float f;
    memcpy(&f, &b, 4);
    return f;
}

static hipError_t build_mats_n(int n, DftMats *out)
{
    const int npad = (n + DBN - 1) / DBN * DBN, kpad = (n + DBK - 1) / DBK * DBK;
    const size_t plane = (size_t)npad * kpad;
    std::vector<uint16_t> h(4 * plane, 0);
    for (int nn = 0; nn < n; ++nn)
        for (int k = 0; k < n; ++k) {
            const long long r = ((long long)nn * k) % n;
            const double ph = 2.0 * M_PI * (double)r / (double)n;
            const double vals[2] = {cos(ph), sin(ph)};
            for (int part = 0; part < 2; ++part) {
                const double x = vals[part];
                const uint16_t hi = host_bf16((float)x);
                const uint16_t lo = host_bf16((float)(x - (double)host_bf16_f(hi)));
                h[(2 * part) * plane + (size_t)nn * kpad + k] = hi;
                h[(2 * part + 1) * plane + (size_t)nn * kpad + k] = lo;
            }
        }
    out->n = n;
    out->npad = npad;
    out->kpad = kpad;
    hipError_t e = hipMalloc(&out->planes, h.size() * sizeof(uint16_t));
    if (e != hipSuccess) return e;
    return hipMemcpy(out->planes, h.data(), h.size() * sizeof(uint16_t), hipMemcpyHostToDevice);
}

hipError_t build_dft_mats(Plan &p)
{
    if (p.dft_mats) return hipSuccess;
    DftMats *m = new DftMats[2];
    hipError_t e = build_mats_n(p.nx, &m[0]);
    if (e == hipSuccess) e = build_mats_n(p.ny, &m[1]);
    if (e != hipSuccess) {
        delete[] m;
        return e;
    }
    p.dft_mats = (void *)m;
    return hipSuccess;
}

void free_dft_mats(Plan &p)
{
    if (!p.dft_mats) return;
    DftMats *m = (DftMats *)p.dft_mats;
    (void)hipFree(m[0].planes);
    (void)hipFree(m[1].planes);
    delete[] m;
    p.dft_mats = nullptr;
}

size_t dft_bf16x3_workspace(int nx, int ny, int batch) { return (size_t)batch * nx * ny * sizeof(float2) + 256; }

static void launch_gemm(int dir, const float2 *X, const DftMats &F, float2 *Yt, int M, int batch, hipStream_t s)
{
    const dim3 grid(F.npad / DBN, (M + DBM - 1) / DBM, batch);
    if (dir > 0)
        hipLaunchKernelGGL(k_dft_gemm<1>, grid, dim3(256), 0, s, X, F.planes, Yt, M, F.n, F.n, F.npad, F.kpad);
    else
        hipLaunchKernelGGL(k_dft_gemm<-1>, grid, dim3(256), 0, s, X, F.planes, Yt, M, F.n, F.n, F.npad, F.kpad);
}

hipError_t launch_dft_bf16x3(Plan &p, int batch, int direction, const float2 *in, float2 *out, void *ws, hipStream_t s)
{
    hipError_t e = build_dft_mats(p);
    if (e != hipSuccess) return e;
    const DftMats *m = (const DftMats *)p.dft_mats;
    float2 *tmp = (float2 *)ws;
    // rows: (S F_x)^T -> tmp [nx][ny]; then (tmp F_y)^T -> out [ny][nx]
    launch_gemm(direction, in, m[0], tmp, p.ny, batch, s);
    launch_gemm(direction, tmp, m[1], out, p.nx, batch, s);
    return hipGetLastError();
}

}  // namespace gws
