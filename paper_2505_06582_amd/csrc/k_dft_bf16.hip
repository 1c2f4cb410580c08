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
// (m n mod N) in FP64 and stored pre-split as four bf16 planes (Re hi, Re lo, Im hi, Im lo),
// transposed ([n][k]) and zero-padded to the block tile.  The data operand is split into its
// four planes once per transform: the input by k_dft_split, the intermediate by the first
// product's epilogue.
#include <math.h>
#include <string.h>

#include <vector>

#include "gws_internal.h"

namespace gws {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));

// Block tile 128 (rows of the data operand) x 128 (DFT columns) x 32 (k); eight wavefronts in
// a 2 x 4 grid, each owning a 64 x 32 block of the result as 4 x 2 MFMA tiles of 16 x 16 (its
// accumulators in 64 registers), so two wavefronts share each SIMD and one's LDS waits overlap
// the other's products.  One work-group per CU.
constexpr int DBM = 128, DBN = 128, DBK = 32;
constexpr int DSTR = DBK + 8;  // padded LDS row stride (bf16 elements): conflict-free 16-byte fragment reads
constexpr int NPA = 4;         // data planes: Re hi, Re lo, Im hi, Im lo
constexpr int NPB = 4;         // DFT-matrix planes: Re hi, Re lo, Im hi, Im lo

struct DftMats {
    int n, npad, kpad;
    uint16_t *planes;  // [NPB][npad][kpad]
};

static __device__ __forceinline__ uint16_t f32_to_bf16_rne(float x)
{
    const uint32_t b = __float_as_uint(x);
    return (uint16_t)((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);
}
static __device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

static __host__ __device__ inline int kpad_of(int k) { return (k + DBK - 1) / DBK * DBK; }

// Data operand split once per transform: X [img][M][K] complex64 -> [img][4][M][kpad] bf16
// planes (x = hi + lo, each rounded to nearest even), zero beyond K.  One thread per 8 k.
__global__ void __launch_bounds__(256) k_dft_split(const float2 *__restrict__ X, uint16_t *__restrict__ P, int M, int K,
                                                   int kpad, int64_t total)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int per_row = kpad / 8;
    const int64_t rowi = t / per_row;
    const int k0 = (int)(t - rowi * per_row) * 8;
    const int64_t img = rowi / M;
    const int row = (int)(rowi - img * M);
    const float2 *src = X + (img * M + row) * (int64_t)K;
    u16x8 rh, rl, ih, il;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int k = k0 + i;
        const float2 v = k < K ? src[k] : make_float2(0.0f, 0.0f);
        const uint16_t hr = f32_to_bf16_rne(v.x), hi_ = f32_to_bf16_rne(v.y);
        rh[i] = hr;
        rl[i] = f32_to_bf16_rne(v.x - bf16_to_f32(hr));
        ih[i] = hi_;
        il[i] = f32_to_bf16_rne(v.y - bf16_to_f32(hi_));
    }
    const int64_t plane = (int64_t)M * kpad, o = (img * NPA * M + row) * (int64_t)kpad + k0;
    *(u16x8 *)(P + o) = rh;
    *(u16x8 *)(P + o + plane) = rl;
    *(u16x8 *)(P + o + 2 * plane) = ih;
    *(u16x8 *)(P + o + 3 * plane) = il;
}

// Yt = (X F)^T for the data planes A [img][4][M][K] (K = kpad of the DFT size) and the DFT
// matrix planes Bt [4][npad][K] (F[m][n] = exp(+j 2 pi m n / N), stored transposed).  With
// F = Fr + j s Fi (s = DIR): Re = Xr Fr - s Xi Fi, Im = s Xr Fi + Xi Fr; the sign is applied to
// the data fragments in registers (a sign-bit flip).  SPLIT_OUT writes Yt as the next
// transform's data planes [img][4][N][kpad_out] (zero beyond M), else as complex64 [img][N][M].
//
// Block order.  Work-groups are dealt to the 8 XCDs round-robin (id % 8), each with its own L2,
// and one operand of a block streams while the other stays cached.  So each XCD takes a
// contiguous run of tiles, and within it tiles go down groups of GROUP_M block rows before the
// next block column: the ~32 blocks an XCD runs at once share a few block rows and columns.
constexpr int GROUP_M = 8;

template <int DIR, bool SPLIT_OUT>
__global__ void __launch_bounds__(512, 2) k_dft_gemm(const uint16_t *__restrict__ A, const uint16_t *__restrict__ Bt,
                                                     void *__restrict__ out, int M, int N, int K, int npad,
                                                     int kpad_out, int mblocks, int rows_total, int per_xcd)
{
    __shared__ __attribute__((aligned(16))) uint16_t As[NPA * DBM * DSTR];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[NPB * DBN * DSTR];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // tile of this work-group: rows_total = batch x mblocks block rows (image-major), npad / DBN
    // block columns
    const int nblocks = npad / DBN;
    const int T = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
    if (T >= rows_total * nblocks) return;
    const int per_group = GROUP_M * nblocks, grp = T / per_group, first = grp * GROUP_M;
    const int gm = min(rows_total - first, GROUP_M), w = T - grp * per_group;
    const int rowblk = first + w % gm, nb = w / gm;
    const int64_t img = rowblk / mblocks;
    const int n0 = nb * DBN, m0 = (rowblk - (int)img * mblocks) * DBM;
    const int64_t aplane = (int64_t)M * K, bplane = (int64_t)npad * K;
    const uint16_t *Ai = A + img * NPA * aplane;
    const int wm = wave & 1, wn = wave >> 1;  // wn: 0..3
    // staging map: 4 planes x 128 rows x 4 chunks of 8 k, for A and for B (4 + 4 per thread)
    int a_off[4], b_off[4], s_lds[4];
    bool a_ok[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int c = tid + 512 * i, p = c >> 9, row = (c >> 2) & (DBM - 1), kq = c & 3;
        a_ok[i] = m0 + row < M;
        a_off[i] = (int)(p * aplane + (int64_t)(m0 + row) * K + kq * 8);
        b_off[i] = (int)(p * bplane + (int64_t)(n0 + row) * K + kq * 8);
        s_lds[i] = p * DBM * DSTR + row * DSTR + kq * 8;
    }
    u16x8 ra[4], rb[4];
    const u16x8 z8 = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        ra[i] = a_ok[i] ? *(const u16x8 *)(Ai + a_off[i]) : z8;
        rb[i] = *(const u16x8 *)(Bt + b_off[i]);
    }
    f32x4 accR[4][2], accI[4][2];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            accR[t][u] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            accI[t][u] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        }
    const int kk = (lane >> 4) * 8;
    const uint32_t sgn = 0x80008000u;
    for (int kc = 0; kc < K; kc += DBK) {
        __syncthreads();  // the previous k-step's fragments are read
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            *(u16x8 *)(As + s_lds[i]) = ra[i];
            *(u16x8 *)(Bs + s_lds[i]) = rb[i];
        }
        __syncthreads();
        if (kc + DBK < K) {  // prefetch the next k-step into registers
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                ra[i] = a_ok[i] ? *(const u16x8 *)(Ai + a_off[i] + kc + DBK) : z8;
                rb[i] = *(const u16x8 *)(Bt + b_off[i] + kc + DBK);
            }
        }
        bf16x8 b[2][NPB];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int c = wn * 32 + u * 16 + (lane & 15);
#pragma unroll
            for (int p = 0; p < NPB; ++p) b[u][p] = *(const bf16x8 *)(Bs + p * DBN * DSTR + c * DSTR + kk);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int r = wm * 64 + t * 16 + (lane & 15);
            bf16x8 a[NPA];
#pragma unroll
            for (int p = 0; p < NPA; ++p) a[p] = *(const bf16x8 *)(As + p * DBM * DSTR + r * DSTR + kk);
            // the negated fragments: -Xi for the real part (DIR = +1), -Xr for the imaginary part (DIR = -1)
            bf16x8 n0v, n1v;
            {
                typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
                const int q = DIR > 0 ? 2 : 0;
                u32x4 w0 = __builtin_bit_cast(u32x4, a[q]), w1 = __builtin_bit_cast(u32x4, a[q + 1]);
                w0 ^= sgn;
                w1 ^= sgn;
                n0v = __builtin_bit_cast(bf16x8, w0);
                n1v = __builtin_bit_cast(bf16x8, w1);
            }
            const bf16x8 xrh = DIR > 0 ? a[0] : n0v, xrl = DIR > 0 ? a[1] : n1v;  // s Xr for Im
            const bf16x8 xih = DIR > 0 ? n0v : a[2], xil = DIR > 0 ? n1v : a[3];  // -s Xi for Re
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                f32x4 cr = accR[t][u], ci = accI[t][u];
                // Re: Xr Fr - s Xi Fi, three split products each
                cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[u][0], cr, 0, 0, 0);
                ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xrh, b[u][2], ci, 0, 0, 0);
                cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[u][1], cr, 0, 0, 0);
                ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xrh, b[u][3], ci, 0, 0, 0);
                cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[u][0], cr, 0, 0, 0);
                ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xrl, b[u][2], ci, 0, 0, 0);
                cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xih, b[u][2], cr, 0, 0, 0);
                ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], b[u][0], ci, 0, 0, 0);
                cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xih, b[u][3], cr, 0, 0, 0);
                ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], b[u][1], ci, 0, 0, 0);
                cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xil, b[u][2], cr, 0, 0, 0);
                ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[3], b[u][0], ci, 0, 0, 0);
                accR[t][u] = cr;
                accI[t][u] = ci;
            }
        }
    }
    // D[row][col] of a 16 x 16 tile: row = (lane / 16) * 4 + i, col = lane % 16; written transposed
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int col = n0 + wn * 32 + u * 16 + (lane & 15);
            const int row0 = m0 + wm * 64 + t * 16 + (lane >> 4) * 4;
            if constexpr (SPLIT_OUT) {
                // the next transform's data planes: 4 consecutive k (= rows here) per lane and plane
                if (col < N && row0 < kpad_out) {
                    u16x4 rh, rl, ih, il;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float vr = accR[t][u][i], vi = accI[t][u][i];
                        rh[i] = f32_to_bf16_rne(vr);
                        rl[i] = f32_to_bf16_rne(vr - bf16_to_f32(rh[i]));
                        ih[i] = f32_to_bf16_rne(vi);
                        il[i] = f32_to_bf16_rne(vi - bf16_to_f32(ih[i]));
                    }
                    uint16_t *Po = (uint16_t *)out;
                    const int64_t plane = (int64_t)N * kpad_out;
                    const int64_t o = img * NPA * plane + (int64_t)col * kpad_out + row0;
                    *(u16x4 *)(Po + o) = rh;
                    *(u16x4 *)(Po + o + plane) = rl;
                    *(u16x4 *)(Po + o + 2 * plane) = ih;
                    *(u16x4 *)(Po + o + 3 * plane) = il;
                }
            } else {
                float2 *Yi = (float2 *)out + img * (int64_t)M * N;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = row0 + i;
                    if (row < M && col < N) Yi[(int64_t)col * M + row] = make_float2(accR[t][u][i], accI[t][u][i]);
                }
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
    const int npad = (n + DBN - 1) / DBN * DBN, kpad = kpad_of(n);
    const size_t plane = (size_t)npad * kpad;
    std::vector<uint16_t> h(NPB * plane, 0);
    for (int nn = 0; nn < n; ++nn)
        for (int k = 0; k < n; ++k) {
            const long long r = ((long long)nn * k) % n;
            const double ph = 2.0 * M_PI * (double)r / (double)n;
            const double vals[2] = {cos(ph), sin(ph)};
            for (int part = 0; part < 2; ++part) {  // Re, Im
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

// Data planes of the input ([batch][4][ny][kpad(nx)] bf16) and of the intermediate
// ([batch][4][nx][kpad(ny)] bf16), 8 bytes per complex element each.
size_t dft_bf16x3_workspace(int nx, int ny, int batch)
{
    const size_t a = (size_t)batch * ny * kpad_of(nx) * 8, b = (size_t)batch * nx * kpad_of(ny) * 8;
    return (a + 255) / 256 * 256 + b + 256;
}

template <bool SPLIT_OUT>
static void launch_gemm(int dir, const uint16_t *A, const DftMats &F, void *out, int M, int kpad_out, int batch,
                        hipStream_t s)
{
    const int mblocks = (M + DBM - 1) / DBM, rows_total = batch * mblocks;
    const int tiles = rows_total * (F.npad / DBN), per_xcd = (tiles + 7) / 8;
    const dim3 grid((unsigned)(8 * per_xcd));
    if (dir > 0)
        hipLaunchKernelGGL((k_dft_gemm<1, SPLIT_OUT>), grid, dim3(512), 0, s, A, F.planes, out, M, F.n, F.kpad, F.npad,
                           kpad_out, mblocks, rows_total, per_xcd);
    else
        hipLaunchKernelGGL((k_dft_gemm<-1, SPLIT_OUT>), grid, dim3(512), 0, s, A, F.planes, out, M, F.n, F.kpad,
                           F.npad, kpad_out, mblocks, rows_total, per_xcd);
}

hipError_t launch_dft_bf16x3(Plan &p, int batch, int direction, const float2 *in, float2 *out, void *ws, hipStream_t s)
{
    hipError_t e = build_dft_mats(p);
    if (e != hipSuccess) return e;
    const DftMats *m = (const DftMats *)p.dft_mats;
    const int nx = p.nx, ny = p.ny, kx = kpad_of(nx), ky = kpad_of(ny);
    uint16_t *pa = (uint16_t *)ws;
    uint16_t *pb = (uint16_t *)((char *)ws + ((size_t)batch * ny * kx * 8 + 255) / 256 * 256);
    // split the rows of the input once, then rows: (S F_x)^T -> pb as the column transform's
    // data planes [nx][ky]; columns: (T^T F_y)^T -> out [ny][nx]
    const int64_t total = (int64_t)batch * ny * (kx / 8);
    hipLaunchKernelGGL(k_dft_split, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, in, pa, ny, nx, kx, total);
    launch_gemm<true>(direction, pa, m[0], pb, ny, ky, batch, s);
    launch_gemm<false>(direction, pb, m[1], out, nx, 0, batch, s);
    return hipGetLastError();
}

}  // namespace gws
