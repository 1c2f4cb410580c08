// Internal declarations shared by the gfx950 kernels and the host side of libgws.
// Nothing here is part of the C ABI (include/gws.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "gws.h"

namespace gws {

// ---------------------------------------------------------------------------------
// Frequency tiling.  The centred frequency plane m' in [-nx/2, nx/2) x [-ny/2, ny/2)
// (index units) is cut into DC-aligned tiles of TILEX x tile_h(F) frequencies: tile
// (tx, ty) covers m'_x in [TILEX tx, TILEX (tx + 1)) and m'_y in [tile_h ty, tile_h (ty + 1)),
// clipped to the grid.  A work-group of 4 wavefronts owns one tile; wavefront w owns the
// SUBX x sub_h(F) sub-tile (w & 1, w >> 1); lane l of a wavefront owns column l % SUBX
// and rows l / SUBX + 4 f for f = 0..F-1 of its sub-tile.  F (frequencies per lane) is
// the tiling parameter the autotuner chooses: 2, 4 or 8.
// ---------------------------------------------------------------------------------
constexpr int SUBX = 16;
constexpr int TILEX = 2 * SUBX;
__host__ __device__ constexpr int sub_h(int f) { return 4 * f; }
// Minimum resident wavefronts per SIMD the evaluation kernels are compiled for: 4 (at most
// 128 VGPRs) for F <= 4; F = 8 keeps 8 frequencies x C wavelengths of per-lane tables in
// registers and is compiled for 2 (at most 256 VGPRs) rather than spill.
__host__ __device__ constexpr int waves_per_simd(int f) { return f >= 8 ? 2 : 4; }
constexpr int WAVES = 4;             // wavefronts per work-group
constexpr int WG = 64 * WAVES;       // threads per work-group
constexpr int NBUCKET = 4096;        // support-radius buckets (index units)

// Adjoint geometry.  Its tile list is the F = 8 tiling (32 x 64 tiles); a region is the left
// or right 16 x 64 half of a tile, two 16 x 32 sub-tiles (the unit of the exact phase base),
// sixteen 4-row blocks.  A work-group of adj_waves(C, depth) wavefronts owns as many sorted
// Gaussians as it has threads (one per thread) and holds one region's per-frequency data in
// LDS; lane l evaluates column l % 16 and rows l / 16 + 4 b of block b.
constexpr int ADJ_F = 8;
constexpr int ADJ_RW = SUBX;           // region columns
constexpr int ADJ_RH = 2 * sub_h(ADJ_F);  // region rows (64)
constexpr int ADJ_SH = sub_h(ADJ_F);   // sub-tile rows (32)
constexpr int ADJ_NB = ADJ_RH / 4;     // 4-row blocks per region
constexpr int ADJ_MIN_CHUNK = 256;     // smallest work-group (and Gaussian chunk) of any variant
static_assert(TILEX == 2 * ADJ_RW, "a tile holds two regions");
// reduced per-Gaussian sums: Re P_c, Sfx, Sfy, Qxx, Qxy, Qyy, then Im P_c and W_c with the
// depth gradient, else sum Im rho
__host__ __device__ constexpr int adj_nv(int c, bool depth) { return (depth ? 3 * c : c) + 5 + (depth ? 0 : 1); }
// LDS of a work-group of w wavefronts: the region's data (12 B per frequency and channel), the
// per-Gaussian sums and the list of accepted Gaussians (16-byte aligned entries).
__host__ __device__ constexpr int adj_lds_bytes(int c, bool depth, int w)
{
    return ADJ_NB * c * 64 * 12 + 64 * w * adj_nv(c, depth) * 4 + 64 * w * ((2 + 2 * c + 3) / 4) * 16;
}
// Eight wavefronts per work-group while that fits 82,000 bytes of LDS, else four.
__host__ __device__ constexpr int adj_waves(int c, bool depth) { return adj_lds_bytes(c, depth, 8) <= 82000 ? 8 : 4; }
__host__ __device__ constexpr int adj_wg(int c, bool depth) { return 64 * adj_waves(c, depth); }
// Wavefronts per SIMD the adjoint is compiled for: two work-groups per CU while each needs at
// most 78 KB of LDS, else one.
__host__ __device__ constexpr int adj_waves_per_simd(int c, bool depth)
{
    return (adj_lds_bytes(c, depth, adj_waves(c, depth)) <= 78 * 1024 ? 2 : 1) * adj_waves(c, depth) / 4;
}
// Region indexing of the packed per-frequency tables: region r = 2 ((ty - ty_min) ntx +
// (tx - tx_min)) + half over the F = 8 tile grid.
struct AdjGeom {
    int32_t tx_min, ty_min, ntx, nreg;
};

// ---------------------------------------------------------------------------------
// Support tests in index units.  The eps-support of a Gaussian's spectrum is the ellipse
// q(x, y) = a x^2 + b2 x y + g y^2 <= lim centred on DC.  q is convex, so over a
// rectangle that does not hold the origin its minimum lies on an edge, where q is a 1-D
// parabola: the test below is exact (up to FP32 rounding).  ia = 1/(2a), ig = 1/(2g).
// ---------------------------------------------------------------------------------
__device__ __forceinline__ bool ellipse_meets_rect_r(float a, float b2, float g, float ia, float ig, float lim,
                                                     float x0, float x1, float y0, float y1)
{
    if (x0 <= 0.0f && x1 >= 0.0f && y0 <= 0.0f && y1 >= 0.0f) return true;
    float m;
    float y = fminf(fmaxf(-b2 * x0 * ig, y0), y1);
    m = x0 * (a * x0 + b2 * y) + g * y * y;
    y = fminf(fmaxf(-b2 * x1 * ig, y0), y1);
    m = fminf(m, x1 * (a * x1 + b2 * y) + g * y * y);
    float x = fminf(fmaxf(-b2 * y0 * ia, x0), x1);
    m = fminf(m, x * (a * x + b2 * y0) + g * y0 * y0);
    x = fminf(fmaxf(-b2 * y1 * ia, x0), x1);
    m = fminf(m, x * (a * x + b2 * y1) + g * y1 * y1);
    return m <= lim;
}

// Bit f is set when the support meets the 4-row block f of a sub-tile: columns [x0, x1],
// rows [sy0 + 4f, sy0 + 4f + 3], rows clipped to the grid [-hy, hy - 1].  With a support
// centred at m_r instead of DC, x0, x1 are passed relative to m_r and ysh = m_r,y.  Lane rows
// l / SUBX + 4 f of the tiling are exactly block f, so a wavefront skips block f of a
// Gaussian whose bit is clear.
//
// The rows the support reaches inside the column strip form an interval [ylo, yhi] (the
// projection of a convex set).  Its top is the ellipse's highest point (x_t, y_t),
// y_t = sqrt(lim / (g - b2^2 / 4a)), x_t = -b2 y_t / 2a, when x_t lies in the strip, else
// the upper root of q(x_b, y) = lim on the strip edge x_b nearest x_t; the bottom mirrors
// it (the ellipse is centred on DC).  The interval is widened by 1e-3 rows so rounding
// never drops a block the exact test would keep.  Only called for a sub-tile the support
// meets, so the strip is never empty.
template <int F>
__device__ __forceinline__ uint32_t row_block_mask(float a, float b2, float g, float lim, float x0, float x1, int sy0,
                                                   int hy, float ysh = 0.0f)
{
    const float dg = g - b2 * b2 * (0.25f / a);
    const float yt = sqrtf(lim / dg), xt = -b2 * yt * (0.5f / a);
    const float ig2 = 0.5f / g;
    float yhi = yt, ylo = -yt;
    if (xt < x0 || xt > x1) {
        const float xb = fminf(fmaxf(xt, x0), x1);
        const float d = fmaxf(b2 * b2 * xb * xb - 4.0f * g * (a * xb * xb - lim), 0.0f);
        yhi = (-b2 * xb + sqrtf(d)) * ig2;
    }
    if (-xt < x0 || -xt > x1) {
        const float xb = fminf(fmaxf(-xt, x0), x1);
        const float d = fmaxf(b2 * b2 * xb * xb - 4.0f * g * (a * xb * xb - lim), 0.0f);
        ylo = (-b2 * xb - sqrtf(d)) * ig2;
    }
    yhi += 1e-3f * (1.0f + fabsf(yhi));
    ylo -= 1e-3f * (1.0f + fabsf(ylo));
    uint32_t m = 0;
#pragma unroll
    for (int f = 0; f < F; ++f) {
        const int r0 = max(sy0 + 4 * f, -hy), r1 = min(sy0 + 4 * f + 3, hy - 1);
        if (r0 <= r1 && (float)r0 - ysh <= yhi && (float)r1 - ysh >= ylo) m |= 1u << f;
    }
    return m;
}

// Sum of a 64-bit counter over the 64 lanes of a wavefront (every lane gets the total).
// Transposed butterfly reduction of V (8 or 16) per-lane values over the 64 lanes of a
// wavefront.  Each transposed step pairs value i with value i + h and lane l with lane
// l ^ d: the lane with the d bit clear keeps and sums the first value of the pair, its
// partner the second, so a step halves the values per lane with one exchange and one add
// per pair.  Steps d = 32 and d = 16 use the gfx950 cross-row swaps (v_permlane32_swap,
// v_permlane16_swap), d = 8 a DPP rotate inside the 16-lane row.  What remains (V / 8
// values per lane) is summed over the 8 lanes of each half-row with three DPP adds
// (half-row mirror, then the two quad swaps).  On return register j of lane l holds the
// total of value (V / 8) (4 b5 + 2 b4 + b3) + j (b_k = bit k of l); no LDS is involved.
static __device__ __forceinline__ float dpp_ror8(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x128, 0xf, 0xf, false));
}
static __device__ __forceinline__ float dpp_half_mirror(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x141, 0xf, 0xf, false));
}
static __device__ __forceinline__ float dpp_xor2(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xf, 0xf, false));
}
static __device__ __forceinline__ float dpp_xor1(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xf, 0xf, false));
}

// With EXTRA, one more value y is carried along: it is summed over lane bits 5, 4 and 3 on
// its own, and in the last stage lanes with bit 2 clear keep x while lanes with bit 2 set
// keep y (the half-row mirror pairs lane i with lane 7 - i, which differ in bit 2), so
// afterwards lanes with bit 2 set hold the total of y.
template <int V, bool EXTRA>
static __device__ __forceinline__ void reduce_transposed(float (&x)[V], float &y, int lane)
{
    static_assert(V == 8 || V == 16, "8 or 16 values");
    static_assert(!EXTRA || V == 8, "the extra value rides with 8 values");
    constexpr int H = V / 2;
#pragma unroll
    for (int i = 0; i < H; ++i) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x[i]), __float_as_uint(x[i + H]), false, false);
        x[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    if (EXTRA) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(y), __float_as_uint(y), false, false);
        y = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
#pragma unroll
    for (int i = 0; i < H / 2; ++i) {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x[i]), __float_as_uint(x[i + H / 2]), false, false);
        x[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    if (EXTRA) {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(y), __float_as_uint(y), false, false);
        y = __uint_as_float(r[0]) + __uint_as_float(r[1]);
        y += dpp_ror8(y);
    }
    const bool b3 = lane & 8;
#pragma unroll
    for (int i = 0; i < H / 4; ++i) {
        const float keep = b3 ? x[i + H / 4] : x[i];
        const float send = b3 ? x[i] : x[i + H / 4];
        x[i] = keep + dpp_ror8(send);
    }
    if (EXTRA) {
        const bool b2 = lane & 4;
        const float keep = b2 ? y : x[0];
        const float send = b2 ? x[0] : y;
        float r = keep + dpp_half_mirror(send);
        r += dpp_xor1(r);
        r += dpp_xor2(r);
        x[0] = r;
        y = r;
    } else {
#pragma unroll
        for (int i = 0; i < V / 8; ++i) {
            float r = x[i];
            r += dpp_half_mirror(r);
            r += dpp_xor1(r);
            r += dpp_xor2(r);
            x[i] = r;
        }
    }
}

__device__ __forceinline__ long long wave_sum_i64(long long v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    return v;
}

// Per-Gaussian record in sorted order, 64 bytes, written by k_records.
struct alignas(16) GRec {
    float alpha, beta2, gamma, z;   // exp2-units quadratic form in index units; depth (m)
    uint32_t rx, ry;                // ramp fraction frac(mu/(N p) + 1/2) in 0.32 fixed point
    float rxf, ryf;                 // the same as signed float in [-1/2, 1/2)
    float kappa[4];                 // carrier frac(phi/2pi - z/lambda_c), revolutions
    float amp[4];                   // a_c o 2 pi sqrt(det) / (px py nx ny)
};
static_assert(sizeof(GRec) == 64, "record must stay 64 B");

// Tilted-Gaussian record (input order), 96 bytes, written by k_tilt_records: the exp2-units
// linear forms u = U . (m_x, m_y, k_z), v = V . (...) and k_oz = N . (...) (m in index units,
// k_z in cycles per metre), depth, ramp (as GRec), carrier and amplitude a_c o 2 pi s_u s_v
// lambda_c / (px py nx ny).
struct alignas(16) TRec {
    float U[3], V[3], N[3], z;
    uint32_t rx, ry;
    float rxf, ryf, pad0, pad1;
    float kappa[4];
    float amp[4];
};
static_assert(sizeof(TRec) == 96, "tilted record must stay 96 B");

// Tilted Gaussians of one call (device arrays, amplitude [C][n]).
struct TView {
    int64_t n;
    const float *mean_x, *mean_y, *depth, *quat_w, *quat_x, *quat_y, *quat_z, *scale_u, *scale_v, *opacity,
        *amplitude, *phase;
};

// Gradient outputs of the tilted adjoint (device arrays, amplitude [C][n]).
struct TGrads {
    float *mean_x, *mean_y, *depth, *quat_w, *quat_x, *quat_y, *quat_z, *scale_u, *scale_v, *opacity, *amplitude,
        *phase;
};

// Forward work item: candidates [chunk*CH, min((chunk+1)*CH, L)) of sorted tile k.
struct Item {
    int32_t tile;    // index into the rho-sorted tile list
    int32_t chunk;
    int32_t slot;    // partial-sum slot, or -1 when the tile has a single item (direct write)
    int32_t pad;
};

// Backward work item: Gaussians [chunk*W, +W) over sorted tiles [k0, k1), W the adjoint's work-group size.
struct BItem {
    int32_t chunk;
    int32_t k0, k1;
    int32_t slot;
};

// Gaussians of one scene: a view into caller arrays; amplitude channel c of Gaussian i is
// amplitude[c * amp_stride + i] (amp_stride = total Gaussians of the concatenated batch).
struct GView {
    int64_t n;
    const float *mean_x, *mean_y, *depth, *cov_xx, *cov_xy, *cov_yy, *opacity, *amplitude, *phase;
    int64_t amp_stride;
};

struct GradView {
    float *mean_x, *mean_y, *depth, *cov_xx, *cov_xy, *cov_yy, *opacity, *amplitude, *phase;
    int64_t amp_stride;
};

constexpr int MAX_SCENES = 64;

// Per-scene pointers of the forward accumulation.
struct FwdScene {
    const GRec *rec;
    const int32_t *tile_L;
    const Item *items;
    const int2 *tile_slots;
    float2 *partials;
    float2 *spectrum;
    long long *counters;
};

// Per-scene pointers of the adjoint.
struct BwdScene {
    const GRec *rec;
    const float2 *gpack;  // (|Gs_c|, arg Gs_c / 2 pi) region-major: [region][block][c][lane]
    const BItem *bitems;
    float *bpartials;
    long long *counters;
    int64_t n;
};

struct FwdTab {
    int32_t n;
    int32_t pad;
    FwdScene s[MAX_SCENES];
};
struct BwdTab {
    int32_t n;
    int32_t pad;
    BwdScene s[MAX_SCENES];
};

// Scalar problem constants passed by value to kernels.
struct Consts {
    int32_t nx, ny, C, pad0;
    double px, py;
    double lambda[4];
    double inv_lambda[4];
    double tau2;        // log2(1/eps)
    double K2;          // 2 pi^2 log2(e)
    int32_t forward;    // 1: cull zero-amplitude Gaussians too
    int32_t phase_mode; // 0 exact base, 1 FP32 base (precision study)
    int32_t depth_grad; // backward: accumulate the depth-gradient sums
    int32_t pad1;
    double nurx, nury;  // reference plane wave's transverse frequency (cycles / m)
    double mrx, mry;    // the same in index units (nu_r N p): centre of every spectral support
};

// Per-shape plan owned by the context.
struct Plan {
    int32_t nx = 0, ny = 0, F = 4, tile_h = 32;
    int32_t ntx = 0, nty = 0, ntiles = 0;
    int32_t tx_min = 0, ty_min = 0;
    // device arrays
    int32_t *tile_xy = nullptr;       // [ntiles] packed (tx & 0xffff) | (ty << 16), rho-sorted
    int32_t *tile_bucket = nullptr;   // [ntiles] floor(rho) of each sorted tile
    int32_t *tile_cum = nullptr;      // [NBUCKET] number of sorted tiles with bucket <= b
    float2 *tw_x = nullptr;           // [nx] exp(-j 2 pi k / nx)
    float2 *tw_y = nullptr;           // [ny]
    int32_t radix_x[16] = {0}, nrad_x = 0;
    int32_t radix_y[16] = {0}, nrad_y = 0;
    // split-bf16 DFT matrices (lazily built)
    void *dft_mats = nullptr;
    size_t dft_bytes = 0;
};

// Workspace layout for one scene batch.
struct Layout {
    size_t total = 0;
    size_t off_keys_a, off_keys_b, off_vals_a, off_vals_b, off_sort_hist, off_bucket_hist, off_cum;
    size_t off_counters, off_records, off_tile_L, off_tile_slots, off_items, off_range_base, off_bitems, off_partials, off_bpartials;
    size_t off_spectrum, off_gspec, off_dtab, off_d0tab, off_chunk_items;
    int32_t nsx = 0, nsy = 0, sx_min = 0, sy_min = 0, F = 4;
    int64_t n = 0;
    int32_t sort_blocks = 0;
    int64_t max_items = 0, max_slots = 0, max_bitems = 0, max_bslots = 0;
    // item-table capacity that covers every tiling sharing this byte budget (F = 2 has the most slots)
    static int64_t max_slots_bound(size_t part_bytes, int C, int ntiles)
    {
        return (int64_t)(part_bytes / ((size_t)C * 2 * WG * 8)) / 2 + ntiles + 1;
    }
};

// Device counters block (int64 for sums; the first entries are the scheduling counters).
enum Counter {
    CTR_WORK = 0,        // forward persistent-queue head
    CTR_BWORK = 1,       // backward persistent-queue head
    CTR_NVALID = 2,
    CTR_NCULLED = 3,
    CTR_NITEMS = 4,
    CTR_CHUNK = 5,
    CTR_NBITEMS = 6,
    CTR_TRB = 7,
    CTR_PAIRS = 8,       // (tile, Gaussian) pairs evaluated
    CTR_CAND = 9,        // (tile, Gaussian) candidates tested
    CTR_CLAMPED = 10,    // exact blending: eps-windows cut at half the grid
    CTR_COUNT = 16
};

// ---- kernel launchers (each enqueues on `stream`, returns hipError_t) ----
hipError_t launch_keys(const GView &g, const Consts &k, uint64_t *keys, uint32_t *vals,
                       uint32_t *bucket_hist, long long *counters, hipStream_t s);
// Blocks (and 256-entry histograms) radix_sort_48 uses for n keys.
int sort_blocks_for(int64_t n);
hipError_t radix_sort_48(uint64_t *keys_a, uint32_t *vals_a, uint64_t *keys_b, uint32_t *vals_b,
                         uint32_t *block_hist, int64_t n, int nblocks, hipStream_t s,
                         uint64_t **keys_out, uint32_t **vals_out);
hipError_t launch_records(const GView &g, const Consts &k, const uint64_t *keys,
                          const uint32_t *vals, GRec *rec, int64_t n, const long long *counters,
                          hipStream_t s);
hipError_t launch_bin_forward(const Plan &p, const uint32_t *bucket_hist, uint32_t *cum, int32_t *tile_L,
                              int2 *tile_slots, Item *items, int64_t max_items, int64_t max_slots, int base_chunk,
                              long long *counters, hipStream_t s);
hipError_t launch_bin_backward(const Plan &p, const uint64_t *keys, BItem *bitems, int2 *chunk_items,
                               int32_t *range_base, int max_ranges, int64_t max_bitems, long long *counters, int64_t n,
                               int chunk, hipStream_t s);
// Writes the scene table and the prefix of per-scene work-item counts, zeroes the queue head.
hipError_t launch_fwd_table(const FwdTab &tab, FwdScene *dst, int32_t *prefix, long long *queue, hipStream_t s);
hipError_t launch_bwd_table(const BwdTab &tab, BwdScene *dst, int32_t *prefix, long long *queue, hipStream_t s);
hipError_t launch_accumulate(const Plan &p, const Consts &k, const FwdScene *scenes, const int32_t *prefix,
                             int n_scenes, long long *queue, int grid, hipStream_t s);
hipError_t launch_reduce_partials(const Plan &p, const Consts &k, const FwdScene *scenes, int n_scenes,
                                  hipStream_t s);

// Exact alpha wave blending (k_exact.hip): device buffers of one call.
struct ExactBuffers {
    uint64_t *keys_a, *keys_b;
    uint32_t *vals_a, *vals_b, *sort_hist;
    int sort_blocks;
    void *rec;     // 64-byte records, front to back
    float *tmap;   // transmittance [ny][nx]
    float2 *pimgs;  // one batch, two Gaussians per image [(B + 1) / 2][ny][nx]: the masked
                    // profiles and their transforms; in the adjoint also the spectra whose
                    // inverse transforms are the real maps r_k
    int4 *colwin, *rowwin;    // per batch Gaussian: window columns / rows as (first, count, 0, 0)
    int4 *pcolwin, *prowwin;  // per packed image: the two Gaussians' windows
    long long *counters;      // CTR_COUNT counters: culled Gaussians, clamped windows
};
size_t exact_batch(int nx, int ny);
// Extra device buffers of the exact-blending adjoint.
struct ExactBwdBuffers {
    float2 *gspec;  // FFT of the field gradient [C][ny][nx]
    float *ckpt;    // the map at every batch start [nbatch][ny][nx]
    float *dmap;    // running back-to-front accumulator [ny][nx]
    float *pspec;   // spectral partial sums [M / 256][64][12]
    float *pspat;   // spatial partial sums [8 x 8 tiles][64][8]
};
int64_t exact_ckpt_count(int64_t n, int nx, int ny);
hipError_t run_exact_backward(const Plan &p, const Consts &k, const GView &g, const ExactBuffers &eb,
                              const ExactBwdBuffers &bb, const float2 *grad_field, const GradView &out, hipStream_t s);
hipError_t run_exact_forward(const Plan &p, const Consts &k, const GView &g, const ExactBuffers &eb, float2 *spec,
                             hipStream_t s);
hipError_t run_probes(int n_cu, hipStream_t s, double *trans_ops, double *valu_ops, double *hbm_bytes);
// Region-major per-frequency tables of the adjoint: dpack [nreg][ADJ_NB][C][64] and d0
// [nreg][2][C] (geometry only), gpack [scene][nreg][ADJ_NB][C][64] from the scenes' Gs.
hipError_t launch_adj_pack(const Consts &k, const AdjGeom &geo, int n_scenes, const float2 *gspecs, float2 *gpack,
                           float *dpack, double *d0, hipStream_t s);
hipError_t launch_adjoint(const Plan &p, const Consts &k, const BwdScene *scenes, const int32_t *prefix, int n_scenes,
                          long long *queue, const float *dpack, const double *d0, const AdjGeom &geo, int grid,
                          hipStream_t s);
hipError_t launch_grad_final(const GView &g, const Consts &k, const uint32_t *vals, const int2 *chunk_items,
                             const int32_t *range_base, const float *bpartials, const GradView &grads, int64_t n,
                             const long long *counters, int chunk, hipStream_t s);
hipError_t launch_sum_counters(long long *const *src, int n, long long *dst, hipStream_t s);
int adjoint_occupancy(int C, int depth);
hipError_t launch_synth(GView g, float *base, int64_t n, uint64_t seed, const Consts &k, hipStream_t s);
int accumulate_occupancy(int C, int F);
hipError_t launch_zero_counters(long long *counters, uint32_t *bucket_hist, hipStream_t s);
hipError_t launch_copy_counters(const long long *src, long long *dst, hipStream_t s);
int fft_col_batch(int n);
size_t l2_workspace_bytes();
hipError_t launch_l2_grad(const float2 *u, const float2 *t, float2 *g, double *loss, void *ws, int64_t n, hipStream_t s);

// Stages timed with HIP events when profiling is on (gws_set_profiling).
enum Stage {
    ST_PREP = 0, ST_BIN, ST_ACCUM, ST_REDUCE, ST_XFORM_INV, ST_XFORM_FWD, ST_DTABLE, ST_ADJOINT, ST_FINAL, ST_LOSS,
    ST_DPAC, ST_FOCAL, ST_HOLO, ST_COUNT
};
hipError_t launch_fft2d(const Plan &p, int batch, int direction, const float2 *in, float2 *out,
                        hipStream_t s);
// Focal stack (angular-spectrum propagation of one field to up to STACK_MAXK planes per launch).
constexpr int STACK_MAXK = 32, STACK_MAXC = 4;
struct StackArgs {
    int32_t K, C, ny, half_band;
    float scale;                         // 1 / (N_x N_y), the inverse transform's normalisation
    float pad0;
    double dnux, dnuy;                   // frequency steps 1 / (N p)
    double inv_l[STACK_MAXC];            // 1 / lambda_c
    double z[STACK_MAXK];                // plane distances (m)
    double piston[STACK_MAXK * STACK_MAXC];  // frac(z_k / lambda_c), reduced on the host in FP64
};
bool focal_stack_fits(int nx);
hipError_t launch_focal_stack(const Plan &p, const float2 *spec, float2 *planes, float *intensity,
                              const StackArgs &sa, hipStream_t s);
// Holographics transform: camera and display parameters (FP64), and the in-plane outputs.
struct HoloArgs {
    double R[9], t[3];            // world to view: p = R mu + t (row-major R)
    double centre[3];             // camera centre in world space, -R^T t
    double fx, fy, cx, cy, near;
    double A[4], b[2];            // ray space to hologram plane (row-major 2 x 2, offset)
    double depth_scale, depth_offset;
    int32_t sh_degree, pad;
};
struct PlaneOut {
    float *mean_x, *mean_y, *depth, *cov_xx, *cov_xy, *cov_yy, *opacity;
};
hipError_t launch_holographics(const HoloArgs &a, int64_t n, const float *mean, const float *quat, const float *scale,
                               const float *sh, const PlaneOut &out, hipStream_t s);

// Display kernels: per-channel max |u| (as float bits), double-phase coding, e^{jP}.
hipError_t launch_amax(const float2 *u, int64_t m, int C, uint32_t *amax_bits, hipStream_t s);
hipError_t launch_dpac(const float2 *u, int nx, int ny, int C, const uint32_t *amax_bits, float amax_fixed,
                       float *phase, hipStream_t s);
hipError_t launch_phase_field(const float *phase, int64_t n, float2 *u, hipStream_t s);

// Windowed transforms of the exact-blending images; a window is one or two periodic intervals
// (start, length, start, length), an unused second interval with length 0.
hipError_t launch_fft2d_cols_out(const Plan &p, int batch, int direction, float2 *buf, const int4 *colwin,
                                 hipStream_t s);
hipError_t launch_fft2d_win(const Plan &p, int batch, int direction, const float2 *in, float2 *out,
                            const int4 *colwin, const int4 *rowwin, hipStream_t s);
hipError_t launch_dft_bf16x3(Plan &p, int batch, int direction, const float2 *in, float2 *out,
                             void *ws, hipStream_t s);
size_t dft_bf16x3_workspace(int nx, int ny, int batch);
hipError_t launch_tilt_records(const TView &g, const Consts &k, TRec *rec, int2 *rect, long long *counters,
                               hipStream_t s);
// Parts a tile's Gaussians are split into (one work item each) for n Gaussians; the forward
// writes one partial spectrum per part (partial: parts x C x ny x nx, NULL for one part) and
// adds them in part order.
int tilt_parts(int64_t n);
hipError_t launch_tilt_accumulate(const Consts &k, const TRec *rec, const int2 *rect, int64_t n, float2 *spectrum,
                                  float2 *partial, long long *counters, int n_cu, hipStream_t s);
hipError_t launch_tilt_offsets(const int2 *rect, int64_t n, int64_t *off, int64_t *bsum, hipStream_t s);
hipError_t launch_tilt_adjoint(const Consts &k, const TRec *rec, const int2 *rect, int64_t n, const float2 *gspec,
                               const int64_t *off, float *part, long long *counters, int n_cu, hipStream_t s);
hipError_t launch_tilt_grad_final(const TView &g, const Consts &k, const int2 *rect, const int64_t *off,
                                  const float *part, const TGrads &gr, hipStream_t s);
int tilt_slot_floats(int C);  // floats per (Gaussian, tile) slot of the tilted adjoint
hipError_t build_dft_mats(Plan &p);
void free_dft_mats(Plan &p);

int occupancy_blocks(const void *kernel, int block, size_t dyn_smem);

}  // namespace gws
