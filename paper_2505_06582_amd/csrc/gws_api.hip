// Host side of libgws: the C ABI of include/gws.h, argument validation, per-shape plans,
// workspace layout and the launch sequence of the forward and backward hot path.
#include <math.h>
#include <cmath>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "gws_internal.h"

using namespace gws;

struct gws_ctx {
    int device = 0;
    int n_cu = 0;
    std::string last_error;
    // per (nx, ny, F, m_r quantised): the tile order depends on the supports' common centre m_r
    std::map<std::tuple<int, int, int, long long, long long>, Plan> plans;
    long long *d_stats = nullptr;  // copy of the counters of the last call
    int64_t last_n = 0;
    int last_tile_config = 1;
    int last_graph = 0;
    std::map<int, int> acc_occ;  // resident work-groups per CU by kernel variant
    std::map<std::tuple<int, int, int, int>, int> tuned;  // (nx, ny, C, log2 n) -> tile_config
    // batched-graph cache
    struct GraphKey {
        std::vector<int64_t> offsets;
        std::vector<uintptr_t> ptrs;
        gws_problem prob;
        int backward;
    };
    std::vector<std::pair<GraphKey, hipGraphExec_t>> graphs;
    // stage profiling
    int profiling = 0;
    struct Rec {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    void *scratch = nullptr;  // this device's copy of the allocation-free forward's scratch array
    float *tilt_part = nullptr;  // per-(Gaussian, tile) sums of the tilted adjoint, grown on demand
    size_t tilt_part_bytes = 0;
};

static hipEvent_t pool_event(gws_ctx *ctx)
{
    if (!ctx->pool.empty()) {
        hipEvent_t e = ctx->pool.back();
        ctx->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Records an event pair around one stage on the caller's stream when profiling is on.
struct StageScope {
    gws_ctx *ctx;
    hipStream_t s;
    int stage;
    hipEvent_t a = nullptr;
    bool on;
    StageScope(gws_ctx *c, hipStream_t st, int sg, bool enable = true) : ctx(c), s(st), stage(sg)
    {
        on = enable && ctx->profiling;
        if (on) {
            a = pool_event(ctx);
            if (a) hipEventRecord(a, s);
        }
    }
    ~StageScope()
    {
        if (on && a) {
            hipEvent_t b = pool_event(ctx);
            if (b) {
                hipEventRecord(b, s);
                ctx->recs.push_back({stage, a, b});
            } else {
                ctx->pool.push_back(a);
            }
        }
    }
};

static thread_local std::string g_tls_error;
static void load_tune_cache(gws_ctx *ctx, const char *path);

static gws_status fail(gws_ctx *ctx, gws_status st, const std::string &msg)
{
    if (ctx) ctx->last_error = msg;
    g_tls_error = msg;
    return st;
}

#define HIP_CHECK(ctx, call)                                                                                 \
    do {                                                                                                     \
        hipError_t e_ = (call);                                                                              \
        if (e_ != hipSuccess)                                                                                \
            return fail((ctx), GWS_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));              \
    } while (0)

extern "C" int gws_abi_version(void) { return GWS_ABI_VERSION; }

extern "C" const char *gws_status_string(gws_status s)
{
    switch (s) {
    case GWS_OK: return "ok";
    case GWS_ERR_INVALID_ARG: return "invalid argument";
    case GWS_ERR_SHAPE: return "unsupported grid shape";
    case GWS_ERR_UNSUPPORTED: return "unsupported request";
    case GWS_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
    case GWS_ERR_NO_DEVICE: return "no gfx950 device";
    case GWS_ERR_HIP: return "HIP runtime error";
    case GWS_ERR_OOM: return "out of device memory";
    default: return "unknown status";
    }
}

extern "C" const char *gws_last_error(const gws_ctx *ctx) { return ctx ? ctx->last_error.c_str() : g_tls_error.c_str(); }

// ---------------------------------------------------------------------------------
// Validation
// ---------------------------------------------------------------------------------
static bool smooth235(int n)
{
    if (n <= 0) return false;
    for (int p : {2, 3, 5})
        while (n % p == 0) n /= p;
    return n == 1;
}

static gws_status check_grid(int nx, int ny)
{
    if (nx < 16 || ny < 16 || nx > 8192 || ny > 8192) return GWS_ERR_SHAPE;
    if ((nx & 1) || (ny & 1)) return GWS_ERR_SHAPE;
    if (!smooth235(nx) || !smooth235(ny)) return GWS_ERR_SHAPE;
    return GWS_OK;
}

extern "C" gws_status gws_check_problem(const gws_problem *p)
{
    if (!p) return GWS_ERR_INVALID_ARG;
    if (!(p->pitch_x > 0.0) || !(p->pitch_y > 0.0) || !isfinite(p->pitch_x) || !isfinite(p->pitch_y))
        return GWS_ERR_INVALID_ARG;
    if (p->n_lambda < 1 || p->n_lambda > GWS_MAX_LAMBDA) return GWS_ERR_INVALID_ARG;
    for (int c = 0; c < p->n_lambda; ++c)
        if (!(p->lambdas[c] > 0.0) || !isfinite(p->lambdas[c])) return GWS_ERR_INVALID_ARG;
    if (p->blend != GWS_BLEND_OIT && p->blend != GWS_BLEND_EXACT) return GWS_ERR_INVALID_ARG;
    if (p->xform != GWS_XFORM_FFT_FP32 && p->xform != GWS_XFORM_DFT_BF16X3) return GWS_ERR_INVALID_ARG;
    if (p->eps_support != 0.0 && !(p->eps_support > 0.0 && p->eps_support <= 1e-3)) return GWS_ERR_INVALID_ARG;
    if (p->phase_mode != 0 && p->phase_mode != 1 && p->phase_mode != 2) return GWS_ERR_INVALID_ARG;
    if (p->tile_config < 0 || p->tile_config > gws_tile_config_count()) return GWS_ERR_INVALID_ARG;
    if (!isfinite(p->ref_nu_x) || !isfinite(p->ref_nu_y) || fabs(p->ref_nu_x) * p->pitch_x > 0.5 ||
        fabs(p->ref_nu_y) * p->pitch_y > 0.5)
        return GWS_ERR_INVALID_ARG;
    if (p->blend == GWS_BLEND_EXACT && (p->ref_nu_x != 0.0 || p->ref_nu_y != 0.0)) return GWS_ERR_UNSUPPORTED;
    const gws_status gs = check_grid(p->nx, p->ny);
    if (gs != GWS_OK) return gs;
    return GWS_OK;
}

// Tilings: frequencies per lane (F) of the forward accumulation and of the adjoint.  The
// work-group tile is 32 x 8F frequencies, the wavefront sub-tile 16 x 4F.
// Forward configurations the autotuner chooses among: (F, frequencies per lane of the
// accumulation: tile 32 x 8F; base chunk, candidates per work item before the binning grows it
// to fit the partial-sum budget).  Small chunks split the long DC tiles into more, shorter
// items (better balance, more partial sums to reduce); large ones the reverse.  The adjoint's
// geometry is fixed (regions of the F = 8 tiling), so a configuration only shapes the forward.
static const int kTileCfg[][2] = {{4, 512}, {4, 1024}, {8, 1024}, {8, 512}, {2, 1024},
                                  {4, 2048}, {2, 512}, {2, 2048}, {8, 2048}};
static const int kNumTileCfg = (int)(sizeof(kTileCfg) / sizeof(kTileCfg[0]));
// Untuned default: F = 4 with 1024-candidate chunks, the fastest measured on MI355X for 1e5
// Gaussians at 1080 x 1920 x 3.
static const int kDefaultTileCfg = 2;

extern "C" int gws_tile_config_count(void) { return kNumTileCfg; }

static Consts make_consts(const gws_problem *p, int forward)
{
    Consts k;
    memset(&k, 0, sizeof(k));
    k.nx = p->nx;
    k.ny = p->ny;
    k.C = p->n_lambda;
    k.px = p->pitch_x;
    k.py = p->pitch_y;
    for (int c = 0; c < 4; ++c) {
        k.lambda[c] = c < p->n_lambda ? p->lambdas[c] : 1.0;
        k.inv_lambda[c] = 1.0 / k.lambda[c];
    }
    const double eps = p->eps_support > 0.0 ? p->eps_support : 1e-7;
    k.tau2 = log2(1.0 / eps);
    k.K2 = 2.0 * M_PI * M_PI / log(2.0);
    k.forward = forward;
    k.phase_mode = p->phase_mode == 1 ? 1 : 0;
    k.nurx = p->ref_nu_x;
    k.nury = p->ref_nu_y;
    k.mrx = p->ref_nu_x * p->nx * p->pitch_x;
    k.mry = p->ref_nu_y * p->ny * p->pitch_y;
    return k;
}

// ---------------------------------------------------------------------------------
// Plans
// ---------------------------------------------------------------------------------
static int floor_div(int a, int b) { return (a >= 0) ? a / b : -((-a + b - 1) / b); }

static int isqrt_floor(long long v)
{
    long long r = (long long)sqrt((double)v);
    while (r * r > v) --r;
    while ((r + 1) * (r + 1) <= v) ++r;
    return (int)r;
}

static void factor_radices(int n, int32_t *r, int32_t *nr)
{
    int k = 0;
    for (const int f : {16, 8, 4, 2, 15, 9, 5, 3})
        while (n % f == 0) { r[k++] = f; n /= f; }
    *nr = k;
}

// Tiles are ordered by their distance (index units) from m_r, the centre every spectral
// support shares (DC under on-axis illumination, nu_r N p under a reference plane wave).
static gws_status build_plan(gws_ctx *ctx, Plan &p, int nx, int ny, int F, double mrx, double mry)
{
    p.nx = nx;
    p.ny = ny;
    p.F = F;
    p.tile_h = 2 * sub_h(F);
    const int TH = p.tile_h;
    const int hx = nx / 2, hy = ny / 2;
    p.tx_min = floor_div(-hx, TILEX);
    p.ty_min = floor_div(-hy, TH);
    const int tx_max = floor_div(hx - 1, TILEX), ty_max = floor_div(hy - 1, TH);
    p.ntx = tx_max - p.tx_min + 1;
    p.nty = ty_max - p.ty_min + 1;
    p.ntiles = p.ntx * p.nty;
    struct T { int bucket, ty, tx; };
    std::vector<T> tiles;
    tiles.reserve(p.ntiles);
    for (int ty = p.ty_min; ty <= ty_max; ++ty)
        for (int tx = p.tx_min; tx <= tx_max; ++tx) {
            const int x0 = std::max(tx * TILEX, -hx), x1 = std::min(tx * TILEX + TILEX - 1, hx - 1);
            const int y0 = std::max(ty * TH, -hy), y1 = std::min(ty * TH + TH - 1, hy - 1);
            int b;
            if (mrx == 0.0 && mry == 0.0) {
                const long long dx = x0 > 0 ? x0 : (x1 < 0 ? -x1 : 0);
                const long long dy = y0 > 0 ? y0 : (y1 < 0 ? -y1 : 0);
                b = isqrt_floor(dx * dx + dy * dy);
            } else {
                const double dx = std::max({x0 - mrx, mrx - x1, 0.0}), dy = std::max({y0 - mry, mry - y1, 0.0});
                b = (int)std::min(floor(sqrt(dx * dx + dy * dy)), (double)(NBUCKET - 1));
            }
            if (b > NBUCKET - 1) b = NBUCKET - 1;
            tiles.push_back({b, ty, tx});
        }
    std::stable_sort(tiles.begin(), tiles.end(), [](const T &a, const T &b) { return a.bucket < b.bucket; });
    std::vector<int32_t> xy(p.ntiles), bk(p.ntiles), cum(NBUCKET, 0);
    for (int i = 0; i < p.ntiles; ++i) {
        xy[i] = (int32_t)((tiles[i].tx & 0xffff) | (tiles[i].ty << 16));
        bk[i] = tiles[i].bucket;
        cum[tiles[i].bucket] += 1;
    }
    for (int b = 1; b < NBUCKET; ++b) cum[b] += cum[b - 1];
    factor_radices(nx, p.radix_x, &p.nrad_x);
    factor_radices(ny, p.radix_y, &p.nrad_y);
    std::vector<float2> twx(nx), twy(ny);
    for (int i = 0; i < nx; ++i) twx[i] = make_float2((float)cos(-2.0 * M_PI * i / nx), (float)sin(-2.0 * M_PI * i / nx));
    for (int i = 0; i < ny; ++i) twy[i] = make_float2((float)cos(-2.0 * M_PI * i / ny), (float)sin(-2.0 * M_PI * i / ny));
    if (hipMalloc(&p.tile_xy, sizeof(int32_t) * p.ntiles) != hipSuccess ||
        hipMalloc(&p.tile_bucket, sizeof(int32_t) * p.ntiles) != hipSuccess ||
        hipMalloc(&p.tile_cum, sizeof(int32_t) * NBUCKET) != hipSuccess ||
        hipMalloc(&p.tw_x, sizeof(float2) * nx) != hipSuccess || hipMalloc(&p.tw_y, sizeof(float2) * ny) != hipSuccess)
        return fail(ctx, GWS_ERR_OOM, "plan allocation failed");
    HIP_CHECK(ctx, hipMemcpy(p.tile_xy, xy.data(), sizeof(int32_t) * p.ntiles, hipMemcpyHostToDevice));
    HIP_CHECK(ctx, hipMemcpy(p.tile_bucket, bk.data(), sizeof(int32_t) * p.ntiles, hipMemcpyHostToDevice));
    HIP_CHECK(ctx, hipMemcpy(p.tile_cum, cum.data(), sizeof(int32_t) * NBUCKET, hipMemcpyHostToDevice));
    HIP_CHECK(ctx, hipMemcpy(p.tw_x, twx.data(), sizeof(float2) * nx, hipMemcpyHostToDevice));
    HIP_CHECK(ctx, hipMemcpy(p.tw_y, twy.data(), sizeof(float2) * ny, hipMemcpyHostToDevice));
    return GWS_OK;
}

static void free_plan(Plan &p)
{
    hipFree(p.tile_xy);
    hipFree(p.tile_bucket);
    hipFree(p.tile_cum);
    hipFree(p.tw_x);
    hipFree(p.tw_y);
    free_dft_mats(p);
}

static long long mr_key(double mr) { return llround(mr * 1048576.0); }

// The plan of a shape if an earlier call built it, else nullptr (never allocates).
static Plan *find_plan(gws_ctx *ctx, int nx, int ny, int F, double mrx = 0.0, double mry = 0.0)
{
    auto it = ctx->plans.find(std::make_tuple(nx, ny, F, mr_key(mrx), mr_key(mry)));
    return it == ctx->plans.end() ? nullptr : &it->second;
}

static gws_status get_plan(gws_ctx *ctx, int nx, int ny, int F, Plan **out, double mrx = 0.0, double mry = 0.0)
{
    auto key = std::make_tuple(nx, ny, F, mr_key(mrx), mr_key(mry));
    auto it = ctx->plans.find(key);
    if (it != ctx->plans.end()) {
        *out = &it->second;
        return GWS_OK;
    }
    HIP_CHECK(ctx, hipSetDevice(ctx->device));
    Plan p;
    const gws_status st = build_plan(ctx, p, nx, ny, F, mrx, mry);
    if (st != GWS_OK) {
        free_plan(p);
        return st;
    }
    auto res = ctx->plans.emplace(key, p);
    *out = &res.first->second;
    return GWS_OK;
}

// ---------------------------------------------------------------------------------
// Workspace layout
// ---------------------------------------------------------------------------------
static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

static int64_t fwd_max_slots_f4(int64_t n) { return std::max<int64_t>(512, std::min<int64_t>(32768, n)); }

static int ntiles_for(int nx, int ny, int F)
{
    const int hx = nx / 2, hy = ny / 2, TH = 2 * sub_h(F);
    const int ntx = floor_div(hx - 1, TILEX) - floor_div(-hx, TILEX) + 1;
    const int nty = floor_div(hy - 1, TH) - floor_div(-hy, TH) + 1;
    return ntx * nty;
}

// Per-scene region.  One region serves forward and backward under every tiling: tile
// arrays are sized for the smallest tiles (F = 2), the partial-sum area is a fixed byte
// budget whose slot count depends on the forward tiling.
static Layout make_layout(const gws_problem *p, int64_t n, int f_fwd, int f_bwd, bool fwd_only = false)
{
    Layout L;
    const int C = p->n_lambda;
    const int ntiles = ntiles_for(p->nx, p->ny, 2);
    L.n = n;
    L.F = f_fwd;
    L.sort_blocks = sort_blocks_for(n);
    const size_t part_bytes = (size_t)fwd_max_slots_f4(n) * C * 4 * WG * sizeof(float2);
    L.max_slots = (int64_t)(part_bytes / ((size_t)C * f_fwd * WG * sizeof(float2)));
    L.max_items = L.max_slots / 2 + ntiles + 1;
    // backward items: (chunk of one adjoint work-group's Gaussians, range of TRB tiles); the
    // binning grows TRB from one tile until the items fit, so up to about 8192 items share the
    // GPU's ~512 work-group slots -- short enough that the heaviest (the widest supports near
    // DC) do not leave the launch's tail to a few work-groups, for small scenes as for large
    // (1k Gaussians at 1080 x 1920 x 3: fwd+bwd 4.2 -> 1.8 ms; 100k: 21.1 -> 20.7 ms)
    const int64_t nchunks = (n + ADJ_MIN_CHUNK - 1) / ADJ_MIN_CHUNK;
    L.max_bitems = nchunks + std::min<int64_t>(8192, nchunks * ntiles);   // no more items than (chunk, tile) pairs
    L.max_bslots = L.max_bitems;
    const int hx = p->nx / 2, hy = p->ny / 2, SY = sub_h(f_bwd);
    L.sx_min = floor_div(-hx, SUBX);
    L.sy_min = floor_div(-hy, SY);
    L.nsx = floor_div(hx - 1, SUBX) - L.sx_min + 1;
    L.nsy = floor_div(hy - 1, SY) - L.sy_min + 1;
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t r = o; o = align256(o + std::max<size_t>(bytes, 1)); return r; };
    L.off_counters = take(sizeof(long long) * CTR_COUNT);
    L.off_bucket_hist = take(sizeof(uint32_t) * NBUCKET);
    L.off_cum = take(sizeof(uint32_t) * NBUCKET);
    L.off_keys_a = take(sizeof(uint64_t) * n);
    L.off_keys_b = take(sizeof(uint64_t) * n);
    L.off_vals_a = take(sizeof(uint32_t) * n);
    L.off_vals_b = take(sizeof(uint32_t) * n);
    L.off_sort_hist = take(sizeof(uint32_t) * 256 * L.sort_blocks);
    L.off_records = take(sizeof(GRec) * n);
    L.off_tile_L = take(sizeof(int32_t) * ntiles);
    L.off_tile_slots = take(sizeof(int2) * ntiles);
    L.off_items = take(sizeof(Item) * (L.max_slots_bound(part_bytes, C, ntiles)));
    L.off_partials = take(part_bytes);
    // the adjoint's areas (empty in a forward-only layout)
    const size_t bw = fwd_only ? 0 : 1;
    L.off_bitems = take(bw * sizeof(BItem) * L.max_bitems);
    L.off_chunk_items = take(bw * sizeof(int2) * (nchunks + 1));
    L.off_range_base = take(bw * sizeof(int32_t) * (ntiles + 2));
    L.off_bpartials = take(bw * sizeof(float) * (size_t)L.max_bslots *
                           std::max(adj_wg(C, true) * adj_nv(C, true), adj_wg(C, false) * adj_nv(C, false)));
    L.total = o;
    return L;
}

// Whole-call layout: a shared head (scene tables, queue heads, spectra, transformed field
// gradients, propagation tables) followed by one region per scene.
struct BatchLayout {
    size_t total = 0;
    size_t off_ctrl = 0, off_ftab = 0, off_btab = 0, off_prefix = 0, off_spectra = 0, off_gspecs = 0, off_gpack = 0,
           off_dpack = 0, off_d0 = 0, off_dftws = 0;
    AdjGeom geo = {};
    int64_t pack_elems = 0;  // packed per-frequency elements of one scene (regions x blocks x C x 64)
    std::vector<size_t> scene_off;
    std::vector<int64_t> n;
};

static BatchLayout make_batch_layout(const gws_problem *p, int S, const int64_t *offsets, bool fwd_only = false)
{
    BatchLayout B;
    const int64_t M = (int64_t)p->nx * p->ny;
    const int C = p->n_lambda;
    const int hx = p->nx / 2, hy = p->ny / 2;
    B.geo.tx_min = floor_div(-hx, TILEX);
    B.geo.ty_min = floor_div(-hy, ADJ_RH);
    B.geo.ntx = floor_div(hx - 1, TILEX) - B.geo.tx_min + 1;
    B.geo.nreg = 2 * B.geo.ntx * (floor_div(hy - 1, ADJ_RH) - B.geo.ty_min + 1);
    B.pack_elems = (int64_t)B.geo.nreg * ADJ_NB * C * 64;
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t r = o; o = align256(o + std::max<size_t>(bytes, 1)); return r; };
    B.off_ctrl = take(sizeof(long long) * 8);
    B.off_ftab = take(sizeof(FwdScene) * S);
    B.off_btab = take(sizeof(BwdScene) * S);
    B.off_prefix = take(sizeof(int32_t) * (S + 1));
    B.off_spectra = take(sizeof(float2) * (size_t)S * C * M);
    // the adjoint's areas (empty in a forward-only layout; the bf16 DFT forward also uses the first)
    const size_t bw = fwd_only ? 0 : 1;
    B.off_gspecs = take(bw * sizeof(float2) * (size_t)S * C * M);
    B.off_gpack = take(bw * sizeof(float2) * (size_t)S * B.pack_elems);
    B.off_dpack = take(bw * sizeof(float) * (size_t)B.pack_elems);
    B.off_d0 = take(bw * sizeof(double) * (size_t)B.geo.nreg * 2 * C);
    // the split-bf16 DFT's operand planes (both directions), when that transform is chosen
    B.off_dftws = take(p->xform == GWS_XFORM_DFT_BF16X3 ? dft_bf16x3_workspace(p->nx, p->ny, S * C) : 0);
    for (int i = 0; i < S; ++i) {
        const int64_t ni = offsets[i + 1] - offsets[i];
        B.n.push_back(ni);
        B.scene_off.push_back(o);
        o = align256(o + make_layout(p, ni, 2, 2, fwd_only).total);
    }
    B.total = o;
    return B;
}

static gws_status check_offsets(int S, const int64_t *offsets, int64_t n)
{
    if (S < 1 || S > MAX_SCENES || !offsets) return GWS_ERR_INVALID_ARG;
    if (offsets[0] != 0 || offsets[S] != n) return GWS_ERR_INVALID_ARG;
    for (int i = 0; i < S; ++i)
        if (offsets[i + 1] < offsets[i]) return GWS_ERR_INVALID_ARG;
    return GWS_OK;
}

// Workspace of exact blending: sort buffers, records, transmittance map, one batch of
// full-grid images (two Gaussians each), the spectrum, the bf16 DFT's intermediate when used,
// and the adjoint's buffers.
struct ExactLayout {
    size_t off_keys_a = 0, off_keys_b = 0, off_vals_a = 0, off_vals_b = 0, off_sort_hist = 0, off_rec = 0,
           off_tmap = 0, off_spec = 0, off_dft = 0, off_gspec = 0, off_ckpt = 0, off_dmap = 0,
           off_pspec = 0, off_pspat = 0, off_win = 0, off_pimgs = 0, off_counters = 0, total = 0;
    int sort_blocks = 1;
};

static ExactLayout exact_layout(const gws_problem *p, int64_t n)
{
    ExactLayout L;
    const size_t M = (size_t)p->nx * p->ny;
    L.sort_blocks = sort_blocks_for(n);
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t r = o; o = align256(o + std::max<size_t>(bytes, 1)); return r; };
    L.off_keys_a = take(sizeof(uint64_t) * n);
    L.off_keys_b = take(sizeof(uint64_t) * n);
    L.off_vals_a = take(sizeof(uint32_t) * n);
    L.off_vals_b = take(sizeof(uint32_t) * n);
    L.off_sort_hist = take(sizeof(uint32_t) * 256 * L.sort_blocks);
    L.off_rec = take((size_t)64 * n);
    L.off_tmap = take(sizeof(float) * M);
    L.off_pimgs = take(sizeof(float2) * M * ((exact_batch(p->nx, p->ny) + 1) / 2));
    L.off_spec = take(sizeof(float2) * M * p->n_lambda);
    L.off_dft = take(p->xform == GWS_XFORM_DFT_BF16X3 ? dft_bf16x3_workspace(p->nx, p->ny, p->n_lambda) : 1);
    L.off_win = take(sizeof(int4) * 4 * 64);
    L.off_counters = take(sizeof(long long) * CTR_COUNT);
    // adjoint: transformed field gradient, map checkpoints, back-to-front accumulator, partial sums
    L.off_gspec = take(sizeof(float2) * M * p->n_lambda);
    L.off_ckpt = take(sizeof(float) * M * (size_t)exact_ckpt_count(n, p->nx, p->ny));
    L.off_dmap = take(sizeof(float) * M);
    L.off_pspec = take(sizeof(float) * ((M + 255) / 256) * 64 * 16);
    L.off_pspat = take(sizeof(float) * (size_t)((p->nx + 7) / 8) * ((p->ny + 7) / 8) * 64 * 8);
    L.total = o;
    return L;
}

extern "C" gws_status gws_workspace_size(const gws_ctx *ctx, const gws_problem *problem, int64_t n, size_t *bytes)
{
    (void)ctx;
    if (!bytes || n < 0) return GWS_ERR_INVALID_ARG;
    const gws_status st = gws_check_problem(problem);
    if (st != GWS_OK) return st;
    if (n > (int64_t)0x7fffffff) return GWS_ERR_INVALID_ARG;
    if (problem->blend == GWS_BLEND_EXACT) {
        *bytes = exact_layout(problem, n).total;
        return GWS_OK;
    }
    const int64_t off[2] = {0, n};
    *bytes = make_batch_layout(problem, 1, off).total;
    return GWS_OK;
}

// Exact blending over several scenes: one scene after another on the stream, sharing the
// workspace (sized for the largest scene).
static size_t exact_batched_bytes(const gws_problem *prob, int S, const int64_t *offsets)
{
    size_t b = 0;
    for (int i = 0; i < S; ++i) b = std::max(b, exact_layout(prob, offsets[i + 1] - offsets[i]).total);
    return b;
}

extern "C" gws_status gws_workspace_size_batched(const gws_ctx *ctx, const gws_problem *problem, int32_t n_scenes,
                                                 const int64_t *offsets, size_t *bytes)
{
    (void)ctx;
    if (!bytes || !offsets || n_scenes < 1) return GWS_ERR_INVALID_ARG;
    const gws_status st = gws_check_problem(problem);
    if (st != GWS_OK) return st;
    if (check_offsets(n_scenes, offsets, offsets[n_scenes]) != GWS_OK) return GWS_ERR_INVALID_ARG;
    *bytes = problem->blend == GWS_BLEND_EXACT ? exact_batched_bytes(problem, n_scenes, offsets)
                                               : make_batch_layout(problem, n_scenes, offsets).total;
    return GWS_OK;
}


// ---------------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------------
// Scratch of gws_forward_noalloc: a file-scope device array, so each GPU the library runs on
// holds its own copy until the process ends.  In host code its name is only a stand-in for the
// symbol; the device address of this GPU's copy is taken once per context (gws_create) with
// hipGetSymbolAddress and only that address is passed to kernels.
static __device__ __align__(256) char scratch[GWS_NOALLOC_SCRATCH_BYTES];

extern "C" gws_status gws_create(gws_ctx **out, int device)
{
    if (!out) return fail(nullptr, GWS_ERR_INVALID_ARG, "ctx pointer is NULL");
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return fail(nullptr, GWS_ERR_NO_DEVICE, "no HIP device");
    if (device < 0 || device >= count) return fail(nullptr, GWS_ERR_NO_DEVICE, "device index out of range");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return fail(nullptr, GWS_ERR_NO_DEVICE, "cannot query device");
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(nullptr, GWS_ERR_NO_DEVICE, std::string("device is ") + prop.gcnArchName + ", not gfx950");
    gws_ctx *ctx = new gws_ctx();
    ctx->device = device;
    ctx->n_cu = prop.multiProcessorCount;
    if (hipSetDevice(device) != hipSuccess || hipMalloc(&ctx->d_stats, sizeof(long long) * CTR_COUNT) != hipSuccess) {
        delete ctx;
        return fail(nullptr, GWS_ERR_OOM, "cannot allocate the statistics buffer");
    }
    (void)hipMemset(ctx->d_stats, 0, sizeof(long long) * CTR_COUNT);
    if (hipGetSymbolAddress(&ctx->scratch, HIP_SYMBOL(scratch)) != hipSuccess || !ctx->scratch) {
        hipFree(ctx->d_stats);
        delete ctx;
        return fail(nullptr, GWS_ERR_HIP, "cannot take the device address of the scratch array");
    }
    load_tune_cache(ctx, getenv("GWS_TUNE_CACHE"));
    *out = ctx;
    return GWS_OK;
}

extern "C" gws_status gws_destroy(gws_ctx *ctx)
{
    if (!ctx) return GWS_OK;
    hipSetDevice(ctx->device);
    for (auto &kv : ctx->plans) free_plan(kv.second);
    for (auto &g : ctx->graphs) hipGraphExecDestroy(g.second);
    for (auto &r : ctx->recs) {
        hipEventDestroy(r.a);
        hipEventDestroy(r.b);
    }
    for (auto e : ctx->pool) hipEventDestroy(e);
    hipFree(ctx->tilt_part);
    hipFree(ctx->d_stats);
    delete ctx;
    return GWS_OK;
}

extern "C" gws_status gws_get_stats(gws_ctx *ctx, gws_stats *out)
{
    if (!ctx || !out) return fail(ctx, GWS_ERR_INVALID_ARG, "null argument");
    long long h[CTR_COUNT];
    HIP_CHECK(ctx, hipSetDevice(ctx->device));
    HIP_CHECK(ctx, hipDeviceSynchronize());
    HIP_CHECK(ctx, hipMemcpy(h, ctx->d_stats, sizeof(h), hipMemcpyDeviceToHost));
    memset(out, 0, sizeof(*out));
    out->n_input = ctx->last_n;
    out->n_culled = h[CTR_NCULLED];
    out->n_items = h[CTR_NITEMS] + h[CTR_NBITEMS];
    out->chunk = h[CTR_CHUNK];
    out->n_pairs_evaluated = h[CTR_PAIRS];
    out->n_candidates = h[CTR_CAND];
    out->tile_config = ctx->last_tile_config;
    out->graph_replayed = ctx->last_graph;
    out->n_window_clamped = h[CTR_CLAMPED];
    out->n_tiles = 0;
    for (auto &kv : ctx->plans) out->n_tiles = std::max<int64_t>(out->n_tiles, kv.second.ntiles);
    return GWS_OK;
}

// ---------------------------------------------------------------------------------
// Forward / backward over a batch of scenes (a single scene is a batch of one)
// ---------------------------------------------------------------------------------
static gws_status check_gaussians(gws_ctx *ctx, const gws_gaussians *g)
{
    if (!g) return fail(ctx, GWS_ERR_INVALID_ARG, "gaussians is NULL");
    if (g->n < 0 || g->n > (int64_t)0x7fffffff) return fail(ctx, GWS_ERR_INVALID_ARG, "bad Gaussian count");
    if (g->n > 0 && (!g->mean_x || !g->mean_y || !g->depth || !g->cov_xx || !g->cov_xy || !g->cov_yy || !g->opacity ||
                     !g->amplitude || !g->phase))
        return fail(ctx, GWS_ERR_INVALID_ARG, "a Gaussian array is NULL");
    return GWS_OK;
}

static gws_status check_grads(gws_ctx *ctx, const gws_grads *gr)
{
    if (!gr || !gr->mean_x || !gr->mean_y || !gr->cov_xx || !gr->cov_xy || !gr->cov_yy || !gr->opacity ||
        !gr->amplitude || !gr->phase)
        return fail(ctx, GWS_ERR_INVALID_ARG, "a gradient array is NULL");
    return GWS_OK;
}

static gws_status check_ws(gws_ctx *ctx, void *ws, size_t ws_bytes, size_t need)
{
    if (!ws || ((uintptr_t)ws & 255) || ws_bytes < need)
        return fail(ctx, GWS_ERR_WORKSPACE, "workspace needs " + std::to_string(need) + " bytes, 256-byte aligned");
    return GWS_OK;
}

struct Bufs {
    long long *counters;
    uint32_t *bucket_hist, *cum, *sort_hist, *vals_a, *vals_b;
    uint64_t *keys_a, *keys_b;
    GRec *rec;
    int32_t *tile_L;
    int2 *tile_slots, *chunk_items;
    int32_t *range_base;
    Item *items;
    BItem *bitems;
    float2 *partials;
    float *bpartials;
};

static Bufs carve(const Layout &L, char *b)
{
    Bufs r;
    r.counters = (long long *)(b + L.off_counters);
    r.bucket_hist = (uint32_t *)(b + L.off_bucket_hist);
    r.cum = (uint32_t *)(b + L.off_cum);
    r.keys_a = (uint64_t *)(b + L.off_keys_a);
    r.keys_b = (uint64_t *)(b + L.off_keys_b);
    r.vals_a = (uint32_t *)(b + L.off_vals_a);
    r.vals_b = (uint32_t *)(b + L.off_vals_b);
    r.sort_hist = (uint32_t *)(b + L.off_sort_hist);
    r.rec = (GRec *)(b + L.off_records);
    r.tile_L = (int32_t *)(b + L.off_tile_L);
    r.tile_slots = (int2 *)(b + L.off_tile_slots);
    r.items = (Item *)(b + L.off_items);
    r.partials = (float2 *)(b + L.off_partials);
    r.bitems = (BItem *)(b + L.off_bitems);
    r.chunk_items = (int2 *)(b + L.off_chunk_items);
    r.range_base = (int32_t *)(b + L.off_range_base);
    r.bpartials = (float *)(b + L.off_bpartials);
    return r;
}

static GView scene_view(const gws_gaussians *g, int64_t off, int64_t n)
{
    GView v;
    v.n = n;
    v.mean_x = g->mean_x ? g->mean_x + off : nullptr;
    v.mean_y = g->mean_y ? g->mean_y + off : nullptr;
    v.depth = g->depth ? g->depth + off : nullptr;
    v.cov_xx = g->cov_xx ? g->cov_xx + off : nullptr;
    v.cov_xy = g->cov_xy ? g->cov_xy + off : nullptr;
    v.cov_yy = g->cov_yy ? g->cov_yy + off : nullptr;
    v.opacity = g->opacity ? g->opacity + off : nullptr;
    v.amplitude = g->amplitude ? g->amplitude + off : nullptr;
    v.phase = g->phase ? g->phase + off : nullptr;
    v.amp_stride = g->n;
    return v;
}

static GradView grad_view(const gws_grads *g, int64_t off, int64_t total)
{
    GradView v;
    v.mean_x = g->mean_x + off;
    v.mean_y = g->mean_y + off;
    v.depth = g->depth ? g->depth + off : nullptr;
    v.cov_xx = g->cov_xx + off;
    v.cov_xy = g->cov_xy + off;
    v.cov_yy = g->cov_yy + off;
    v.opacity = g->opacity + off;
    v.amplitude = g->amplitude + off;
    v.phase = g->phase + off;
    v.amp_stride = total;
    return v;
}

// Preprocess + sort + records of one scene: shared by forward and backward.
static gws_status run_prep(gws_ctx *ctx, const Consts &k, const GView &g, const Layout &L, const Bufs &B, hipStream_t s,
                           uint64_t **keys_sorted, uint32_t **vals_sorted)
{
    HIP_CHECK(ctx, launch_zero_counters(B.counters, B.bucket_hist, s));
    HIP_CHECK(ctx, launch_keys(g, k, B.keys_a, B.vals_a, B.bucket_hist, B.counters, s));
    HIP_CHECK(ctx, radix_sort_48(B.keys_a, B.vals_a, B.keys_b, B.vals_b, B.sort_hist, g.n, L.sort_blocks, s, keys_sorted,
                                 vals_sorted));
    HIP_CHECK(ctx, launch_records(g, k, *keys_sorted, *vals_sorted, B.rec, g.n, B.counters, s));
    return GWS_OK;
}

static int acc_grid(gws_ctx *ctx, int C, int F)
{
    const int key = C * 16 + F;
    auto it = ctx->acc_occ.find(key);
    if (it == ctx->acc_occ.end()) it = ctx->acc_occ.emplace(key, accumulate_occupancy(C, F)).first;
    return ctx->n_cu * it->second;
}

static int adj_grid(gws_ctx *ctx, int C, int depth)
{
    const int key = 256 + C * 2 + (depth ? 1 : 0);
    auto it = ctx->acc_occ.find(key);
    if (it == ctx->acc_occ.end()) it = ctx->acc_occ.emplace(key, adjoint_occupancy(C, depth)).first;
    return ctx->n_cu * it->second;
}

static int n_bucket(int64_t n)
{
    int b = 0;
    while (b < 40 && (1ll << (b + 1)) <= std::max<int64_t>(n, 1)) ++b;
    return b;
}

// Tiling for this call: the explicit one, else the autotuner's choice for this grid and
// channel count at the nearest size class, else the default.
static int resolve_tile_config(const gws_ctx *ctx, const gws_problem *prob, int64_t n)
{
    if (prob->tile_config > 0) return prob->tile_config;
    if (ctx) {
        const int b = n_bucket(n);
        int best = -1, dist = 1 << 30;
        for (auto &kv : ctx->tuned) {
            if (std::get<0>(kv.first) != prob->nx || std::get<1>(kv.first) != prob->ny ||
                std::get<2>(kv.first) != prob->n_lambda)
                continue;
            const int d = std::abs(std::get<3>(kv.first) - b);
            if (d < dist) {
                dist = d;
                best = kv.second;
            }
        }
        if (best > 0) return best;
    }
    return kDefaultTileCfg;
}

static int64_t max_scene(int S, const int64_t *offsets)
{
    int64_t m = 0;
    for (int i = 0; i < S; ++i) m = std::max<int64_t>(m, offsets[i + 1] - offsets[i]);
    return m;
}

// noalloc: the allocation-free variant (forward-only layout in the given scratch, the plan
// looked up but never built, no profiling events).
static gws_status forward_run(gws_ctx *ctx, const gws_problem *prob, int S, const int64_t *offsets,
                              const gws_gaussians *g, const gws_output *out, void *ws, size_t ws_bytes, hipStream_t s,
                              bool noalloc = false)
{
    const int cfg = resolve_tile_config(ctx, prob, max_scene(S, offsets));
    const int F = kTileCfg[cfg - 1][0];
    Plan *p = nullptr;
    gws_status st = GWS_OK;
    const double mrx = prob->ref_nu_x * prob->nx * prob->pitch_x, mry = prob->ref_nu_y * prob->ny * prob->pitch_y;
    if (noalloc) {
        p = find_plan(ctx, prob->nx, prob->ny, F, mrx, mry);
        if (!p)
            return fail(ctx, GWS_ERR_UNSUPPORTED,
                        "no plan for this grid and tiling yet: call gws_forward once for this shape first");
    } else {
        st = get_plan(ctx, prob->nx, prob->ny, F, &p, mrx, mry);
        if (st != GWS_OK) return st;
    }
    const BatchLayout BL = make_batch_layout(prob, S, offsets, noalloc);
    st = check_ws(ctx, ws, ws_bytes, BL.total);
    if (st != GWS_OK) return st;
    char *base = (char *)ws;
    const Consts k = make_consts(prob, 1);
    const int64_t CM = (int64_t)k.C * prob->nx * prob->ny;
    float2 *spectra = out->spectrum ? (float2 *)out->spectrum : (float2 *)(base + BL.off_spectra);
    FwdTab tab;
    memset(&tab, 0, sizeof(tab));
    tab.n = S;
    std::vector<long long *> ctrs(S);
    {
        StageScope sc(ctx, s, ST_PREP, !noalloc);
        for (int i = 0; i < S; ++i) {
            const Layout L = make_layout(prob, BL.n[i], F, ADJ_F, noalloc);
            const Bufs B = carve(L, base + BL.scene_off[i]);
            uint64_t *keys = nullptr;
            uint32_t *vals = nullptr;
            st = run_prep(ctx, k, scene_view(g, offsets[i], BL.n[i]), L, B, s, &keys, &vals);
            if (st != GWS_OK) return st;
            // the configuration's chunk of candidates per work item, capped at n / 16 (at least 128)
            // so that a small scene's crowded tiles still split into several items
            const int chunk = (int)std::min<int64_t>(kTileCfg[cfg - 1][1], std::max<int64_t>(128, BL.n[i] / 16));
            HIP_CHECK(ctx, launch_bin_forward(*p, B.bucket_hist, B.cum, B.tile_L, B.tile_slots, B.items, L.max_items,
                                              L.max_slots, chunk, B.counters, s));
            tab.s[i] = FwdScene{B.rec, B.tile_L, B.items, B.tile_slots, B.partials, spectra + (int64_t)i * CM, B.counters};
            ctrs[i] = B.counters;
        }
    }
    FwdScene *dtab = (FwdScene *)(base + BL.off_ftab);
    int32_t *prefix = (int32_t *)(base + BL.off_prefix);
    long long *queue = (long long *)(base + BL.off_ctrl);
    {
        StageScope sc(ctx, s, ST_BIN, !noalloc);
        HIP_CHECK(ctx, launch_fwd_table(tab, dtab, prefix, queue, s));
    }
    {
        StageScope sc(ctx, s, ST_ACCUM, !noalloc);
        HIP_CHECK(ctx, launch_accumulate(*p, k, dtab, prefix, S, queue, acc_grid(ctx, k.C, F), s));
    }
    {
        StageScope sc(ctx, s, ST_REDUCE, !noalloc);
        HIP_CHECK(ctx, launch_reduce_partials(*p, k, dtab, S, s));
    }
    {
        StageScope sc(ctx, s, ST_XFORM_INV, !noalloc);
        if (prob->xform == GWS_XFORM_FFT_FP32)
            HIP_CHECK(ctx, launch_fft2d(*p, S * k.C, +1, spectra, (float2 *)out->field, s));
        else
            HIP_CHECK(ctx, launch_dft_bf16x3(*p, S * k.C, +1, spectra, (float2 *)out->field,
                                             (void *)(base + BL.off_dftws), s));
    }
    HIP_CHECK(ctx, launch_sum_counters(ctrs.data(), S, ctx->d_stats, s));
    ctx->last_n = g->n;
    ctx->last_tile_config = cfg;
    return GWS_OK;
}

static gws_status backward_run(gws_ctx *ctx, const gws_problem *prob, int S, const int64_t *offsets,
                               const gws_gaussians *g, const void *grad_field, const gws_grads *grads, void *ws,
                               size_t ws_bytes, hipStream_t s)
{
    if (prob->n_lambda > 3 && grads->depth)
        return fail(ctx, GWS_ERR_UNSUPPORTED,
                    "the order-invariant adjoint takes the depth gradient for at most 3 wavelengths");
    // the adjoint's geometry is fixed (regions of the F = 8 tiling); the tiling chooses the forward's
    const int cfg = resolve_tile_config(ctx, prob, max_scene(S, offsets));
    Plan *p = nullptr;
    gws_status st = get_plan(ctx, prob->nx, prob->ny, ADJ_F, &p, prob->ref_nu_x * prob->nx * prob->pitch_x,
                             prob->ref_nu_y * prob->ny * prob->pitch_y);
    if (st != GWS_OK) return st;
    const BatchLayout BL = make_batch_layout(prob, S, offsets);
    st = check_ws(ctx, ws, ws_bytes, BL.total);
    if (st != GWS_OK) return st;
    char *base = (char *)ws;
    Consts k = make_consts(prob, 0);
    k.depth_grad = grads->depth != nullptr;
    float2 *gspecs = (float2 *)(base + BL.off_gspecs);
    float2 *gpack = (float2 *)(base + BL.off_gpack);
    float *dpack = (float *)(base + BL.off_dpack);
    double *d0 = (double *)(base + BL.off_d0);
    BwdTab tab;
    memset(&tab, 0, sizeof(tab));
    tab.n = S;
    std::vector<long long *> ctrs(S);
    std::vector<uint32_t *> vals_sorted(S);
    {
        StageScope sc(ctx, s, ST_PREP);
        for (int i = 0; i < S; ++i) {
            const Layout L = make_layout(prob, BL.n[i], kTileCfg[cfg - 1][0], ADJ_F);
            const Bufs B = carve(L, base + BL.scene_off[i]);
            uint64_t *keys = nullptr;
            uint32_t *vals = nullptr;
            st = run_prep(ctx, k, scene_view(g, offsets[i], BL.n[i]), L, B, s, &keys, &vals);
            if (st != GWS_OK) return st;
            HIP_CHECK(ctx, launch_bin_backward(*p, keys, B.bitems, B.chunk_items, B.range_base, p->ntiles + 1,
                                               L.max_bitems, B.counters, BL.n[i], adj_wg(k.C, k.depth_grad != 0), s));
            tab.s[i] = BwdScene{B.rec, gpack + (int64_t)i * BL.pack_elems, B.bitems, B.bpartials, B.counters, BL.n[i]};
            ctrs[i] = B.counters;
            vals_sorted[i] = vals;
        }
    }
    {
        // Gs = forward DFT of the field gradient (adjoint of the unnormalised inverse DFT)
        StageScope sc(ctx, s, ST_XFORM_FWD);
        if (prob->xform == GWS_XFORM_FFT_FP32)
            HIP_CHECK(ctx, launch_fft2d(*p, S * k.C, -1, (const float2 *)grad_field, gspecs, s));
        else
            HIP_CHECK(ctx, launch_dft_bf16x3(*p, S * k.C, -1, (const float2 *)grad_field, gspecs,
                                             (void *)(base + BL.off_dftws), s));
    }
    {
        StageScope sc(ctx, s, ST_DTABLE);
        HIP_CHECK(ctx, launch_adj_pack(k, BL.geo, S, gspecs, gpack, dpack, d0, s));
    }
    BwdScene *dscenes = (BwdScene *)(base + BL.off_btab);
    int32_t *prefix = (int32_t *)(base + BL.off_prefix);
    long long *queue = (long long *)(base + BL.off_ctrl) + 1;
    {
        StageScope sc(ctx, s, ST_ADJOINT);
        HIP_CHECK(ctx, launch_bwd_table(tab, dscenes, prefix, queue, s));
        HIP_CHECK(ctx, launch_adjoint(*p, k, dscenes, prefix, S, queue, dpack, d0, BL.geo,
                                      adj_grid(ctx, k.C, k.depth_grad), s));
    }
    {
        StageScope sc(ctx, s, ST_FINAL);
        for (int i = 0; i < S; ++i) {
            const Layout L = make_layout(prob, BL.n[i], kTileCfg[cfg - 1][0], ADJ_F);
            const Bufs B = carve(L, base + BL.scene_off[i]);
            HIP_CHECK(ctx, launch_grad_final(scene_view(g, offsets[i], BL.n[i]), k, vals_sorted[i], B.chunk_items,
                                             B.range_base, B.bpartials, grad_view(grads, offsets[i], g->n), BL.n[i],
                                             B.counters, adj_wg(k.C, k.depth_grad != 0), s));
        }
    }
    HIP_CHECK(ctx, launch_sum_counters(ctrs.data(), S, ctx->d_stats, s));
    ctx->last_n = g->n;
    ctx->last_tile_config = cfg;
    return GWS_OK;
}

// Gaussians [off, off + n) of g, one scene; field (and optionally spectrum) of that scene.
static gws_status exact_forward_run(gws_ctx *ctx, const gws_problem *prob, const gws_gaussians *g, int64_t off,
                                    int64_t n, void *field, void *spectrum, void *ws, size_t ws_bytes, hipStream_t s)
{
    Plan *p = nullptr;
    gws_status st = get_plan(ctx, prob->nx, prob->ny, 4, &p);  // for its transform tables
    if (st != GWS_OK) return st;
    const ExactLayout L = exact_layout(prob, n);
    st = check_ws(ctx, ws, ws_bytes, L.total);
    if (st != GWS_OK) return st;
    char *base = (char *)ws;
    const Consts k = make_consts(prob, 1);
    ExactBuffers eb;
    eb.keys_a = (uint64_t *)(base + L.off_keys_a);
    eb.keys_b = (uint64_t *)(base + L.off_keys_b);
    eb.vals_a = (uint32_t *)(base + L.off_vals_a);
    eb.vals_b = (uint32_t *)(base + L.off_vals_b);
    eb.sort_hist = (uint32_t *)(base + L.off_sort_hist);
    eb.sort_blocks = L.sort_blocks;
    eb.rec = (void *)(base + L.off_rec);
    eb.tmap = (float *)(base + L.off_tmap);
    eb.pimgs = (float2 *)(base + L.off_pimgs);
    eb.colwin = (int4 *)(base + L.off_win);
    eb.rowwin = eb.colwin + 64;
    eb.pcolwin = eb.rowwin + 64;
    eb.prowwin = eb.pcolwin + 64;
    eb.counters = (long long *)(base + L.off_counters);
    float2 *spec = spectrum ? (float2 *)spectrum : (float2 *)(base + L.off_spec);
    {
        StageScope sc(ctx, s, ST_ACCUM);
        HIP_CHECK(ctx, run_exact_forward(*p, k, scene_view(g, off, n), eb, spec, s));
    }
    {
        StageScope sc(ctx, s, ST_XFORM_INV);
        if (prob->xform == GWS_XFORM_FFT_FP32)
            HIP_CHECK(ctx, launch_fft2d(*p, k.C, +1, spec, (float2 *)field, s));
        else
            HIP_CHECK(ctx, launch_dft_bf16x3(*p, k.C, +1, spec, (float2 *)field, (void *)(base + L.off_dft), s));
    }
    HIP_CHECK(ctx, launch_sum_counters(&eb.counters, 1, ctx->d_stats, s));
    ctx->last_tile_config = 0;
    return GWS_OK;
}

// Gaussians [off, off + n) of g, one scene with its field gradient; their gradients.
static gws_status exact_backward_run(gws_ctx *ctx, const gws_problem *prob, const gws_gaussians *g, int64_t off,
                                     int64_t n, const void *grad_field, const gws_grads *grads, void *ws,
                                     size_t ws_bytes, hipStream_t s)
{
    Plan *p = nullptr;
    gws_status st = get_plan(ctx, prob->nx, prob->ny, 4, &p);
    if (st != GWS_OK) return st;
    const ExactLayout L = exact_layout(prob, n);
    st = check_ws(ctx, ws, ws_bytes, L.total);
    if (st != GWS_OK) return st;
    char *base = (char *)ws;
    const Consts k = make_consts(prob, 1);
    ExactBuffers eb;
    eb.keys_a = (uint64_t *)(base + L.off_keys_a);
    eb.keys_b = (uint64_t *)(base + L.off_keys_b);
    eb.vals_a = (uint32_t *)(base + L.off_vals_a);
    eb.vals_b = (uint32_t *)(base + L.off_vals_b);
    eb.sort_hist = (uint32_t *)(base + L.off_sort_hist);
    eb.sort_blocks = L.sort_blocks;
    eb.rec = (void *)(base + L.off_rec);
    eb.tmap = (float *)(base + L.off_tmap);
    eb.pimgs = (float2 *)(base + L.off_pimgs);
    eb.colwin = (int4 *)(base + L.off_win);
    eb.rowwin = eb.colwin + 64;
    eb.pcolwin = eb.rowwin + 64;
    eb.prowwin = eb.pcolwin + 64;
    eb.counters = (long long *)(base + L.off_counters);
    ExactBwdBuffers bb;
    bb.gspec = (float2 *)(base + L.off_gspec);
    bb.ckpt = (float *)(base + L.off_ckpt);
    bb.dmap = (float *)(base + L.off_dmap);
    bb.pspec = (float *)(base + L.off_pspec);
    bb.pspat = (float *)(base + L.off_pspat);
    const GradView gv = grad_view(grads, off, g->n);  // amplitude rows are strided by the whole batch
    {
        StageScope sc(ctx, s, ST_ADJOINT);
        HIP_CHECK(ctx, run_exact_backward(*p, k, scene_view(g, off, n), eb, bb, (const float2 *)grad_field, gv, s));
    }
    HIP_CHECK(ctx, launch_sum_counters(&eb.counters, 1, ctx->d_stats, s));
    ctx->last_tile_config = 0;
    return GWS_OK;
}


extern "C" gws_status gws_forward(gws_ctx *ctx, const gws_problem *prob, const gws_gaussians *g, const gws_output *out,
                                  void *ws, size_t ws_bytes, void *stream)
{
    if (!ctx) return fail(nullptr, GWS_ERR_INVALID_ARG, "ctx is NULL");
    gws_status st = gws_check_problem(prob);
    if (st != GWS_OK) return fail(ctx, st, std::string("problem rejected: ") + gws_status_string(st));
    st = check_gaussians(ctx, g);
    if (st != GWS_OK) return st;
    if (!out || !out->field) return fail(ctx, GWS_ERR_INVALID_ARG, "output field is NULL");
    HIP_CHECK(ctx, hipSetDevice(ctx->device));
    const int64_t off[2] = {0, g->n};
    ctx->last_graph = 0;
    if (prob->blend == GWS_BLEND_EXACT) {
        ctx->last_n = g->n;
        return exact_forward_run(ctx, prob, g, 0, g->n, out->field, out->spectrum, ws, ws_bytes, (hipStream_t)stream);
    }
    return forward_run(ctx, prob, 1, off, g, out, ws, ws_bytes, (hipStream_t)stream);
}

extern "C" gws_status gws_forward_noalloc(gws_ctx *ctx, const gws_problem *prob, const gws_gaussians *g,
                                          const gws_output *out, void *stream)
{
    if (!ctx) return fail(nullptr, GWS_ERR_INVALID_ARG, "ctx is NULL");
    gws_status st = gws_check_problem(prob);
    if (st != GWS_OK) return fail(ctx, st, std::string("problem rejected: ") + gws_status_string(st));
    st = check_gaussians(ctx, g);
    if (st != GWS_OK) return st;
    if (!out || !out->field) return fail(ctx, GWS_ERR_INVALID_ARG, "output field is NULL");
    if (prob->blend != GWS_BLEND_OIT || prob->xform != GWS_XFORM_FFT_FP32)
        return fail(ctx, GWS_ERR_UNSUPPORTED, "gws_forward_noalloc takes the order-invariant blend with the FP32 FFT");
    const int64_t off[2] = {0, g->n};
    const size_t need = make_batch_layout(prob, 1, off, true).total;
    if (need > (size_t)GWS_NOALLOC_SCRATCH_BYTES)
        return fail(ctx, GWS_ERR_WORKSPACE,
                    "gws_forward_noalloc: this problem needs " + std::to_string(need) + " bytes of scratch, more than the " +
                        std::to_string((size_t)GWS_NOALLOC_SCRATCH_BYTES) + " the library holds; use gws_forward");
    HIP_CHECK(ctx, hipSetDevice(ctx->device));
    ctx->last_graph = 0;
    return forward_run(ctx, prob, 1, off, g, out, ctx->scratch, (size_t)GWS_NOALLOC_SCRATCH_BYTES, (hipStream_t)stream,
                       true);
}

// ---------------------------------------------------------------------------------
// Tilted Gaussians
// ---------------------------------------------------------------------------------
struct TiltLayout {
    size_t off_rec, off_rect, off_counters, off_spectrum, off_partial, off_dftws, off_off, off_bsum, total;
};

static TiltLayout tilt_layout(const gws_problem *p, int64_t n)
{
    TiltLayout L{};
    size_t o = 0;
    auto take = [&](size_t b) { const size_t at = o; o += align256(b); return at; };
    L.off_rec = take((size_t)std::max<int64_t>(n, 1) * sizeof(TRec));
    L.off_rect = take((size_t)std::max<int64_t>(n, 1) * sizeof(int2));
    L.off_counters = take(CTR_COUNT * sizeof(long long));
    L.off_spectrum = take((size_t)p->n_lambda * p->nx * p->ny * sizeof(float2));
    // the forward's partial spectra when a tile's Gaussians are split into parts
    const int np = tilt_parts(n);
    L.off_partial = take(np > 1 ? (size_t)np * p->n_lambda * p->nx * p->ny * sizeof(float2) : 0);
    L.off_dftws = take(p->xform == GWS_XFORM_DFT_BF16X3 ? dft_bf16x3_workspace(p->nx, p->ny, p->n_lambda) : 0);
    // the adjoint's slot offsets (n + 1) and the scan's block totals
    L.off_off = take((size_t)(n + 1) * sizeof(int64_t));
    L.off_bsum = take((size_t)((n + 1023) / 1024 + 1) * sizeof(int64_t));
    L.total = o;
    return L;
}

static gws_status check_tilted(gws_ctx *ctx, const gws_problem *prob, const gws_tilted_gaussians *g)
{
    if (!g) return fail(ctx, GWS_ERR_INVALID_ARG, "gaussians is NULL");
    if (g->n < 0 || g->n > (int64_t)0x7fffffff) return fail(ctx, GWS_ERR_INVALID_ARG, "bad Gaussian count");
    if (g->n > 0 && (!g->mean_x || !g->mean_y || !g->depth || !g->quat_w || !g->quat_x || !g->quat_y || !g->quat_z ||
                     !g->scale_u || !g->scale_v || !g->opacity || !g->amplitude || !g->phase))
        return fail(ctx, GWS_ERR_INVALID_ARG, "a Gaussian array is NULL");
    if (prob->blend != GWS_BLEND_OIT)
        return fail(ctx, GWS_ERR_UNSUPPORTED, "tilted Gaussians take the order-invariant blend only");
    if (prob->ref_nu_x != 0.0 || prob->ref_nu_y != 0.0)
        return fail(ctx, GWS_ERR_UNSUPPORTED, "tilted Gaussians take on-axis illumination only (ref_nu = 0)");
    return GWS_OK;
}

extern "C" gws_status gws_workspace_size_tilted(const gws_ctx *ctx, const gws_problem *problem, int64_t n,
                                                size_t *bytes)
{
    (void)ctx;
    if (!bytes || n < 0 || n > (int64_t)0x7fffffff) return GWS_ERR_INVALID_ARG;
    const gws_status st = gws_check_problem(problem);
    if (st != GWS_OK) return st;
    *bytes = tilt_layout(problem, n).total;
    return GWS_OK;
}

extern "C" gws_status gws_forward_tilted(gws_ctx *ctx, const gws_problem *prob, const gws_tilted_gaussians *g,
                                         const gws_output *out, void *ws, size_t ws_bytes, void *stream)
{
    if (!ctx) return fail(nullptr, GWS_ERR_INVALID_ARG, "ctx is NULL");
    gws_status st = gws_check_problem(prob);
    if (st != GWS_OK) return fail(ctx, st, std::string("problem rejected: ") + gws_status_string(st));
    st = check_tilted(ctx, prob, g);
    if (st != GWS_OK) return st;
    if (!out || !out->field) return fail(ctx, GWS_ERR_INVALID_ARG, "output field is NULL");
    const TiltLayout L = tilt_layout(prob, g->n);
    st = check_ws(ctx, ws, ws_bytes, L.total);
    if (st != GWS_OK) return st;
    HIP_CHECK(ctx, hipSetDevice(ctx->device));
    const hipStream_t s = (hipStream_t)stream;
    Plan *p = nullptr;  // the transform's tables (the tiling is not used here)
    st = get_plan(ctx, prob->nx, prob->ny, kTileCfg[kDefaultTileCfg - 1][0], &p);
    if (st != GWS_OK) return st;
    char *base = (char *)ws;
    const Consts k = make_consts(prob, 1);
    TRec *rec = (TRec *)(base + L.off_rec);
    int2 *rect = (int2 *)(base + L.off_rect);
    long long *counters = (long long *)(base + L.off_counters);
    float2 *spectrum = out->spectrum ? (float2 *)out->spectrum : (float2 *)(base + L.off_spectrum);
    const TView tv{g->n,       g->mean_x,  g->mean_y,  g->depth,   g->quat_w,    g->quat_x, g->quat_y,
                   g->quat_z,  g->scale_u, g->scale_v, g->opacity, g->amplitude, g->phase};
    ctx->last_graph = 0;
    {
        StageScope sc(ctx, s, ST_PREP);
        HIP_CHECK(ctx, launch_tilt_records(tv, k, rec, rect, counters, s));
    }
    {
        StageScope sc(ctx, s, ST_ACCUM);
        float2 *partial = tilt_parts(g->n) > 1 ? (float2 *)(base + L.off_partial) : nullptr;
        HIP_CHECK(ctx, launch_tilt_accumulate(k, rec, rect, g->n, spectrum, partial, counters, ctx->n_cu, s));
    }
    {
        StageScope sc(ctx, s, ST_XFORM_INV);
        if (prob->xform == GWS_XFORM_FFT_FP32)
            HIP_CHECK(ctx, launch_fft2d(*p, k.C, +1, spectrum, (float2 *)out->field, s));
        else
            HIP_CHECK(ctx, launch_dft_bf16x3(*p, k.C, +1, spectrum, (float2 *)out->field, (void *)(base + L.off_dftws), s));
    }
    long long *ctrs[1] = {counters};
    HIP_CHECK(ctx, launch_sum_counters(ctrs, 1, ctx->d_stats, s));
    ctx->last_n = g->n;
    ctx->last_tile_config = 0;
    return GWS_OK;
}

static gws_status check_tilted_grads(gws_ctx *ctx, const gws_tilted_grads *gr)
{
    if (!gr || !gr->mean_x || !gr->mean_y || !gr->depth || !gr->quat_w || !gr->quat_x || !gr->quat_y || !gr->quat_z ||
        !gr->scale_u || !gr->scale_v || !gr->opacity || !gr->amplitude || !gr->phase)
        return fail(ctx, GWS_ERR_INVALID_ARG, "a gradient array is NULL");
    return GWS_OK;
}

extern "C" gws_status gws_backward_tilted(gws_ctx *ctx, const gws_problem *prob, const gws_tilted_gaussians *g,
                                          const void *grad_field, const gws_tilted_grads *grads, void *ws,
                                          size_t ws_bytes, void *stream)
{
    if (!ctx) return fail(nullptr, GWS_ERR_INVALID_ARG, "ctx is NULL");
    gws_status st = gws_check_problem(prob);
    if (st != GWS_OK) return fail(ctx, st, std::string("problem rejected: ") + gws_status_string(st));
    st = check_tilted(ctx, prob, g);
    if (st != GWS_OK) return st;
    if (g->n == 0) return GWS_OK;
    if (!grad_field) return fail(ctx, GWS_ERR_INVALID_ARG, "grad_field is NULL");
    st = check_tilted_grads(ctx, grads);
    if (st != GWS_OK) return st;
    const TiltLayout L = tilt_layout(prob, g->n);
    st = check_ws(ctx, ws, ws_bytes, L.total);
    if (st != GWS_OK) return st;
    HIP_CHECK(ctx, hipSetDevice(ctx->device));
    const hipStream_t s = (hipStream_t)stream;
    Plan *p = nullptr;
    st = get_plan(ctx, prob->nx, prob->ny, kTileCfg[kDefaultTileCfg - 1][0], &p);
    if (st != GWS_OK) return st;
    char *base = (char *)ws;
    const Consts k = make_consts(prob, 0);  // keep Gaussians that add nothing: their gradients do not vanish
    TRec *rec = (TRec *)(base + L.off_rec);
    int2 *rect = (int2 *)(base + L.off_rect);
    long long *counters = (long long *)(base + L.off_counters);
    float2 *gspec = (float2 *)(base + L.off_spectrum);
    int64_t *off = (int64_t *)(base + L.off_off);
    int64_t *bsum = (int64_t *)(base + L.off_bsum);
    const TView tv{g->n,       g->mean_x,  g->mean_y,  g->depth,   g->quat_w,    g->quat_x, g->quat_y,
                   g->quat_z,  g->scale_u, g->scale_v, g->opacity, g->amplitude, g->phase};
    const TGrads tg{grads->mean_x, grads->mean_y, grads->depth,   grads->quat_w,  grads->quat_x,    grads->quat_y,
                    grads->quat_z, grads->scale_u, grads->scale_v, grads->opacity, grads->amplitude, grads->phase};
    ctx->last_graph = 0;
    {
        StageScope sc(ctx, s, ST_PREP);
        HIP_CHECK(ctx, launch_tilt_records(tv, k, rec, rect, counters, s));
        HIP_CHECK(ctx, launch_tilt_offsets(rect, g->n, off, bsum, s));
    }
    {
        // Gs = forward DFT of the field gradient (adjoint of the unnormalised inverse DFT)
        StageScope sc(ctx, s, ST_XFORM_FWD);
        if (prob->xform == GWS_XFORM_FFT_FP32)
            HIP_CHECK(ctx, launch_fft2d(*p, k.C, -1, (const float2 *)grad_field, gspec, s));
        else
            HIP_CHECK(ctx, launch_dft_bf16x3(*p, k.C, -1, (const float2 *)grad_field, gspec,
                                             (void *)(base + L.off_dftws), s));
    }
    // the number of (Gaussian, tile) slots sizes the context's partial-sum buffer: one read-back
    int64_t nslots = 0;
    HIP_CHECK(ctx, hipMemcpyAsync(&nslots, off + g->n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_CHECK(ctx, hipStreamSynchronize(s));
    const size_t need = (size_t)std::max<int64_t>(nslots, 1) * tilt_slot_floats(k.C) * sizeof(float);
    if (need > ctx->tilt_part_bytes) {
        HIP_CHECK(ctx, hipFree(ctx->tilt_part));
        ctx->tilt_part = nullptr;
        ctx->tilt_part_bytes = 0;
        if (hipMalloc(&ctx->tilt_part, need) != hipSuccess) {
            ctx->tilt_part = nullptr;
            return fail(ctx, GWS_ERR_OOM, "tilted adjoint: " + std::to_string(need) + " bytes of partial sums");
        }
        ctx->tilt_part_bytes = need;
    }
    {
        StageScope sc(ctx, s, ST_ADJOINT);
        HIP_CHECK(ctx, launch_tilt_adjoint(k, rec, rect, g->n, gspec, off, ctx->tilt_part, counters, ctx->n_cu, s));
    }
    {
        StageScope sc(ctx, s, ST_FINAL);
        HIP_CHECK(ctx, launch_tilt_grad_final(tv, k, rect, off, ctx->tilt_part, tg, s));
    }
    long long *ctrs[1] = {counters};
    HIP_CHECK(ctx, launch_sum_counters(ctrs, 1, ctx->d_stats, s));
    ctx->last_n = g->n;
    ctx->last_tile_config = 0;
    return GWS_OK;
}

extern "C" gws_status gws_backward(gws_ctx *ctx, const gws_problem *prob, const gws_gaussians *g, const void *grad_field,
                                   const gws_grads *grads, void *ws, size_t ws_bytes, void *stream)
{
    if (!ctx) return fail(nullptr, GWS_ERR_INVALID_ARG, "ctx is NULL");
    gws_status st = gws_check_problem(prob);
    if (st != GWS_OK) return fail(ctx, st, std::string("problem rejected: ") + gws_status_string(st));
    st = check_gaussians(ctx, g);
    if (st != GWS_OK) return st;
    st = check_grads(ctx, grads);
    if (st != GWS_OK) return st;
    if (!grad_field) return fail(ctx, GWS_ERR_INVALID_ARG, "grad_field is NULL");
    HIP_CHECK(ctx, hipSetDevice(ctx->device));
    const int64_t off[2] = {0, g->n};
    ctx->last_graph = 0;
    if (prob->blend == GWS_BLEND_EXACT) {
        ctx->last_n = g->n;
        return exact_backward_run(ctx, prob, g, 0, g->n, grad_field, grads, ws, ws_bytes, (hipStream_t)stream);
    }
    return backward_run(ctx, prob, 1, off, g, grad_field, grads, ws, ws_bytes, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------------
// Batched calls, captured into a hipGraph on first use and replayed afterwards
// ---------------------------------------------------------------------------------
static bool same_key(const gws_ctx::GraphKey &a, const gws_ctx::GraphKey &b)
{
    return a.backward == b.backward && a.offsets == b.offsets && a.ptrs == b.ptrs &&
           memcmp(&a.prob, &b.prob, sizeof(gws_problem)) == 0;
}

template <class Fn>
static gws_status run_graph(gws_ctx *ctx, const gws_ctx::GraphKey &key, hipStream_t s, Fn &&enqueue)
{
    for (auto &e : ctx->graphs)
        if (same_key(e.first, key)) {
            HIP_CHECK(ctx, hipGraphLaunch(e.second, s));
            ctx->last_graph = 1;
            return GWS_OK;
        }
    ctx->last_graph = 0;
    if (s == nullptr) return enqueue();  // the legacy default stream cannot be captured: run directly
    const int prof = ctx->profiling;
    ctx->profiling = 0;  // events are not recorded inside a captured graph
    hipGraph_t graph = nullptr;
    HIP_CHECK(ctx, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    const gws_status st = enqueue();
    const hipError_t ce = hipStreamEndCapture(s, &graph);
    ctx->profiling = prof;
    if (st != GWS_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (ce != hipSuccess || !graph) return fail(ctx, GWS_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(ce));
    hipGraphExec_t exec = nullptr;
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return fail(ctx, GWS_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(ie));
    ctx->graphs.emplace_back(key, exec);
    HIP_CHECK(ctx, hipGraphLaunch(exec, s));
    return GWS_OK;
}

static void key_ptrs_g(std::vector<uintptr_t> &v, const gws_gaussians *g)
{
    for (const void *q : {(const void *)g->mean_x, (const void *)g->mean_y, (const void *)g->depth, (const void *)g->cov_xx,
                          (const void *)g->cov_xy, (const void *)g->cov_yy, (const void *)g->opacity,
                          (const void *)g->amplitude, (const void *)g->phase})
        v.push_back((uintptr_t)q);
    v.push_back((uintptr_t)g->n);
}

// Plans and DFT matrices are built outside the capture (they allocate and copy).
static gws_status prepare_plans(gws_ctx *ctx, const gws_problem *prob, int S, const int64_t *offsets)
{
    const int cfg = resolve_tile_config(ctx, prob, max_scene(S, offsets));
    const double mrx = prob->ref_nu_x * prob->nx * prob->pitch_x, mry = prob->ref_nu_y * prob->ny * prob->pitch_y;
    for (int d = 0; d < 2; ++d) {
        Plan *p = nullptr;
        // the forward's tiling, and the adjoint's fixed one
        const gws_status st = get_plan(ctx, prob->nx, prob->ny, d == 0 ? kTileCfg[cfg - 1][0] : ADJ_F, &p, mrx, mry);
        if (st != GWS_OK) return st;
        if (prob->xform == GWS_XFORM_DFT_BF16X3) HIP_CHECK(ctx, build_dft_mats(*p));
        (void)acc_grid(ctx, prob->n_lambda, kTileCfg[cfg - 1][0]);
    }
    return GWS_OK;
}

extern "C" gws_status gws_forward_batched(gws_ctx *ctx, const gws_problem *prob, int32_t n_scenes, const int64_t *offsets,
                                          const gws_gaussians *g, const gws_output *out, void *ws, size_t ws_bytes,
                                          void *stream)
{
    if (!ctx) return fail(nullptr, GWS_ERR_INVALID_ARG, "ctx is NULL");
    gws_status st = gws_check_problem(prob);
    if (st != GWS_OK) return fail(ctx, st, std::string("problem rejected: ") + gws_status_string(st));
    st = check_gaussians(ctx, g);
    if (st != GWS_OK) return st;
    if (!out || !out->field) return fail(ctx, GWS_ERR_INVALID_ARG, "output field is NULL");
    if (check_offsets(n_scenes, offsets, g->n) != GWS_OK)
        return fail(ctx, GWS_ERR_INVALID_ARG, "offsets must be a CSR array of n_scenes + 1 entries (1..64 scenes)");
    HIP_CHECK(ctx, hipSetDevice(ctx->device));
    if (prob->blend == GWS_BLEND_EXACT) {
        st = check_ws(ctx, ws, ws_bytes, exact_batched_bytes(prob, n_scenes, offsets));
        if (st != GWS_OK) return st;
        const size_t img = (size_t)prob->n_lambda * prob->nx * prob->ny * sizeof(float2);
        ctx->last_graph = 0;
        ctx->last_n = g->n;
        for (int i = 0; i < n_scenes; ++i) {
            st = exact_forward_run(ctx, prob, g, offsets[i], offsets[i + 1] - offsets[i], (char *)out->field + i * img,
                                   out->spectrum ? (char *)out->spectrum + i * img : nullptr, ws, ws_bytes,
                                   (hipStream_t)stream);
            if (st != GWS_OK) return st;
        }
        return GWS_OK;
    }
    st = prepare_plans(ctx, prob, n_scenes, offsets);
    if (st != GWS_OK) return st;
    gws_ctx::GraphKey key;
    key.offsets.assign(offsets, offsets + n_scenes + 1);
    key_ptrs_g(key.ptrs, g);
    key.ptrs.push_back((uintptr_t)out->field);
    key.ptrs.push_back((uintptr_t)out->spectrum);
    key.ptrs.push_back((uintptr_t)ws);
    key.ptrs.push_back((uintptr_t)ws_bytes);
    key.prob = *prob;
    key.backward = 0;
    hipStream_t s = (hipStream_t)stream;
    return run_graph(ctx, key, s, [&]() { return forward_run(ctx, prob, n_scenes, offsets, g, out, ws, ws_bytes, s); });
}

extern "C" gws_status gws_backward_batched(gws_ctx *ctx, const gws_problem *prob, int32_t n_scenes, const int64_t *offsets,
                                           const gws_gaussians *g, const void *grad_field, const gws_grads *grads,
                                           void *ws, size_t ws_bytes, void *stream)
{
    if (!ctx) return fail(nullptr, GWS_ERR_INVALID_ARG, "ctx is NULL");
    gws_status st = gws_check_problem(prob);
    if (st != GWS_OK) return fail(ctx, st, std::string("problem rejected: ") + gws_status_string(st));
    st = check_gaussians(ctx, g);
    if (st != GWS_OK) return st;
    st = check_grads(ctx, grads);
    if (st != GWS_OK) return st;
    if (!grad_field) return fail(ctx, GWS_ERR_INVALID_ARG, "grad_field is NULL");
    if (check_offsets(n_scenes, offsets, g->n) != GWS_OK)
        return fail(ctx, GWS_ERR_INVALID_ARG, "offsets must be a CSR array of n_scenes + 1 entries (1..64 scenes)");
    HIP_CHECK(ctx, hipSetDevice(ctx->device));
    if (prob->blend == GWS_BLEND_EXACT) {
        st = check_ws(ctx, ws, ws_bytes, exact_batched_bytes(prob, n_scenes, offsets));
        if (st != GWS_OK) return st;
        const size_t img = (size_t)prob->n_lambda * prob->nx * prob->ny * sizeof(float2);
        ctx->last_graph = 0;
        ctx->last_n = g->n;
        for (int i = 0; i < n_scenes; ++i) {
            st = exact_backward_run(ctx, prob, g, offsets[i], offsets[i + 1] - offsets[i],
                                    (const char *)grad_field + i * img, grads, ws, ws_bytes, (hipStream_t)stream);
            if (st != GWS_OK) return st;
        }
        return GWS_OK;
    }
    st = prepare_plans(ctx, prob, n_scenes, offsets);
    if (st != GWS_OK) return st;
    gws_ctx::GraphKey key;
    key.offsets.assign(offsets, offsets + n_scenes + 1);
    key_ptrs_g(key.ptrs, g);
    key.ptrs.push_back((uintptr_t)grad_field);
    for (const void *q : {(const void *)grads->mean_x, (const void *)grads->mean_y, (const void *)grads->depth,
                          (const void *)grads->cov_xx, (const void *)grads->cov_xy, (const void *)grads->cov_yy,
                          (const void *)grads->opacity, (const void *)grads->amplitude, (const void *)grads->phase})
        key.ptrs.push_back((uintptr_t)q);
    key.ptrs.push_back((uintptr_t)ws);
    key.ptrs.push_back((uintptr_t)ws_bytes);
    key.prob = *prob;
    key.backward = 1;
    hipStream_t s = (hipStream_t)stream;
    return run_graph(ctx, key, s,
                     [&]() { return backward_run(ctx, prob, n_scenes, offsets, g, grad_field, grads, ws, ws_bytes, s); });
}

// ---------------------------------------------------------------------------------
// Stand-alone 2D DFT
// ---------------------------------------------------------------------------------
// Row and column launches index rows and slabs of the whole batch with 32-bit grid sizes.
static bool dft_batch_fits(int32_t nx, int32_t ny, int32_t batch)
{
    return (int64_t)batch * std::max(nx, ny) < ((int64_t)1 << 31);
}

extern "C" gws_status gws_dft_workspace_size(const gws_ctx *ctx, int32_t nx, int32_t ny, int32_t batch, int32_t xform,
                                             size_t *bytes)
{
    (void)ctx;
    if (!bytes || batch < 1) return GWS_ERR_INVALID_ARG;
    if (check_grid(nx, ny) != GWS_OK || !dft_batch_fits(nx, ny, batch)) return GWS_ERR_SHAPE;
    if (xform == GWS_XFORM_FFT_FP32) *bytes = 0;
    else if (xform == GWS_XFORM_DFT_BF16X3) *bytes = dft_bf16x3_workspace(nx, ny, batch);
    else return GWS_ERR_INVALID_ARG;
    return GWS_OK;
}

extern "C" gws_status gws_dft2d(gws_ctx *ctx, int32_t nx, int32_t ny, int32_t batch, int32_t direction, int32_t xform,
                                const void *in, void *out, void *ws, size_t ws_bytes, void *stream)
{
    if (!ctx) return fail(nullptr, GWS_ERR_INVALID_ARG, "ctx is NULL");
    if (!in || !out || batch < 1 || (direction != 1 && direction != -1))
        return fail(ctx, GWS_ERR_INVALID_ARG, "bad DFT arguments");
    if (check_grid(nx, ny) != GWS_OK) return fail(ctx, GWS_ERR_SHAPE, "unsupported DFT shape");
    if (!dft_batch_fits(nx, ny, batch)) return fail(ctx, GWS_ERR_SHAPE, "DFT batch too large");
    HIP_CHECK(ctx, hipSetDevice(ctx->device));
    Plan *p = nullptr;
    gws_status st = get_plan(ctx, nx, ny, 4, &p);
    if (st != GWS_OK) return st;
    if (xform == GWS_XFORM_FFT_FP32) {
        HIP_CHECK(ctx, launch_fft2d(*p, batch, direction, (const float2 *)in, (float2 *)out, (hipStream_t)stream));
    } else if (xform == GWS_XFORM_DFT_BF16X3) {
        const size_t need = dft_bf16x3_workspace(nx, ny, batch);
        st = check_ws(ctx, ws, ws_bytes, need);
        if (st != GWS_OK) return st;
        HIP_CHECK(ctx, launch_dft_bf16x3(*p, batch, direction, (const float2 *)in, (float2 *)out, ws, (hipStream_t)stream));
    } else {
        return fail(ctx, GWS_ERR_INVALID_ARG, "bad xform");
    }
    return GWS_OK;
}

// ---------------------------------------------------------------------------------
// Autotuner: time each accumulation tiling and each adjoint tiling on synthetic
// Gaussians of the requested count, keep the fastest pair for this grid and size class.
// ---------------------------------------------------------------------------------
static std::string tune_line(const gws_problem *p, int nb, int cfg, const double *tf)
{
    std::string l = "{\"arch\": \"gfx950\", \"nx\": " + std::to_string(p->nx) + ", \"ny\": " + std::to_string(p->ny) +
                    ", \"n_lambda\": " + std::to_string(p->n_lambda) + ", \"n_bucket\": " + std::to_string(nb) +
                    ", \"tile_config\": " + std::to_string(cfg) + ", \"fwd_ms\": {";
    for (int c = 0; c < kNumTileCfg; ++c) {
        char buf[96];
        snprintf(buf, sizeof(buf), "%s\"F%d/chunk%d\": %.4f", c ? ", " : "", kTileCfg[c][0], kTileCfg[c][1], tf[c]);
        l += buf;
    }
    return l + "}}";
}

static bool parse_tune_line(const std::string &l, int *nx, int *ny, int *C, int *nb, int *cfg)
{
    return sscanf(l.c_str(),
                  "{\"arch\": \"gfx950\", \"nx\": %d, \"ny\": %d, \"n_lambda\": %d, \"n_bucket\": %d, \"tile_config\": %d",
                  nx, ny, C, nb, cfg) == 5;
}

static void load_tune_cache(gws_ctx *ctx, const char *path)
{
    FILE *f = path ? fopen(path, "r") : nullptr;
    if (!f) return;
    char line[1024];
    while (fgets(line, sizeof(line), f)) {
        int nx, ny, C, nb, cfg;
        if (parse_tune_line(line, &nx, &ny, &C, &nb, &cfg) && cfg >= 1 && cfg <= kNumTileCfg)
            ctx->tuned[std::make_tuple(nx, ny, C, nb)] = cfg;
    }
    fclose(f);
}

static void merge_tune_cache(const char *path, const gws_problem *p, int nb, const std::string &entry)
{
    std::vector<std::string> keep;
    if (FILE *f = fopen(path, "r")) {
        char line[1024];
        while (fgets(line, sizeof(line), f)) {
            std::string l(line);
            while (!l.empty() && (l.back() == '\n' || l.back() == '\r')) l.pop_back();
            int nx, ny, C, b, cfg;
            if (!parse_tune_line(l, &nx, &ny, &C, &b, &cfg)) continue;
            if (nx == p->nx && ny == p->ny && C == p->n_lambda && b == nb) continue;
            keep.push_back(l);
        }
        fclose(f);
    }
    keep.push_back(entry);
    if (FILE *f = fopen(path, "w")) {
        for (auto &l : keep) fprintf(f, "%s\n", l.c_str());
        fclose(f);
    }
}

extern "C" gws_status gws_autotune(gws_ctx *ctx, const gws_problem *prob, int64_t n_hint, const char *cache_path,
                                   void *stream)
{
    if (!ctx) return fail(nullptr, GWS_ERR_INVALID_ARG, "ctx is NULL");
    gws_status st = gws_check_problem(prob);
    if (st != GWS_OK) return fail(ctx, st, std::string("problem rejected: ") + gws_status_string(st));
    if (n_hint < 1 || n_hint > (int64_t)0x7fffffff) return fail(ctx, GWS_ERR_INVALID_ARG, "n_hint out of range");
    if (prob->blend == GWS_BLEND_EXACT) return fail(ctx, GWS_ERR_UNSUPPORTED, "the tilings tuned are those of Eq. 12");
    HIP_CHECK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    const int C = prob->n_lambda;
    const int64_t n = n_hint, M = (int64_t)prob->nx * prob->ny;
    const int64_t off[2] = {0, n};
    const size_t ws_bytes = make_batch_layout(prob, 1, off).total;
    float *gbuf = nullptr, *grbuf = nullptr;
    float2 *field = nullptr;
    void *ws = nullptr;
    auto cleanup = [&]() {
        (void)hipFree(gbuf);
        (void)hipFree(grbuf);
        (void)hipFree(field);
        (void)hipFree(ws);
    };
    if (hipMalloc(&gbuf, sizeof(float) * (8 + C) * n) != hipSuccess ||
        hipMalloc(&grbuf, sizeof(float) * (8 + C) * n) != hipSuccess ||
        hipMalloc(&field, sizeof(float2) * C * M) != hipSuccess || hipMalloc(&ws, ws_bytes) != hipSuccess) {
        cleanup();
        return fail(ctx, GWS_ERR_OOM, "autotune buffers");
    }
    gws_gaussians g;
    g.n = n;
    g.mean_x = gbuf; g.mean_y = gbuf + n; g.depth = gbuf + 2 * n; g.cov_xx = gbuf + 3 * n; g.cov_xy = gbuf + 4 * n;
    g.cov_yy = gbuf + 5 * n; g.opacity = gbuf + 6 * n; g.phase = gbuf + 7 * n; g.amplitude = gbuf + 8 * n;
    gws_grads gr;
    gr.mean_x = grbuf; gr.mean_y = grbuf + n; gr.depth = nullptr; gr.cov_xx = grbuf + 3 * n; gr.cov_xy = grbuf + 4 * n;
    gr.cov_yy = grbuf + 5 * n; gr.opacity = grbuf + 6 * n; gr.phase = grbuf + 7 * n; gr.amplitude = grbuf + 8 * n;
    const Consts k = make_consts(prob, 1);
    GView dummy;
    memset(&dummy, 0, sizeof(dummy));
    if (launch_synth(dummy, gbuf, n, 0x5eed5eedull, k, s) != hipSuccess) {
        cleanup();
        return fail(ctx, GWS_ERR_HIP, "synthetic Gaussians");
    }
    gws_output out{field, nullptr};
    double tf[kNumTileCfg];
    hipEvent_t e0 = nullptr, e1 = nullptr;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const int prof = ctx->profiling;
    ctx->profiling = 0;
    gws_problem q = *prob;
    // every forward configuration (the adjoint's geometry does not depend on it): one untimed
    // call (plan and first-touch), then the mean of two
    for (int c = 0; c < kNumTileCfg && st == GWS_OK; ++c) {
        q.tile_config = c + 1;
        for (int rep = 0; rep < 3 && st == GWS_OK; ++rep) {
            if (rep == 1) (void)hipEventRecord(e0, s);
            st = forward_run(ctx, &q, 1, off, &g, &out, ws, ws_bytes, s);
        }
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        tf[c] = ms / 2.0;
    }
    ctx->profiling = prof;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const hipError_t se = hipStreamSynchronize(s);
    cleanup();
    if (st != GWS_OK) return st;
    if (se != hipSuccess) return fail(ctx, GWS_ERR_HIP, hipGetErrorString(se));
    const int best = (int)(std::min_element(tf, tf + kNumTileCfg) - tf) + 1;
    const int nb = n_bucket(n);
    ctx->tuned[std::make_tuple(prob->nx, prob->ny, C, nb)] = best;
    if (cache_path) merge_tune_cache(cache_path, prob, nb, tune_line(prob, nb, best, tf));
    return GWS_OK;
}

// ---------------------------------------------------------------------------------
// Loss and profiling
// ---------------------------------------------------------------------------------
extern "C" size_t gws_l2_workspace_size(void) { return align256(l2_workspace_bytes()); }

extern "C" gws_status gws_l2_loss_grad(gws_ctx *ctx, int64_t n, const void *field, const void *target, void *grad,
                                       double *loss, void *ws, size_t ws_bytes, void *stream)
{
    if (!ctx) return fail(nullptr, GWS_ERR_INVALID_ARG, "ctx is NULL");
    if (n < 0 || (n > 0 && (!field || !target)) || !loss) return fail(ctx, GWS_ERR_INVALID_ARG, "bad loss arguments");
    gws_status st = check_ws(ctx, ws, ws_bytes, gws_l2_workspace_size());
    if (st != GWS_OK) return st;
    HIP_CHECK(ctx, hipSetDevice(ctx->device));
    StageScope sc(ctx, (hipStream_t)stream, ST_LOSS);
    HIP_CHECK(ctx, launch_l2_grad((const float2 *)field, (const float2 *)target, (float2 *)grad, loss, ws, n,
                                  (hipStream_t)stream));
    return GWS_OK;
}

// ---------------------------------------------------------------------------------
// Holographics transform
// ---------------------------------------------------------------------------------
extern "C" gws_status gws_holographics(gws_ctx *ctx, const gws_view *view, const gws_world_gaussians *in,
                                       const gws_plane_gaussians *out, void *stream)
{
    if (!ctx) return fail(nullptr, GWS_ERR_INVALID_ARG, "ctx is NULL");
    if (!view || !in || !out || in->n < 0) return fail(ctx, GWS_ERR_INVALID_ARG, "bad holographics arguments");
    if (!(view->fx > 0.0) || !(view->fy > 0.0) || !(view->near >= 0.0) || view->sh_degree < 0 || view->sh_degree > 3)
        return fail(ctx, GWS_ERR_INVALID_ARG, "bad camera: fx, fy > 0, near >= 0, sh_degree 0..3");
    for (int i = 0; i < 12; ++i)
        if (!std::isfinite(view->world_to_view[i])) return fail(ctx, GWS_ERR_INVALID_ARG, "non-finite view matrix");
    if (in->n == 0) return GWS_OK;
    if (!in->mean || !in->quat || !in->scale || !in->opacity_sh || !out->mean_x || !out->mean_y || !out->depth ||
        !out->cov_xx || !out->cov_xy || !out->cov_yy || !out->opacity)
        return fail(ctx, GWS_ERR_INVALID_ARG, "a Gaussian array is NULL");
    HoloArgs a{};
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) a.R[3 * r + c] = view->world_to_view[4 * r + c];
        a.t[r] = view->world_to_view[4 * r + 3];
    }
    for (int c = 0; c < 3; ++c) a.centre[c] = -(a.R[c] * a.t[0] + a.R[3 + c] * a.t[1] + a.R[6 + c] * a.t[2]);
    a.fx = view->fx;
    a.fy = view->fy;
    a.cx = view->cx;
    a.cy = view->cy;
    a.near = view->near;
    a.A[0] = view->ray_to_holo[0];
    a.A[1] = view->ray_to_holo[1];
    a.b[0] = view->ray_to_holo[2];
    a.A[2] = view->ray_to_holo[3];
    a.A[3] = view->ray_to_holo[4];
    a.b[1] = view->ray_to_holo[5];
    a.depth_scale = view->depth_scale;
    a.depth_offset = view->depth_offset;
    a.sh_degree = view->sh_degree;
    const PlaneOut po{out->mean_x, out->mean_y, out->depth, out->cov_xx, out->cov_xy, out->cov_yy, out->opacity};
    HIP_CHECK(ctx, hipSetDevice(ctx->device));
    const hipStream_t s = (hipStream_t)stream;
    StageScope sc(ctx, s, ST_HOLO);
    HIP_CHECK(ctx, launch_holographics(a, in->n, in->mean, in->quat, in->scale, in->opacity_sh, po, s));
    return GWS_OK;
}

// ---------------------------------------------------------------------------------
// Display side: double-phase coding and focal stacks
// ---------------------------------------------------------------------------------
extern "C" size_t gws_dpac_workspace_size(int32_t n_lambda)
{
    return align256(sizeof(uint32_t) * (size_t)std::max<int32_t>(n_lambda, 1));
}

extern "C" gws_status gws_dpac_encode(gws_ctx *ctx, int32_t nx, int32_t ny, int32_t n_lambda, const void *field,
                                      float a_max, float *phase, void *ws, size_t ws_bytes, void *stream)
{
    if (!ctx) return fail(nullptr, GWS_ERR_INVALID_ARG, "ctx is NULL");
    if (nx < 1 || ny < 1 || n_lambda < 1 || n_lambda > GWS_MAX_LAMBDA || !field || !phase || !(a_max == a_max))
        return fail(ctx, GWS_ERR_INVALID_ARG, "bad double-phase arguments");
    if ((int64_t)n_lambda * ny > 65535) return fail(ctx, GWS_ERR_SHAPE, "double-phase coding needs n_lambda * ny <= 65535");
    const bool auto_max = !(a_max > 0.0f);
    if (auto_max) {
        const gws_status st = check_ws(ctx, ws, ws_bytes, gws_dpac_workspace_size(n_lambda));
        if (st != GWS_OK) return st;
    }
    HIP_CHECK(ctx, hipSetDevice(ctx->device));
    const hipStream_t s = (hipStream_t)stream;
    StageScope sc(ctx, s, ST_DPAC);
    const int64_t m = (int64_t)nx * ny;
    uint32_t *bits = auto_max ? (uint32_t *)ws : nullptr;
    if (auto_max) HIP_CHECK(ctx, launch_amax((const float2 *)field, m, n_lambda, bits, s));
    HIP_CHECK(ctx, launch_dpac((const float2 *)field, nx, ny, n_lambda, bits, auto_max ? 0.0f : a_max, phase, s));
    return GWS_OK;
}

static size_t focal_stack_bytes(const gws_problem *p, int32_t n_planes, int32_t flags)
{
    const size_t img = (size_t)p->nx * p->ny * p->n_lambda * sizeof(float2);
    size_t bytes = align256(img);  // the spectrum DFT(u)
    if (!(flags & GWS_FS_COMPLEX_OUTPUT))
        bytes += align256(img * (size_t)std::min<int32_t>(std::max<int32_t>(n_planes, 1), STACK_MAXK));
    return bytes;
}

static gws_status check_focal(gws_ctx *ctx, const gws_problem *p, int32_t n_planes, int32_t flags)
{
    const gws_status st = gws_check_problem(p);
    if (st != GWS_OK) return fail(ctx, st, "invalid problem");
    if (!focal_stack_fits(p->nx)) return fail(ctx, GWS_ERR_SHAPE, "focal stacks need nx <= 4096");
    if (n_planes < 0 || (flags & ~(GWS_FS_PHASE_INPUT | GWS_FS_HALF_BAND | GWS_FS_COMPLEX_OUTPUT)))
        return fail(ctx, GWS_ERR_INVALID_ARG, "bad focal-stack arguments");
    return GWS_OK;
}

extern "C" gws_status gws_focal_stack_workspace_size(const gws_ctx *ctx, const gws_problem *problem, int32_t n_planes,
                                                     int32_t flags, size_t *bytes)
{
    if (!bytes) return GWS_ERR_INVALID_ARG;
    const gws_status st = check_focal(const_cast<gws_ctx *>(ctx), problem, n_planes, flags);
    if (st != GWS_OK) return st;
    *bytes = focal_stack_bytes(problem, n_planes, flags);
    return GWS_OK;
}

extern "C" gws_status gws_focal_stack(gws_ctx *ctx, const gws_problem *prob, const void *input, int32_t n_planes,
                                      const double *depths, int32_t flags, void *out, void *ws, size_t ws_bytes,
                                      void *stream)
{
    if (!ctx) return fail(nullptr, GWS_ERR_INVALID_ARG, "ctx is NULL");
    gws_status st = check_focal(ctx, prob, n_planes, flags);
    if (st != GWS_OK) return st;
    if (n_planes == 0) return GWS_OK;
    if (!input || !out || !depths) return fail(ctx, GWS_ERR_INVALID_ARG, "input, depths and out are required");
    for (int k = 0; k < n_planes; ++k)
        if (!std::isfinite(depths[k])) return fail(ctx, GWS_ERR_INVALID_ARG, "depths must be finite");
    st = check_ws(ctx, ws, ws_bytes, focal_stack_bytes(prob, n_planes, flags));
    if (st != GWS_OK) return st;
    HIP_CHECK(ctx, hipSetDevice(ctx->device));
    Plan *p = nullptr;
    st = get_plan(ctx, prob->nx, prob->ny, 4, &p);
    if (st != GWS_OK) return st;
    const hipStream_t s = (hipStream_t)stream;
    StageScope sc(ctx, s, ST_FOCAL);
    const int C = prob->n_lambda;
    const int64_t m = (int64_t)prob->nx * prob->ny;
    float2 *spec = (float2 *)ws;
    float2 *planes = (float2 *)((char *)ws + align256((size_t)m * C * sizeof(float2)));
    if (flags & GWS_FS_PHASE_INPUT) {
        HIP_CHECK(ctx, launch_phase_field((const float *)input, m * C, spec, s));
        HIP_CHECK(ctx, launch_fft2d(*p, C, -1, spec, spec, s));
    } else {
        HIP_CHECK(ctx, launch_fft2d(*p, C, -1, (const float2 *)input, spec, s));
    }
    StackArgs sa{};
    sa.C = C;
    sa.ny = prob->ny;
    sa.half_band = (flags & GWS_FS_HALF_BAND) ? 1 : 0;
    sa.scale = (float)(1.0 / ((double)prob->nx * prob->ny));
    sa.dnux = 1.0 / (prob->nx * prob->pitch_x);
    sa.dnuy = 1.0 / (prob->ny * prob->pitch_y);
    for (int c = 0; c < C; ++c) sa.inv_l[c] = 1.0 / prob->lambdas[c];
    for (int k0 = 0; k0 < n_planes; k0 += STACK_MAXK) {
        sa.K = std::min(STACK_MAXK, n_planes - k0);
        for (int k = 0; k < sa.K; ++k) {
            const double z = depths[k0 + k];
            sa.z[k] = z;
            for (int c = 0; c < C; ++c) {
                const double t = z * sa.inv_l[c];  // z / lambda to FP64 rounding (|z / lambda| << 2^52)
                sa.piston[k * STACK_MAXC + c] = t - std::floor(t);
            }
        }
        if (flags & GWS_FS_COMPLEX_OUTPUT) {
            float2 *dst = (float2 *)out + (int64_t)k0 * C * m;
            HIP_CHECK(ctx, launch_focal_stack(*p, spec, dst, nullptr, sa, s));
        } else {
            float *dst = (float *)out + (int64_t)k0 * C * m;
            HIP_CHECK(ctx, launch_focal_stack(*p, spec, planes, dst, sa, s));
        }
    }
    return GWS_OK;
}

extern "C" gws_status gws_set_profiling(gws_ctx *ctx, int enable)
{
    if (!ctx) return fail(nullptr, GWS_ERR_INVALID_ARG, "ctx is NULL");
    ctx->profiling = enable ? 1 : 0;
    return GWS_OK;
}

extern "C" gws_status gws_read_profile(gws_ctx *ctx, double *ms, int64_t *count)
{
    if (!ctx || !ms || !count) return fail(ctx, GWS_ERR_INVALID_ARG, "null argument");
    for (int i = 0; i < GWS_N_STAGES; ++i) {
        ms[i] = 0.0;
        count[i] = 0;
    }
    HIP_CHECK(ctx, hipSetDevice(ctx->device));
    for (auto &r : ctx->recs) {
        HIP_CHECK(ctx, hipEventSynchronize(r.b));
        float t = 0.0f;
        HIP_CHECK(ctx, hipEventElapsedTime(&t, r.a, r.b));
        if (r.stage >= 0 && r.stage < GWS_N_STAGES) {
            ms[r.stage] += t;
            count[r.stage] += 1;
        }
        ctx->pool.push_back(r.a);
        ctx->pool.push_back(r.b);
    }
    ctx->recs.clear();
    return GWS_OK;
}

extern "C" gws_status gws_measure_peaks(gws_ctx *ctx, gws_peaks *out, void *stream)
{
    if (!ctx || !out) return fail(ctx, GWS_ERR_INVALID_ARG, "null argument");
    HIP_CHECK(ctx, hipSetDevice(ctx->device));
    HIP_CHECK(ctx, run_probes(ctx->n_cu, (hipStream_t)stream, &out->trans_ops_per_s, &out->valu_ops_per_s,
                              &out->hbm_bytes_per_s));
    return GWS_OK;
}
