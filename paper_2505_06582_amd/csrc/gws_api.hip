// Host side of libgws: the C ABI of include/gws.h, argument validation, per-shape plans,
// workspace layout and the launch sequence of the forward and backward hot path.
#include <math.h>
#include <stdio.h>
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
    std::map<std::tuple<int, int, int>, Plan> plans;
    long long *d_stats = nullptr;  // copy of the counters of the last call
    int64_t last_n = 0;
    int last_tile_config = 1;
    int last_graph = 0;
    std::map<int, int> acc_occ;
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
    StageScope(gws_ctx *c, hipStream_t st, int sg) : ctx(c), s(st), stage(sg)
    {
        if (ctx->profiling) {
            a = pool_event(ctx);
            if (a) hipEventRecord(a, s);
        }
    }
    ~StageScope()
    {
        if (ctx->profiling && a) {
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
    const gws_status gs = check_grid(p->nx, p->ny);
    if (gs != GWS_OK) return gs;
    if (p->blend == GWS_BLEND_EXACT) return GWS_ERR_UNSUPPORTED;
    return GWS_OK;
}

// Tilings: frequencies per lane (F) of the forward accumulation and of the adjoint.  The
// work-group tile is 32 x 8F frequencies, the wavefront sub-tile 16 x 4F.
static const int kTileCfg[][2] = {{4, 4}, {4, 8}, {8, 8}, {8, 4}, {2, 4}, {4, 2}, {2, 2}, {2, 8}, {8, 2}};
static const int kNumTileCfg = (int)(sizeof(kTileCfg) / sizeof(kTileCfg[0]));
// Untuned default: F = 2 for the accumulation (finest culling), F = 4 for the adjoint
// (fewer cross-lane reductions per evaluated term); the fastest pair measured on MI355X
// for 1e4..1e5 Gaussians at 1080 x 1920.
static const int kDefaultTileCfg = 5;

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
    while (n % 8 == 0) { r[k++] = 8; n /= 8; }
    while (n % 4 == 0) { r[k++] = 4; n /= 4; }
    while (n % 2 == 0) { r[k++] = 2; n /= 2; }
    while (n % 5 == 0) { r[k++] = 5; n /= 5; }
    while (n % 3 == 0) { r[k++] = 3; n /= 3; }
    *nr = k;
}

static gws_status build_plan(gws_ctx *ctx, Plan &p, int nx, int ny, int F)
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
            const long long dx = x0 > 0 ? x0 : (x1 < 0 ? -x1 : 0);
            const long long dy = y0 > 0 ? y0 : (y1 < 0 ? -y1 : 0);
            int b = isqrt_floor(dx * dx + dy * dy);
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

static gws_status get_plan(gws_ctx *ctx, int nx, int ny, int F, Plan **out)
{
    auto key = std::make_tuple(nx, ny, F);
    auto it = ctx->plans.find(key);
    if (it != ctx->plans.end()) {
        *out = &it->second;
        return GWS_OK;
    }
    HIP_CHECK(ctx, hipSetDevice(ctx->device));
    Plan p;
    const gws_status st = build_plan(ctx, p, nx, ny, F);
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

// One workspace serves forward and backward under every tiling: tile arrays are sized
// for the smallest tiles (F = 2), the partial-sum area is a fixed byte budget whose slot
// count depends on the forward tiling, and the propagation table on the adjoint tiling.
static Layout make_layout(const gws_problem *p, int64_t n, int f_fwd, int f_bwd)
{
    Layout L;
    const int64_t M = (int64_t)p->nx * p->ny;
    const int C = p->n_lambda;
    const int ntiles = ntiles_for(p->nx, p->ny, 2);
    L.n = n;
    L.F = f_fwd;
    L.sort_blocks = (int)std::max<int64_t>(1, (n + 4095) / 4096);
    const size_t part_bytes = (size_t)fwd_max_slots_f4(n) * C * 4 * WG * sizeof(float2);
    L.max_slots = (int64_t)(part_bytes / ((size_t)C * f_fwd * WG * sizeof(float2)));
    L.max_items = L.max_slots / 2 + ntiles + 1;
    const int64_t nchunks = (n + BWD_CHUNK - 1) / BWD_CHUNK;
    L.max_bitems = std::max<int64_t>(nchunks + 1024, std::min<int64_t>(65536, nchunks * 64 + 1024));
    L.max_bslots = L.max_bitems;
    const int hx = p->nx / 2, hy = p->ny / 2, SY = sub_h(f_bwd);
    L.sx_min = floor_div(-hx, SUBX);
    L.sy_min = floor_div(-hy, SY);
    L.nsx = floor_div(hx - 1, SUBX) - L.sx_min + 1;
    L.nsy = floor_div(hy - 1, SY) - L.sy_min + 1;
    const int nsy_max = floor_div(hy - 1, sub_h(2)) - floor_div(-hy, sub_h(2)) + 1;
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
    L.off_bitems = take(sizeof(BItem) * L.max_bitems);
    L.off_chunk_items = take(sizeof(int2) * (nchunks + 1));
    L.off_bpartials = take(sizeof(float) * (size_t)L.max_bslots * 64 * NACC);
    L.off_spectrum = take(sizeof(float2) * (size_t)C * M);
    L.off_gspec = take(sizeof(float2) * (size_t)C * M);
    L.off_dtab = take(sizeof(float) * (size_t)C * M);
    L.off_d0tab = take(sizeof(double) * (size_t)C * L.nsx * nsy_max);
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
    *bytes = make_layout(problem, n, 2, 2).total;
    return GWS_OK;
}

// ---------------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------------
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
    hipMemset(ctx->d_stats, 0, sizeof(long long) * CTR_COUNT);
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
    out->n_tile_gaussian = h[CTR_PAIRS];
    out->n_candidates = h[CTR_CAND];
    out->tile_config = ctx->last_tile_config;
    out->graph_replayed = ctx->last_graph;
    out->n_tiles = 0;
    for (auto &kv : ctx->plans) out->n_tiles = std::max<int64_t>(out->n_tiles, kv.second.ntiles);
    return GWS_OK;
}

// ---------------------------------------------------------------------------------
// Forward / backward
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
    Item *items;
    BItem *bitems;
    float2 *partials, *spectrum, *gspec;
    float *bpartials, *dtab;
    double *d0tab;
};

static Bufs carve(const Layout &L, void *ws)
{
    char *b = (char *)ws;
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
    r.bpartials = (float *)(b + L.off_bpartials);
    r.spectrum = (float2 *)(b + L.off_spectrum);
    r.gspec = (float2 *)(b + L.off_gspec);
    r.dtab = (float *)(b + L.off_dtab);
    r.d0tab = (double *)(b + L.off_d0tab);
    return r;
}

// Preprocess + sort + records: shared by forward and backward.
static gws_status run_prep(gws_ctx *ctx, const Consts &k, const gws_gaussians *g, const Layout &L, const Bufs &B,
                           hipStream_t s, uint64_t **keys_sorted, uint32_t **vals_sorted)
{
    StageScope sc(ctx, s, ST_PREP);
    HIP_CHECK(ctx, launch_zero_counters(B.counters, B.bucket_hist, s));
    HIP_CHECK(ctx, launch_keys(*g, k, B.keys_a, B.vals_a, B.bucket_hist, B.counters, s));
    HIP_CHECK(ctx, radix_sort_48(B.keys_a, B.vals_a, B.keys_b, B.vals_b, B.sort_hist, g->n, L.sort_blocks, s, keys_sorted,
                                 vals_sorted));
    HIP_CHECK(ctx, launch_records(*g, k, *keys_sorted, *vals_sorted, B.rec, g->n, B.counters, s));
    return GWS_OK;
}

static int acc_grid(gws_ctx *ctx, int C, int F)
{
    const int key = C * 16 + F;
    auto it = ctx->acc_occ.find(key);
    if (it == ctx->acc_occ.end()) it = ctx->acc_occ.emplace(key, accumulate_occupancy(C, F)).first;
    return ctx->n_cu * it->second;
}

static int n_bucket(int64_t n)
{
    int b = 0;
    while (b < 40 && (1ll << (b + 1)) <= std::max<int64_t>(n, 1)) ++b;
    return b;
}

// Tiling for this call: the explicit one, else the one the autotuner chose for this shape
// and size class, else the default.
static int resolve_tile_config(const gws_ctx *ctx, const gws_problem *prob, int64_t n)
{
    if (prob->tile_config > 0) return prob->tile_config;
    if (ctx) {
        auto it = ctx->tuned.find(std::make_tuple(prob->nx, prob->ny, prob->n_lambda, n_bucket(n)));
        if (it != ctx->tuned.end()) return it->second;
    }
    return kDefaultTileCfg;
}

static gws_status forward_impl(gws_ctx *ctx, const gws_problem *prob, const gws_gaussians *g, const gws_output *out,
                               void *ws, size_t ws_bytes, hipStream_t s)
{
    const int cfg = resolve_tile_config(ctx, prob, g->n);
    const int F = kTileCfg[cfg - 1][0];
    Plan *p = nullptr;
    gws_status st = get_plan(ctx, prob->nx, prob->ny, F, &p);
    if (st != GWS_OK) return st;
    const Layout L = make_layout(prob, g->n, F, kTileCfg[cfg - 1][1]);
    st = check_ws(ctx, ws, ws_bytes, make_layout(prob, g->n, 2, 2).total);
    if (st != GWS_OK) return st;
    const Bufs B = carve(L, ws);
    const Consts k = make_consts(prob, 1);
    uint64_t *keys = nullptr;
    uint32_t *vals = nullptr;
    st = run_prep(ctx, k, g, L, B, s, &keys, &vals);
    if (st != GWS_OK) return st;
    {
        StageScope sc(ctx, s, ST_BIN);
        HIP_CHECK(ctx, launch_bin_forward(*p, B.bucket_hist, B.cum, B.tile_L, B.tile_slots, B.items, L.max_items,
                                          L.max_slots, B.counters, s));
    }
    float2 *spec = out->spectrum ? (float2 *)out->spectrum : B.spectrum;
    {
        StageScope sc(ctx, s, ST_ACCUM);
        HIP_CHECK(ctx, launch_accumulate(*p, k, B.rec, B.tile_L, B.items, B.partials, spec, B.counters,
                                         acc_grid(ctx, k.C, F), s));
    }
    {
        StageScope sc(ctx, s, ST_REDUCE);
        HIP_CHECK(ctx, launch_reduce_partials(*p, k, B.tile_slots, B.partials, spec, s));
    }
    {
        StageScope sc(ctx, s, ST_XFORM_INV);
        if (prob->xform == GWS_XFORM_FFT_FP32) {
            HIP_CHECK(ctx, launch_fft2d(*p, k.C, +1, spec, (float2 *)out->field, s));
        } else {
            // the bf16 DFT keeps its split operands in the spare gspec/dtab region of the workspace
            HIP_CHECK(ctx, launch_dft_bf16x3(*p, k.C, +1, spec, (float2 *)out->field, (void *)B.gspec, s));
        }
    }
    HIP_CHECK(ctx, launch_copy_counters(B.counters, ctx->d_stats, s));
    ctx->last_n = g->n;
    ctx->last_tile_config = cfg;
    ctx->last_graph = 0;
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
    return forward_impl(ctx, prob, g, out, ws, ws_bytes, (hipStream_t)stream);
}

static gws_status check_grads(gws_ctx *ctx, const gws_grads *gr)
{
    if (!gr || !gr->mean_x || !gr->mean_y || !gr->cov_xx || !gr->cov_xy || !gr->cov_yy || !gr->opacity ||
        !gr->amplitude || !gr->phase)
        return fail(ctx, GWS_ERR_INVALID_ARG, "a gradient array is NULL");
    return GWS_OK;
}

static gws_status backward_impl(gws_ctx *ctx, const gws_problem *prob, const gws_gaussians *g, const void *grad_field,
                                const gws_grads *grads, void *ws, size_t ws_bytes, hipStream_t s)
{
    const int cfg = resolve_tile_config(ctx, prob, g->n);
    const int F = kTileCfg[cfg - 1][1];
    Plan *p = nullptr;
    gws_status st = get_plan(ctx, prob->nx, prob->ny, F, &p);
    if (st != GWS_OK) return st;
    const Layout L = make_layout(prob, g->n, kTileCfg[cfg - 1][0], F);
    st = check_ws(ctx, ws, ws_bytes, make_layout(prob, g->n, 2, 2).total);
    if (st != GWS_OK) return st;
    const Bufs B = carve(L, ws);
    Consts k = make_consts(prob, 0);
    k.depth_grad = grads->depth != nullptr;
    uint64_t *keys = nullptr;
    uint32_t *vals = nullptr;
    st = run_prep(ctx, k, g, L, B, s, &keys, &vals);
    if (st != GWS_OK) return st;
    {
        StageScope sc(ctx, s, ST_BIN);
        HIP_CHECK(ctx, launch_bin_backward(*p, keys, B.bitems, B.chunk_items, L.max_bitems, B.counters, g->n, s));
    }
    {
        // Gs = forward DFT of the field gradient (adjoint of the unnormalised inverse DFT)
        StageScope sc(ctx, s, ST_XFORM_FWD);
        if (prob->xform == GWS_XFORM_FFT_FP32)
            HIP_CHECK(ctx, launch_fft2d(*p, k.C, -1, (const float2 *)grad_field, B.gspec, s));
        else
            HIP_CHECK(ctx, launch_dft_bf16x3(*p, k.C, -1, (const float2 *)grad_field, B.gspec, (void *)B.spectrum, s));
    }
    {
        StageScope sc(ctx, s, ST_DTABLE);
        HIP_CHECK(ctx, launch_dtable(k, B.dtab, B.d0tab, L.nsx, L.nsy, L.sx_min, L.sy_min, sub_h(F), s));
    }
    {
        StageScope sc(ctx, s, ST_ADJOINT);
        HIP_CHECK(ctx, launch_adjoint2(*p, k, B.rec, B.gspec, B.dtab, B.d0tab, L.nsx, L.nsy, L.sx_min, L.sy_min,
                                       B.bitems, B.bpartials, B.counters, g->n, ctx->n_cu * 4, s));
    }
    {
        StageScope sc(ctx, s, ST_FINAL);
        HIP_CHECK(ctx, launch_grad_final2(*g, k, vals, B.chunk_items, B.bpartials, *grads, g->n, B.counters, s));
    }
    HIP_CHECK(ctx, launch_copy_counters(B.counters, ctx->d_stats, s));
    ctx->last_n = g->n;
    ctx->last_tile_config = cfg;
    ctx->last_graph = 0;
    return GWS_OK;
}

extern "C" gws_status gws_backward(gws_ctx *ctx, const gws_problem *prob, const gws_gaussians *g, const void *grad_field,
                                   const gws_grads *grads, void *ws, size_t ws_bytes, void *stream)
{
    if (!ctx) return fail(nullptr, GWS_ERR_INVALID_ARG, "ctx is NULL");
    gws_status st = gws_check_problem(prob);
    if (st != GWS_OK) return fail(ctx, st, std::string("problem rejected: ") + gws_status_string(st));
    if (prob->n_lambda > 3) return fail(ctx, GWS_ERR_UNSUPPORTED, "backward supports at most 3 wavelengths");
    st = check_gaussians(ctx, g);
    if (st != GWS_OK) return st;
    st = check_grads(ctx, grads);
    if (st != GWS_OK) return st;
    if (!grad_field) return fail(ctx, GWS_ERR_INVALID_ARG, "grad_field is NULL");
    HIP_CHECK(ctx, hipSetDevice(ctx->device));
    return backward_impl(ctx, prob, g, grad_field, grads, ws, ws_bytes, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------------
// Stand-alone 2D DFT
// ---------------------------------------------------------------------------------
extern "C" gws_status gws_dft_workspace_size(const gws_ctx *ctx, int32_t nx, int32_t ny, int32_t batch, int32_t xform,
                                             size_t *bytes)
{
    (void)ctx;
    if (!bytes || batch < 1) return GWS_ERR_INVALID_ARG;
    if (check_grid(nx, ny) != GWS_OK) return GWS_ERR_SHAPE;
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
// Batched scenes and autotuning: not yet available.
// ---------------------------------------------------------------------------------
extern "C" gws_status gws_workspace_size_batched(const gws_ctx *, const gws_problem *, int32_t, const int64_t *, size_t *)
{
    return GWS_ERR_UNSUPPORTED;
}
extern "C" gws_status gws_forward_batched(gws_ctx *ctx, const gws_problem *, int32_t, const int64_t *, const gws_gaussians *,
                                          const gws_output *, void *, size_t, void *)
{
    return fail(ctx, GWS_ERR_UNSUPPORTED, "batched forward not built");
}
extern "C" gws_status gws_backward_batched(gws_ctx *ctx, const gws_problem *, int32_t, const int64_t *, const gws_gaussians *,
                                           const void *, const gws_grads *, void *, size_t, void *)
{
    return fail(ctx, GWS_ERR_UNSUPPORTED, "batched backward not built");
}
extern "C" gws_status gws_autotune(gws_ctx *ctx, const gws_problem *, int64_t, const char *, void *)
{
    return fail(ctx, GWS_ERR_UNSUPPORTED, "autotuner not built");
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
