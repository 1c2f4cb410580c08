// Per-Gaussian preprocessing, depth sort and binning of spectral supports (gfx950).
//
// k_keys     one thread per Gaussian: validity, spectral-support radius bucket, sort key
//            (support radius descending, then depth descending = front to back).
// radix sort stable LSD radix sort of the 48-bit keys, 8-bit digits, wave-ballot ranking.
// k_records  one thread per sorted Gaussian: the 64-byte record the accumulation reads,
//            with every large phase quantity reduced exactly in FP64 / fixed point.
// k_bin_*    one work-group: candidate counts per tile, chunk size, work-item lists.
//
// The spectrum of Gaussian i (Sec. 4.1, Eq. 10, in-plane so det J = 1) has modulus
// 2 pi sqrt(det S) exp(-2 pi^2 nu^T S nu): an ellipse centred on DC.  In index units
// (nu_x = m_x'/(nx px), nu_y = m_y'/(ny py)) the exponent, written in powers of two, is
// q(m') = alpha m_x'^2 + beta2 m_x' m_y' + gamma m_y'^2 and the term is below eps of its
// peak outside q <= log2(1/eps).  The circumscribed circle of that ellipse has radius
// sqrt(log2(1/eps) / lambda_min) and sets the Gaussian's bucket.
#include "gws_internal.h"

namespace gws {

static __device__ __forceinline__ bool finite_f(float v) { return (__float_as_uint(v) & 0x7f800000u) != 0x7f800000u; }

static __device__ __forceinline__ double frac_d(double v) { return v - floor(v); }

__global__ void __launch_bounds__(256) k_keys(GView g, Consts k, uint64_t *__restrict__ keys,
                                               uint32_t *__restrict__ vals, uint32_t *__restrict__ bucket_hist,
                                               long long *__restrict__ counters)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.n) return;
    const float sxx = g.cov_xx[i], sxy = g.cov_xy[i], syy = g.cov_yy[i];
    const float mx = g.mean_x[i], my = g.mean_y[i], z = g.depth[i], o = g.opacity[i], ph = g.phase[i];
    bool ok = finite_f(sxx) && finite_f(sxy) && finite_f(syy) && finite_f(mx) && finite_f(my) &&
              finite_f(z) && finite_f(o) && finite_f(ph);
    bool any_amp = false;
    for (int c = 0; c < k.C; ++c) {
        const float a = g.amplitude[(int64_t)c * g.amp_stride + i];
        ok = ok && finite_f(a);
        any_amp = any_amp || (a != 0.0f);
    }
    const double det = (double)sxx * syy - (double)sxy * sxy;
    ok = ok && sxx > 0.0f && det > 0.0;
    if (k.forward) ok = ok && o != 0.0f && any_amp;
    uint32_t hi;
    if (ok) {
        const double Wx = k.nx * k.px, Wy = k.ny * k.py;
        const double a = k.K2 * sxx / (Wx * Wx), b = k.K2 * sxy / (Wx * Wy), c = k.K2 * syy / (Wy * Wy);
        const double lmin = 0.5 * (a + c) - sqrt(0.25 * (a - c) * (a - c) + b * b);
        int bucket = NBUCKET - 1;
        if (lmin > 0.0) {
            const double R = sqrt(k.tau2 / lmin);
            if (R < (double)(NBUCKET - 1)) bucket = (int)R;
        }
        hi = (uint32_t)(NBUCKET - 1 - bucket);
        atomicAdd(&bucket_hist[bucket], 1u);
    } else {
        hi = 0xffffu;
        atomicAdd((unsigned long long *)&counters[CTR_NCULLED], 1ull);
    }
    // depth, descending: map the float to an ascending unsigned key, then complement
    const uint32_t u = __float_as_uint(z);
    const uint32_t asc = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    keys[i] = ((uint64_t)hi << 32) | (uint64_t)(~asc);
    vals[i] = (uint32_t)i;
}

hipError_t launch_keys(const GView &g, const Consts &k, uint64_t *keys, uint32_t *vals,
                       uint32_t *bucket_hist, long long *counters, hipStream_t s)
{
    const int64_t blocks = (g.n + 255) / 256;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_keys, dim3((unsigned)blocks), dim3(256), 0, s, g, k, keys, vals, bucket_hist, counters);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Stable LSD radix sort, 8-bit digits.  Each block owns ITEMS x 256 consecutive keys: 16 per
// thread, or 4 for up to 32768 keys, where more, shorter blocks finish each pass sooner.
// ---------------------------------------------------------------------------------
constexpr int SORT_THREADS = 256;
static int sort_items(int64_t n) { return n <= 32768 ? 4 : 16; }
int sort_blocks_for(int64_t n)
{
    const int64_t tile = (int64_t)SORT_THREADS * sort_items(n);
    return (int)std::max<int64_t>(1, (n + tile - 1) / tile);
}

template <int ITEMS>
__global__ void __launch_bounds__(SORT_THREADS) k_sort_hist(const uint64_t *__restrict__ keys, int64_t n, int shift,
                                                            uint32_t *__restrict__ block_hist, int nblocks)
{
    constexpr int SORT_ITEMS = ITEMS, SORT_TILE = SORT_THREADS * ITEMS;
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * SORT_TILE;
    for (int it = 0; it < SORT_ITEMS; ++it) {
        const int64_t i = base + (int64_t)it * SORT_THREADS + threadIdx.x;
        if (i < n) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & 0xffu], 1u);
    }
    __syncthreads();
    block_hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of block_hist (digit-major) in place; one block of 1024 threads.
__global__ void __launch_bounds__(1024) k_sort_scan(uint32_t *__restrict__ block_hist, int total)
{
    __shared__ uint32_t part[1024];
    const int per = (total + 1023) / 1024;
    const int b = threadIdx.x * per;
    uint32_t sum = 0;
    for (int j = 0; j < per && b + j < total; ++j) sum += block_hist[b + j];
    part[threadIdx.x] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = part[threadIdx.x] - sum;
    for (int j = 0; j < per && b + j < total; ++j) {
        const uint32_t v = block_hist[b + j];
        block_hist[b + j] = run;
        run += v;
    }
}

template <int ITEMS>
__global__ void __launch_bounds__(SORT_THREADS) k_sort_scatter(const uint64_t *__restrict__ keys_in,
                                                               const uint32_t *__restrict__ vals_in,
                                                               uint64_t *__restrict__ keys_out,
                                                               uint32_t *__restrict__ vals_out, int64_t n,
                                                               int shift, const uint32_t *__restrict__ block_hist,
                                                               int nblocks)
{
    constexpr int SORT_ITEMS = ITEMS, SORT_TILE = SORT_THREADS * ITEMS;
    __shared__ uint32_t run[256];          // running output offset per digit for this block
    __shared__ uint32_t wave_cnt[SORT_THREADS / 64][256];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    run[threadIdx.x] = block_hist[(int64_t)threadIdx.x * nblocks + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * SORT_TILE;
    for (int it = 0; it < SORT_ITEMS; ++it) {
        const int64_t i = base + (int64_t)it * SORT_THREADS + threadIdx.x;
        const bool valid = i < n;
        uint64_t key = valid ? keys_in[i] : 0;
        const uint32_t val = valid ? vals_in[i] : 0;
        const uint32_t d = (uint32_t)(key >> shift) & 0xffu;
        // lanes of this wave holding the same digit
        uint64_t same = __ballot(valid);
        for (int bit = 0; bit < 8; ++bit) {
            const uint64_t bb = __ballot((d >> bit) & 1u);
            same &= ((d >> bit) & 1u) ? bb : ~bb;
        }
        const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        const uint32_t rank_in_wave = (uint32_t)__popcll(same & lt);
        // zero the per-wave counts, then the lowest lane of each digit group publishes its size
        for (int j = lane; j < 256; j += 64) wave_cnt[wave][j] = 0;
        __syncthreads();
        if (valid && rank_in_wave == 0) wave_cnt[wave][d] = (uint32_t)__popcll(same);
        __syncthreads();
        if (valid) {
            uint32_t off = run[d];
            for (int w = 0; w < wave; ++w) off += wave_cnt[w][d];
            const uint32_t pos = off + rank_in_wave;
            keys_out[pos] = key;
            vals_out[pos] = val;
        }
        __syncthreads();
        // advance the running offsets by this iteration's digit counts
        {
            uint32_t add = 0;
            for (int w = 0; w < SORT_THREADS / 64; ++w) add += wave_cnt[w][threadIdx.x];
            run[threadIdx.x] += add;
        }
        __syncthreads();
    }
}

hipError_t radix_sort_48(uint64_t *keys_a, uint32_t *vals_a, uint64_t *keys_b, uint32_t *vals_b,
                         uint32_t *block_hist, int64_t n, int nblocks, hipStream_t s, uint64_t **keys_out,
                         uint32_t **vals_out)
{
    uint64_t *ki = keys_a, *ko = keys_b;
    uint32_t *vi = vals_a, *vo = vals_b;
    if (n > 0) {
        if (nblocks != sort_blocks_for(n)) return hipErrorInvalidValue;   // the caller's histogram area
        const bool small = sort_items(n) == 4;
        for (int pass = 0; pass < 6; ++pass) {
            const int shift = 8 * pass;
            if (small)
                hipLaunchKernelGGL(k_sort_hist<4>, dim3(nblocks), dim3(SORT_THREADS), 0, s, ki, n, shift, block_hist,
                                   nblocks);
            else
                hipLaunchKernelGGL(k_sort_hist<16>, dim3(nblocks), dim3(SORT_THREADS), 0, s, ki, n, shift, block_hist,
                                   nblocks);
            hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(1024), 0, s, block_hist, 256 * nblocks);
            if (small)
                hipLaunchKernelGGL(k_sort_scatter<4>, dim3(nblocks), dim3(SORT_THREADS), 0, s, ki, vi, ko, vo, n, shift,
                                   block_hist, nblocks);
            else
                hipLaunchKernelGGL(k_sort_scatter<16>, dim3(nblocks), dim3(SORT_THREADS), 0, s, ki, vi, ko, vo, n,
                                   shift, block_hist, nblocks);
            uint64_t *tk = ki; ki = ko; ko = tk;
            uint32_t *tv = vi; vi = vo; vo = tv;
        }
    }
    *keys_out = ki;
    *vals_out = vi;
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Records, in sorted order.
// ---------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_records(GView g, Consts k, const uint64_t *__restrict__ keys,
                                                  const uint32_t *__restrict__ vals, GRec *__restrict__ rec,
                                                  int64_t n, const long long *__restrict__ counters)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nvalid = n - counters[CTR_NCULLED];
    if (s >= nvalid) return;
    const int64_t i = vals[s];
    const double sxx = g.cov_xx[i], sxy = g.cov_xy[i], syy = g.cov_yy[i];
    const double det = sxx * syy - sxy * sxy;
    const double Wx = k.nx * k.px, Wy = k.ny * k.py;
    GRec r;
    r.alpha = (float)(k.K2 * sxx / (Wx * Wx));
    r.beta2 = (float)(2.0 * k.K2 * sxy / (Wx * Wy));
    r.gamma = (float)(k.K2 * syy / (Wy * Wy));
    const float z = g.depth[i];
    r.z = z;
    // ramp: the centring factor (-1)^m' of the SLM-centred field is folded in as +1/2
    const double fx = frac_d((double)g.mean_x[i] / Wx + 0.5);
    const double fy = frac_d((double)g.mean_y[i] / Wy + 0.5);
    r.rx = (uint32_t)(uint64_t)llrint(fx * 4294967296.0);
    r.ry = (uint32_t)(uint64_t)llrint(fy * 4294967296.0);
    r.rxf = (float)((double)(int32_t)r.rx * (1.0 / 4294967296.0));
    r.ryf = (float)((double)(int32_t)r.ry * (1.0 / 4294967296.0));
    const double o = g.opacity[i];
    const double norm = 6.283185307179586 * sqrt(det) / (k.px * k.py * (double)k.nx * (double)k.ny);
    // carrier: the Gaussian's phase, the propagation's z / lambda, and under reference-wave
    // illumination (spectrum taken at nu - nu_r) the ramp's constant part +nu_r . mu
    const double phi_rev =
        frac_d((double)g.phase[i] * 0.15915494309189535 + k.nurx * (double)g.mean_x[i] + k.nury * (double)g.mean_y[i]);
    for (int c = 0; c < 4; ++c) {
        if (c < k.C) {
            r.kappa[c] = (float)frac_d(phi_rev - (double)z * k.inv_lambda[c]);
            r.amp[c] = (float)((double)g.amplitude[(int64_t)c * g.amp_stride + i] * o * norm);
        } else {
            r.kappa[c] = 0.0f;
            r.amp[c] = 0.0f;
        }
    }
    rec[s] = r;
}

hipError_t launch_records(const GView &g, const Consts &k, const uint64_t *keys, const uint32_t *vals,
                          GRec *rec, int64_t n, const long long *counters, hipStream_t s)
{
    const int64_t blocks = (n + 255) / 256;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_records, dim3((unsigned)blocks), dim3(256), 0, s, g, k, keys, vals, rec, n, counters);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Forward binning.  Tiles are held in order of increasing distance rho from DC, so the
// candidates of tile k -- Gaussians whose support circle reaches the tile -- are a prefix
// L_k of the sorted Gaussians, and the heaviest tiles come first.  Each tile's
// candidates are split into chunks of CH; CH grows until the tiles with more than one
// chunk need at most max_slots partial-sum slots (bounded workspace).
// ---------------------------------------------------------------------------------
static __device__ uint32_t block_excl_scan_1024(uint32_t v, uint32_t *tmp, uint32_t *total)
{
    tmp[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t t = threadIdx.x >= off ? tmp[threadIdx.x - off] : 0u;
        __syncthreads();
        tmp[threadIdx.x] += t;
        __syncthreads();
    }
    const uint32_t incl = tmp[threadIdx.x];
    *total = tmp[1023];
    __syncthreads();
    return incl - v;
}

__global__ void __launch_bounds__(1024) k_bin_forward(const int32_t *__restrict__ tile_bucket, int ntiles,
                                                      const uint32_t *__restrict__ bucket_hist, uint32_t *__restrict__ cum,
                                                      int32_t *__restrict__ tile_L, int2 *__restrict__ tile_slots,
                                                      Item *__restrict__ items,
                                                      int64_t max_items, int64_t max_slots, int base_chunk,
                                                      long long *__restrict__ counters)
{
    __shared__ uint32_t tmp[1024];
    __shared__ unsigned long long red[1024];
    __shared__ int32_t chunk_sh;
    uint32_t total;
    // suffix sums over buckets: cum[b] = #valid Gaussians with bucket >= b
    {
        const int per = NBUCKET / 1024;
        const int b0 = (1023 - threadIdx.x) * per;  // thread 0 owns the highest buckets
        uint32_t s = 0;
        for (int j = 0; j < per; ++j) s += bucket_hist[b0 + j];
        const uint32_t ex = block_excl_scan_1024(s, tmp, &total);
        uint32_t run = ex;
        for (int j = per - 1; j >= 0; --j) {
            run += bucket_hist[b0 + j];
            cum[b0 + j] = run;
        }
    }
    __syncthreads();
    // candidates per tile and their total
    unsigned long long sumL = 0;
    for (int t = threadIdx.x; t < ntiles; t += 1024) {
        const uint32_t L = cum[tile_bucket[t]];
        tile_L[t] = (int32_t)L;
        sumL += L;
    }
    red[threadIdx.x] = sumL;
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const unsigned long long S = red[0];
        // multi-chunk tiles need <= 2 S / CH slots: the configured base chunk, grown to fit
        long long ch = base_chunk;
        const long long need = (long long)((2ull * S + (unsigned long long)max_slots - 1) / (unsigned long long)max_slots);
        if (need > ch) ch = (need + 255) / 256 * 256;
        if (ch > (1ll << 30)) ch = 1ll << 30;
        chunk_sh = (int32_t)ch;
        counters[CTR_CHUNK] = ch;
        counters[CTR_CAND] = (long long)S;
    }
    __syncthreads();
    const int CH = chunk_sh;
    // items per tile (tiles are processed in slices of 1024 with a running offset)
    uint32_t item_base = 0, slot_base = 0;
    for (int t0 = 0; t0 < ntiles; t0 += 1024) {
        const int t = t0 + threadIdx.x;
        const uint32_t L = t < ntiles ? (uint32_t)tile_L[t] : 0u;
        const uint32_t nk = (L + CH - 1) / CH;
        uint32_t tot_items, tot_slots;
        const uint32_t ex_items = block_excl_scan_1024(nk, tmp, &tot_items);
        const uint32_t ex_slots = block_excl_scan_1024(nk > 1 ? nk : 0u, tmp, &tot_slots);
        if (t < ntiles) tile_slots[t] = make_int2((int)nk, (int)(slot_base + ex_slots));
        for (uint32_t j = 0; j < nk; ++j) {
            const uint64_t it = (uint64_t)item_base + ex_items + j;
            if (it < (uint64_t)max_items) {
                Item e;
                e.tile = t;
                e.chunk = (int32_t)j;
                e.slot = nk > 1 ? (int32_t)(slot_base + ex_slots + j) : -1;
                e.pad = 0;
                items[it] = e;
            }
        }
        item_base += tot_items;
        slot_base += tot_slots;
    }
    if (threadIdx.x == 0) {
        counters[CTR_NITEMS] = (long long)(item_base < max_items ? item_base : max_items);
        counters[CTR_WORK] = 0;
    }
}

hipError_t launch_bin_forward(const Plan &p, const uint32_t *bucket_hist, uint32_t *cum, int32_t *tile_L,
                              int2 *tile_slots, Item *items, int64_t max_items, int64_t max_slots, int base_chunk,
                              long long *counters, hipStream_t s)
{
    hipLaunchKernelGGL(k_bin_forward, dim3(1), dim3(1024), 0, s, p.tile_bucket, p.ntiles, bucket_hist, cum, tile_L,
                       tile_slots, items, max_items, max_slots, base_chunk, counters);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Backward binning: chunk b of `chunk` sorted Gaussians reaches the first K_b sorted
// tiles (K_b = tiles whose bucket is at most the chunk's largest bucket).  Those tiles are
// split into ranges of TRB tiles (TRB grows until the items fit max_bitems).  Items are
// ordered range-major -- range r of every chunk that has one, then range r + 1 -- so the
// wavefronts in flight at any time read the same tiles of the field gradient (L2 reuse).
// Because K_b does not increase with b (chunks are sorted by support radius), the chunks
// that have range r form a prefix [0, P_r) and item (r, b) sits at range_base[r] + b.
// ---------------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) k_bin_backward(const int32_t *__restrict__ tile_cum,
                                                       const uint64_t *__restrict__ keys, BItem *__restrict__ bitems,
                                                       int2 *__restrict__ chunk_items, int32_t *__restrict__ range_base,
                                                       int max_ranges, int64_t max_bitems,
                                                       long long *__restrict__ counters, int64_t n, int chunk)
{
    __shared__ uint32_t tmp[1024];
    __shared__ unsigned long long red[1024];
    __shared__ int32_t trb_sh, nr_sh;
    const int64_t nvalid = n - counters[CTR_NCULLED];
    const int nchunks = (int)((nvalid + chunk - 1) / chunk);
    auto K_of = [&](int b) { return tile_cum[NBUCKET - 1 - (int)(keys[(int64_t)b * chunk] >> 32)]; };
    unsigned long long sumK = 0;
    for (int b = threadIdx.x; b < nchunks; b += 1024) sumK += (unsigned long long)K_of(b);
    red[threadIdx.x] = sumK;
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const unsigned long long S = red[0];
        long long trb = 1;
        // items <= S / TRB + nchunks <= max_bitems
        const long long room = max_bitems - nchunks;
        if (room > 0) {
            const long long need = (long long)((S + (unsigned long long)room - 1) / (unsigned long long)room);
            if (need > trb) trb = need;
        } else {
            trb = 1 << 30;
        }
        trb_sh = (int32_t)trb;
        nr_sh = nchunks > 0 ? (int32_t)((K_of(0) + trb - 1) / trb) : 0;
        counters[CTR_TRB] = trb;
    }
    __syncthreads();
    const int TRB = trb_sh, NR = min(nr_sh, max_ranges);
    // P_r = number of chunks with more than r ranges (a prefix, found by bisection)
    uint32_t base = 0;
    for (int r0 = 0; r0 < NR; r0 += 1024) {
        const int r = r0 + threadIdx.x;
        uint32_t P = 0;
        if (r < NR) {
            int lo = 0, hi = nchunks;  // first b with ceil(K_b / TRB) <= r
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if ((K_of(mid) + TRB - 1) / TRB > r) lo = mid + 1;
                else hi = mid;
            }
            P = (uint32_t)lo;
        }
        uint32_t tot;
        const uint32_t ex = block_excl_scan_1024(P, tmp, &tot);
        if (r < NR) range_base[r] = (int32_t)(base + ex);
        base += tot;
    }
    if (threadIdx.x == 0) range_base[NR] = (int32_t)base;
    __syncthreads();
    for (int b = threadIdx.x; b < nchunks; b += 1024) {
        const int K = K_of(b);
        const int nk = min((K + TRB - 1) / TRB, NR);
        chunk_items[b] = make_int2(0, nk);
        for (int r = 0; r < nk; ++r) {
            const int64_t it = (int64_t)range_base[r] + b;
            if (it < max_bitems) {
                BItem e;
                e.chunk = b;
                e.k0 = r * TRB;
                e.k1 = min((r + 1) * TRB, K);
                e.slot = (int32_t)it;
                bitems[it] = e;
            }
        }
    }
    if (threadIdx.x == 0) {
        counters[CTR_NBITEMS] = (long long)(base < max_bitems ? base : max_bitems);
        counters[CTR_BWORK] = 0;
    }
}

hipError_t launch_bin_backward(const Plan &p, const uint64_t *keys, BItem *bitems, int2 *chunk_items,
                               int32_t *range_base, int max_ranges, int64_t max_bitems, long long *counters, int64_t n,
                               int chunk, hipStream_t s)
{
    hipLaunchKernelGGL(k_bin_backward, dim3(1), dim3(1024), 0, s, p.tile_cum, keys, bitems, chunk_items, range_base,
                       max_ranges, max_bitems, counters, n, chunk);
    return hipGetLastError();
}

__global__ void k_zero_counters(long long *__restrict__ counters, uint32_t *__restrict__ bucket_hist)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < CTR_COUNT) counters[t] = 0;
    if (t < NBUCKET) bucket_hist[t] = 0;
}

__global__ void k_copy_counters(const long long *__restrict__ src, long long *__restrict__ dst)
{
    const int t = threadIdx.x;
    if (t < CTR_COUNT) dst[t] = src[t];
}

hipError_t launch_zero_counters(long long *counters, uint32_t *bucket_hist, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_counters, dim3(NBUCKET / 256), dim3(256), 0, s, counters, bucket_hist);
    return hipGetLastError();
}

hipError_t launch_copy_counters(const long long *src, long long *dst, hipStream_t s)
{
    hipLaunchKernelGGL(k_copy_counters, dim3(1), dim3(64), 0, s, src, dst);
    return hipGetLastError();
}

// Scene tables: copy the by-value table to device memory and form the prefix sums of the
// per-scene work-item counts (so one persistent launch can walk every scene's items).
__global__ void k_fwd_table(FwdTab tab, FwdScene *__restrict__ dst, int32_t *__restrict__ prefix,
                            long long *__restrict__ queue)
{
    if (threadIdx.x == 0) {
        int32_t run = 0;
        for (int i = 0; i < tab.n; ++i) {
            dst[i] = tab.s[i];
            prefix[i] = run;
            run += (int32_t)tab.s[i].counters[CTR_NITEMS];
        }
        prefix[tab.n] = run;
        *queue = 0;
    }
}

__global__ void k_bwd_table(BwdTab tab, BwdScene *__restrict__ dst, int32_t *__restrict__ prefix,
                            long long *__restrict__ queue)
{
    if (threadIdx.x == 0) {
        int32_t run = 0;
        for (int i = 0; i < tab.n; ++i) {
            dst[i] = tab.s[i];
            prefix[i] = run;
            run += (int32_t)tab.s[i].counters[CTR_NBITEMS];
        }
        prefix[tab.n] = run;
        *queue = 0;
    }
}

hipError_t launch_fwd_table(const FwdTab &tab, FwdScene *dst, int32_t *prefix, long long *queue, hipStream_t s)
{
    hipLaunchKernelGGL(k_fwd_table, dim3(1), dim3(64), 0, s, tab, dst, prefix, queue);
    return hipGetLastError();
}

hipError_t launch_bwd_table(const BwdTab &tab, BwdScene *dst, int32_t *prefix, long long *queue, hipStream_t s)
{
    hipLaunchKernelGGL(k_bwd_table, dim3(1), dim3(64), 0, s, tab, dst, prefix, queue);
    return hipGetLastError();
}

struct CtrPtrs {
    int n;
    long long *p[MAX_SCENES];
};

// Statistics of a call: counters summed over its scenes.
__global__ void k_sum_counters(CtrPtrs src, long long *__restrict__ dst)
{
    const int t = threadIdx.x;
    if (t < CTR_COUNT) {
        long long v = 0;
        for (int i = 0; i < src.n; ++i) v += src.p[i][t];
        dst[t] = v;
    }
}

hipError_t launch_sum_counters(long long *const *src, int n, long long *dst, hipStream_t s)
{
    CtrPtrs c;
    c.n = n;
    for (int i = 0; i < n && i < MAX_SCENES; ++i) c.p[i] = src[i];
    hipLaunchKernelGGL(k_sum_counters, dim3(1), dim3(64), 0, s, c, dst);
    return hipGetLastError();
}

// Synthetic Gaussians for the autotuner, drawn on the device with a counter-based
// generator (SplitMix64 of seed, index and draw number): means uniform over the field,
// depth U(-10, 10) mm, standard deviations U(2, 20) pixels per axis, rotation U(0, pi),
// opacity U(0.1, 1), amplitudes U(0, 1), phase U(0, 2 pi).
static __device__ __forceinline__ double u01(uint64_t seed, uint64_t i, uint64_t d)
{
    uint64_t z = seed + 0x9e3779b97f4a7c15ull * (i * 16 + d + 1);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

__global__ void k_synth(float *__restrict__ base, int64_t n, uint64_t seed, Consts k)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double PI = 3.14159265358979323846;
    const double W = k.nx * k.px, H = k.ny * k.py;
    const double su = (2.0 + 18.0 * u01(seed, i, 3)) * k.px, sv = (2.0 + 18.0 * u01(seed, i, 4)) * k.py;
    const double th = PI * u01(seed, i, 5);
    const double c = cos(th), s = sin(th);
    float *mx = base, *my = base + n, *z = base + 2 * n, *sxx = base + 3 * n, *sxy = base + 4 * n, *syy = base + 5 * n;
    float *o = base + 6 * n, *ph = base + 7 * n, *amp = base + 8 * n;
    mx[i] = (float)((u01(seed, i, 0) - 0.5) * W);
    my[i] = (float)((u01(seed, i, 1) - 0.5) * H);
    z[i] = (float)((u01(seed, i, 2) - 0.5) * 0.02);
    sxx[i] = (float)(c * c * su * su + s * s * sv * sv);
    sxy[i] = (float)(c * s * (su * su - sv * sv));
    syy[i] = (float)(s * s * su * su + c * c * sv * sv);
    o[i] = (float)(0.1 + 0.9 * u01(seed, i, 6));
    ph[i] = (float)(2.0 * PI * u01(seed, i, 7));
    for (int ch = 0; ch < k.C; ++ch) amp[(int64_t)ch * n + i] = (float)u01(seed, i, 8 + ch);
}

hipError_t launch_synth(GView g, float *base, int64_t n, uint64_t seed, const Consts &k, hipStream_t s)
{
    (void)g;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_synth, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, base, n, seed, k);
    return hipGetLastError();
}

}  // namespace gws
