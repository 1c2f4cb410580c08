/*
 * gws.h -- C ABI of the MI355X (gfx950) Gaussian Wave Splatting library.
 *
 * The library turns a set of in-plane 2D Gaussians into the complex field they produce
 * at the SLM plane, with the fast (order-invariant transparency) form of alpha wave
 * blending: every Gaussian's closed-form angular spectrum (Sec. 4.1, Eq. 10) is
 * multiplied by its colour, opacity and the angular-spectrum transfer function for its
 * depth (Eq. 3-4 at distance -z), summed per frequency (Sec. 4.2, Eq. 12; Alg. 1 and
 * Alg. 4 of the supplement) and brought to the SLM plane by one inverse 2D DFT.  It also
 * gives the exact adjoint of that map (gradients of a real loss with respect to every
 * Gaussian parameter).
 *
 * Conventions (the paper mixes angular and ordinary frequency; these are fixed here):
 *   - spatial frequency nu in cycles per metre; frequency index m in FFT order, with
 *     signed index m' = m if 2m < N else m - N and nu = m' / (N * pitch);
 *   - a Gaussian centred at mu carries the ramp exp(-j 2 pi nu . mu);
 *   - H(nu, d) = exp(+j 2 pi d sqrt(1/lambda^2 - |nu|^2)) for |nu| < 1/lambda, else 0,
 *     applied with d = -z_i (the viewer sits at +z);
 *   - the field sample n (row n_y, column n_x) sits at x = ((n_x - nx/2) px, (n_y - ny/2) py),
 *     so the SLM centre is pixel (nx/2, ny/2);
 *   - u_c[n] = 1/(nx ny px py) * sum_m U_c(nu_m) exp(+j 2 pi nu_m . x_n): a z = 0 Gaussian
 *     with amplitude a and opacity o peaks at a*o.
 *
 * Results are deterministic: every reduction (partial spectra of a frequency tile, the
 * per-Gaussian gradient sums, the loss) runs in a fixed order independent of scheduling,
 * so the same inputs on the same device give bitwise the same outputs, batched or not.
 * There is no non-deterministic mode.
 *
 * Every pointer is a device pointer unless its comment says "host".  The caller owns
 * every input, output and workspace buffer; the context owns only per-shape plans
 * (tile order, twiddle tables, DFT matrices), the tuning cache and a small statistics
 * buffer.  All work is enqueued on the caller's stream (a hipStream_t passed as void*);
 * no call synchronises the device except gws_get_stats, gws_autotune and gws_create.
 * One context must not be used from two host threads at once.
 */
#ifndef GWS_H
#define GWS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GWS_ABI_VERSION 4
#define GWS_MAX_LAMBDA 4

/* Return codes.  Launch-time validation returns the code at once and leaves the
 * outputs untouched; an asynchronous device fault surfaces at a later call or at the
 * caller's synchronisation, and gws_last_error() holds its text. */
typedef enum gws_status {
    GWS_OK = 0,
    GWS_ERR_INVALID_ARG = -1, /* null pointer, non-positive size, bad enum value */
    GWS_ERR_SHAPE = -2,       /* grid not supported: odd, < 16, > 8192, or a prime factor > 5 */
    GWS_ERR_UNSUPPORTED = -3, /* valid request this build does not implement (see gws_blend) */
    GWS_ERR_WORKSPACE = -4,   /* workspace null, misaligned (256 B) or smaller than required */
    GWS_ERR_NO_DEVICE = -5,   /* no HIP device, or the device is not gfx950 */
    GWS_ERR_HIP = -6,         /* a HIP runtime call failed; see gws_last_error */
    GWS_ERR_OOM = -7,         /* the context could not allocate a per-shape plan */
    GWS_STATUS_MAX_ENUM = 0x7fffffff /* not a status: makes the enum a full 32-bit int, so any
                                        int a caller passes (e.g. to gws_status_string) is a
                                        valid value of the type */
} gws_status;

/* Blending model.  OIT is Eq. 12 (transmittance taken as 1).  EXACT is alpha wave
 * blending with a spatial transmittance map (Eq. 5-6, supplement Alg. 2): Gaussians front to
 * back (descending depth, ties by index); each splats its own wavefront e^{j phi} g(x)
 * (profile truncated below eps_support of its peak, and at most nx/2 - 1, ny/2 - 1 pixels from
 * its centre: the nearest periodic image only; gws_stats.n_window_clamped counts the
 * Gaussians cut there) masked by the map, propagated by H(nu, -z) and scaled by a_c o;
 * alpha = o g in FP32, dropped unless above 1/255 (at pixels within FP32 rounding of the
 * threshold either decision can be taken), then updates the map.  EXACT is supported by
 * gws_forward, gws_backward (the map recomputed from per-batch checkpoints, never divided
 * by 1 - alpha), the batched calls (scene after scene) and the workspace queries;
 * gws_autotune returns GWS_ERR_UNSUPPORTED for it (it has no tiling). */
typedef enum gws_blend { GWS_BLEND_OIT = 0, GWS_BLEND_EXACT = 1 } gws_blend;

/* Inverse transform: mixed-radix FP32 FFT, or the DFT as two dense complex GEMMs on the
 * matrix cores with bf16 hi/lo operand splitting (three products, FP32 accumulation). */
typedef enum gws_xform { GWS_XFORM_FFT_FP32 = 0, GWS_XFORM_DFT_BF16X3 = 1 } gws_xform;

typedef struct gws_problem {
    int32_t nx, ny;            /* hologram columns and rows; even, 16..8192, factors 2,3,5 */
    double pitch_x, pitch_y;   /* SLM pixel pitch in metres, > 0 */
    int32_t n_lambda;          /* number of wavelengths (colour channels), 1..4 */
    double lambdas[GWS_MAX_LAMBDA]; /* wavelengths in metres, > 0 */
    int32_t blend;             /* gws_blend */
    int32_t xform;             /* gws_xform */
    double eps_support;        /* spectral-support cut: terms whose Gaussian envelope is below
                                  eps * (its peak) are skipped; 0 selects 1e-7; must be in
                                  (0, 1e-3].  The relative L2 error it adds is about eps. */
    int32_t phase_mode;        /* 0: every large phase term (carrier z/lambda, ramp, propagation
                                  at the tile centre) reduced exactly per (tile, Gaussian) in
                                  fixed point and FP64, small per-frequency deltas in FP32
                                  (default); 1: the same terms in plain FP32 (precision study
                                  only: loses accuracy for far off-axis, deep Gaussians);
                                  2: same as 0 */
    int32_t tile_config;       /* 0: the autotuned configuration for this shape if gws_autotune
                                  ran, else the default; k in 1..gws_tile_config_count():
                                  forward configuration k, a pair (frequencies per lane of the
                                  accumulation F, tile 32 x 8F; base chunk of candidates per
                                  work item) from {(4,512),(4,1024),(8,1024),(8,512),(2,1024),
                                  (4,2048),(2,512),(2,2048),(8,2048)}; the default is 2 =
                                  (4,1024).  The chunk is capped at n / 16 (at least 128) for
                                  each scene of n Gaussians, so a small scene's crowded tiles
                                  still split into several work items.  The order-invariant
                                  adjoint's geometry is fixed. */
    double ref_nu_x, ref_nu_y; /* transverse frequency (cycles per metre) of the reference plane
                                  wave that illuminates every Gaussian (Sec. 4.1): each
                                  Gaussian's wavefront is multiplied by exp(+j 2 pi nu_r . x), x
                                  from the SLM centre, so its spectrum is evaluated at nu - nu_r
                                  while H keeps the full nu; (0, 0) is on-axis illumination.
                                  Finite, |nu_r| at most half the grid's band along each axis
                                  (|nu_r,x| <= 1 / (2 pitch_x), likewise y); the order-invariant
                                  blend only (GWS_BLEND_EXACT returns GWS_ERR_UNSUPPORTED for a
                                  non-zero nu_r) */
} gws_problem;

/* Gaussians as structure-of-arrays float32 device buffers of length n.  amplitude is
 * [n_lambda][n] (channel-major).  Covariance is the 2x2 matrix [[cov_xx, cov_xy],
 * [cov_xy, cov_yy]] in m^2; mean and depth in metres; phase in radians; opacity is used
 * as given (no sigmoid).  A Gaussian whose covariance is not positive definite or whose
 * values are not finite is skipped and counted in gws_stats.n_culled; forward also skips
 * Gaussians with zero opacity or all-zero amplitude (they add exactly nothing). */
typedef struct gws_gaussians {
    int64_t n;
    const float *mean_x, *mean_y, *depth;
    const float *cov_xx, *cov_xy, *cov_yy;
    const float *opacity, *amplitude, *phase;
} gws_gaussians;

typedef struct gws_output {
    void *field;    /* complex64 [n_lambda][ny][nx], (re, im) interleaved, row-major, x fastest */
    void *spectrum; /* optional (NULL to skip): complex64 [n_lambda][ny][nx] in FFT index order,
                       holding U_c(nu_m) * (-1)^(m_x'+m_y') / (nx ny px py), i.e. exactly the
                       array whose unnormalised inverse DFT is the field */
} gws_output;

/* Gradient outputs, float32, same layout as the inputs; overwritten, never accumulated.
 * depth may be NULL to skip the depth gradient; every other pointer is required. */
typedef struct gws_grads {
    float *mean_x, *mean_y, *depth;
    float *cov_xx, *cov_xy, *cov_yy;
    float *opacity, *amplitude, *phase;
} gws_grads;

typedef struct gws_stats {
    int64_t n_input;          /* Gaussians passed to the last forward/backward */
    int64_t n_culled;         /* skipped (see gws_gaussians) */
    int64_t n_tiles;          /* frequency tiles of the grid */
    int64_t n_items;          /* accumulation work items launched */
    int64_t chunk;            /* candidate Gaussians per work item */
    int64_t n_pairs_evaluated; /* (Gaussian, frequency) pairs evaluated: accepted Gaussians x the
                                  frequencies of each wavefront sub-tile they were tested on;
                                  gws_forward_tilted counts (Gaussian, frequency, wavelength)
                                  triples (its exponent depends on the wavelength) */
    int64_t n_candidates;     /* (tile, Gaussian) pairs tested */
    int32_t tile_config;      /* tiling used */
    int32_t graph_replayed;   /* batched call replayed a captured graph */
    int64_t n_window_clamped; /* GWS_BLEND_EXACT: Gaussians whose eps-window (the profile's
                                 extent above eps_support of its peak) reached past nx/2 - 1 or
                                 ny/2 - 1 pixels from its centre and was cut there, so their
                                 profile is truncated (a standard deviation above about
                                 N / (2 sqrt(2 ln(1/eps))), N/11 at eps = 1e-7); 0 for OIT */
} gws_stats;

typedef struct gws_ctx gws_ctx;

/* ABI version this library was built with (GWS_ABI_VERSION). */
int gws_abi_version(void);

/* Static text for a status code; never NULL. */
const char *gws_status_string(gws_status status);

/* Create a context bound to HIP device `device`.  Returns GWS_ERR_NO_DEVICE when there is
 * no such device or it is not gfx950, GWS_ERR_INVALID_ARG when ctx is NULL.  Allocates a
 * small statistics buffer on the device. */
gws_status gws_create(gws_ctx **ctx, int device);

/* Free the context and every plan it holds.  NULL is accepted. */
gws_status gws_destroy(gws_ctx *ctx);

/* Text of the last error recorded on ctx (empty string if none); ctx may be NULL for the
 * last error of a call that had no context. */
const char *gws_last_error(const gws_ctx *ctx);

/* Validate a problem description without touching the device.  Returns the code the
 * other entry points would return for it. */
gws_status gws_check_problem(const gws_problem *problem);

/* Bytes of workspace gws_forward / gws_backward need for n Gaussians (host-only; ctx may
 * be NULL).  The same workspace serves both calls. */
gws_status gws_workspace_size(const gws_ctx *ctx, const gws_problem *problem, int64_t n, size_t *bytes);

/* Forward: the field (and optionally the spectrum) of n Gaussians, Eq. 12 + inverse DFT.
 * Steps on the stream: per-Gaussian preprocessing and keys, depth-within-support-radius
 * radix sort, binning into frequency tiles, spectrum accumulation, inverse 2D transform.
 * With blend = GWS_BLEND_EXACT (Eq. 5-6): depth sort, then per batch of up to 64 Gaussians
 * the masked wavefronts with the transmittance map, their batched forward FFT and the
 * propagated splat into the spectrum, then the inverse 2D transform.  The workspace for
 * EXACT holds one batch of full-grid complex images, two Gaussians per image (0.53 GB at
 * 1080 x 1920, at most 1 GiB). */
gws_status gws_forward(gws_ctx *ctx, const gws_problem *problem, const gws_gaussians *g,
                       const gws_output *out, void *workspace, size_t workspace_bytes, void *stream);

/* Bytes of the device scratch array gws_forward_noalloc works in (each GPU holds one). */
#define GWS_NOALLOC_SCRATCH_BYTES (256u << 20)

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): gws_forward with the order-invariant blend and the
 * FP32 FFT, working in a scratch array of GWS_NOALLOC_SCRATCH_BYTES that the library holds on
 * each device from gws_create until the process ends, instead of a caller workspace.  It calls
 * no allocating routine: the per-shape plan must already exist, built by an earlier gws_forward
 * on this context with the same grid and tiling (else GWS_ERR_UNSUPPORTED), and a problem whose
 * forward-only workspace exceeds the scratch size is refused with GWS_ERR_WORKSPACE (at
 * 1080 x 1920 x 3 it takes up to about 8800 Gaussians).  Everything it needs zeroed it clears
 * itself on the stream.  The scratch is shared by every context and stream on the device: calls
 * that overlap on one GPU (two streams, or two host threads) race and must be serialised by the
 * caller.  Results are bitwise those of gws_forward. */
gws_status gws_forward_noalloc(gws_ctx *ctx, const gws_problem *problem, const gws_gaussians *g,
                               const gws_output *out, void *stream);

/* ---- Tilted Gaussians (Sec. 4.1, Eq. 8-10; the supplement's translation, rotation and
 * scaling steps) ----
 *
 * A tilted Gaussian is the canonical 2D Gaussian of the plane z_c = 0 placed in hologram space
 * by x = R S x_c + mu: S = diag(scale_u, scale_v, 0), R the rotation of the quaternion (w, x,
 * y, z) (normalised here; any non-zero norm), mu = (mean_x, mean_y, depth).  Its spectrum on
 * the plane z = depth is |det J| G_o(R^T k) e^{-j 2 pi nu . mu_xy} with k = (nu, k_z),
 * det J = k_oz / k_z (taken in magnitude: R and R diag(1, -1, -1) describe the same disk),
 * G_o the scaled canonical spectrum 2 pi s_u s_v exp(-2 pi^2 (s_u^2 k_ox^2 + s_v^2 k_oy^2));
 * it is then propagated by H(nu, -depth), weighted by amplitude_c * opacity * e^{j phase}
 * and summed order-invariantly (Eq. 12).  A rotation about z alone is exactly the in-plane
 * Gaussian with Sigma = R S^2 R^T.  Device float32 arrays of n elements, amplitude
 * [n_lambda][n].  Gaussians with a non-finite value, a scale <= 0, a zero quaternion, zero
 * opacity or all-zero amplitudes are culled and counted in gws_stats.n_culled. */
typedef struct gws_tilted_gaussians {
    int64_t n;
    const float *mean_x, *mean_y, *depth;
    const float *quat_w, *quat_x, *quat_y, *quat_z;
    const float *scale_u, *scale_v;
    const float *opacity, *amplitude, *phase;
} gws_tilted_gaussians;

/* Bytes of workspace gws_forward_tilted and gws_backward_tilted need for n Gaussians
 * (host-only; ctx may be NULL): 112 bytes per Gaussian (record, tile rectangle, slot offset),
 * the spectrum, from 16384 Gaussians up to 8 partial spectra (one per 8192 Gaussians: the
 * Gaussians reaching a tile are split into parts worked on separately and added in part
 * order), and the split-bf16 DFT's planes when problem->xform selects it. */
gws_status gws_workspace_size_tilted(const gws_ctx *ctx, const gws_problem *problem, int64_t n, size_t *bytes);

/* Forward of tilted Gaussians: field (and optionally spectrum) as gws_forward.  Takes the
 * order-invariant blend and on-axis illumination only: blend = GWS_BLEND_EXACT or a non-zero
 * ref_nu returns GWS_ERR_UNSUPPORTED.  eps_support cuts each term where its Gaussian factor
 * is below eps (the Jacobian factor |det J| is not part of the test).  Steps on the stream:
 * records and tile rectangles in input order, spectrum accumulation (one persistent launch;
 * each part of the Gaussians writes every frequency of a tile once, sums in input order, and
 * the parts' spectra are added in part order: bitwise reproducible), inverse 2D transform.
 * No host synchronisation. */
gws_status gws_forward_tilted(gws_ctx *ctx, const gws_problem *problem, const gws_tilted_gaussians *g,
                              const gws_output *out, void *workspace, size_t workspace_bytes, void *stream);

/* Gradient outputs of gws_backward_tilted: float32 device arrays shaped like the inputs
 * (amplitude [n_lambda][n]); overwritten, never accumulated.  All are required. */
typedef struct gws_tilted_grads {
    float *mean_x, *mean_y, *depth;
    float *quat_w, *quat_x, *quat_y, *quat_z;
    float *scale_u, *scale_v;
    float *opacity, *amplitude, *phase;
} gws_tilted_grads;

/* Backward of gws_forward_tilted: given grad_field = dL/dRe(u) + j dL/dIm(u) (complex64
 * [n_lambda][ny][nx]), write dL/d(parameter) for every tilted Gaussian, the quaternion's
 * gradient taken through its normalisation.  The workspace is the one gws_forward_tilted uses
 * (gws_workspace_size_tilted).  Recomputes every term; per (Gaussian, frequency tile of 32 x 32
 * reached by its support rectangle) it stores C + 13 floats of partial sums in a buffer the
 * context owns and grows (hipMalloc when a call needs more; freed by gws_destroy), so it
 * synchronises the stream once to read the slot count.  Culled Gaussians, and Gaussians whose
 * support lies outside the band, get zero gradients.  Bitwise reproducible. */
gws_status gws_backward_tilted(gws_ctx *ctx, const gws_problem *problem, const gws_tilted_gaussians *g,
                               const void *grad_field, const gws_tilted_grads *grads, void *workspace,
                               size_t workspace_bytes, void *stream);

/* Backward: given grad_field = dL/dRe(u) + j dL/dIm(u) (complex64 [n_lambda][ny][nx], the
 * convention torch uses for complex tensors), write dL/d(parameter) for every Gaussian.
 * Recomputes preprocessing, sort and binning (no state is kept from gws_forward) and
 * recomputes every (Gaussian, frequency) term instead of storing it.  With
 * GWS_BLEND_EXACT: a forward sweep checkpoints the transmittance map at every batch start
 * (about 8 MB per 64 Gaussians at 1080 x 1920), then the batches run back to front,
 * recomputing the masked wavefronts, the map within the batch and a back-to-front
 * accumulator instead of storing or dividing them; the 1/255 decision is held fixed (its
 * derivative is taken as zero).  The order-invariant adjoint takes the depth gradient for at
 * most three wavelengths: n_lambda = 4 with grads->depth non-NULL returns GWS_ERR_UNSUPPORTED
 * (pass depth = NULL to skip it; every other gradient is available at four). */
gws_status gws_backward(gws_ctx *ctx, const gws_problem *problem, const gws_gaussians *g,
                        const void *grad_field, const gws_grads *grads,
                        void *workspace, size_t workspace_bytes, void *stream);

/* Several independent scenes sharing one problem: scene s owns Gaussians
 * [offsets[s], offsets[s+1]) of g (offsets is a host array of n_scenes + 1 entries,
 * offsets[0] = 0, non-decreasing, offsets[n_scenes] = g->n).  Fields are written to
 * out->field + s * n_lambda*ny*nx complex64 (spectrum likewise if non-NULL).  All scenes
 * run through one persistent accumulation launch; the whole sequence is captured into a
 * hipGraph on first use for a given (problem, offsets, pointers) and replayed after.  With
 * GWS_BLEND_EXACT the scenes run one after another on the stream, sharing a workspace sized
 * for the largest, without graph capture. */
gws_status gws_workspace_size_batched(const gws_ctx *ctx, const gws_problem *problem, int32_t n_scenes,
                                      const int64_t *offsets, size_t *bytes);
gws_status gws_forward_batched(gws_ctx *ctx, const gws_problem *problem, int32_t n_scenes,
                               const int64_t *offsets, const gws_gaussians *g, const gws_output *out,
                               void *workspace, size_t workspace_bytes, void *stream);
/* grad_field holds n_scenes consecutive fields; grads are per Gaussian of the concatenation. */
gws_status gws_backward_batched(gws_ctx *ctx, const gws_problem *problem, int32_t n_scenes,
                                const int64_t *offsets, const gws_gaussians *g, const void *grad_field,
                                const gws_grads *grads, void *workspace, size_t workspace_bytes,
                                void *stream);

/* Unnormalised 2D DFT of `batch` complex64 arrays [ny][nx] (in and out may alias):
 * direction +1: out[n] = sum_m in[m] exp(+j 2 pi m.n/N); -1: exp(-j 2 pi ...).
 * xform selects the FP32 FFT or the split-bf16 matrix-core DFT.  workspace may be NULL
 * for the FFT; the bf16 DFT needs gws_dft_workspace_size bytes.  nx, ny as for a problem;
 * batch >= 1 with batch * max(nx, ny) < 2^31 (else GWS_ERR_SHAPE). */
gws_status gws_dft_workspace_size(const gws_ctx *ctx, int32_t nx, int32_t ny, int32_t batch,
                                  int32_t xform, size_t *bytes);
gws_status gws_dft2d(gws_ctx *ctx, int32_t nx, int32_t ny, int32_t batch, int32_t direction,
                     int32_t xform, const void *in, void *out, void *workspace, size_t workspace_bytes,
                     void *stream);

/* Number of explicit tilings gws_problem.tile_config may name (1..count). */
int gws_tile_config_count(void);

/* Time every forward configuration (tile_config 1..count: frequencies per lane and base
 * chunk) on the device for this problem with n_hint synthetic Gaussians drawn on the device,
 * keep the fastest in the context for problems of this shape and size class, and if
 * cache_path (host string) is non-NULL merge the choice into that JSON file, which later
 * contexts read at gws_create time if GWS_TUNE_CACHE names it.  Synchronises. */
gws_status gws_autotune(gws_ctx *ctx, const gws_problem *problem, int64_t n_hint, const char *cache_path,
                        void *stream);

/* Copy the statistics of the last forward/backward on ctx to *out (host).  Synchronises
 * the device. */
gws_status gws_get_stats(gws_ctx *ctx, gws_stats *out);

/* Field loss of the training step around the hot path: over n complex64 elements,
 * *loss = sum |u - t|^2 (one double, device) and, if grad is non-NULL,
 * grad = 2 (u - t) (complex64, device; may alias u).  The sum is reduced in a fixed
 * order.  workspace needs gws_l2_workspace_size() bytes (device, 256-byte aligned). */
size_t gws_l2_workspace_size(void);
gws_status gws_l2_loss_grad(gws_ctx *ctx, int64_t n, const void *field, const void *target, void *grad,
                            double *loss, void *workspace, size_t workspace_bytes, void *stream);

/* Stage timing with HIP events on the caller's stream.  While enabled, every library call
 * records an event pair around each of its stages (0 preprocess+sort+records, 1 binning,
 * 2 spectrum accumulation, 3 partial-sum reduction, 4 inverse transform, 5 forward
 * transform, 6 propagation table, 7 adjoint accumulation, 8 gradient chain rule, 9 loss,
 * 10 double-phase coding, 11 focal stack, 12 holographics transform).
 * gws_read_profile synchronises, returns per stage the summed milliseconds and the number
 * of launches since the last read (host arrays of GWS_N_STAGES entries), and clears them. */
#define GWS_N_STAGES 13
gws_status gws_set_profiling(gws_ctx *ctx, int enable);
gws_status gws_read_profile(gws_ctx *ctx, double *ms, int64_t *count);

/* Roofline denominators measured on the context's device (the derived ones come from unit
 * counts and clock).  trans_ops_per_s: v_exp_f32, v_sin_f32 and v_cos_f32 in the spectrum
 * accumulation's 1:3:3 mix, as independent chains at full occupancy; valu_ops_per_s:
 * independent FP32 FMAs (one op each); hbm_bytes_per_s: a 1 GiB device-to-device copy,
 * bytes read plus bytes written.  Best of three launches each, timed with HIP events on
 * `stream`.  Allocates 2 GiB + 64 KiB of device memory for the duration of the call and
 * synchronises; takes a few tens of milliseconds. */
typedef struct gws_peaks {
    double trans_ops_per_s;
    double valu_ops_per_s;
    double hbm_bytes_per_s;
} gws_peaks;
gws_status gws_measure_peaks(gws_ctx *ctx, gws_peaks *out, void *stream);

/* ---- Holographics: world-space Gaussians to hologram-space in-plane Gaussians ---- */

/* Camera and display of the holographics transform (supplement, Holographics pipeline). */
typedef struct gws_view {
    double world_to_view[12]; /* [R | t], 3 x 4 row-major: p = R mu + t; the camera looks along -z */
    double fx, fy;            /* pinhole focal lengths, ray-space units (e.g. pixels); > 0 */
    double cx, cy;            /* principal point, ray-space units */
    double near;              /* Gaussians with view distance -p_z < near are culled; >= 0 */
    double ray_to_holo[6];    /* 2 x 3 row-major: (x_h, y_h) = A (u, v) + b, metres on the SLM */
    double depth_scale;       /* hologram depth z_h = depth_scale * p_z + depth_offset (metres) */
    double depth_offset;
    int32_t sh_degree;        /* 0..3: (sh_degree + 1)^2 opacity coefficients per Gaussian */
    int32_t pad;
} gws_view;

/* World-space Gaussians, float32 rows (device pointers). */
typedef struct gws_world_gaussians {
    int64_t n;
    const float *mean;        /* [n][3] */
    const float *quat;        /* [n][4] rotation quaternion (w, x, y, z); normalised here */
    const float *scale;       /* [n][3] standard deviations along the rotated axes (flat 2D
                                 Gaussians: third scale 0) */
    const float *opacity_sh;  /* [n][(sh_degree + 1)^2] view-dependent opacity coefficients */
} gws_world_gaussians;

/* In-plane hologram-space Gaussians written by gws_holographics (device, float32 [n] each;
 * overwritten).  They are the mean_x .. opacity fields of gws_gaussians; amplitude and phase
 * are not part of the transform and pass through unchanged. */
typedef struct gws_plane_gaussians {
    float *mean_x, *mean_y, *depth, *cov_xx, *cov_xy, *cov_yy, *opacity;
} gws_plane_gaussians;

/* The holographics transform (supplement, Holographics pipeline; Sec. 4 view-dependent
 * opacity), in FP64 per Gaussian: model transform Sigma_w = R_w S_w S_w^T R_w^T; view transform;
 * pinhole projection Pi(p) = (fx p_x / -p_z + cx, fy p_y / -p_z + cy) with the local affine
 * (EWA) approximation Sigma_r = J R Sigma_w R^T J^T, J = dPi/dp; lift with the view depth p_z
 * and zero z-scale; the hologram transform (an in-plane 2 x 2 map with offset and an affine
 * depth map, which keep every Gaussian in-plane); opacity = sum_k o_k Y_k(d) clamped to [0, 1],
 * Y_k the real spherical harmonics (Condon-Shortley phase, k = l^2 + l + m) of the unit
 * direction d from the camera centre -R^T t to the mean.  Gaussians closer than `near` in
 * front of the camera get opacity 0 and a zero covariance (culled by gws_forward).  n = 0
 * does nothing.  GWS_ERR_INVALID_ARG for NULL pointers, fx or fy <= 0, near < 0 or a
 * sh_degree outside 0..3. */
gws_status gws_holographics(gws_ctx *ctx, const gws_view *view, const gws_world_gaussians *in,
                            const gws_plane_gaussians *out, void *stream);

/* ---- Display side: phase-only encoding and focal stacks of a hologram ---- */

/* Double-phase amplitude coding (Sec. 5, phase-only encoding; supplement, display
 * section, read in the standard double-phase form of the works it cites, since the printed
 * pair of phases is garbled).  field: complex64 [n_lambda][ny][nx] (device); phase: float32
 * radians, same shape (device, overwritten).  With r = min(|u| / a_max, 1) (r = 0 when
 * a_max = 0), phase = arg u - arccos r where n_x + n_y is even and arg u + arccos r where it
 * is odd, so that a_max (e^{jP-} + e^{jP+}) / 2 = u at every pixel.  Phases are not
 * wrapped: they lie in (-2 pi, 2 pi].  a_max > 0 is used for every channel; a_max <= 0
 * takes each channel's largest |u|, computed on the device into the workspace
 * (gws_dpac_workspace_size bytes, 256-byte aligned; may be NULL when a_max > 0).
 * nx, ny >= 1 and n_lambda in [1, GWS_MAX_LAMBDA] (GWS_ERR_INVALID_ARG otherwise), and
 * n_lambda * ny <= 65535 (GWS_ERR_SHAPE otherwise). */
size_t gws_dpac_workspace_size(int32_t n_lambda);
gws_status gws_dpac_encode(gws_ctx *ctx, int32_t nx, int32_t ny, int32_t n_lambda, const void *field, float a_max,
                           float *phase, void *workspace, size_t workspace_bytes, void *stream);

/* Focal stack by the angular-spectrum method (Eq. 3-4) on the hologram's periodic grid:
 * plane k holds P(u; d_k) = IDFT(DFT(u) H(nu, d_k)), H = exp(j 2 pi d sqrt(1/lambda^2 -
 * |nu|^2)) inside the propagating band and 0 outside, for every wavelength of the problem
 * (its nx, ny, pitches and lambdas are used; blend and xform are ignored).  A Gaussian whose
 * hologram term carries H(nu, -z) (Eq. 5, 12) is in focus in plane d = z.
 * input: complex64 field [n_lambda][ny][nx], or with GWS_FS_PHASE_INPUT a float32 phase-only
 * pattern P of that shape (u = e^{jP}).  GWS_FS_HALF_BAND keeps only |m'_x| < nx/4 and
 * |m'_y| < ny/4 (signed FFT indices), the Fourier filter of double-phase coding.
 * depths: host array of n_planes distances in metres.  out (device, overwritten): float32
 * intensities |P(u; d_k)|^2 [n_planes][n_lambda][ny][nx], or with GWS_FS_COMPLEX_OUTPUT the
 * complex64 fields.  The phase of each plane is reduced in FP64.  nx <= 4096 (GWS_ERR_SHAPE
 * otherwise); n_planes = 0 does nothing.  workspace: gws_focal_stack_workspace_size bytes. */
#define GWS_FS_PHASE_INPUT 1
#define GWS_FS_HALF_BAND 2
#define GWS_FS_COMPLEX_OUTPUT 4
gws_status gws_focal_stack_workspace_size(const gws_ctx *ctx, const gws_problem *problem, int32_t n_planes,
                                          int32_t flags, size_t *bytes);
gws_status gws_focal_stack(gws_ctx *ctx, const gws_problem *problem, const void *input, int32_t n_planes,
                           const double *depths, int32_t flags, void *out, void *workspace, size_t workspace_bytes,
                           void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GWS_H */
