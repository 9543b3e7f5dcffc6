/*
 * gi.h -- C ABI of an MI355X (gfx950) differentiable renderer of N anisotropic 2-D Gaussians by
 * accumulated summation, the image representation of GaussianImage (arXiv 2403.08551).
 *
 * What is computed (paper Sec. 3.1, Eq. cholesky; Sec. 3.2, Eq. rasterization2 and
 * rasterization4; App. A):
 *   Each Gaussian n is a record of 8 floats (mu_x, mu_y, l1, l2, l3, c0, c1, c2) in pixel units:
 *   mean mu, Cholesky factor L = [[l1, 0], [l2, l3]] of Sigma = L L^T, and weighted colour c'
 *   (unbounded; Sec. 3.2 after Eq. rasterization4).  Pixel (x, y) of an H x W image has centre
 *   p = (x + 0.5, y + 0.5) and value
 *       C(p) = sum_n c'_n exp(-sigma_n(p)),   sigma_n(p) = 1/2 d^T Sigma_n^{-1} d,  d = p - mu_n,
 *   with no depth order and no alpha blending (Sec. 3.2).  The sum runs over the Gaussians whose
 *   3-sigma box touches the 16x16 tile of p: the box half-width is r = ceil(3 sqrt(lambda_max))
 *   pixels, decided exactly in float64, and Gaussian n covers tiles
 *   [floor((mu - r) / 16), floor((mu + r) / 16)] clipped to the image.  A Gaussian with a
 *   non-finite number, |l1| or |l3| < 2^-24, or |l2|, |mu_x|, |mu_y| > 2^24 takes no part.
 *   Gradients follow App. A (with dC/dsigma = -c' exp(-sigma) and dL/dl2 = 2 g2 l1 + 2 g3 l2).
 *
 *   Rotation-scale records (GI_OPT_COVARIANCE = GI_COV_ROTATION_SCALE; Sec. 3.1, Eq. RSSR):
 *   the record is (mu_x, mu_y, s1, s2, theta, c0, c1, c2) with Sigma = (R S)(R S)^T, R the
 *   rotation by theta (radians, counter-clockwise in (x, y)) and S = diag(s1, s2).  Since the
 *   eigenvalues of Sigma are s1^2 and s2^2, the box half-width is the least integer r with
 *   r^2 >= 9 max(s1^2, s2^2) (exact in float64).  Such a Gaussian takes no part when a number
 *   is not finite, |s1| or |s2| < 2^-24, or |theta|, |mu_x|, |mu_y| > 2^24.  Gradients are
 *   with respect to (s1, s2, theta) in slots 2..4; the rest is as above.
 *
 * Conventions for every call:
 *   - Pointers named *_dev are device pointers owned by the caller (for example torch tensor
 *     storage); the library never frees them.  Pointers named *_host are host memory.
 *   - Images are row-major [H][W][3] float32; batches concatenate images in order.
 *   - Parameters are [N][8] float32 rows in the record order above; outputs are overwritten,
 *     never accumulated into.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).  Work is enqueued
 *     on it and the call returns without waiting, except where a call says it synchronises.
 *   - Every argument is checked before anything is enqueued; a bad argument returns
 *     GI_ERR_INVALID_ARG and enqueues nothing.
 *   - A context is used from one host thread at a time; contexts are independent.
 *   - Forward results are bitwise deterministic: the per-tile lists are in ascending Gaussian
 *     order and each tile sums in that order.  Gradients are deterministic too: per (tile,
 *     Gaussian) partial sums are reduced in a fixed order, with no floating-point atomics.
 */
#ifndef GI_H
#define GI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes returned by every int-valued call. */
enum {
    GI_OK = 0,
    GI_ERR_INVALID_ARG = -1,  /* a bad pointer, size or option; nothing was enqueued */
    GI_ERR_CAPACITY = -2,     /* keys exceed the reserved capacity in a non-growing call */
    GI_ERR_HIP = -3,          /* a HIP runtime call failed (gi_last_error has the text) */
    GI_ERR_NONFINITE = -4,    /* a parameter was not finite (reported by gi_query) */
    GI_ERR_UNSUPPORTED = -5,  /* valid request the library does not handle */
    GI_ERR_NO_DEVICE = -6     /* no usable gfx950 device */
};

/* Sticky device flags read by gi_query. */
#define GI_FLAG_KEY_OVERFLOW 1u /* more (tile, Gaussian) keys than capacity: outputs undefined */
#define GI_FLAG_NONFINITE 2u    /* some parameter was NaN or Inf (that Gaussian took no part) */
#define GI_FLAG_SCAN_STALL 4u   /* a one-pass scan block waited past its bound: outputs undefined */
#define GI_FLAG_BAD_CODE 8u     /* a compressed Gaussian had a code or index out of range (it took
                                   no part) */

typedef struct gi_ctx gi_ctx;
typedef struct gi_graph gi_graph;

/* Adam hyper-parameters of the fused update (fit calls).  lr_* are per group: position (mu),
 * covariance slots 2..4 ((l1, l2, l3) or (s1, s2, theta)) and colour (c').  After each update
 * |l1| and |l3| (|s1| and |s2| in the rotation-scale form) are raised to at least l_min
 * (0 disables), keeping Sigma away from singular (the paper adds 0.5 to the diagonal for the
 * same reason, App. C).  Bias correction uses the step number t >= 1. */
typedef struct gi_adam {
    float lr_mu, lr_l, lr_c;
    float beta1, beta2, eps;
    float l_min;
} gi_adam;

/* A batch of B independent images fitted or rendered together (host arrays).  Image b is
 * height[b] x width[b] and owns Gaussians [gauss_off[b], gauss_off[b+1]) of the concatenated
 * parameter array; gauss_off[0] = 0.  Pixels of image b start at pixel sum_{b'<b} H W. */
typedef struct gi_batch {
    int32_t count;
    const int32_t *height_host;
    const int32_t *width_host;
    const int64_t *gauss_off_host;
} gi_batch;

/* Options for gi_set_option. */
enum {
    GI_OPT_SYNC = 1,          /* 1 (default): calls read back the key count (4 bytes, waits on
                                 the stream) and grow the key buffers; 0: use the reserved
                                 capacity, never wait, report overflow through flags */
    GI_OPT_SORT_BITS = 2,     /* radix digit width 1..11, 0 = automatic */
    GI_OPT_FWD_PIXELS = 3,    /* pixels per lane in the forward kernels: 1, 2 or 4; 0 = auto */
    GI_OPT_BINNING = 4,       /* 0 = auto (one pass when the tiles number at most 2048, else
                                 row binning when every image is at most 1024 tiles wide, else
                                 radix), 1 = key duplication + LSD radix sort, 2 = one pass if
                                 possible, else radix, 3 = row binning if possible, else radix */
    GI_OPT_TIMING = 5,        /* 1: bracket each stage of non-captured calls with HIP events on
                                 the call's stream (read with gi_timing); 0 (default): off */
    GI_OPT_COVARIANCE = 6,    /* how params[2..4] describe Sigma (Sec. 3.1): GI_COV_CHOLESKY
                                 (default) or GI_COV_ROTATION_SCALE; read by every later call,
                                 and fixed into a captured step when it is created */
    GI_OPT_TILE_ORDER = 7,    /* order in which the raster workgroups take the tiles: 0 = auto
                                 (tuned, else 3 up to 16384 tiles and 1 above), 1 = tile index,
                                 2 = longest list first (one small sorting kernel after the
                                 binning), 3 = longest list first by the previous fit step's
                                 lists (written by that step's update kernel at no extra launch,
                                 up to 16384 tiles; a call whose tile count differs from the
                                 previous one's sorts once as with 2, and above 16384 tiles that
                                 first order stays).  Never changes a result: each tile's
                                 arithmetic is the same in any order */
    GI_OPT_FIT_WAVES = 8      /* resident waves per SIMD the fused fit kernel is compiled for:
                                 0 = auto (tuned, else 4), 4 (up to 128 VGPRs: the most
                                 registers for scheduling) or 6 (up to 80 VGPRs: more tiles in
                                 flight, which pays when tile lists are short).  Never changes a
                                 result: the two builds execute the same arithmetic */
};

/* Values of GI_OPT_COVARIANCE. */
enum {
    GI_COV_CHOLESKY = 0,        /* (l1, l2, l3): Sigma = L L^T, L = [[l1, 0], [l2, l3]] */
    GI_COV_ROTATION_SCALE = 1   /* (s1, s2, theta): Sigma = R(theta) diag(s1^2, s2^2) R^T */
};

/* Stages timed when GI_OPT_TIMING is on. */
enum {
    GI_STAGE_BINNING = 0,     /* projection through the gather into tile order */
    GI_STAGE_RASTER_FWD = 1,  /* forward kernel of gi_render */
    GI_STAGE_RASTER_BWD = 2,  /* adjoint kernel of gi_grad */
    GI_STAGE_RASTER_FIT = 3,  /* fused forward + loss gradient + adjoint of the fit calls */
    GI_STAGE_UPDATE = 4,      /* per-Gaussian gradient reduction (and Adam) */
    GI_STAGE_COUNT = 5
};

/* ---- context ------------------------------------------------------------------------------ */

/* Create a context on HIP device `device`.  Allocates a small fixed workspace.  Returns
 * GI_ERR_NO_DEVICE when the device is missing or not gfx950. */
int gi_create(gi_ctx **out, int device);
/* Release the context and its workspace (waits for its work to finish).  NULL is accepted. */
int gi_destroy(gi_ctx *ctx);
/* Set an option (GI_OPT_*).  Host only. */
int gi_set_option(gi_ctx *ctx, int option, int64_t value);
/* Grow the workspace to hold n_gauss Gaussians, n_tiles tiles and key_capacity (tile,
 * Gaussian) keys.  Host call that allocates; never call it while a graph is being captured. */
int gi_reserve(gi_ctx *ctx, int64_t n_gauss, int64_t n_tiles, int64_t key_capacity);
/* Wait for the context's work, then report the key count of the last binning and the sticky
 * flags (GI_FLAG_*); clear = 1 resets the flags. */
int gi_query(gi_ctx *ctx, int64_t *last_keys, uint32_t *flags, int clear);
/* Read an option (GI_OPT_*); for the tunable options 0 means "automatic". */
int gi_get_option(gi_ctx *ctx, int option, int64_t *value);

/* A schedule of the tunable knobs (0 = the knob's automatic rule): binning path (GI_OPT_BINNING
 * values 1..3), forward pixels per lane (1, 2, 4), radix digit width (radix path only), tile
 * order (GI_OPT_TILE_ORDER values 1, 2, 3), fit kernel waves per SIMD (GI_OPT_FIT_WAVES values
 * 4, 6); ms_per_step is the fit step time it was chosen with. */
typedef struct gi_schedule {
    int32_t binning;
    int32_t fwd_pixels;
    int32_t sort_bits;
    int32_t tile_order;
    int32_t fit_waves;
    float ms_per_step;
} gi_schedule;

/* Autotuner: time fit steps of this workload (batch == NULL: the single image n x height x
 * width; else the batch) under the tunable knobs, one knob at a time in this order, each
 * starting from the best of the knobs before it: the binning path (one pass when the tiles
 * number at most 2048, row binning when the images allow it, radix always), the radix digit
 * width (automatic, 4, 6, 8, 11; radix path only), forward pixels per lane (1, 2, 4), the
 * tile order (index, longest list first) and the fit kernel's waves per SIMD (4, 6).  Runs on scratch copies of the parameters (the
 * caller's buffers are read, never written) with zero learning rates, so every timed step does
 * the same work: one untimed step, then `reps` timed steps per trial.  After three untimed
 * trials of the default schedule (clocks and caches warm up), each candidate is timed in turn
 * with the best schedule so far (candidate, best, candidate, best; the faster trial of each
 * counts) and replaces it only when faster by more than 1.5%.  The fastest schedule is kept in the context for the workload's size class (covariance form, Gaussian count and
 * pixel count, each rounded to a power of sqrt(2)) and used by later calls whose options are
 * automatic; every schedule gives the same results bit for bit.  Allocates scratch memory and
 * synchronises; never call it during graph capture.  *chosen (may be NULL) receives it. */
int gi_autotune(gi_ctx *ctx, const float *params_dev, const float *target_dev, int64_t n,
                int32_t height, int32_t width, const gi_batch *batch, int32_t reps,
                void *stream, gi_schedule *chosen);

/* Write the context's tuned schedules to a text file (one JSON object per line, with the
 * device's architecture name), replacing it; GI_ERR_INVALID_ARG if it cannot be written. */
int gi_autotune_save(gi_ctx *ctx, const char *path);
/* Read schedules written by gi_autotune_save for this device's architecture into the context
 * (entries for other architectures are skipped; an entry replaces the context's schedule of
 * its size class).  *loaded (may be NULL) receives the number of entries taken.
 * GI_ERR_INVALID_ARG if the file cannot be read or a line for this architecture is malformed. */
int gi_autotune_load(gi_ctx *ctx, const char *path, int32_t *loaded);

/* Wait for the timed events, then report the summed milliseconds and the number of timed
 * launches of `stage` (GI_STAGE_*) since the last reset; reset = 1 clears the totals. */
int gi_timing(gi_ctx *ctx, int stage, double *total_ms, int64_t *launches, int reset);
/* Static text for a status code. */
const char *gi_status_string(int status);
/* Text of the last HIP error seen by this context ("" if none). */
const char *gi_last_error(gi_ctx *ctx);

/* ---- single image (Sec. 3.2 forward, App. A backward) -------------------------------------- */

/* render(params, H, W) -> image: Eq. rasterization4 over the tile support.
 * params_dev [N][8], image_dev [H][W][3].  N >= 0 (N = 0 gives a zero image), 1 <= H, W <= 32768. */
int gi_render(gi_ctx *ctx, const float *params_dev, int64_t n, int32_t height, int32_t width,
              float *image_dev, void *stream);

/* grad(params, dL/dimage) -> dparams (App. A): dparams_dev [N][8] in record order,
 * dl_dimage_dev [H][W][3]. */
int gi_grad(gi_ctx *ctx, const float *params_dev, int64_t n, int32_t height, int32_t width,
            const float *dl_dimage_dev, float *dparams_dev, void *stream);

/* One fit step (Sec. 3.4, L2 loss): render, loss = mean over H*W*3 of (C - target)^2,
 * dL/dC = 2 (C - target) / (3 H W), gradients, then the Adam update of params_dev in place with
 * moments m_dev, v_dev ([N][8], caller-initialised, usually zeros).  step_dev points to one
 * int32 on the device holding the step number t >= 1, used for bias correction and then
 * incremented, so that replays of a captured step advance it.  image_out_dev ([H][W][3]) and
 * loss_out_dev (one float) receive the render and loss before the update; either may be NULL.
 * If the key overflow flag is set the update is skipped (parameters unchanged). */
int gi_fit_step(gi_ctx *ctx, float *params_dev, float *m_dev, float *v_dev,
                const float *target_dev, int64_t n, int32_t height, int32_t width,
                const gi_adam *hp, int32_t *step_dev, float *image_out_dev, float *loss_out_dev,
                void *stream);

/* ---- batched: B images, one launch per stage ---------------------------------------------- */

/* Same as gi_render for every image of the batch; images_dev is the concatenation. */
int gi_render_batched(gi_ctx *ctx, const float *params_dev, const gi_batch *batch,
                      float *images_dev, void *stream);
/* Same as gi_grad for every image; dl_dimages_dev and dparams_dev are concatenations. */
int gi_grad_batched(gi_ctx *ctx, const float *params_dev, const gi_batch *batch,
                    const float *dl_dimages_dev, float *dparams_dev, void *stream);
/* Same as gi_fit_step for every image (each image's loss is its own mean);
 * loss_out_dev receives B floats (may be NULL). */
int gi_fit_step_batched(gi_ctx *ctx, float *params_dev, float *m_dev, float *v_dev,
                        const float *targets_dev, const gi_batch *batch, const gi_adam *hp,
                        int32_t *step_dev, float *images_out_dev, float *loss_out_dev,
                        void *stream);

/* ---- opacity renderings (Sec. 3.2, the ablation rows of Table 3) --------------------------- */

/* Values of `blend`. */
enum {
    GI_BLEND_SUM = 1,    /* C = sum_n c_n o_n exp(-sigma_n): summation with a separate opacity
                            (Eq. rasterization3) */
    GI_BLEND_ALPHA = 2   /* C = sum_n c_n alpha_n T_n, T_n = prod_{m<n} (1 - alpha_m),
                            alpha_n = min(o_n exp(-sigma_n), 0.99): alpha blending
                            (Eq. rasterization1, rasterization2) in ascending Gaussian order
                            within each tile (no depth exists); the clamp keeps 1 - alpha >= 0.01.
                            No alpha threshold and no early stop. */
};

/* Render with colours c (params slots 5..7, not merged with the opacity) and opacities
 * opacity_dev [N] (float32).  Support, records and covariance form as in gi_render.  A
 * non-finite opacity makes its Gaussian take no part (GI_FLAG_NONFINITE). */
int gi_render_opacity(gi_ctx *ctx, const float *params_dev, const float *opacity_dev, int64_t n,
                      int32_t height, int32_t width, int32_t blend, float *image_dev,
                      void *stream);
/* Gradients of an opacity rendering: dparams_dev [N][8] (slots 5..7 = dL/dc) and
 * dopacity_dev [N].  Where alpha is clamped it depends on neither o nor sigma. */
int gi_grad_opacity(gi_ctx *ctx, const float *params_dev, const float *opacity_dev, int64_t n,
                    int32_t height, int32_t width, int32_t blend, const float *dl_dimage_dev,
                    float *dparams_dev, float *dopacity_dev, void *stream);

/* One fit step of an opacity rendering (as gi_fit_step): loss, gradients, then Adam on params
 * (moments m_dev, v_dev [N][8]) and on the opacities (moments m_opacity_dev, v_opacity_dev [N],
 * learning rate lr_c, no floor). */
int gi_fit_step_opacity(gi_ctx *ctx, float *params_dev, float *opacity_dev, float *m_dev,
                        float *v_dev, float *m_opacity_dev, float *v_opacity_dev,
                        const float *target_dev, int64_t n, int32_t height, int32_t width,
                        int32_t blend, const gi_adam *hp, int32_t *step_dev,
                        float *image_out_dev, float *loss_out_dev, void *stream);

/* ---- the paper's fitting recipe (Sec. 4.1, App. C) ---------------------------------------- */

/* Adan hyper-parameters (Xie et al. 2022, as used in Sec. 4.1): decay rates beta1..beta3 of the
 * gradient, gradient-difference and squared-Nesterov-gradient moments (published defaults 0.98,
 * 0.92, 0.99), learning rate lr (1e-3 in the paper) halved every halve_every steps (20000;
 * 0 = constant), decoupled weight decay. */
typedef struct gi_adan {
    float lr, beta1, beta2, beta3, eps, weight_decay;
    int32_t halve_every;
} gi_adan;

/* One fit step on raw records (App. C): the renderer sees mu = extent (tanh(rho) + 1) / 2 per
 * axis, l1 + 0.5 and l3 + 0.5 (s1 + 0.5 and s2 + 0.5 in the rotation-scale form), the rest as
 * stored; L2 loss and gradients as gi_fit_step, chained to the raw records; then Adan:
 *   m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) d,  n = b3 n + (1 - b3) (g + b2 d)^2,
 *   raw = (raw - lr_k (m / (1 - b1^k) + b2 v / (1 - b2^k)) / (sqrt(n / (1 - b3^k)) + eps))
 *         / (1 + lr_k wd),
 * with d = g - (previous gradient) (0 on step 1) and k = *step_dev (then incremented).
 * state_dev holds m, v, n and the previous gradient, each [N][8] float32, one after another
 * (caller-initialised, usually zeros). */
int gi_fit_step_recipe(gi_ctx *ctx, float *raw_dev, float *state_dev, const float *target_dev,
                       int64_t n, int32_t height, int32_t width, const gi_adan *hp,
                       int32_t *step_dev, float *image_out_dev, float *loss_out_dev,
                       void *stream);
/* Effective records [N][8] of raw recipe records (for gi_render and the other calls). */
int gi_recipe_params(gi_ctx *ctx, const float *raw_dev, int64_t n, int32_t height, int32_t width,
                     float *params_dev, void *stream);

/* ---- quantisation-aware fine-tuning (Sec. 3.3, Sec. 4.1) ------------------------------------ */

/* The quantiser being fine-tuned, on the device (caller owned, float32):
 *   quant_dev   [6 + 3 M B]: gamma[3], beta[3] of the b-bit covariance codes (LSQ+), then the
 *               residual-VQ codebooks [M][B][3]
 *   quant_m_dev, quant_v_dev [6]: Adam moments of gamma and beta (caller-initialised, zeros)
 *   ema_dev     [M][B][4]: each codebook entry's running count and running residual sum (3)
 *               of the moving-average update (set by gi_qat_init; not read by gi_qat_encode)
 * 1 <= bits <= 8, 1 <= stages <= 8, 1 <= codebook_size <= 64, stages * codebook_size <= 64;
 * 0 <= decay <= 1.  lambda weights the commitment loss in the reported loss; lr_q is the Adam
 * rate of gamma and beta; decay is the codebooks' moving-average decay (Sec. 3.4). */
typedef struct gi_qat {
    float *quant_dev;
    float *quant_m_dev, *quant_v_dev;
    int32_t bits, stages, codebook_size;
    float lambda, lr_q;
    float *ema_dev;
    float decay;
} gi_qat;

/* Initialise quant_dev and ema_dev from float records params_dev [N][8] (N >= 1): beta_i = min
 * of slot i, gamma_i = the least float32 >= (max - min) / (2^b - 1); codebooks by kmeans_iters
 * Lloyd iterations per stage on the residual colours (float64), seeded with the points
 * floor(j N / B), an emptied centroid staying put; each entry's running count = the number of
 * residuals nearest its final centroid, running sum = count x the float32 entry.  Allocates
 * scratch on first use. */
int gi_qat_init(gi_ctx *ctx, const float *params_dev, int64_t n, const gi_qat *q,
                int32_t kmeans_iters, void *stream);
/* One fine-tuning step (as gi_fit_step, on float records; Sec. 3.3 and Sec. 3.4): render the
 * fake-quantised records (binary16 positions; covariance slot i as code * gamma_i + beta_i,
 * code = round-half-even(clamp((l - beta_i) / gamma_i, 0, 2^b - 1)); colours by greedy residual
 * VQ, nearest entry by squared distance, lowest index on ties; all in float64, rounded once);
 * reported loss = mean (C - target)^2 + lambda L_c, L_c = 1/(N B) sum over stages and Gaussians
 * of |C^m[i^m] - r^{m-1}|^2 (r the residual before stage m); straight-through gradients to the
 * records (covariance slots only inside the code range) and LSQ+ gradients to gamma and beta,
 * each taking an Adam step (records with hp, gamma and beta with lr_q and hp's moments); the
 * codebooks by the moving average: per stage m and entry j, with n_j the Gaussians that chose
 * it and s_j the sum of their residuals r^{m-1}, count <- decay count + (1 - decay) n_j,
 * sum <- decay sum + (1 - decay) s_j, entry = sum / count (kept while the count is 0); float64
 * arithmetic, float32 state.  A step whose keys overflow updates nothing (flag raised). */
int gi_fit_step_qat(gi_ctx *ctx, float *params_dev, float *m_dev, float *v_dev,
                    const float *target_dev, int64_t n, int32_t height, int32_t width,
                    const gi_adam *hp, const gi_qat *q, int32_t *step_dev, float *image_out_dev,
                    float *loss_out_dev, void *stream);
/* Encode float records with the quantiser into the codec layout of gi_codec: mu_dev [N][2]
 * binary16 bits (4-byte aligned), codes_dev [N][3], index_dev [N][M]; gi_render_codec of the
 * result with this quantiser's gamma, beta and codebooks renders what the fine-tuning rendered. */
int gi_qat_encode(gi_ctx *ctx, const float *params_dev, int64_t n, const gi_qat *q,
                  uint16_t *mu_dev, uint8_t *codes_dev, uint8_t *index_dev, void *stream);

/* ---- codec decode (Sec. 3.3) ------------------------------------------------------------- */

/* A compressed Gaussian set (Sec. 3.3, attribute quantisation).  Device arrays, caller owned:
 *   mu_dev        [N][2] uint16   IEEE binary16 bit patterns of (mu_x, mu_y) (16-bit positions);
 *                                 the array must be 4-byte aligned
 *   codes_dev     [N][3] uint8    b-bit codes of params[2..4] (LSQ+ with a scale gamma[i] and an
 *                                 offset beta[i] shared by all Gaussians): value = code * gamma
 *                                 + beta
 *   index_dev     [N][M] uint8    residual vector quantisation indices, stage 0 first
 *   codebook_dev  [M][B][3] float stage codebooks; the colour is the sum over stages of
 *                                 codebook[m][index[m]]
 * gamma and beta are host values.  Dequantisation and the colour sum are formed in float64
 * (exact products; sums in stage order) and rounded once to float32.  1 <= bits <= 8,
 * 1 <= stages <= 8, 1 <= codebook_size <= 256.  A Gaussian with a code above 2^bits - 1 or an
 * index >= codebook_size takes no part and raises GI_FLAG_BAD_CODE.  Slots 2..4 are read in
 * the context's GI_OPT_COVARIANCE form. */
typedef struct gi_codec {
    const uint16_t *mu_dev;
    const uint8_t *codes_dev;
    const uint8_t *index_dev;
    const float *codebook_dev;
    float gamma[3], beta[3];
    int32_t bits, stages, codebook_size;
} gi_codec;

/* Decode a compressed set into float records params_dev [N][8] (16-byte aligned); a Gaussian
 * with an invalid code or index decodes to NaN in every slot. */
int gi_codec_decode(gi_ctx *ctx, const gi_codec *codec, int64_t n, float *params_dev,
                    void *stream);
/* Decode and render (the paper's decoder, Table 2): as gi_render of the decoded records, with
 * the dequantisation fused into the projection so that no [N][8] intermediate is written. */
int gi_render_codec(gi_ctx *ctx, const gi_codec *codec, int64_t n, int32_t height,
                    int32_t width, float *image_dev, void *stream);

/* ---- captured fit steps ------------------------------------------------------------------- */

/* Capture one fit step (batch == NULL: the single image n x height x width; else the batch)
 * into a HIP graph.  The graph owns a private workspace (a context created on ctx's device with
 * ctx's options and autotuned settings), sized by one synchronous binning pass of the current
 * parameters with a 1.25x margin on the key count, so later calls on ctx never move memory the
 * graph uses.  Its kernels never wait on the host: if the key count outgrows the capacity the
 * overflow flag is set and the update skipped (read it with gi_fit_graph_query, then re-create
 * the graph).  The caller's pointers are baked into the graph and must stay valid. */
int gi_fit_graph_create(gi_ctx *ctx, float *params_dev, float *m_dev, float *v_dev,
                        const float *target_dev, int64_t n, int32_t height, int32_t width,
                        const gi_batch *batch, const gi_adam *hp, int32_t *step_dev,
                        float *image_out_dev, float *loss_out_dev, void *stream,
                        gi_graph **out);
/* The same for one step of the paper's fitting recipe (gi_fit_step_recipe: raw records, Adan;
 * Sec. 4.1, App. C) and one quantisation-aware fine-tuning step (gi_fit_step_qat; Sec. 3.3) on a
 * single image; the sizing pass bins the records as those steps project them (the recipe's
 * parametrisation, the fake-quantised records).  The quantiser's buffers in q are baked in. */
int gi_fit_graph_create_recipe(gi_ctx *ctx, float *raw_dev, float *state_dev,
                               const float *target_dev, int64_t n, int32_t height, int32_t width,
                               const gi_adan *hp, int32_t *step_dev, float *image_out_dev,
                               float *loss_out_dev, void *stream, gi_graph **out);
int gi_fit_graph_create_qat(gi_ctx *ctx, float *params_dev, float *m_dev, float *v_dev,
                            const float *target_dev, int64_t n, int32_t height, int32_t width,
                            const gi_adam *hp, const gi_qat *q, int32_t *step_dev,
                            float *image_out_dev, float *loss_out_dev, void *stream,
                            gi_graph **out);
/* Replay the captured step `steps` times on `stream`.  Runs of 16 steps go out as one launch of
 * a graph that holds the step 16 times (a graph launch leaves the device idle for a few
 * microseconds at its boundary); the work done is the same. */
int gi_fit_graph_launch(gi_graph *graph, int32_t steps, void *stream);
/* gi_query on the graph's private workspace (waits for the device). */
int gi_fit_graph_query(gi_graph *graph, int64_t *last_keys, uint32_t *flags, int clear);
/* Wait for the device, then release the graph and its workspace. */
int gi_fit_graph_destroy(gi_graph *graph);

/* ---- render without allocation --------------------------------------------------------------- */

/* Limits of gi_render_noalloc: the bytes of its static device array (held by every device the
 * library runs on, from the library's first use there until the process ends), and the largest
 * Gaussian and tile counts it accepts. */
#define GI_NOALLOC_SCRATCH_BYTES (64ll << 20)
#define GI_NOALLOC_MAX_GAUSSIANS (1ll << 18)
#define GI_NOALLOC_MAX_TILES 2048ll

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): gi_render without a context and without any
 * allocation.  It renders params_dev [N][8] (Cholesky records, as gi_render) into image_dev
 * [H][W][3] on the current HIP device with the same kernels as gi_render's one-pass binning and
 * gives the same bits.  Every intermediate buffer lives in one static device array of
 * GI_NOALLOC_SCRATCH_BYTES per device; the call allocates nothing, never waits and enqueues only
 * kernels (no memset or copy nodes), so it can be captured.
 * Limits: N <= GI_NOALLOC_MAX_GAUSSIANS and ceil(H/16) ceil(W/16) <= GI_NOALLOC_MAX_TILES, else
 * GI_ERR_CAPACITY and nothing is enqueued; (tile, Gaussian) keys beyond what the array holds
 * after the per-Gaussian buffers (about 1.0 million at the largest N, 1.8 million at
 * N = 70 000)
 * raise GI_FLAG_KEY_OVERFLOW and leave the image undefined.
 * flags_dev (one uint32 on the device, may be NULL) receives the call's GI_FLAG_* bits when the
 * call's work has run.  GI_ERR_NO_DEVICE when the current device is not gfx950.
 * All calls on one device share its array: calls whose work overlaps in time on one device (on
 * different streams, or from different host threads without ordering) race and give undefined
 * results; calls ordered on one stream are safe. */
int gi_render_noalloc(const float *params_dev, int64_t n, int32_t height, int32_t width,
                      float *image_dev, uint32_t *flags_dev, void *stream);

/* ---- the binning stages, for inspection and testing ---------------------------------------- */

/* Run projection, key duplication, the stable radix sort and tile-range extraction (the
 * binning stages; Sec. 3.2 drops the depth key, so the sort key is the tile id alone), then copy out:
 * rects_dev [N][4] int32 (tx0, ty0, tx1, ty1; (0, 0, -1, -1) when the Gaussian covers nothing),
 * counts_dev [N] uint32, offsets_dev [N] uint32 (exclusive prefix sum of counts),
 * ranges_dev [T][2] uint32 ([start, end) into the sorted list, T = ceil(H/16) ceil(W/16)),
 * ids_dev [ids_capacity] uint32 (Gaussian ids, tile-major, ascending within a tile).
 * *keys_host receives the key count K (synchronises).  Any output pointer may be NULL; if
 * ids_capacity < K the ids are not copied and GI_ERR_CAPACITY is returned. */
int gi_binning(gi_ctx *ctx, const float *params_dev, int64_t n, int32_t height, int32_t width,
               int32_t *rects_dev, uint32_t *counts_dev, uint32_t *offsets_dev,
               uint32_t *ranges_dev, uint32_t *ids_dev, int64_t ids_capacity,
               int64_t *keys_host, void *stream);

/* Exclusive prefix sum of n uint32 values (out may alias in); total_dev (one uint64, may be
 * NULL) receives the sum. */
int gi_scan_u32(gi_ctx *ctx, const uint32_t *in_dev, uint32_t *out_dev, int64_t n,
                uint64_t *total_dev, void *stream);

/* Stable LSD radix sort of n (key, value) uint32 pairs by the low key_bits (1..32) bits of the
 * key.  Outputs must not alias inputs. */
int gi_sort_pairs(gi_ctx *ctx, const uint32_t *keys_in_dev, const uint32_t *vals_in_dev,
                  uint32_t *keys_out_dev, uint32_t *vals_out_dev, int64_t n, int32_t key_bits,
                  void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GI_H */
