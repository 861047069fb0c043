/*
 * r4d.h -- C ABI of the MI355X 4D-rotor Gaussian splatting renderer.
 *
 * One render slices rotor-parameterised 4D Gaussians at a time t into 3D
 * Gaussians (paper Sec. 3.2.2, Eq. center-motion and App. A), projects them with
 * the EWA approximation, shades them with spherical harmonics and alpha-
 * composites them front to back in depth order (paper Sec. 3.1), tile by tile.
 * The backward pass returns the gradient of a scalar loss with respect to every
 * Gaussian parameter, given the loss gradient with respect to the images (the
 * paper back-propagates image-loss gradients through this renderer, Sec. 3 and
 * Fig. "Framework Overview").
 *
 * Conventions shared by every entry point:
 *  - Array arguments are DEVICE pointers owned by the caller, contiguous,
 *    component-major ("SoA"): element (c, i) of an [C][n] array is ptr[c*n + i].
 *  - r4d_view / r4d_settings / r4d_gaussians / r4d_grads structs themselves
 *    live in HOST memory; they are read during the call and not retained.
 *  - Every call is stream-ordered on the caller's hipStream_t (passed as
 *    void*; NULL = the legacy default stream).  All calls on one context must
 *    use one stream, or the caller must order them.
 *  - No call throws or aborts.  Each returns an r4d_status; on failure the
 *    message is available from r4d_last_error(ctx).  Inputs are never
 *    modified.
 *  - A failed call leaves outputs unspecified.
 */
#ifndef R4D_H
#define R4D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  R4D_OK = 0,
  R4D_ERR_INVALID_ARG = -1, /* null pointer, bad size, unsupported setting   */
  R4D_ERR_HIP = -2,         /* a HIP runtime call failed                      */
  R4D_ERR_OOM = -3,         /* device allocation failed                       */
  R4D_ERR_CAPACITY = -4,    /* duplicate count beyond what one render holds   */
  R4D_ERR_STATE = -5        /* saved state does not match the call            */
} r4d_status;

/* The Gaussian set (paper Sec. 3.2.1: a 4D centre, 4D scaling, a rotor of 8
 * coefficients, an opacity and SH coefficients).
 *   means      [4][n]   x, y, z, t
 *   log_scales [4][n]   log s_x, log s_y, log s_z, log s_t   (s = exp(.))
 *   rotors     [8][n]   s, b01, b02, b12, b03, b13, b23, p   (component order of
 *                       the rotor definition in Sec. 3.2.1; unnormalised: the
 *                       library applies the normalisation of App. A)
 *   opacity    [n]      already activated, in (0, 1)
 *   sh         [3k][n]  row = coefficient*3 + channel, k = (sh_degree+1)^2
 * n may be 0 (the image is the background). sh_degree is 0..3. */
typedef struct {
  int32_t n;
  int32_t sh_degree;
  const float *means;
  const float *log_scales;
  const float *rotors;
  const float *opacity;
  const float *sh;
} r4d_gaussians;

/* One render: a pinhole camera and a time.  world_to_cam is the row-major
 * 3x4 [R|t] mapping world points into camera space with OpenCV axes (x right,
 * y down, z forward).  Pixel (x, y) is sampled at (x + 0.5, y + 0.5).
 * Images are planar [3][height][width]. */
typedef struct {
  int32_t width, height;
  float fx, fy, cx, cy;
  float world_to_cam[12];
  float t;
  float bg[3];
} r4d_view;

/* Cut-offs and conventions (values in parentheses are the defaults that
 * r4d_default_settings writes).
 *   tile_size     8, 16 or 32 pixels, or 0: picked by the autotuner, which times
 *                 forward + backward of the call's renders at every tile size and
 *                 tile-sort chunking and keeps the fastest for calls of the same
 *                 shape: device, float type, views' sizes, SH degree, mode and
 *                 Gaussian count within a half octave (16).  Choices persist
 *                 across processes in a text file: the path in the environment
 *                 variable R4D_TUNE_CACHE (empty: none), else
 *                 $XDG_CACHE_HOME/r4d/autotune.txt or ~/.cache/r4d/autotune.txt;
 *                 a call whose shape the file holds is not tuned again.
 *                 The image does not depend on the tile size.
 *   near_plane    camera-space depth at or below which a Gaussian is dropped (0.2)
 *   time_cull     a Gaussian is dropped if lambda (t - mu_t)^2 > time_cull (16;
 *                 the visibility threshold of Sec. 3.2.2)
 *   extent_sigma  a Gaussian reaches a pixel only if its Mahalanobis distance
 *                 q satisfies q <= extent_sigma^2 (3)
 *   alpha_min     contributions with alpha < alpha_min are skipped (1/255)
 *   alpha_max     alpha is clamped to alpha_max (0.99)
 *   T_min         compositing of a pixel stops before the Gaussian that would
 *                 take the transmittance below T_min (1e-4)
 *   dilation      added to the diagonal of every 2D covariance (0.3)
 *   guard_band    x/z and y/z entering the projection Jacobian are clamped to
 *                 guard_band * half image size / focal (1.3)
 *   fwd_pixels_per_thread, bwd_pixels_per_thread
 *                 pixels each lane of the forward / backward rasteriser handles:
 *                 0 = automatic (forward 1; backward 1 for tile 8, 4 for tiles 16
 *                 and 32); otherwise 1 for tile 8 and 1, 2 or 4 for tiles 16 and
 *                 32.  Neither changes the image. */
typedef struct {
  int32_t tile_size;
  float near_plane;
  float time_cull;
  float extent_sigma;
  float alpha_min;
  float alpha_max;
  float T_min;
  float dilation;
  float guard_band;
  int32_t fwd_pixels_per_thread;
  int32_t bwd_pixels_per_thread;
  int32_t mode;        /* R4D_MODE_* (R4D_MODE_PER_VIEW)                          */
  int32_t sort_items;  /* tile sort: 0 = packed 32-bit entries with the emission
                          fused into the first pass (renders of at most 65536
                          tiles and at most 2^24 Gaussians; otherwise as 16);
                          8 or 16 = (tile id, index) pairs sorted by a onesweep
                          radix sort with this many keys per lane.  With
                          tile_size 0 the autotuner picks 0 or 16.  (0)           */
  float front_fraction; /* front lists: with n_vis visible Gaussians in depth
                          order, those at positions from r0 = ceil(front_fraction
                          * n_vis) on are listed only in tiles covered by at most
                          front_keep tile boxes of the Gaussians before r0 (a tile
                          that few front Gaussians reach may not fill up); any
                          other tile's list ends there, and when its pixels
                          outlast that front list the forward collects the
                          rest of the list itself.  The rasteriser sees every list in full up to
                          where its pixels stop (Sec. 3.1 compositing rule), so
                          images and gradients do not depend on this; it saves
                          sorting entries that lie behind saturated pixels.
                          >= 1: whole lists.  Renders whose
                          (tiles_x + 1) * (tiles_y + 1) exceeds 16384 get
                          whole lists.  (0.1)                                    */
  int32_t front_keep;   /* see front_fraction; negative: no tile is kept whole
                          (1024)                                                 */
} r4d_settings;

/* How a call with several views is executed.
 *   R4D_MODE_PER_VIEW  one launch sequence per view; the entry count of each
 *                      view is read back to size its tile lists exactly (one
 *                      stream synchronisation per view).
 *   R4D_MODE_FUSED     all views in one launch sequence (every stage is one
 *                      launch over all views, rasterisation one persistent
 *                      launch over the tiles of all views); one synchronisation
 *                      per call.
 *   R4D_MODE_GRAPH     the fused sequence captured once in a HIP graph per call
 *                      shape (views' sizes, Gaussian count, settings, argument
 *                      pointers) and replayed; no synchronisation.  The tile lists
 *                      have a fixed capacity (1.25x the entry count of the call
 *                      that captured the graph, doubled after an overflow); a
 *                      replay that overflows renders the background only and is
 *                      reported by the backward of its saved state (or
 *                      r4d_saved_check); one without saved state, by the
 *                      context's next render call (or r4d_check_pending).  The
 *                      next forward of that shape grows the capacity and
 *                      captures again.  The saved state of a graph
 *                      forward refers to the graph's buffers: it is valid until the
 *                      next forward of the same shape (backward returns
 *                      R4D_ERR_STATE after that).  The backward is captured too.
 * Images and gradients do not depend on the mode (the last bits of gradients
 * aside, which are summed with atomics). */
enum { R4D_MODE_PER_VIEW = 0, R4D_MODE_FUSED = 1, R4D_MODE_GRAPH = 2 };

/* Gradients, same layouts as r4d_gaussians (means [4][n], log_scales [4][n],
 * rotors [8][n], opacity [n], sh [3k][n]); all DEVICE pointers, overwritten. */
typedef struct {
  float *means;
  float *log_scales;
  float *rotors;
  float *opacity;
  float *sh;
} r4d_grads;

/* Double-precision twins used by finite-difference checks.  The same kernel
 * templates run in float64; depths are still ordered by their float32 value. */
typedef struct {
  int32_t n;
  int32_t sh_degree;
  const double *means;
  const double *log_scales;
  const double *rotors;
  const double *opacity;
  const double *sh;
} r4d_gaussians_f64;

typedef struct {
  double *means;
  double *log_scales;
  double *rotors;
  double *opacity;
  double *sh;
} r4d_grads_f64;

typedef struct r4d_ctx r4d_ctx;
typedef struct r4d_saved r4d_saved;

/* Fills *s with the defaults listed above. */
void r4d_default_settings(r4d_settings *s);

/* Creates a context on HIP device `device`.  The context owns a grow-only
 * device workspace and a cache of saved-state arenas; it is released by
 * r4d_destroy.  Returns R4D_ERR_HIP if the device cannot be selected. */
r4d_status r4d_create(r4d_ctx **ctx, int device);
void r4d_destroy(r4d_ctx *ctx);

/* Forward render of 1 <= n_views <= 64 views of one Gaussian set.
 *   images  DEVICE float, view v at offset sum_{u<v} 3*H_u*W_u, planar [3][H][W]
 *   saved   if non-NULL, receives an opaque handle holding what the backward
 *           pass needs (per view: projected records, sorted tile lists, tile
 *           ranges, final transmittance and last-contributor count per pixel);
 *           release it with r4d_saved_release.  NULL = inference only.
 * Synchronisation: see R4D_MODE_*.
 * Errors: R4D_ERR_INVALID_ARG (null pointers, n < 0, bad degree, bad view size,
 * unsupported tile size / pixels per lane / mode), R4D_ERR_CAPACITY (a view
 * with 2^30 or more tile entries, or a call with 2^32 or more), R4D_ERR_OOM,
 * R4D_ERR_HIP.  A forward's own overflow or sort failure is found on the
 * device after the call returns; it is reported by the backward of its saved
 * state, by r4d_saved_check, or -- for a call without saved state, or a saved
 * state released unchecked -- by the context's next forward or backward call
 * (which then does nothing else and returns R4D_ERR_CAPACITY for an
 * overflow, R4D_ERR_HIP for a sort whose predecessor never published) or by
 * r4d_check_pending. */
r4d_status r4d_render_forward(r4d_ctx *ctx, const r4d_gaussians *g, const r4d_view *views,
                              int n_views, const r4d_settings *settings, float *images,
                              r4d_saved **saved, void *stream);

/* Backward of r4d_render_forward.  g, views, n_views and settings must be
 * those of the forward call that produced `saved` (R4D_ERR_STATE otherwise).
 *   dL_dimages  DEVICE float, same layout as the forward images
 *   out         gradients w.r.t. means, log_scales, rotors, opacity and sh,
 *               summed over the views; overwritten (not accumulated).
 * Gradients through the alpha clamp, the rgb clamp at 0 and every cull or skip
 * are zero.  Per-Gaussian screen-space sums are accumulated with atomics, so
 * the last bits can vary from run to run.
 * After enqueueing its kernels the call waits for the forward to finish on the
 * device (the backward is queued behind it, so the device stays busy) and
 * returns R4D_ERR_CAPACITY if the forward's tile lists overflowed (graph mode)
 * or R4D_ERR_HIP if its sort failed: the gradients in `out` are then invalid.
 * It also returns an unreported failure of an earlier forward of the context
 * (see r4d_render_forward), before enqueueing anything. */
r4d_status r4d_render_backward(r4d_ctx *ctx, const r4d_gaussians *g, const r4d_view *views,
                               int n_views, const r4d_settings *settings,
                               const r4d_saved *saved, const float *dL_dimages, r4d_grads *out,
                               void *stream);

/* Same as the two calls above in float64 (test use: finite differences). */
r4d_status r4d_render_forward_f64(r4d_ctx *ctx, const r4d_gaussians_f64 *g,
                                  const r4d_view *views, int n_views,
                                  const r4d_settings *settings, double *images,
                                  r4d_saved **saved, void *stream);
r4d_status r4d_render_backward_f64(r4d_ctx *ctx, const r4d_gaussians_f64 *g,
                                   const r4d_view *views, int n_views,
                                   const r4d_settings *settings, const r4d_saved *saved,
                                   const double *dL_dimages, r4d_grads_f64 *out, void *stream);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): r4d_render_forward without saved state
 * (inference), allocating nothing.  Every buffer of the call lives in one
 * region of R4D_NOALLOC_BYTES that the library reserves statically on each GPU
 * it runs on (held until the process ends; r4d_create looks up its address).
 * The caller passes the inputs and `images` as for r4d_render_forward.
 *   settings  tile_size must be 8, 16 or 32 (the autotuner allocates);
 *             mode R4D_MODE_FUSED renders all views in one run,
 *             R4D_MODE_PER_VIEW one view after the other, each in the whole
 *             region; R4D_MODE_GRAPH is rejected (R4D_ERR_INVALID_ARG).
 * Images equal those of r4d_render_forward with the same settings.
 * Limits: the per-Gaussian and per-pixel buffers of a run (about 100 bytes per
 * Gaussian and 20 per pixel, per view) and its tile lists (about 30 bytes per
 * tile entry at tile 16) must fit in the region together.  A call whose
 * Gaussians and pixels do not fit returns R4D_ERR_CAPACITY before launching
 * anything; one whose tile entries (known after the preprocess, which the call
 * waits for, like plain mode) do not fit returns R4D_ERR_CAPACITY without
 * rasterising.  Other errors as r4d_render_forward; a sort failure is reported
 * by the context's next call.
 * Every call on one GPU uses that GPU's one region, whatever the context:
 * calls that overlap on one GPU (other streams, other host threads, other
 * contexts) race and give wrong images.  Calls on one stream are ordered. */
#define R4D_NOALLOC_BYTES (256u << 20)
r4d_status r4d_render_forward_noalloc(r4d_ctx *ctx, const r4d_gaussians *g,
                                      const r4d_view *views, int n_views,
                                      const r4d_settings *settings, float *images, void *stream);

/* Speed-field (optical flow) render, Sec. 3.2.2: the sliced mean of a
 * Gaussian moves with speed V / W (V the space-time block of its 4D covariance,
 * W its time variance), so its projected mean moves at
 *   flow = (fx (vx z - x vz) / z^2, fy (vy z - y vz) / z^2)
 * pixels per unit of t, with (x, y, z) the camera-space mean and (vx, vy, vz)
 * = world_to_cam rotation times V / W.  Each pixel receives the flows of the
 * Gaussians blended there, weighted exactly as their colours (alpha times the
 * transmittance in front), over a background of 0.  The colour images are
 * rendered in the same pass, identical to r4d_render_forward's.
 *   flows  DEVICE float, view v at offset sum_{u<v} 2*H_u*W_u, planar [2][H][W]
 *          (x then y component)
 * Other arguments, layout and errors as r4d_render_forward (flows NULL:
 * R4D_ERR_INVALID_ARG).  The saved state also serves r4d_render_backward
 * (colour gradient only). */
r4d_status r4d_render_forward_flow(r4d_ctx *ctx, const r4d_gaussians *g, const r4d_view *views,
                                   int n_views, const r4d_settings *settings, float *images,
                                   float *flows, r4d_saved **saved, void *stream);

/* Backward of r4d_render_forward_flow: gradients of a loss on both the colour
 * images and the flow images.
 *   dL_dflows  DEVICE float, same layout as the forward flows (not NULL)
 * Other arguments and errors as r4d_render_backward; R4D_ERR_STATE if `saved`
 * comes from a forward without flow. */
r4d_status r4d_render_backward_flow(r4d_ctx *ctx, const r4d_gaussians *g, const r4d_view *views,
                                    int n_views, const r4d_settings *settings,
                                    const r4d_saved *saved, const float *dL_dimages,
                                    const float *dL_dflows, r4d_grads *out, void *stream);

/* The two flow calls in float64 (test use: finite differences). */
r4d_status r4d_render_forward_flow_f64(r4d_ctx *ctx, const r4d_gaussians_f64 *g,
                                       const r4d_view *views, int n_views,
                                       const r4d_settings *settings, double *images,
                                       double *flows, r4d_saved **saved, void *stream);
r4d_status r4d_render_backward_flow_f64(r4d_ctx *ctx, const r4d_gaussians_f64 *g,
                                        const r4d_view *views, int n_views,
                                        const r4d_settings *settings, const r4d_saved *saved,
                                        const double *dL_dimages, const double *dL_dflows,
                                        r4d_grads_f64 *out, void *stream);

/* 4D nearest neighbours for the 4D consistency loss (Sec. 3.3, "4D Consistency
 * Loss"): the neighbour set of Gaussian i is its k nearest other Gaussians in
 * 4D, Euclidean distance after dividing x, y, z by spatial_scale and t by
 * temporal_scale.  Computed exactly in float32: coordinates u = x * fl(1 /
 * scale), squared distance ((d0^2 + d1^2) + d2^2) + d3^2 with every operation
 * rounded to float32, ties broken by the smaller index, i itself excluded.
 *   means       DEVICE float [4][n] (the Gaussians' means, component-major;
 *               finite values)
 *   neighbours  DEVICE int32 [n][k], written: row i = the k neighbours of i,
 *               nearest first
 * Requires n >= 2, 1 <= k <= 32, k < n, n * k < 2^31 and positive finite
 * scales (R4D_ERR_INVALID_ARG / R4D_ERR_CAPACITY otherwise).  Temporary
 * buffers come from the context's cache; the call is ordered on `stream`. */
r4d_status r4d_knn4d(r4d_ctx *ctx, const float *means, int32_t n, int32_t k,
                     float spatial_scale, float temporal_scale, int32_t *neighbours,
                     void *stream);

/* The 4D consistency loss (Sec. 3.3, "4D Consistency Loss") and its gradient:
 *   L = (1/n) sum_i || s_i - (1/k) sum_{j in neighbours[i]} s_j ||_1,
 * s_i = V_i / W_i the speed of Gaussian i's slice (Sec. 3.2.2; V the
 * space-time block of Sigma_4, W its time variance), computed from g's rotors
 * and log-scales (the other arrays of g are not read).
 *   neighbours  DEVICE int32 [n][k] (e.g. from r4d_knn4d); entries outside
 *               [0, n) are skipped
 *   loss        DEVICE float scalar receiving L, or NULL
 *   grads       NULL, or gradient arrays of which only rotors [8][n] and
 *               log_scales [4][n] are used: they are ADDED to, += weight *
 *               dL/d(rotors, log_scales).  The neighbour lists are constants
 *               (no gradient reaches the means); |.| has derivative 0 at 0.
 * Requires n >= 2 and 1 <= k < n.  The gradient's neighbour sums are exact
 * (integer atomics): results do not depend on the order of execution. */
r4d_status r4d_consistency4d_loss_grad(r4d_ctx *ctx, const r4d_gaussians *g,
                                       const int32_t *neighbours, int32_t k, float weight,
                                       float *loss, r4d_grads *grads, void *stream);
/* The same in float64 (test use: finite differences). */
r4d_status r4d_consistency4d_loss_grad_f64(r4d_ctx *ctx, const r4d_gaussians_f64 *g,
                                           const int32_t *neighbours, int32_t k, double weight,
                                           double *loss, r4d_grads_f64 *grads, void *stream);

/* ---- optimisation step (Sec. 3.3 losses; the optimiser conventions the paper
 * takes from 3D Gaussian Splatting, Sec. 4 "Implementation Details") ---- */

/* Adam settings.  Learning rates per parameter group; the position (4D mean)
 * rate decays exponentially from lr_means_init at step 0 to lr_means_final at
 * step lr_means_steps (constant after): lr(t) = exp((1 - u) ln init + u ln
 * final), u = min(t / steps, 1).  SH degree-0 coefficients (rows 0..2 of the
 * [3k][n] array) use lr_sh_dc, the higher bands lr_sh_rest.  Update:
 * m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps), t the 1-based step. */
typedef struct {
  float lr_means_init;
  float lr_means_final;
  int32_t lr_means_steps;
  float lr_log_scales;
  float lr_rotors;
  float lr_opacity;
  float lr_sh_dc;
  float lr_sh_rest;
  float beta1;
  float beta2;
  float eps;
} r4d_adam_config;

/* 3D Gaussian Splatting's values: means 1.6e-4 -> 1.6e-6 over 30000 steps
 * (before any scene-extent factor, which the caller applies), log-scales
 * 5e-3, rotors 1e-3, opacity 0.05, SH degree 0 2.5e-3 and higher bands
 * 2.5e-3 / 20, betas 0.9 / 0.999, eps 1e-15. */
void r4d_default_adam_config(r4d_adam_config *c);

/* Optimiser state of n Gaussians (all DEVICE float unless noted):
 *   means..sh      the render's parameter arrays (layouts of r4d_gaussians),
 *                  updated in place
 *   opacity_logit  [n]: the optimiser's opacity parameter l, with
 *                  opacity = 1 / (1 + exp(-l)) kept in sync by every call
 *   adam_m, adam_v [n (17 + 3k)]: the moments, groups back to back in the
 *                  order means, log_scales, rotors, opacity (of the logit),
 *                  sh, each laid out like its parameter; zero initially
 *   step           DEVICE int32: steps taken (0 initially), incremented by
 *                  every r4d_adam_step on the device (so a step can be
 *                  captured in a graph and replayed) */
typedef struct {
  int32_t n;
  int32_t sh_degree;
  float *means;
  float *log_scales;
  float *rotors;
  float *opacity;
  float *sh;
  float *opacity_logit;
  float *adam_m;
  float *adam_v;
  int32_t *step;
} r4d_train_state;

/* Initial optimiser state of a parameter set (the opacity-as-logit
 * convention the paper takes from 3D Gaussian Splatting, Sec. 4): writes
 * opacity_logit[i] = ln(o_i / (1 - o_i)) from state->opacity (o clamped to
 * [1e-7, 1 - 1e-7], evaluated in float64 and rounded to float32), zeroes
 * adam_m and adam_v over all n (17 + 3k) elements and sets *step = 0.  One
 * launch, ordered on `stream`; opacity and the other parameters are read
 * only.  n = 0 only resets the step count. */
r4d_status r4d_train_state_init(r4d_ctx *ctx, const r4d_train_state *state, void *stream);

/* One Adam step of all five groups (one fused launch).  grads: the gradients
 * of r4d_render_backward (plus any regulariser's), the opacity one w.r.t. the
 * activated opacity (the call multiplies by o (1 - o) for the logit). */
r4d_status r4d_adam_step(r4d_ctx *ctx, const r4d_train_state *state, const r4d_grads *grads,
                         const r4d_adam_config *cfg, void *stream);

/* Opacity reset: opacity = min(opacity, cap) (through the logit), and the
 * opacity moments cleared for every Gaussian; 0 < cap < 1. */
r4d_status r4d_opacity_reset(r4d_ctx *ctx, const r4d_train_state *state, float cap, void *stream);

/* Entropy loss (Sec. 3.3 "Entropy Loss"): L = (1/n) sum_i -o_i ln o_i over
 * DEVICE float opacity [n] (values in (0, 1]).  loss: DEVICE float scalar or
 * NULL; grad_opacity: DEVICE float [n] or NULL, += weight * dL/do
 * (= -weight (ln o + 1) / n). */
r4d_status r4d_entropy_loss_grad(r4d_ctx *ctx, const float *opacity, int32_t n, float weight,
                                 float *loss, float *grad_opacity, void *stream);

/* ---- density control (3D Gaussian Splatting's adaptive density control,
 * which the paper applies to its 4D Gaussians, Sec. 4) ---- */

/* r4d_render_backward (or, with dL_dflows non-NULL, r4d_render_backward_flow)
 * that also accumulates the densification statistics: for every render in
 * which Gaussian i is listed in some tile,
 *   grad_accum[i] += || (dL/dmean2d.x * W/2, dL/dmean2d.y * H/2) ||
 * (the projected-mean gradient in normalised device coordinates) and
 * vis_count[i] += 1.  grad_accum: DEVICE float [n]; vis_count: DEVICE int32
 * [n]; both added to (the caller zeroes them when a statistics period starts). */
r4d_status r4d_render_backward_stats(r4d_ctx *ctx, const r4d_gaussians *g, const r4d_view *views,
                                     int n_views, const r4d_settings *settings,
                                     const r4d_saved *saved, const float *dL_dimages,
                                     const float *dL_dflows, r4d_grads *out, float *grad_accum,
                                     int32_t *vis_count, void *stream);

typedef struct {
  float grad_threshold;  /* densify when accum / count >= this (2e-4)         */
  float size_threshold;  /* clone when the largest spatial scale <= this,
                            else split (0.01; 3DGS: 0.01 x scene extent)       */
  float min_opacity;     /* drop Gaussians with opacity below this (0.005)     */
  float max_size;        /* drop Gaussians whose largest spatial scale exceeds
                            this; 0 disables (0)                               */
} r4d_densify_config;
void r4d_default_densify_config(r4d_densify_config *c);

/* Clone, split and prune.  Decisions in float32 on the stored values:
 * selected = count > 0 and accum / count >= grad_threshold; a selected
 * Gaussian whose largest spatial log-scale <= fl(ln size_threshold) is cloned
 * (identical copy, zero moments); a larger one is split into 2 children
 * placed at mu + R diag(s) z_c (mu the 4D mean, R the rotor's 4x4 rotation, s
 * the scales, z_c = normals[:, 2i + c]), log-scales reduced by fl(ln 1.6),
 * everything else copied, zero moments, the parent removed.  Every result is
 * then dropped if its opacity < min_opacity or (max_size > 0 and its largest
 * spatial log-scale > fl(ln max_size)).  Order of the new set: surviving
 * originals (moments kept), then clones, then children (two per parent), each
 * in index order.
 *   in       the current train state (read)
 *   normals  DEVICE float [4][2 n] standard normal draws (the caller's random
 *            numbers)
 *   out      a second train state: out->n is its capacity in Gaussians (every
 *            array sized for it, e.g. 2 n, which always suffices); the new set
 *            is written with row stride *n_out; out->step receives in->step
 *   n_out    HOST: the new Gaussian count
 * Synchronises with `stream` once (to learn the count).  R4D_ERR_CAPACITY with
 * *n_out = the count needed when it exceeds the capacity (nothing written). */
r4d_status r4d_densify(r4d_ctx *ctx, const r4d_train_state *in, const float *grad_accum,
                       const int32_t *vis_count, const float *normals,
                       const r4d_densify_config *cfg, const r4d_train_state *out,
                       int32_t *n_out, void *stream);

/* ---- static 3D Gaussians (the 3D/4D unification of Sec. 3.2.1: a rotor with
 * no temporal part is a quaternion and the Gaussian does not move) ---- */

/* A static set: means [3][n], log_scales [3][n], quats [4][n] as (w, x, y, z)
 * (any norm; normalised inside; |q|^2 < 1e-12 acts as the identity), opacity
 * [n], sh [3k][n]; all DEVICE, component-major like r4d_gaussians. */
typedef struct {
  int32_t n;
  int32_t sh_degree;
  const float *means;
  const float *log_scales;
  const float *quats;
  const float *opacity;
  const float *sh;
} r4d_gaussians3d;
typedef struct {
  float *means;
  float *log_scales;
  float *quats;
  float *opacity;
  float *sh;
} r4d_grads3d;
typedef struct {
  int32_t n;
  int32_t sh_degree;
  const double *means;
  const double *log_scales;
  const double *quats;
  const double *opacity;
  const double *sh;
} r4d_gaussians3d_f64;
typedef struct {
  double *means;
  double *log_scales;
  double *quats;
  double *opacity;
  double *sh;
} r4d_grads3d_f64;

/* Render of a static set: every view at every time sees the same 3D
 * Gaussians, Sigma_3D = R(q) diag(s^2) R(q)^T, no opacity decay and no time
 * cull -- the 4D render of the rotors (w, -z, y, -x, 0, 0, 0, 0) with an
 * unbounded time scale, computed without the rotor, Sigma_4 and the slice.
 * Same binning, sort and rasteriser as r4d_render_forward; arguments, layout,
 * modes and errors as there (views' t is ignored).  The saved state serves
 * only r4d_render_backward_3d (R4D_ERR_STATE otherwise, and vice versa). */
r4d_status r4d_render_forward_3d(r4d_ctx *ctx, const r4d_gaussians3d *g, const r4d_view *views,
                                 int n_views, const r4d_settings *settings, float *images,
                                 r4d_saved **saved, void *stream);
/* Backward of r4d_render_forward_3d: gradients w.r.t. means, log_scales,
 * quats (raw), opacity and sh, overwritten, summed over the views. */
r4d_status r4d_render_backward_3d(r4d_ctx *ctx, const r4d_gaussians3d *g, const r4d_view *views,
                                  int n_views, const r4d_settings *settings,
                                  const r4d_saved *saved, const float *dL_dimages,
                                  r4d_grads3d *out, void *stream);
/* The two static calls in float64 (test use: finite differences). */
r4d_status r4d_render_forward_3d_f64(r4d_ctx *ctx, const r4d_gaussians3d_f64 *g,
                                     const r4d_view *views, int n_views,
                                     const r4d_settings *settings, double *images,
                                     r4d_saved **saved, void *stream);
r4d_status r4d_render_backward_3d_f64(r4d_ctx *ctx, const r4d_gaussians3d_f64 *g,
                                      const r4d_view *views, int n_views,
                                      const r4d_settings *settings, const r4d_saved *saved,
                                      const double *dL_dimages, r4d_grads3d_f64 *out,
                                      void *stream);

/* Returns the saved arena to its context's cache.  NULL is ignored.  A saved
 * handle may outlive its context: r4d_destroy frees its device memory and a
 * later release only frees the handle.  If neither a backward nor
 * r4d_saved_check read the forward's status, the context's next call does. */
void r4d_saved_release(r4d_saved *saved);

/* Gradient of the mean absolute error L = sum |image - target| / count
 * (the L1 term of the paper's loss, Sec. 3.3 "Total Loss"):
 *   dL_dimage[i] = sign(image[i] - target[i]) / count   (0 where equal)
 * image, target, dL_dimage: DEVICE float [count].  loss: DEVICE float scalar
 * or NULL; if given it receives L (accumulated with atomics, so it is
 * overwritten first). */
r4d_status r4d_l1_loss_grad(r4d_ctx *ctx, const float *image, const float *target, int64_t count,
                            float *dL_dimage, float *loss, void *stream);

/* Gradient of L = sum over views v of mean_v |image - target| (each view's
 * mean over its own 3*H*W values), for images laid out as in
 * r4d_render_forward: dL_dimage = sign(image - target) / (3 H_v W_v).  One
 * launch for all views.  loss: DEVICE float scalar or NULL. */
r4d_status r4d_l1_loss_grad_views(r4d_ctx *ctx, const float *images, const float *targets,
                                  const r4d_view *views, int n_views, float *dL_dimages,
                                  float *loss, void *stream);

/* Waits until the forward call that produced `saved` has finished on the
 * device and reports what it could not report when it returned:
 * R4D_ERR_CAPACITY if its tile lists overflowed (graph mode), R4D_ERR_HIP if
 * its sort timed out waiting for a predecessor, R4D_OK otherwise.  Each graph
 * replay keeps its own status words, so this also answers for a saved state
 * whose buffers a later forward has reused. */
r4d_status r4d_saved_check(const r4d_saved *saved);

/* Waits for every forward of the context whose status nobody has read yet
 * (calls without saved state, saved states released unchecked) and reports
 * the first overflow (R4D_ERR_CAPACITY) or sort failure (R4D_ERR_HIP) among
 * them; R4D_OK if none.  Each such forward is reported once, here or by the
 * context's next forward or backward call. */
r4d_status r4d_check_pending(r4d_ctx *ctx);

/* The tile size, tile-sort keys per lane and mode the forward call used (the
 * autotuner's choice when tile_size was 0).  Any pointer may be NULL. */
r4d_status r4d_saved_config(const r4d_saved *saved, int32_t *tile_size, int32_t *sort_items,
                            int32_t *mode);

/* Introspection of saved state (tests and the benchmark).
 * r4d_saved_stats writes, for view v: n_visible (Gaussians with at least one
 * tile), n_dup (tile entries D of the whole lists), tiles_x, tiles_y.  It waits
 * for the forward call to finish. */
r4d_status r4d_saved_stats(const r4d_saved *saved, int view, int64_t *n_visible, int64_t *n_dup,
                           int32_t *tiles_x, int32_t *tiles_y);

/* Front lists of view v (see front_fraction): n_front, the entries emitted and
 * sorted (n_dup with whole lists); n_values, the length of R4D_BUF_VALUES;
 * rest_tiles, the tiles whose forward collected a rest; rest_entries, the
 * rest area those took (each tile's share rounded up to 256).  Any pointer
 * may be NULL.  Waits for the forward call to finish. */
r4d_status r4d_saved_front_stats(const r4d_saved *saved, int view, int64_t *n_front,
                                 int64_t *n_values, int64_t *rest_tiles, int64_t *rest_entries);

/* Copies one saved buffer of view v into dst (DEVICE, at least `bytes`).
 *   R4D_BUF_RECORDS   per Gaussian, 12 floats (or doubles for the f64 path):
 *                     mean2d.x, mean2d.y, conic a, conic b, conic c,
 *                     opacity_t, depth, q_max, r, g, b, (unused) -- record i
 *                     at [12*i]; q = a dx^2 + 2 b dx dy + c dy^2 and q_max =
 *                     min(extent^2, 2 ln(opacity_t / alpha_min)) rounded up,
 *                     the largest q at which the Gaussian is blended.  Only
 *                     records with a depth key other than 0xffffffff are set.
 *   R4D_BUF_RECT      per Gaussian, 4 uint16: tile x0, y0, x1, y1 (x1, y1
 *                     exclusive; all zero when culled), the bounding box of
 *                     the tiles the Gaussian is listed in: in each of its
 *                     rows, the run of tiles holding a pixel centre within one
 *                     pixel of the ellipse q <= q_max (Sec. 3.1 compositing
 *                     rule; every row of the box holds a run)
 *   R4D_BUF_DEPTHKEY  per Gaussian uint32: float32 bit pattern of the depth,
 *                     0xffffffff when culled
 *   R4D_BUF_VALUES    n_values uint32 (r4d_saved_front_stats; D with whole
 *                     lists): Gaussian index of each tile entry, sorted by
 *                     (tile, depth, index); with front lists the front lists,
 *                     then the rest area
 *   R4D_BUF_RANGES    tiles_x*tiles_y pairs of uint32 [start, end) into VALUES
 *                     (of this view): each tile's whole or front list
 *   R4D_BUF_REST      tiles_x*tiles_y pairs of uint32 [start, end) into VALUES:
 *                     the rest the forward collected for a tile's front list
 *                     ([0, 0) for none); front and rest together are the
 *                     list's first entries, up to past the tile's last
 *                     contributor
 *   R4D_BUF_TFINAL    H*W float (double): final transmittance per pixel
 *   R4D_BUF_NCONTRIB  H*W uint32: tile-list entries up to the last contributor
 *   R4D_BUF_NEVAL     H*W uint32: tile-list entries the forward evaluated for the
 *                     pixel (only if timing was enabled for the forward call,
 *                     R4D_ERR_STATE otherwise; never for a flow render)
 *   R4D_BUF_NBLEND    H*W uint32: Gaussians the forward blended into the pixel
 *                     (conditions as R4D_BUF_NEVAL)
 *   R4D_BUF_FLOW      per Gaussian, 2 floats (doubles): its 2D flow, record i
 *                     at [2*i], set where RECORDS is (flow renders only,
 *                     R4D_ERR_STATE otherwise)
 * `bytes` must equal the buffer size (R4D_ERR_INVALID_ARG otherwise).  The
 * call waits for the forward call to finish. */
enum {
  R4D_BUF_RECORDS = 0,
  R4D_BUF_RECT = 1,
  R4D_BUF_DEPTHKEY = 2,
  R4D_BUF_VALUES = 3,
  R4D_BUF_RANGES = 4,
  R4D_BUF_TFINAL = 5,
  R4D_BUF_NCONTRIB = 6,
  R4D_BUF_NEVAL = 7,
  R4D_BUF_FLOW = 8,
  R4D_BUF_NBLEND = 9,
  R4D_BUF_REST = 10
};
r4d_status r4d_saved_copy(const r4d_saved *saved, int view, int buffer, void *dst, size_t bytes,
                          void *stream);

/* Per-stage timing with HIP events recorded on the call's stream around each
 * kernel launch (measurement aid; off by default, adds no synchronisation to
 * the render calls; ignored in graph mode).  Stages: 0 preprocess_fwd, 1 depth_sort, 2 count_scan,
 * 3 emit, 4 tile_sort, 5 tile_ranges, 6 raster_fwd, 7 raster_bwd,
 * 8 preprocess_bwd.  r4d_get_timings synchronises on the recorded events and
 * writes, per stage, the summed milliseconds and the number of launches since
 * the last reset (arrays of R4D_NUM_STAGES entries). */
#define R4D_NUM_STAGES 9
r4d_status r4d_set_timing(r4d_ctx *ctx, int enable);
r4d_status r4d_get_timings(r4d_ctx *ctx, double *ms, int64_t *launches, int reset);
const char *r4d_stage_name(int stage);

/* Human-readable status name; never NULL. */
const char *r4d_status_string(r4d_status s);
/* Last error message recorded on ctx (empty string if none); never NULL. */
const char *r4d_last_error(const r4d_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* R4D_H */
