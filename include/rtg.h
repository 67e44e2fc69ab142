/*
 * rtg.h - C ABI of the MI355X (gfx950) Gaussian-splatting rasterizer used by
 * RT-GuIDE (arXiv 2409.18122) to build its map and to score candidate views.
 *
 * The calls follow the paper's statement of the problem:
 *   - h(x, G) "synthesises a measurement given a pose and a map" (Sec. III,
 *     eq. (1)): rtg_project + rtg_bin_sort + rtg_render;
 *   - the mapping problem argmin_G sum_s L(y_s, h(x_s, G)) (Sec. III eq. (2))
 *     with the L1 part of the loss of eq. (4): rtg_loss + rtg_render_backward;
 *   - choosing the next view by the information proxy of Sec. IV-A eq. (7):
 *     rtg_score_views (one call for many candidate poses).
 * A pose is (R_k, T_k), the camera rotation and position in the world frame
 * (Sec. III, Gaussian Splatting paragraph).
 *
 * Conventions for every entry point:
 *   - Pointers to Gaussian parameters, images, gradients and scores are
 *     DEVICE pointers owned by the caller; the library never frees them.
 *     Camera and settings structs are HOST pointers, read during the call.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the default
 *     stream) and is asynchronous unless a host output is requested; calls
 *     that size internal buffers synchronise `stream` once or twice (noted).
 *   - Errors are returned as rtg_status; rtg_last_error() gives a message
 *     (thread-local). Arguments are validated on the host before any launch.
 *     Non-finite Gaussian geometry and zero quaternions are not errors: such
 *     Gaussians are culled.
 *   - A context is bound to one device and is not thread-safe; use one
 *     context per host thread / stream.
 */
#ifndef RTG_H
#define RTG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rtg_status;
#define RTG_OK 0
#define RTG_ERR_INVALID (-1)     /* bad argument (null pointer, size, tile, NaN camera) */
#define RTG_ERR_HIP (-2)         /* a HIP runtime call failed (message has the code) */
#define RTG_ERR_CAPACITY (-3)    /* a fixed-capacity buffer overflowed (graph replay) */
/* RTG_ERR_UNSUPPORTED is also returned when a frame would hold 2^31 or more
 * records (view-Gaussian pairs) or (tile, Gaussian) pairs: list offsets are
 * 32-bit, and the count scans detect the carry in 64 bits. */
#define RTG_ERR_OOM (-4)         /* device allocation failed */
#define RTG_ERR_UNSUPPORTED (-5) /* request outside what this build supports */

/* Pinhole camera with pose (R_k, T_k) of Sec. III.  R is camera-to-world,
 * row-major (column k = camera axis k in world coordinates), T the camera
 * centre in the world.  Camera axes: x right, y down, z forward.  Pixel
 * centres are at integer coordinates: the centre of pixel (u, v) is (u, v). */
typedef struct rtg_camera {
    int32_t width, height;
    float fx, fy, cx, cy;
    float R[9];
    float T[3];
} rtg_camera;

/* Rasterizer settings (rtg_default_settings fills the defaults shown).
 *   tile_w x tile_h: screen tile, one of 8x8, 16x16 (default), 32x8; 0x0
 *     asks for the tile chosen by rtg_autotune (16x16 if never tuned);
 *   batch: Gaussians staged per LDS batch by the forward and scoring
 *     kernels: 0 = one per thread of the tile, else 32, 64, 128 or 256, not
 *     above the tile's pixel count (the backward stages 64 per wave);
 *   T_min = 1e-4: compositing stops before the Gaussian that would take the
 *     transmittance below T_min;
 *   alpha_min = 1/255: a Gaussian whose alpha at a pixel is below it is
 *     skipped there (and this fixes its screen-space support);
 *   alpha_max = 0.99: alpha is clamped to it;
 *   z_near = 0.2: Gaussians with camera depth <= z_near are culled;
 *   eps2d = 0: added to the diagonal of the 2D covariance;
 *   max_instances: capacity of (tile, Gaussian) pairs for captured graphs
 *     (0 = sized by a first eager pass);
 *   isotropic = 0: 1 selects the paper's 8-parameter Gaussian of Sec. III
 *     (colour, mean, radius, opacity): the first n log_scales values are the
 *     log-radii, quats is not read (may be NULL) and the splat projects with
 *     r_2D = f r / d per image axis, Sigma_2D = diag((fx r/d)^2, (fy r/d)^2)
 *     (+ eps2d); the backward then writes only the first n log-scale
 *     gradients and no quaternion gradient;
 *   reserved: 0. */
typedef struct rtg_settings {
    int32_t tile_w, tile_h;
    int32_t batch;
    float T_min, alpha_min, alpha_max, z_near, eps2d;
    int64_t max_instances;
    int32_t isotropic;
    int32_t reserved;
} rtg_settings;

/* The Gaussian map (Sec. III: colour, position, size, opacity; the
 * anisotropic form of the cited 3DGS work), planar structure of arrays of n
 * float32 entries per component:
 *   means 3 x n, log_scales 3 x n, quats 4 x n (w, x, y, z; any norm),
 *   opacity n (activated, in (0, 1]), colors 3 x n, uncert n (per-Gaussian
 *   uncertainty u_i of Sec. IV-A; may be NULL when no uncertainty image or
 *   score is requested).  With settings.isotropic = 1, log_scales holds n
 *   log-radii (1 x n; a 3 x n array is read in its first row) and quats may
 *   be NULL. */
typedef struct rtg_gaussians {
    int64_t n;
    const float *means, *log_scales, *quats, *opacity, *colors, *uncert;
} rtg_gaussians;

/* Gradients, same layouts as rtg_gaussians; ADDED to (+=), so several calls
 * accumulate.  Any pointer may be NULL to skip that group. */
typedef struct rtg_grads {
    float *d_means, *d_log_scales, *d_quats, *d_opacity, *d_colors;
} rtg_grads;

typedef struct rtg_ctx rtg_ctx;
typedef struct rtg_frame rtg_frame;
typedef struct rtg_graph rtg_graph;

/* Message of the last error on this thread ("" if none). */
const char *rtg_last_error(void);

/* Fills *s with the defaults listed above. */
rtg_status rtg_default_settings(rtg_settings *s);

/* Number of HIP devices (0 when none; never an error). */
int32_t rtg_device_count(void);

/* Creates a context on `device`.  RTG_ERR_HIP if there is no such device. */
rtg_status rtg_create(int32_t device, rtg_ctx **out);
void rtg_destroy(rtg_ctx *ctx);

/* Device allocator of a context's scratch (projected records, pair lists,
 * sort buffers, per-pixel state, gradients in screen space).  By default the
 * library calls hipMalloc and keeps released blocks for reuse; with an
 * allocator set, blocks come from alloc(user, bytes) (device memory of the
 * context's device, 256-byte aligned, or NULL when it cannot allocate) and go
 * back through free(user, ptr) when the context trims its cache or is
 * destroyed; a caching allocator such as PyTorch's can serve them.  Both
 * NULL restores hipMalloc.  RTG_ERR_INVALID while any frame or graph of the
 * context holds scratch (destroy them first), or if only one of alloc / free
 * is given.  Synchronises the device. */
typedef void *(*rtg_alloc_fn)(void *user, size_t bytes);
typedef void (*rtg_free_fn)(void *user, void *ptr);
rtg_status rtg_set_allocator(rtg_ctx *ctx, rtg_alloc_fn alloc, rtg_free_fn free, void *user);

/* Projection and culling (Sec. III: mu_2D = K R^T (mu - T) / d with the EWA
 * 2D covariance).  Projects every Gaussian into each of the n_views cameras
 * and keeps the (view, Gaussian) pairs whose alpha >= alpha_min support
 * meets the image.  Creates *out, which holds the projected records and
 * references g's arrays: they must stay valid and unchanged until the frame
 * is destroyed.  Images of several views are packed view after view (see
 * rtg_render).  n_views in [1, 1024].  Synchronises `stream` once (to size
 * the record buffer).  RTG_ERR_UNSUPPORTED when the records number 2^31 or
 * more (nothing is allocated for them). */
rtg_status rtg_project(rtg_ctx *ctx, const rtg_gaussians *g, const rtg_camera *cams,
                       int32_t n_views, const rtg_settings *settings, rtg_frame **out,
                       void *stream);

/* Depth ordering and tile binning (Sec. III: "sorted in increasing order of
 * depth relative to the camera").  Builds, for every screen tile of every
 * view, the list of Gaussians whose support meets it, in ascending binary32
 * camera depth, ties by Gaussian index.  A Gaussian is listed in a tile when
 * its support ellipse {alpha >= alpha_min} reaches the tile's pixel-centre
 * columns on one of the tile's pixel rows inside its pixel box, by a
 * conservative binary32 test (every pixel that composites it is kept): a
 * subset of the tiles its pixel box meets, and at least one tile per visible
 * Gaussian.  *n_instances (host, nullable)
 * receives the number of (tile, Gaussian) pairs.  Synchronises `stream`
 * once (to size the pair buffers).  RTG_ERR_UNSUPPORTED when the pairs
 * number 2^31 or more (nothing is allocated for them). */
rtg_status rtg_bin_sort(rtg_ctx *ctx, rtg_frame *f, int64_t *n_instances, void *stream);

/* Forward compositing (Sec. III: C(p) = sum_i c_i a_i prod_{j<i} (1 - a_j),
 * depth with c_i -> d_i): per pixel, RGB, depth (not normalised), alpha
 * = 1 - T_final and uncertainty sum_i u_i a_i T_i.  Outputs are float32,
 * planar per view and packed view after view: view v starts at pixel offset
 * P_0 + ... + P_{v-1} (P = width*height); rgb holds 3 planes per view, so
 * view v's RGB starts at 3*offset_v.  Any output may be NULL.  Saves the
 * per-pixel state the backward needs inside the frame.  Requires
 * rtg_bin_sort first. */
rtg_status rtg_render(rtg_ctx *ctx, rtg_frame *f, float *rgb, float *depth, float *alpha,
                      float *unc, void *stream);

/* L1 part of the mapping loss of Sec. III eq. (4):
 *   L = sum_views (1/P_v) sum_p [ sum_ch |C - C*| + w_depth |D - D*| ]
 * and dL/dC, dL/dD (sign(0) = 0), all in rtg_render's packed layout.
 * loss: device pointer to one double (written).  d_rgb/d_depth may be NULL. */
rtg_status rtg_loss(rtg_ctx *ctx, rtg_frame *f, const float *rgb, const float *depth,
                    const float *target_rgb, const float *target_depth, float w_depth,
                    float *d_rgb, float *d_depth, double *loss, void *stream);

/* The full mapping loss of Sec. III eq. (4), per view v of P_v pixels:
 *   L = sum_v [ (1/P_v) sum_p ( w_depth |D - D*| + lambda_1 sum_ch |C - C*| )
 *               + lambda_2 (1 - SSIM_v(C, C*)) ]
 * (the paper: w_depth = 1, lambda_1 = 0.4, lambda_2 = 0.1), and dL/dC, dL/dD
 * (sign(0) = 0) in rtg_render's packed layout.  SSIM_v is the mean over the
 * three channels and P_v pixels of the structural similarity index of Wang
 * et al. with an 11x11 Gaussian window (sigma 1.5, separable, normalised),
 * pixels outside the view read as 0, C1 = 0.01^2, C2 = 0.03^2 (colours in
 * [0, 1]).  Binary32 filtering; the loss is summed in binary64 in a fixed
 * order.  loss: device pointer to one double (written).  d_rgb / d_depth may
 * be NULL (both NULL: the loss only).  Scratch: 36 bytes per pixel, kept in
 * the frame. */
rtg_status rtg_loss_ssim(rtg_ctx *ctx, rtg_frame *f, const float *rgb, const float *depth,
                         const float *target_rgb, const float *target_depth, float w_depth,
                         float lambda_1, float lambda_2, float *d_rgb, float *d_depth, double *loss,
                         void *stream);

/* Reverse mode of rtg_render and rtg_project (the map is "refined through
 * backpropagation", Sec. IV-A): given dL/d(image) in rtg_render's layout
 * (d_alpha and d_unc nullable = zero), ADDS dL/d(means, log_scales, raw
 * quaternion, opacity, colors) into *out, summed over the frame's views.
 * Threshold decisions (alpha_min, T_min, alpha_max clamp, culling) are
 * treated as constants.  Requires rtg_render on the same frame first. */
rtg_status rtg_render_backward(rtg_ctx *ctx, rtg_frame *f, const float *d_rgb,
                               const float *d_depth, const float *d_alpha,
                               const float *d_unc, const rtg_grads *out, void *stream);

/* Releases a frame (NULL is a no-op). */
void rtg_frame_destroy(rtg_frame *f);

/* Copies the frame's binning to caller DEVICE buffers (any may be NULL):
 *   keys[k] = (global_tile << 32) | binary32 depth bits, vals[k] = Gaussian
 *   index, for the n_instances pairs in sorted order; ranges[2*t], [2*t+1] =
 *   [start, end) of global tile t (tiles of view v follow those of views
 *   0..v-1, row-major inside a view).  Sizes come from rtg_frame_info. */
rtg_status rtg_frame_export(rtg_ctx *ctx, rtg_frame *f, uint64_t *keys, uint32_t *vals,
                            uint32_t *ranges, void *stream);

/* Copies the frame's projected records (Sec. III projection: one per visible
 * (view, Gaussian) pair, Gaussian-major, views ascending within a Gaussian)
 * to caller DEVICE buffers, for inspection and key parity; any pointer may be
 * NULL.  R = rtg_frame_info()[0]; arrays are planar:
 *   mean2d: 2 x R doubles, mu_2D = (fx t_x / d + cx, fy t_y / d + cy), held by
 *     the kernels as the sum of two binary32 values (about 48 bits);
 *   conic: 3 x R doubles, Sigma_2D^-1 entries (xx, xy, yy), binary64;
 *   pbox: 4 x R int32, (u0, u1, v0, v1): the inclusive pixel box of
 *     {alpha >= alpha_min}, u0 = ceil(mu_x - h_x), u1 = floor(mu_x + h_x)
 *     clipped to the image, h_x = sqrt(2 ln(o / alpha_min) Sigma_xx), and
 *     the same in y;
 *   depth_bits: R uint32, bits of the binary32 camera depth (the sort key);
 *   gid, view: R uint32, Gaussian and view index;
 *   ntiles: R uint32, (tile, Gaussian) pairs of the record.
 * Asynchronous on `stream`. */
rtg_status rtg_frame_export_records(rtg_ctx *ctx, rtg_frame *f, double *mean2d, double *conic,
                                    int32_t *pbox, uint32_t *depth_bits, uint32_t *gid,
                                    uint32_t *view, uint32_t *ntiles, void *stream);

/* Host-side sizes of a frame: [0] records (visible view-Gaussian pairs),
 * [1] instances (tile-Gaussian pairs, -1 before rtg_bin_sort), [2] total
 * tiles, [3] total pixels, [4] tile_w, [5] tile_h. */
rtg_status rtg_frame_info(const rtg_frame *f, int64_t info[6]);

/* View scoring by the trace proxy of Sec. IV-A eq. (7), summed over the
 * pixels p of view v in binary64:
 *   mode 0 (rendered): score_v = sum_p sum_i u_i a_i(p) T_i(p), the
 *     per-Gaussian uncertainty composited like a colour channel;
 *   mode 1 (binary-J): score_v = sum_p sum of u_i over the Gaussians i that
 *     contribute at p (pass the alpha_min test before termination) - the
 *     Jacobian in the trace replaced by its binary sparsity pattern.
 * scores: device array of n_views doubles.  persistent = 1: all views go
 * through one projection, one sort and one persistent compositing launch;
 * persistent = 0: a plain loop of per-view launches (for comparison).
 * Results are identical either way.  A mode other than 0 or 1 is
 * RTG_ERR_INVALID.  Synchronises `stream` to size buffers.  A view whose
 * binning reported an internal inconsistency gets a NaN score. */
rtg_status rtg_score_views(rtg_ctx *ctx, const rtg_gaussians *g, const rtg_camera *cams,
                           int32_t n_views, const rtg_settings *settings, double *scores,
                           int32_t persistent, int32_t mode, void *stream);

/* Captured scoring pipeline: the whole batched path of rtg_score_views in
 * one hipGraph with device-side sizes, replayed for new poses.
 * create: fixes the map g (its arrays must stay valid and unchanged), at
 * most max_views views, each at most max_width x max_height pixels, and the
 * settings, and the score mode (as in rtg_score_views).  Buffers have
 * fixed capacities: the (tile, Gaussian) pair
 * capacity is settings->max_instances if > 0, else twice the count measured
 * by an eager pass over the n_probe `probe` cameras, scaled to max_views
 * (probe must then be non-NULL).  launch: uploads cams (host, n_views <=
 * max_views, each within the size limits), replays the graph on `stream` and
 * copies the n_views scores to the device array `scores`.  A replay whose
 * buffers overflow writes NaN scores, and the overflow is sticky: the graph
 * keeps reporting it until destroyed.  launch never waits for a running
 * replay (it waits only for the one before the previous, whose pinned
 * camera area it reuses) and returns RTG_ERR_CAPACITY, without replaying,
 * once an earlier replay's overflow has reached the host (an overflow of
 * 2^31 or more pairs is RTG_ERR_UNSUPPORTED); create a graph with larger
 * capacity then.  status: waits for the last replay and returns the same
 * codes, so it also reports an overflow of that last replay. */
rtg_status rtg_score_graph_create(rtg_ctx *ctx, const rtg_gaussians *g, int32_t max_views,
                                  int32_t max_width, int32_t max_height,
                                  const rtg_settings *settings, int32_t mode,
                                  const rtg_camera *probe, int32_t n_probe, rtg_graph **out,
                                  void *stream);
/* Captured mapping iteration for fixed keyframes: the gradient of the
 * mapping problem of Sec. III eq. (2) with the L1 part of eq. (4), as one
 * hipGraph replayed once per optimiser iteration.  One replay runs
 * projection, depth sort and tile binning, forward compositing into rgb and
 * depth (caller device buffers in rtg_render's packed layout), the loss into
 * *loss (device double), and the backward, ADDING the gradients into *grads
 * (device arrays shaped like the map; any group may be NULL).  The map, the
 * targets, the outputs and the gradient arrays are captured by address: they
 * must stay allocated, and the map may be updated in place between replays.
 * Buffer capacities are 1.5x the counts of an eager pass at creation (or
 * settings->max_instances pairs when > 0).  A replay that overflows them
 * leaves its outputs invalid and adds nothing to the gradients, and so does
 * every later replay (the overflow is sticky); rtg_map_graph_launch returns
 * RTG_ERR_CAPACITY without replaying once an overflow has reached the host
 * (it never waits), and rtg_map_graph_status waits for the last replay and
 * reports it. */
rtg_status rtg_map_graph_create(rtg_ctx *ctx, const rtg_gaussians *g, const rtg_camera *cams,
                                int32_t n_views, const rtg_settings *settings,
                                const float *target_rgb, const float *target_depth, float w_depth,
                                float *rgb, float *depth, double *loss, const rtg_grads *grads,
                                rtg_graph **out, void *stream);
/* The same captured mapping iteration with the full loss of eq. (4) as
 * computed by rtg_loss_ssim (L1 depth weighted by w_depth, L1 colour by
 * lambda_1, 1 - SSIM by lambda_2; the paper: 1, 0.4, 0.1).  Launch, status
 * and destroy as for rtg_map_graph_create. */
rtg_status rtg_map_graph_create_ssim(rtg_ctx *ctx, const rtg_gaussians *g, const rtg_camera *cams,
                                     int32_t n_views, const rtg_settings *settings,
                                     const float *target_rgb, const float *target_depth,
                                     float w_depth, float lambda_1, float lambda_2, float *rgb,
                                     float *depth, double *loss, const rtg_grads *grads,
                                     rtg_graph **out, void *stream);
rtg_status rtg_map_graph_launch(rtg_graph *gr, void *stream);
rtg_status rtg_map_graph_status(rtg_graph *gr);
void rtg_map_graph_destroy(rtg_graph *gr);

rtg_status rtg_score_graph_launch(rtg_graph *gr, const rtg_camera *cams, int32_t n_views,
                                  double *scores, void *stream);
rtg_status rtg_score_graph_status(rtg_graph *gr);
void rtg_score_graph_destroy(rtg_graph *gr);

/* Autotuner: times `mode` (0 forward, 1 forward+backward, 2 scoring) on the
 * given map and cameras for every tile in {8x8, 16x16, 32x8} with every
 * staging batch in {0 (one splat per thread of the tile), 32, 64, 128} below
 * the tile's pixel count (10 candidates); a candidate's cost is the median
 * over three calls (after one warm-up) of its kernels' device time, taken
 * with the library's per-group events (the eager calls' host reads are left
 * out, as in a captured graph).  Writes the fastest into
 * settings->tile_w/tile_h/batch and makes it the context's choice for
 * settings with tile 0x0.  The caller's rtg_timing totals are left as they
 * were.  Images, scores and gradients do not depend on the choice.
 * Synchronises `stream`. */
rtg_status rtg_autotune(rtg_ctx *ctx, const rtg_gaussians *g, const rtg_camera *cams,
                        int32_t n_views, int32_t mode, rtg_settings *settings, void *stream);

/* Paper-literal view utility of Sec. IV-B eq. (8), which does not render:
 *   v(x, g) = 1 when Gaussian g is in the field of view of camera x - its
 *   camera depth is in (settings->z_near, range] (range: the sensor's
 *   perception range; no occlusion test) and its projected mean lies inside
 *   the image, 0 <= u <= W-1, 0 <= v <= H-1;
 *   H = {g : u_g > lo_hi[1]}, L = {g : u_g < lo_hi[0]};
 *   n_high[v] = sum_{g in H} v(x_v, g), n_low[v] = sum_{g in L} v(x_v, g),
 *   sum_u[v] = sum_g u_g v(x_v, g) (the "-sum" variant of Sec. V-A, in 2^-40
 *   fixed point), xi[v] = n_high[v] - lambda_xi n_low[v].
 * lo_hi: device array of the two thresholds (see rtg_uncertainty_thresholds).
 * All outputs are device arrays of n_views entries; any may be NULL.  Only the
 * means and uncert arrays of g are read.  The visibility decision is taken
 * in binary64 wherever binary32 cannot decide it. */
rtg_status rtg_view_utility(rtg_ctx *ctx, const rtg_gaussians *g, const rtg_camera *cams,
                            int32_t n_views, const rtg_settings *settings, float range,
                            const double *lo_hi, double lambda_xi, int64_t *n_high,
                            int64_t *n_low, double *sum_u, double *xi, void *stream);

/* Thresholds of the high / low uncertainty sets (Sec. IV-C: half a standard
 * deviation above and below the mean): lo_hi[0] = mean - k_std sd,
 * lo_hi[1] = mean + k_std sd over u[0..n), binary64, population standard
 * deviation, fixed reduction order.  lo_hi: device array of 2 doubles. */
rtg_status rtg_uncertainty_thresholds(rtg_ctx *ctx, const float *uncert, int64_t n, double k_std,
                                      double *lo_hi, void *stream);

/* Trajectory selection of Sec. IV-B eq. (10): traj_utility[t] = sum of xi
 * over the states offsets[t] .. offsets[t+1]-1 (device int32 array of
 * n_traj + 1 offsets), summed in order; *best (device int32) = the first
 * trajectory of maximal utility.  traj_utility may be NULL. */
rtg_status rtg_trajectory_select(rtg_ctx *ctx, const double *xi, const int32_t *offsets,
                                 int32_t n_traj, double *traj_utility, int32_t *best,
                                 void *stream);

/* Uncertainty bookkeeping of Sec. IV-A: the uncertainty of a Gaussian is the
 * magnitude of the change of its mean over a map update,
 *   u_out[i] = ||mu_cur[i] - mu_prev[i]||_2  (squared when squared != 0: the
 *              -sq variant of Sec. V-A),
 * except that a Gaussian whose mean did not change in the update (all three
 * components equal) keeps u_out[i] = u_prev[i].  Formed in binary64 as
 * sqrt((dx^2 + dy^2) + dz^2) and rounded once to binary32.  means_prev and
 * means_cur: device, planar 3 x n; u_prev, u_out: device, n floats (u_out
 * may equal u_prev).  Asynchronous on `stream`. */
rtg_status rtg_uncertainty_update(rtg_ctx *ctx, int64_t n, const float *means_prev,
                                  const float *means_cur, const float *u_prev, int32_t squared,
                                  float *u_out, void *stream);

/* Region grid of Sec. IV-B (high-level planner: the known enclosing space
 * evenly partitioned into cuboids), host only: the box [lo, hi) (box = lo x,
 * y, z, hi x, y, z) is partitioned into cuboids of edge `size` (2.5 m, set in
 * Sec. IV-C), dims[a] = ceil((hi_a - lo_a) / size).  RTG_ERR_INVALID for a
 * non-positive size or extent. */
rtg_status rtg_region_grid(const double *box, double size, int32_t *dims);

/* Region utility Omega_k of Sec. IV-B (high-level planner; region size from
 * Sec. IV-C): for each cuboid region r = ix + nx (iy + ny iz)
 * of rtg_region_grid(box, size), count[r] = M = the number of Gaussians whose
 * mean lies in it (i = floor((mu_a - lo_a) / size) in binary64, half-open
 * cells; means outside the grid count nowhere), sum[r] = the sum of their u,
 * mean[r] = Omega = sum / M (0 for an empty region).  Sums are accumulated in
 * fixed point with 2^-32 resolution, independent of the order of the
 * atomics; a region holding a non-finite u or |u| >= 2^20 reports NaN.
 * means (planar 3 x n), u (n): device; box: host, 6 doubles; count, sum,
 * mean: device arrays of nx ny nz entries, any may be NULL.  Asynchronous on
 * `stream`. */
rtg_status rtg_region_utility(rtg_ctx *ctx, int64_t n, const float *means, const float *u,
                              const double *box, double size, int64_t *count, double *sum,
                              double *mean, void *stream);

/* Collision check of Sec. IV-B (trajectory planner, Collision Checking): a
 * Gaussian is treated as a sphere about its mean of radius lambda_g r_i, r_i = exp(max of its three log-scales) (the
 * principal axis); a point sampled on a path collides when a sphere of radius
 * r_robot about it meets one of them:
 *   collide[j]   = 1 if ||p_j - mu_i||^2 < (r_robot + lambda_g r_i)^2 for
 *                  some i, else 0 (strict; decided in binary64 wherever the
 *                  binary32 distance is within a relative 4e-6 of the bound);
 *   clearance[j] = min_i (||p_j - mu_i|| - lambda_g r_i), binary32, +inf when
 *                  no Gaussian is left.
 * Gaussians with a non-finite mean or log-scale are ignored.  points: device,
 * planar 3 x n_points; collide: device, n_points int32 (required);
 * clearance: device, n_points floats or NULL.  Only g->means and
 * g->log_scales are read.  r_robot, lambda_g: finite and >= 0 (the paper
 * uses lambda_g = 3).  Every point is tested against every Gaussian (no
 * spatial index).  Asynchronous on `stream`. */
rtg_status rtg_collision_check(rtg_ctx *ctx, const rtg_gaussians *g, const float *points,
                               int64_t n_points, float r_robot, float lambda_g, int32_t *collide,
                               float *clearance, void *stream);

/* rtg_collision_check for callers that cannot allocate device memory (code
 * under hipGraph capture, tight planning loops, hosts that forbid
 * allocation): the same check and results, with its scratch (24 bytes per
 * Gaussian + 4 per point, each part 256-byte aligned) taken from a fixed
 * 96 MiB device array that every GPU the library runs on holds from the
 * library's load until the process ends; it calls no hipMalloc, hipFree or
 * allocating routine.  Larger inputs return RTG_ERR_UNSUPPORTED before any
 * launch (use rtg_collision_check).  All calls on one GPU share that array:
 * calls that overlap on one GPU (several streams, threads or contexts) race,
 * so the caller must order them.  The caller still passes the inputs and
 * outputs, as for rtg_collision_check. */
rtg_status rtg_collision_check_noalloc(rtg_ctx *ctx, const rtg_gaussians *g, const float *points,
                                       int64_t n_points, float r_robot, float lambda_g,
                                       int32_t *collide, float *clearance, void *stream);

/* Work counters of a rendered frame (host output, synchronises `stream`):
 *   out[0] records (visible view-Gaussian pairs), out[1] instances
 *   (tile-Gaussian pairs), out[2] contributing pixel-Gaussian pairs (terms of
 *   the compositing sums of Sec. III over all pixels), out[3] splat list
 *   entries walked by the backward (sum over pixels of the position after the
 *   last contributor).  Requires rtg_render.  Also reports a binning
 *   inconsistency found after rtg_bin_sort returned (RTG_ERR_HIP; the
 *   frame's images are then unwritten). */
rtg_status rtg_frame_stats(rtg_ctx *ctx, rtg_frame *f, int64_t out[4], void *stream);

/* Kernel timing for measurement: while enabled, the library brackets its
 * kernels with HIP events on the stream they are launched on and accumulates
 * the elapsed time per kernel id:
 *   0 projection (count + emit), 1 depth sort, 2 tile binning and sort,
 *   3 forward compositing, 4 loss, 5 backward compositing, 6 projection
 *   backward, 7 view-scoring compositing (persistent or per-view; a whole
 *   scoring-graph replay), 8 a whole mapping-graph replay.
 * rtg_timing_read waits for pending events and returns the accumulated
 * milliseconds and launch count of one id; rtg_timing_reset clears all. */
rtg_status rtg_timing_enable(rtg_ctx *ctx, int32_t on);
rtg_status rtg_timing_read(rtg_ctx *ctx, int32_t id, double *total_ms, int64_t *count);
rtg_status rtg_timing_reset(rtg_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* RTG_H */
