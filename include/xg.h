/*
 * xg.h -- C ABI of libxg, the gfx950 (MI355X) implementation of
 * Differentiable Radiative Rasterization (DRR): tile-based splatting of
 * radiative 3-D Gaussians through a circular cone-beam X-ray camera, and
 * its backward pass to every Gaussian parameter.
 *
 * Paper: "Radiative Gaussian Splatting for Efficient X-ray Novel View
 * Synthesis" (X-Gaussian).  The rendered image is I = F_DRR(M_ext, M_int,
 * {G_i(mu_i, Sigma_i, alpha_i, f_i)}) of Eq. 5; the calls below split F_DRR
 * into the stages of Sec. 3.2 and add its adjoint.
 *
 * Conventions for every call:
 *  - Pointers are DEVICE pointers to caller-owned memory unless marked
 *    [host].  The library never allocates, never frees and never
 *    synchronises; compute calls only enqueue work on `stream` (a
 *    hipStream_t; NULL = the null stream) and are safe under HIP graph
 *    capture.
 *  - Arguments are validated on the host before any HIP call; invalid
 *    arguments return XG_EINVAL and enqueue nothing.  XG_EHIP reports a
 *    failed kernel launch.  XG_ECAPACITY is raised asynchronously: when the
 *    number of (view, Gaussian, tile) pairs exceeds the workspace capacity
 *    the device status word is set (read it with xg_ws_layout offsets after
 *    synchronising) and later stages leave their outputs undefined.
 *  - Degenerate Gaussians (camera depth <= near_z, zero quaternion,
 *    non-positive 2-D determinant, opacity < alpha_min, non-finite input,
 *    footprint outside the detector) are culled: no pairs, zero gradient.
 *  - Float arithmetic is IEEE binary32 except where noted; the depth and
 *    bounding-rectangle computation ("key path") is a fixed binary32
 *    operation sequence with no contraction, so sort keys are reproducible
 *    bit for bit by any IEEE implementation.
 */
#ifndef XG_H
#define XG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define XG_ABI_VERSION 4

typedef enum {
    XG_OK = 0,
    XG_EINVAL = 1,     /* invalid argument (synchronous, nothing enqueued) */
    XG_ECAPACITY = 2,  /* pair capacity exceeded (device status word)      */
    XG_EHIP = 3        /* a HIP runtime call or kernel launch failed       */
} xg_status;

/* One view.  Rotation/translation are rows 0..2 of M_ext and the focal
 * lengths / principal point are M_int, both of Eq. 12.  pixel_offset and
 * tile_offset place the view in the concatenated image buffers and in the
 * global tile numbering; fill them with xg_layout_views.  80 bytes. */
typedef struct {
    float rot[9];          /* rotation block of M_ext, row-major            */
    float trans[3];        /* translation column of M_ext: (0, 0, L_SO)      */
    float fx, fy;          /* focal lengths, pixels                          */
    float cx, cy;          /* principal point, pixels (W/2, H/2)             */
    int32_t width, height; /* detector pixels                                */
    int32_t pixel_offset;  /* index of pixel (0,0) in concatenated images    */
    int32_t tile_offset;   /* global id of tile (0,0) for settings.tile      */
} xg_camera;

/* Renderer constants.  Defaults (xg_default_settings): tile 16,
 * lds_batch 256, lowpass 0.3 px^2 added to the diagonal of the 2-D
 * covariance, alpha_min 1/255, alpha_max 0.99, t_min 1e-4, near_z 0.2. */
typedef struct {
    int32_t tile;          /* 8 | 16 | 32: tile side and workgroup footprint */
    int32_t lds_batch;     /* 64 | 128 | 256 Gaussians staged in LDS at once */
    float lowpass;         /* k of Sigma'' + k I (>= 0)                       */
    float alpha_min;       /* skip an evaluation with alpha < alpha_min      */
    float alpha_max;       /* clamp alpha to alpha_max (< 1)                  */
    float t_min;           /* stop before transmittance drops below t_min
                              (below the smallest normal float32, 2^-126,
                              it acts as 2^-126)                              */
    float near_z;          /* cull Gaussians with camera depth <= near_z     */
    uint32_t flags;        /* XG_F_* bits                                     */
} xg_settings;

#define XG_F_PERSISTENT 1u /* render with a persistent grid over a tile queue */

/* Gaussian parameters, float32, structure of arrays, contiguous:
 * means[n][3], scales[n][3] (activated, > 0), quats[n][4] (w, x, y, z;
 * any non-zero norm, normalised inside), opacity[n] (activated, in (0,1]),
 * intensity[n] (activated view-independent radiation intensity, Eq. 3). */
typedef struct {
    const float *means, *scales, *quats, *opacity, *intensity;
    int32_t n;
} xg_gaussians;

/* Gradients of the same shapes; xg_render_bwd and xg_preprocess_bwd
 * ACCUMULATE (+=) into them. */
typedef struct {
    float *means, *scales, *quats, *opacity, *intensity;
} xg_grads;

/* Everything that describes one rendering of n Gaussians into n_views
 * views.  cams is a [host] array used for validation and launch shapes;
 * cams_dev must hold the same n_views records in device memory.  ws is a
 * device workspace of ws_bytes >= xg_workspace_size(...) bytes, 256-byte
 * aligned; pair_capacity bounds the (view, Gaussian, tile) pairs it holds. */
typedef struct {
    int32_t n;
    int32_t n_views;
    const xg_camera *cams;      /* [host]   */
    const xg_camera *cams_dev;  /* [device] */
    xg_settings settings;
    void *ws;
    size_t ws_bytes;
    int64_t pair_capacity;      /* 0 < pair_capacity < 2^31 */
} xg_frame;

/* Workspace sub-buffer offsets (bytes from ws), for inspection and tests.
 * Pair p of the sorted order has a global tile id and a Gaussian index.
 * When pair_index_bits = b > 0 they share one word: pair_tiles[p] =
 * tile << b | index (tile bits + b <= 32; pair_values is the same array);
 * when b = 0 they are parallel arrays pair_tiles[p], pair_values[p].  The
 * pair's sort key is (tile << 32) | float32 bits of the camera depth of
 * (view of that tile, that Gaussian), which is word 7 of that (view,
 * Gaussian)'s 64-byte render record. */
typedef struct {
    size_t status;      /* int32: XG_OK or XG_ECAPACITY                       */
    size_t n_pairs;     /* int32: pairs emitted (may exceed the capacity)     */
    size_t depth_range; /* uint32[2]: min, max depth bits of kept Gaussians */
                        /* (set by xg_bin_sort)                               */
    size_t records;     /* 64-byte render records per (view, Gaussian)        */
    size_t counts;      /* uint32[n_views*n]: tiles touched (0 = culled)      */
    size_t offsets;     /* uint32[n_views*n]: scan of counts in depth order   */
    size_t pair_tiles;  /* uint32[pair_capacity]: tile ids, sorted            */
    size_t pair_values; /* uint32[pair_capacity]: Gaussian indices, sorted    */
    size_t ranges;      /* uint32[total_tiles][2]: [start, end) per tile      */
    size_t grad2d;      /* float[n_views*n][8]: per-view 2-D gradients        */
    size_t total;       /* bytes needed                                       */
    size_t pair_index_bits; /* b above: index bits of a packed pair, 0 = two arrays */
} xg_ws_layout;

/* Returns XG_ABI_VERSION. */
int32_t xg_abi_version(void);

/* Human-readable name of a status code (static string). */
const char *xg_status_string(xg_status s);

/* Name and description of the last HIP error seen by a call on this host
 * thread that returned XG_EHIP ("hipSuccess" if none); static storage. */
const char *xg_last_error(void);

/* Default renderer constants. */
xg_settings xg_default_settings(void);

/* Camera of a circular cone-beam scanner (Eq. 12, W of Eq. 9): source at
 * azimuth phi on a circle of radius l_so about the world z axis, elevation
 * 0, flat detector of det_w x det_h scene units at distance l_sd from the
 * source, sampled by width x height pixels.  Rows of M_ext are
 * (-sin phi, cos phi, 0), (0, 0, -1), (-cos phi, -sin phi, 0) with
 * translation (0, 0, l_so); focal lengths (l_sd * width) / det_w and
 * (l_sd * height) / det_h pixels (the paper's L_SD with the pixel pitch made
 * explicit); principal point (width/2, height/2).  float64 math rounded
 * once to float32.  Leaves pixel_offset/tile_offset at 0.
 * XG_EINVAL if out is NULL, width/height <= 0, or a length is not > 0. */
xg_status xg_camera_from_scanner(double phi, double l_so, double l_sd, int32_t width,
                                 int32_t height, double det_w, double det_h,
                                 xg_camera *out /* [host] */);

/* Fills pixel_offset and tile_offset of n_views [host] cameras for tile
 * size `tile`: views are concatenated in order, tiles numbered row-major
 * within a view.  Writes the totals if the pointers are non-NULL. */
xg_status xg_layout_views(xg_camera *cams /* [host] */, int32_t n_views, int32_t tile,
                          int64_t *total_pixels, int64_t *total_tiles);

/* Workspace layout and size for a frame (only n, n_views, cams, settings
 * and pair_capacity are read; ws may be NULL). */
xg_status xg_ws_layout_of(const xg_frame *f /* [host] */, xg_ws_layout *out /* [host] */);

/* Total workspace bytes for a frame (same inputs as xg_ws_layout_of). */
xg_status xg_workspace_size(const xg_frame *f /* [host] */, size_t *bytes /* [host] */);

/* Stage 1 (Eq. 7-9, Sec. 3.2): per (view, Gaussian) camera-space centre,
 * depth, culling, 2-D covariance Sigma'' = J W Sigma W^T J^T (rows/cols 1-2)
 * plus lowpass*I, its inverse in factored form, image-space centre, the
 * integer bounding rectangle of the alpha >= alpha_min footprint and the
 * number of tiles it touches.  Also clears the per-view 2-D gradient
 * accumulators used by xg_render_bwd, and leaves the depth bounds of its
 * workgroups for xg_bin_sort, whose first launch resets the status word
 * and sets the frame's depth range (with no items, this call resets
 * them). */
xg_status xg_preprocess(const xg_frame *f /* [host] */, const xg_gaussians *g /* [host] */,
                        void *stream);

/* Stage 2 (Sec. 3.2): the per-tile lists of Gaussians sorted by camera
 * depth.  The (view, Gaussian) items of each view are radix-sorted stably
 * by depth on the depth bits that vary, and their tile counts are scanned
 * in that order (offsets).  One (global tile id, Gaussian index) pair per
 * (view, Gaussian, tile) is then placed in tile order: when every view has
 * at most 4096 tiles, directly at its list position by a stable counting
 * sort of each view's pairs by tile; otherwise emitted in item order and
 * radix-sorted stably by tile id.  A tile lists only Gaussians of its own
 * view, so either way the result equals a sort of the keys (tile << 32 |
 * float32 bits of the depth), ties by ascending Gaussian index.  Also
 * fills the per-tile [start, end) ranges and the pair count; more pairs
 * than the capacity raise XG_ECAPACITY (no pair is written, every range
 * is empty).  A sort whose partitions cannot complete reports XG_EHIP in
 * the status word.  Last, the order in which the blend launches take the
 * tiles: each XCD's contiguous block of tiles (workgroup b runs on XCD
 * b % 8) from the longest list to the shortest, so no long tile starts
 * near the end of a launch; the render calls read it (any order gives the
 * same results). */
xg_status xg_bin_sort(const xg_frame *f /* [host] */, void *stream);

/* Stage 3 (Eq. 10): front-to-back blending of every pixel over its tile's
 * sorted list: at pixel centre p + 1/2, alpha = min(alpha_max, o G) with
 * G the projected 2-D Gaussian; evaluations outside the Gaussian's
 * rectangle or with alpha < alpha_min are skipped; blending stops before a
 * Gaussian that would take the transmittance below t_min.  Writes, per
 * pixel of the concatenated images: image (sum of intensity*alpha*T,
 * background 0), final_t (transmittance after the last contributor) and
 * n_contrib (1-based position in the tile list of the last contributor,
 * 0 if none).  Also leaves in the workspace, for every list entry it
 * stages, which 8 x 8 pixel blocks the entry can reach alpha_min in; the
 * backward reads them (as do the _l1 and _store forms). */
xg_status xg_render_fwd(const xg_frame *f /* [host] */, const xg_gaussians *g /* [host] */,
                        float *image, float *final_t, int32_t *n_contrib, void *stream);

/* xg_render_fwd followed by the L1 term of Eq. 11 in the same launch:
 * also writes dl_dimage = scale * sign(image - target) (sign(0) = 0), equal
 * bit for bit to xg_l1_grad on the image it writes; target and dl_dimage
 * [device] have the image layout.  EINVAL: as xg_render_fwd, null target
 * or dl_dimage, non-finite scale. */
xg_status xg_render_fwd_l1(const xg_frame *f /* [host] */, const xg_gaussians *g /* [host] */,
                           float *image, float *final_t, int32_t *n_contrib, const float *target,
                           float scale, float *dl_dimage, void *stream);

/* Stage 4 (adjoint of Eq. 10 and of Eq. 7-9): the gradient of
 * L = sum_p dl_dimage[p] I(p) with respect to every Gaussian parameter,
 * ADDED to `grads` (the caller zeroes them).  Runs xg_render_bwd_2d, then
 * xg_preprocess_bwd.  dl_dimage has the image layout; final_t and
 * n_contrib are the outputs of the forward of this frame since the last
 * xg_preprocess.  Recomputes the transmittance by division (only the final
 * T and the last contributor are kept from the forward).  Call once per
 * xg_preprocess (which clears the 2-D accumulators).  EINVAL: as
 * xg_render_bwd_2d and xg_preprocess_bwd, checked before anything is
 * enqueued. */
xg_status xg_render_bwd(const xg_frame *f /* [host] */, const xg_gaussians *g /* [host] */,
                        const float *dl_dimage, const float *final_t, const int32_t *n_contrib,
                        const xg_grads *grads /* [host] struct of device ptrs */, void *stream);

/* The first half of xg_render_bwd (adjoint of Eq. 10 alone): walks each
 * pixel's list backwards from n_contrib, recovering the transmittance by
 * division instead of reading stored per-contributor values, and
 * accumulates per (view, Gaussian) the 2-D gradients (image-space centre,
 * inverse 2-D covariance moments, opacity times the opacity gradient,
 * intensity) in the workspace,
 * reduced across each wavefront before one atomic add per (Gaussian,
 * wavefront).  Reads the per-entry block masks the forward left in the
 * workspace: final_t and n_contrib must come from xg_render_fwd,
 * xg_render_fwd_l1 or xg_render_fwd_store on these lists (after the last
 * xg_bin_sort); the comparison model's forward does not write them.
 * Follow with xg_preprocess_bwd or xg_preprocess_bwd_write. */
xg_status xg_render_bwd_2d(const xg_frame *f /* [host] */, const float *dl_dimage,
                           const float *final_t, const int32_t *n_contrib, void *stream);

/* Stored-transmittance variant of stages 3 and 4.  The forward
 * additionally keeps, for every pixel, the transmittance in front of each
 * of its first `slots` contributors (the T_j of Eq. 10 that the adjoint
 * needs); the backward reads them instead of dividing the transmittance
 * back, and divides only for contributors beyond `slots`.  Results equal
 * xg_render_fwd / xg_render_bwd up to the rounding of that division.
 * store: device buffer of at least xg_store_size(f, slots) bytes,
 * 256-byte aligned, caller-owned, written by the forward and read by the
 * backward of the same frame and tile size (its layout is per tile:
 * int32 contributor counts, then float transmittances slot-major).
 * EINVAL: slots outside [1, XG_MAX_STORE_SLOTS], a short or misaligned
 * store, or XG_F_PERSISTENT set. */
#define XG_MAX_STORE_SLOTS 4096
xg_status xg_store_size(const xg_frame *f /* [host] */, int32_t slots, int64_t *bytes /* [host] */);
xg_status xg_render_fwd_store(const xg_frame *f /* [host] */, const xg_gaussians *g /* [host] */,
                              float *image, float *final_t, int32_t *n_contrib, void *store,
                              int32_t slots, int64_t store_bytes, void *stream);
/* xg_render_bwd with the stored transmittances: the 2-D stage
 * (xg_render_bwd_store_2d) then xg_preprocess_bwd, adding to `grads`. */
xg_status xg_render_bwd_store(const xg_frame *f /* [host] */, const xg_gaussians *g /* [host] */,
                              const float *dl_dimage, const float *final_t,
                              const int32_t *n_contrib, const void *store, int32_t slots,
                              int64_t store_bytes, const xg_grads *grads /* [host] */, void *stream);
/* The 2-D stage alone (as xg_render_bwd_2d, reading the store). */
xg_status xg_render_bwd_store_2d(const xg_frame *f /* [host] */, const float *dl_dimage,
                                 const float *final_t, const int32_t *n_contrib, const void *store,
                                 int32_t slots, int64_t store_bytes, void *stream);

/* Stage 5 (adjoint of Eq. 7-9): maps the 2-D gradients of every view to
 * means, scales, quaternions (through their normalisation), opacity and
 * intensity, summing over views in registers (one thread per Gaussian, no
 * atomics), and ACCUMULATES into `grads` (caller zeroes them). */
xg_status xg_preprocess_bwd(const xg_frame *f /* [host] */, const xg_gaussians *g /* [host] */,
                            const xg_grads *grads /* [host] */, void *stream);
/* The same adjoint, WRITING the gradients instead of adding to them (zeros
 * for a Gaussian no view touched): the caller need not clear them first. */
xg_status xg_preprocess_bwd_write(const xg_frame *f /* [host] */, const xg_gaussians *g /* [host] */,
                                  const xg_grads *grads /* [host] */, void *stream);

/* Work counts, for throughput accounting and tests.  counts is int32
 * [XG_COUNT_ROWS][total pixels] (device).  Rows 0-3 follow from the
 * definition of Eq. 10 and the sorted lists alone; rows 4-7 describe how
 * the blending kernels walk the lists (wavefronts of 8 x 8 pixel blocks,
 * 8-aligned in each view; entries whose footprint cannot reach alpha_min
 * anywhere in the block are not visited).  "Per block" rows hold the
 * block's value at its first pixel and 0 at its other pixels.
 *   0: per pixel, evaluations: Gaussians of the list whose rectangle holds
 *      the pixel, up to and including the one that ends blending
 *   1: per pixel, contributors
 *   2: per pixel, evaluations up to the last contributor (what the
 *      backward revisits)
 *   3: per block, Gaussians that contribute to at least one pixel of the
 *      block (the backward's wavefront reductions)
 *   4: per block, list entries the backward wavefront visits (up to the
 *      block's last contributing entry; every pixel's upstream gradient
 *      taken as nonzero)
 *   5: per block, list entries the forward wavefront visits (up to the
 *      entry at which the block's last pixel stops, or the list end)
 *   6: per pixel, evaluations the forward makes for it in those visits
 *   7: per pixel, evaluations the backward makes for it in its visits (in
 *      the rectangle, up to the pixel's last contributor) */
#define XG_COUNT_ROWS 8
xg_status xg_render_counts(const xg_frame *f /* [host] */, int32_t *counts, void *stream);

/* Device pointers into a frame's workspace, for inspection and tests (no
 * HIP call; read them after synchronising with the stream that wrote
 * them).  pair_tiles/pair_values as in xg_ws_layout; ranges
 * uint32[total_tiles][2]; records 64-byte render records per (view,
 * Gaussian); grad2d float[n_views*n][8].  The workspace holds no 64-bit
 * sort keys (the lists are built by two 32-bit sorts); xg_pair_keys writes
 * them out. */
typedef struct {
    const int32_t *status, *n_pairs;
    const uint32_t *pair_tiles, *pair_values, *ranges;
    const void *records;
    const float *grad2d;
    int32_t pair_index_bits;
    int64_t total_tiles, total_pixels;
    const int32_t *tile_order;   /* int32[total_tiles], written by xg_bin_sort */
} xg_ws_view;
xg_status xg_ws_inspect(const xg_frame *f /* [host] */, xg_ws_view *out /* [host] */);

/* The sorted lists as (key, value) pairs (Sec. 3.2): for every sorted pair
 * p below the device pair count, keys[p] = (global tile id << 32) | float32
 * bits of the camera depth of (view of that tile, Gaussian), values[p] =
 * Gaussian index, ascending by (key, value).  keys uint64[capacity] and
 * values uint32[capacity] are device buffers; pairs past `capacity` and
 * entries past the pair count are not written; nothing is written when the
 * status word is not XG_OK.  EINVAL: null buffers, capacity < 0. */
xg_status xg_pair_keys(const xg_frame *f /* [host] */, uint64_t *keys, uint32_t *values,
                       int64_t capacity, void *stream);

/* Radiation intensity response (Eq. 3): each Gaussian has a feature
 * vector f[n_features] and its intensity is sigmoid(sum_k w[k] f[k]) with
 * constant weights w (the paper's lambda; it adopts 16 features).
 * features: device float[n][n_features]; weights: device
 * float[n_features]; intensity: device float[n].  EINVAL: null pointers,
 * n < 0, n_features outside [1, XG_MAX_FEATURES]. */
#define XG_MAX_FEATURES 64
xg_status xg_rirf_fwd(const float *features, const float *weights, int32_t n, int32_t n_features,
                      float *intensity, void *stream);
/* Adjoint: grad_features[i][k] += dl_dintensity[i] * s (1 - s) * w[k] with
 * s the intensity recomputed from the features (accumulates; the caller
 * clears grad_features). */
xg_status xg_rirf_bwd(const float *features, const float *weights, int32_t n, int32_t n_features,
                      const float *dl_dintensity, float *grad_features, void *stream);

/* Raw (unconstrained) trainable parameters, float32 SoA, contiguous:
 * means[n][3], log_scales[n][3] (scales = exp), quats[n][4] (the renderer
 * normalises), opacity_logit[n] (opacity = sigmoid), features[n][n_features]
 * (intensity = sigmoid(weights . features), Eq. 3); weights is the
 * constant device float[n_features]. */
typedef struct {
    float *means, *log_scales, *quats, *opacity_logit, *features;
    const float *weights;
    int32_t n;
    int32_t n_features;
} xg_params;

/* Adam settings.  The paper's (Sec. 4.1): beta1 0.9, beta2 0.999, eps
 * 1e-15; learning rates: positions 1.9e-4 decaying exponentially to 1.9e-6
 * over 2e4 steps, feature 2e-3, opacity 8e-3, scaling 5e-3, rotation 1e-3.
 * The position rate at step t (1-based) is
 * exp((1 - f) ln(lr_means_start) + f ln(lr_means_end)),
 * f = min(t - 1, lr_means_steps) / lr_means_steps.  The betas are double:
 * 0.999 rounded to float moves 1 - beta2 by 1.3e-5 relative, so the
 * library forms 1 - beta, beta^t and the rate schedule in double and rounds
 * the results once to float. */
typedef struct {
    float lr_means_start, lr_means_end;
    int32_t lr_means_steps;
    float lr_scales, lr_quats, lr_opacity, lr_feature;
    float eps;
    int32_t reserved;       /* 0 */
    double beta1, beta2;
} xg_adam;

/* Fused optimiser step (gradients from xg_preprocess_bwd are with respect
 * to the activated parameters).  With t = *step + 1 read from device
 * memory: per raw scalar, chain rule through the activation at the current
 * value, m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps); then writes the
 * activated copies scales[n][3], opacity[n], intensity[n] (means and quats
 * are used raw) and advances *step.  m and v are float[(11 + n_features) n]
 * in the order means, log_scales, quats, opacity_logit, features; *step
 * starts at 0.
 * The step count lives on the device so a captured step replays correctly.
 * gate (device, nullable): when it reads nonzero at execution time the
 * step is skipped (nothing written, *step unchanged); pass the frame's
 * status word (xg_ws_layout.status) so a step whose pairs overflowed the
 * capacity never reaches the parameters.  All array pointers device;
 * updates in place.  EINVAL: null pointers, beta outside [0, 1), eps < 0,
 * non-finite or negative rates, lr_means_steps < 1, reserved != 0,
 * n_features outside [1, XG_MAX_FEATURES]. */
xg_status xg_adam_step(const xg_params *p /* [host] struct of device ptrs */,
                       const xg_grads *g /* [host] struct of device ptrs */, float *m, float *v,
                       int32_t *step, const xg_adam *c /* [host] */, float *scales, float *opacity,
                       float *intensity, const int32_t *gate, void *stream);

/* Comparison model (the RGB Gaussians of 3D Gaussian splatting, Sec. 3.1
 * Eq. 2, measured against the radiative model in Tab. 3a), forward only.
 * xg_preprocess_rgb: xg_preprocess, then every (view, Gaussian)'s colour
 * c = max(sum_{l <= degree} sum_{|m| <= l} k_l^m Y_l^m(d) + 1/2, 0) per
 * channel, d the unit direction from the view's source (-R^T t) to the
 * Gaussian centre, Y_l^m the real spherical harmonics with the
 * Condon-Shortley phase; the colours live in the workspace until the next
 * preprocess.  sh [device] float32 [n][(degree+1)^2][3], basis index
 * l^2 + l + m, channel fastest; degree in 0..3.  g->intensity is not used
 * by the RGB blend but must be a valid pointer.
 * xg_render_fwd_rgb: Eq. 10 with the colour channels in place of the
 * intensity, after xg_preprocess_rgb and xg_bin_sort; image [device] is
 * planar float32 [3][total pixels], final_t and n_contrib as for
 * xg_render_fwd.  EINVAL: as xg_preprocess / xg_render_fwd, null sh, degree
 * outside 0..3, XG_F_PERSISTENT set (one workgroup per tile only). */
xg_status xg_preprocess_rgb(const xg_frame *f /* [host] */, const xg_gaussians *g /* [host] */,
                            const float *sh, int32_t degree, void *stream);
xg_status xg_render_fwd_rgb(const xg_frame *f /* [host] */, const xg_gaussians *g /* [host] */,
                            float *image, float *final_t, int32_t *n_contrib, void *stream);

/* ACUI initialisation of the Gaussian centres (Sec. 3.3, Eq. 13): a
 * cuboid of size size[0] x size[1] x size[2] centred on the origin, divided
 * into a grid[0] x grid[1] x grid[2] voxel grid, sampled at interval d:
 * points (n1 S1 d / M1, n2 S2 d / M2, n3 S3 d / M3) for all integers
 * |n_i| <= K_i = floor(M_i / (2 d)) + 1.  size, grid [host]; means [device]
 * float32 [count][3], n1 slowest and n3 fastest, each n_i ascending; every
 * coordinate is ((n S) d) / M evaluated in double and rounded once.
 * xg_acui_count gives count = prod (2 K_i + 1) [host].  EINVAL: a size, d
 * not finite and positive, a grid entry < 1, a count above INT32_MAX, null
 * means or capacity (in points) below the count. */
xg_status xg_acui_count(const double size[3], const int32_t grid[3], double d, int64_t *count);
xg_status xg_acui_grid(const double size[3], const int32_t grid[3], double d, float *means,
                       int64_t capacity, void *stream);

/* Training objective of Eq. 11, L = (1 - gamma) L1 + gamma L_SSIM (the
 * paper's gamma is 0.2), and its gradient with respect to the rendered
 * images, for every view of the frame (image and target have the image
 * layout).  L1 is the mean absolute difference over all pixels (sign(0) =
 * 0); L_SSIM = 1 - the mean of the SSIM map of Wang et al., each view's map
 * over its own image with an 11 x 11 Gaussian window (standard deviation
 * 1.5), zero padding, C1 = 0.01^2, C2 = 0.03^2.  Writes dl_dimage; if loss
 * (device float, nullable) is given, writes L there (per-tile shares added
 * in double in a fixed order: deterministic).  Uses the frame's workspace
 * for three per-pixel maps.  EINVAL: gamma outside [0, 1], null
 * images. */
xg_status xg_loss_grad(const xg_frame *f /* [host] */, const float *image, const float *target,
                       float gamma, float *dl_dimage, float *loss, void *stream);

/* Allocation-free form of xg_loss_grad, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, and
 * harnesses that forbid hipMalloc.  Same arguments, results and errors as
 * xg_loss_grad, but the three per-pixel maps and the per-strip loss shares
 * live in a static device array of XG_STATIC_SCRATCH_BYTES held by the
 * library (one copy per device, resident until the process ends) instead
 * of the frame's workspace: f->ws and f->ws_bytes are not read (may be
 * NULL / 0); f->cams and f->cams_dev are.  Allocates and frees nothing;
 * the first call on a device resolves that device's address of the array
 * (the current device must be the one `stream` belongs to).  Every value
 * read from the array is written earlier in the same call, so nothing is
 * cleared.  All calls on one device share the array: calls that overlap
 * in time on one device (different streams, or host threads) race and
 * give undefined results; calls in order on one stream are safe.
 * XG_ECAPACITY (synchronous, nothing enqueued) when 12 * total pixels +
 * 4 * ceil(W / 48) * ceil(H / 8) summed over views exceeds
 * XG_STATIC_SCRATCH_BYTES (e.g. 8 views of 512 x 512 need 25.2 MB). */
#define XG_STATIC_SCRATCH_BYTES (32u << 20)
xg_status xg_loss_grad_static(const xg_frame *f /* [host] */, const float *image, const float *target,
                              float gamma, float *dl_dimage, float *loss, void *stream);

/* L1 term of Eq. 11: dl_dimage[p] = scale * sign(image[p] - target[p])
 * (0 where equal), for n_pixels pixels. */
xg_status xg_l1_grad(const float *image, const float *target, float *dl_dimage,
                     int64_t n_pixels, float scale, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* XG_H */
