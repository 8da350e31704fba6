/*
 * omnigs.h -- C ABI of libomnigs.so, the MI355X (gfx950) rasterizer that
 * splats 3D Gaussians onto an equirectangular (ERP) image through the
 * spherical camera model of OmniGS (arXiv 2404.03202, Sec. 3), and its
 * backward pass.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Pointers documented "device" are HIP device addresses; "host" are
 *   ordinary CPU pointers read during the call only.
 * - `stream` is a hipStream_t passed as void*; NULL means the legacy default
 *   stream.  All GPU work is enqueued on it.  Calls do not synchronise the
 *   stream except where stated (the instance-count readback of
 *   omnigs_forward).
 * - The caller owns every buffer.  Device memory the library needs beyond
 *   the caller's inputs and outputs is obtained through the caller's
 *   allocator callback and never freed by the library:
 *     OMNIGS_MEM_SCRATCH allocations are dead once every kernel the call
 *       enqueued has run (a stream-ordered caching allocator may recycle
 *       them as soon as the call returns);
 *     OMNIGS_MEM_STATE allocations back an omnigs_state and must stay alive
 *       until the last omnigs_backward that uses that state has run.
 *   omnigs_backward_noalloc is the exception: it allocates nothing and takes
 *   its scratch from a fixed device array of the library.
 * - Errors: every entry point returns an omnigs_status.  On a non-OK status
 *   nothing valid was produced, and omnigs_last_error() returns a
 *   thread-local message.  No exception crosses the ABI.
 * - Image layout is planar [3][H][W] float32, row-major, pixel (x, y) sampled
 *   at the continuous ERP coordinate (x + 1/2, y + 1/2) (Eq. 5).
 * - Requirements: width % 16 == 0 (16x16 tiles that wrap across the
 *   longitude seam), width <= 65520 and 1 <= height <= 65520.
 */
#ifndef OMNIGS_H
#define OMNIGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    OMNIGS_OK = 0,
    OMNIGS_ERR_INVALID = 1,  /* bad argument (null pointer, size, degree, non-finite camera, ...) */
    OMNIGS_ERR_ALLOC = 2,    /* the allocator callback returned NULL */
    OMNIGS_ERR_HIP = 3,      /* a HIP runtime call or kernel launch failed */
    OMNIGS_ERR_CAPACITY = 4  /* more tile instances than the caller's capacity */
} omnigs_status;

enum { OMNIGS_MEM_SCRATCH = 0, OMNIGS_MEM_STATE = 1 };

/* Device allocator: returns `bytes` of device memory aligned to 256 bytes,
 * or NULL.  `kind` is OMNIGS_MEM_SCRATCH or OMNIGS_MEM_STATE. */
typedef void *(*omnigs_alloc_fn)(void *user, size_t bytes, int32_t kind);
typedef struct {
    omnigs_alloc_fn alloc;
    void *user;
} omnigs_allocator;

/* The Gaussian set (Sec. 3.1): centre m, scale S, rotation q, opacity o and
 * SH colour coefficients.  All device, float32, densely packed. */
typedef struct {
    const float *means;     /* [n][3] world positions m                              */
    const float *scales;    /* [n][3] activated (positive) scales S                  */
    const float *quats;     /* [n][4] rotation q = (w, x, y, z); normalised inside   */
    const float *opacities; /* [n]    activated opacity o in (0, 1)                  */
    const float *sh;        /* [n][sh_coeffs][3] real SH, index l*l+l+m, RGB last     */
    int64_t n;              /* 0 <= n < 2^31                                          */
    int32_t sh_degree;      /* active degree D, 0..3                                  */
    int32_t sh_coeffs;      /* stored coefficients per Gaussian: (D+1)^2 <= it <= 16 */
} omnigs_gaussians;

/* Camera models. */
#define OMNIGS_CAMERA_ERP 0     /* equirectangular image of Eq. 3-5 (the paper's) */
#define OMNIGS_CAMERA_PINHOLE 1 /* perspective image of Eq. 2 (perspective crops) */

/* Camera pose T_cw of Eq. 1 (host, float64): t = R_cw m + t_cw, camera axes
 * +X right, +Y down, +Z forward (Fig. 2); for the ERP camera the X-Z plane is
 * the equator.  A zero-initialised model selects the ERP camera.
 *   ERP:     width a multiple of 16 (the seam wraps whole tile columns);
 *            Gaussians ordered by t_r; the fx..cy fields are ignored.
 *   PINHOLE: p = (fx t_x / t_z + cx, fy t_y / t_z + cy) (Eq. 2), pixel (x, y)
 *            sampled at (x + 1/2, y + 1/2); any width (the last tile column
 *            may be partial); Gaussians ordered by t_z; t_z <= near_plane
 *            culled; fx, fy > 0 and cx, cy finite (pixels).
 * rows: the number of image rows rendered, from the top (0 = all H).  The
 * mapping still uses H; the outputs then have `rows` rows and the rows below
 * cost nothing, forward or backward (the paper's 360Roam evaluation leaves
 * the bottom rows out of the loss, Sec. 4).
 * OMNIGS_ERR_INVALID for an unknown model, rows outside [0, H] or bad
 * intrinsics. */
typedef struct {
    double R_cw[9]; /* row-major rotation W of Eq. 1 */
    double t_cw[3];
    int32_t width;  /* image W, <= 65520 */
    int32_t height; /* image H, <= 65520 */
    int32_t model;  /* OMNIGS_CAMERA_ERP or OMNIGS_CAMERA_PINHOLE */
    int32_t rows;   /* rendered rows from the top, 0 = all */
    double fx, fy, cx, cy; /* pinhole intrinsics of Eq. 2 */
} omnigs_camera;

/* Rasterisation settings (host).  The paper fixes the stop threshold (Sec.
 * 3.3, "alpha = 0.9999", i.e. T_min = 1e-4); the others are this library's
 * readings, with the defaults given by omnigs_default_settings():
 *   alpha_min 1/255, alpha_max 0.99, T_min 1e-4, dilation 0.3 px^2,
 *   near_plane 0.2, bg = 0. */
typedef struct {
    double alpha_min;  /* instances with alpha < alpha_min are skipped                 */
    double alpha_max;  /* alpha is clamped to alpha_max                                  */
    double T_min;      /* stop before an instance that would bring T below T_min        */
    double dilation;   /* added to the diagonal of the 2D covariance (px^2)             */
    double near_plane; /* Gaussians with t_r <= near_plane are culled                    */
    double bg[3];      /* background colour seen through the final transmittance       */
} omnigs_settings;

/* Per-pixel outputs of the forward pass (device, caller-allocated; H is the
 * rendered rows).  The alpha image is 1 - final_T. */
typedef struct {
    float *image;       /* [3][H][W]  C + T_final * bg  (Eq. 6)                   */
    float *final_T;     /* [H][W]     transmittance after the last blended one   */
    int32_t *n_contrib; /* [H][W]     1 + tile-list position of the last blended */
    int32_t *n_blended; /* [H][W]     instances blended (alpha >= alpha_min);
                           optional: NULL skips it                              */
    float *depth;       /* [H][W]     depth image sum_i d_i alpha_i T_i, d the
                           sort depth (t_r, or t_z for a pinhole camera), not
                           normalised by the alpha; optional: NULL skips it    */
} omnigs_image_out;

/* Saved forward state (filled by omnigs_forward, read by omnigs_backward).
 * The buffers are OMNIGS_MEM_STATE allocations from the caller's allocator;
 * the typed views below point into them. */
typedef struct {
    int64_t n;           /* Gaussians                                    */
    int64_t n_instances; /* M: (Gaussian, covered tile) instances         */
    int64_t n_entries;   /* S: (Gaussian, touched 8x8-tile block) entries  */
    int32_t width, height, tiles_x, tiles_y; /* height: the rendered rows */
    const void *records;         /* [n] 48-byte blend records (opaque)              */
    const uint32_t *n_tiles;     /* [n] tiles covered per Gaussian, 0 when culled    */
    const uint32_t *depth_order; /* [n] Gaussian ids sorted by (t_r, id), culled last */
    const uint32_t *inst_gauss;  /* [M] Gaussian ids: each tile's list contiguous,
                                    in (t_r, id) order; tiles stored 8x8 block
                                    by 8x8 block                                    */
    const uint32_t *tile_range;  /* [tiles][2] [start, end) of tile ty*tiles_x+tx
                                    in inst_gauss                                   */
    const uint32_t *tile_work;   /* [tiles] largest n_contrib of the tile (the
                                    backward's walk length)                        */
    const float *radii;          /* [n] screen radius in pixels (the larger half
                                    extent of the alpha = alpha_min box), 0 when
                                    culled                                          */
    const float *depth;          /* [n] sort depth d (t_r or t_z) of each Gaussian */
    const uint32_t *counts;      /* [3] S and M as counted on the device, then
                                    fault bits (bit 0: a lookback wait of the sort
                                    or scan gave up; the lists are then invalid)
                                    (device words; n_entries and n_instances are
                                    -1 when the call read nothing back)             */
    const uint8_t *inst_quad;    /* [M] per instance, the 8x8 quadrants of its tile
                                    that its alpha >= alpha_min region can reach
                                    (bits 0-3, quadrant 2*row + column), written
                                    by the forward's blend for each instance it
                                    walked; the backward reads them instead of
                                    testing again.  NULL (a state built by hand):
                                    the backward tests                             */
} omnigs_state;

/* Capacities of a forward call that reads nothing back (host struct).  With
 * instances > 0 the instance buffers hold that many (Gaussian, tile)
 * instances and the block-entry buffers `entries` (Gaussian, 8x8-tile
 * block) entries (entries == 0: as many as instances; S <= M always), the
 * counts stay on the device and the call only enqueues work.  If M or S
 * exceeds its capacity the call still stays within its buffers, but its
 * outputs (and a backward from its state) are invalid and *overflow is 1.
 * overflow (device int32, may be NULL) is set on the call's stream to 0, or
 * to a nonzero value when the outputs are invalid: bit 0 a capacity was
 * exceeded, bit 1 a lookback wait of the sort or scan gave up (see
 * omnigs_selftest_lookback).
 * Both capacities must stay below 2^31 - 1. */
typedef struct {
    int64_t instances;
    int64_t entries;
    int32_t *overflow;
} omnigs_capacity;

/* Parameter gradients (device, caller-allocated, overwritten). */
typedef struct {
    float *dmeans;     /* [n][3]                                                  */
    float *dscales;    /* [n][3]  w.r.t. the activated scales                     */
    float *dquats;     /* [n][4]  w.r.t. the raw quaternion                       */
    float *dopacities; /* [n]     w.r.t. the activated opacity                    */
    float *dsh;        /* [n][sh_coeffs][3]; coefficients above degree D are 0    */
    float *dscreen;    /* [n][2]  dL/ds, s the uniform screen coordinate (Eq. 4) */
} omnigs_grads;

/* Default settings (see omnigs_settings). */
omnigs_settings omnigs_default_settings(void);

/* Forward render of the ERP image (Sec. 3.3).
 * Stages, each a HIP kernel on `stream`:
 *   1. project: Eq. 1 (world -> camera), Eq. 3-5 (ERP pixel), Eq. 9-16
 *      (2D covariance through the spherical Jacobian), SH colour, and the
 *      radius of influence (the box of the alpha = alpha_min iso-ellipse),
 *      with its tile span wrapped across the longitude seam;
 *   2. depth sort of the Gaussians by t_r (Sec. 3.3: ERP sorts by distance,
 *      not t_z), then one instance per (Gaussian, covered tile), in two
 *      levels: an entry per touched block of 8x8 tiles, emitted in depth
 *      order and stably sorted by block, then each block's list expanded
 *      into its tiles' lists (each instance written once): each tile's list
 *      is in (t_r, id) order; per-tile [start, end) ranges;
 *   3. front-to-back alpha blending of Eq. 6-8, one 16x16 tile per
 *      workgroup, stopping per pixel before T would drop below T_min.
 * cap == NULL or cap->instances == 0: the instance counts are read back to
 * size the instance buffers, the only host synchronisation of the call;
 * otherwise the buffers take the capacities of *cap and nothing is read
 * back (see omnigs_capacity).
 * Inputs: g (device arrays), cam and s (host).  Outputs: out (device,
 * caller-allocated) and *state (host struct; device buffers from `alloc`).
 * Returns OMNIGS_ERR_INVALID for null pointers, n < 0, sh_degree outside
 * 0..3, sh_coeffs out of range, width % 16 != 0, height outside [1, 65520] or a non-finite
 * camera; OMNIGS_ERR_ALLOC if `alloc` fails; OMNIGS_ERR_HIP on a runtime
 * failure. */
omnigs_status omnigs_forward(const omnigs_gaussians *g, const omnigs_camera *cam, const omnigs_settings *s,
                             omnigs_allocator alloc, omnigs_image_out *out, omnigs_state *state,
                             const omnigs_capacity *cap, void *stream);

/* Backward pass of the render (Sec. 3.4, Eq. 18-20) for an image-space
 * cotangent dL_dimage [3][H][W] (device) and, each optional (NULL), the
 * cotangents dL_ddepth [H][W] of the depth image and dL_dalpha [H][W] of the
 * alpha image 1 - final_T: both flow back as colour channels with colour d_i
 * (respectively 1) over a black background, and dL/dd_i reaches the mean
 * through d t_r / dt = t / t_r (t_z: (0, 0, 1)).  Re-walks each pixel's tile list
 * back to front from the saved final T and n_contrib (recomputing alpha and
 * T rather than reading stored per-pixel lists), accumulates per-Gaussian
 * dL/dp, dL/dSigma2D^-1, dL/do, dL/dcolour with one atomic per field per
 * (tile, Gaussian), then chains them per Gaussian through the omnidirectional
 * terms dSigma2D/dSigma, dJ/dt, dp/ds, ds/dt to means, scales, quaternions,
 * opacities and SH.  g, cam and s must be those of the forward call that
 * produced `state` and `fwd`.  Gradients are overwritten.  Zero gradient
 * flows through the alpha_max clamp and through colour channels clamped at 0.
 * Scratch (the accumulators) comes from `alloc`.  Errors as omnigs_forward. */
omnigs_status omnigs_backward(const omnigs_gaussians *g, const omnigs_camera *cam, const omnigs_settings *s,
                              const omnigs_state *state, const omnigs_image_out *fwd, const float *dL_dimage,
                              const float *dL_ddepth, const float *dL_dalpha, omnigs_grads *grads,
                              omnigs_allocator alloc, void *stream);

/* omnigs_backward for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving or training loops, harnesses that forbid
 * hipMalloc): the same checks, kernels and results, with the gradient
 * accumulators and the tile launch order in a fixed 64 MiB device array of
 * the library instead of `alloc` scratch; no device memory is allocated.
 * It holds (10 n + tiles) 32-bit words, about 1.6M Gaussians at 2048x1024;
 * a larger call returns OMNIGS_ERR_INVALID before enqueuing anything.  Each
 * device has its own array, shared by every call on that device and cleared
 * by each call before use: calls that overlap on one device (other streams,
 * other host threads) race and must be serialised by the caller.  Arguments,
 * outputs and other errors as omnigs_backward. */
omnigs_status omnigs_backward_noalloc(const omnigs_gaussians *g, const omnigs_camera *cam, const omnigs_settings *s,
                                      const omnigs_state *state, const omnigs_image_out *fwd, const float *dL_dimage,
                                      const float *dL_ddepth, const float *dL_dalpha, omnigs_grads *grads,
                                      void *stream);

/* L1 photometric term of Eq. 17 (lambda = 0): *loss = mean |image - target|
 * over `count` float32 entries, and dL_dimage = sign(image - target) / count
 * with sign(0) = 0.  image, target, dL_dimage (may be NULL) and loss are
 * device pointers; the sum is reduced in a fixed order (deterministic).
 * Scratch comes from `alloc`. */
omnigs_status omnigs_l1_loss(const float *image, const float *target, int64_t count, float *dL_dimage, float *loss,
                             omnigs_allocator alloc, void *stream);

/* Photometric loss of Eq. 17, L = (1 - lambda) L1 + lambda (1 - SSIM), for
 * [channels][height][width] float32 images (device): L1 is the mean |image -
 * target|; SSIM is the mean over channels and pixels of the structural
 * similarity on 11x11 Gaussian windows (sigma 1.5; C1 = 0.01^2, C2 = 0.03^2)
 * over zero-padded images (the paper gives the weight lambda in its absent
 * supplement: a parameter here).  mask (device, [height][width], may be
 * NULL): per-pixel loss weights m >= 0 with a positive sum, shared by the
 * channels: both means become m-weighted, L1 = sum m |x - y| / (C sum m) and
 * SSIM = sum m S / (C sum m), the windows still over the whole images (the
 * paper leaves the 360Roam images' bottom rows out of the loss, Sec. 4; a
 * camera's `rows` skips such rows outright).  *loss (device) receives L and
 * dL_dimage (device, may be NULL) its gradient.  Scratch comes from `alloc`:
 * per-tile partial sums, plus with a gradient 12 bytes per image element
 * (three window-filtered planes).
 * OMNIGS_ERR_INVALID for null pointers, sizes < 1 or lambda outside [0, 1]. */
omnigs_status omnigs_photometric_loss(const float *image, const float *target, int32_t channels, int32_t height,
                                      int32_t width, double lambda, const float *mask, float *dL_dimage, float *loss,
                                      omnigs_allocator alloc, void *stream);

/* Batched forward render of `batch` cameras (1 <= batch <= OMNIGS_MAX_BATCH,
 * mixed resolutions) over one resident Gaussian set: the path of
 * omnigs_forward (Sec. 3.2-3.3) run once for all of them.  One projection
 * launch covers every (camera, Gaussian) pair; one depth sort orders all of
 * them; block entries and instances are emitted into the concatenation of
 * the cameras' block and tile spaces (camera b's follow those of cameras
 * 0..b-1), so one binning pass and one blend launch serve the whole batch.  A tile's list holds the same
 * records in the same order as when its camera is rendered alone, so every
 * output equals that of omnigs_forward for the camera, bit for bit.
 * cams[b] (host) and outs[b] (device, caller-allocated) per camera.
 * instance_capacity == 0: the total instance count M is read back to size
 *   the instance buffers (one host synchronisation of `stream`).
 * instance_capacity > 0: the instance buffers hold that many instances and
 *   nothing is read back (no host synchronisation: the call only enqueues);
 *   if M exceeds it, the call still stays within its buffers, but the
 *   outputs are invalid and *overflow is 1.
 * overflow (device int32, may be NULL) is set on `stream` to 0, or nonzero
 * with the bits of omnigs_capacity's overflow.
 * n_instances (host, may be NULL) receives M when it was read back, else -1.
 * M must stay below 2^32.  No backward state is kept; all memory beyond the
 * outputs is OMNIGS_MEM_SCRATCH.  Errors as omnigs_forward, plus
 * OMNIGS_ERR_INVALID for batch out of range or batch * n >= 2^32. */
#define OMNIGS_MAX_BATCH 16
omnigs_status omnigs_forward_batch(const omnigs_gaussians *g, const omnigs_camera *cams, int32_t batch,
                                   const omnigs_settings *s, omnigs_allocator alloc, omnigs_image_out *outs,
                                   int64_t instance_capacity, int32_t *overflow, int64_t *n_instances,
                                   void *stream);

/* Device bytes that omnigs_forward_batch with these cameras (host, checked
 * as there), n Gaussians and instance_capacity > 0 requests from its
 * allocator (the sum of its requests, each rounded up to 256 bytes), so that
 * a scheduler can admit a batch by HBM footprint before enqueuing it; the
 * caller's outputs come on top.  Host arithmetic only: nothing is enqueued.
 * OMNIGS_ERR_INVALID for n outside [0, 2^31), instance_capacity outside
 * [1, 2^32), batch out of range, a bad camera or batch * n >= 2^32. */
omnigs_status omnigs_forward_batch_bytes(int64_t n, const omnigs_camera *cams, int32_t batch,
                                         int64_t instance_capacity, uint64_t *bytes);

/* ------------------------------------------------------------------------
 * Optimisation around the rasterizer (Sec. 4, Alg. 1).  The paper leaves
 * the optimizer and the densification rules to 3DGS (and to its absent
 * supplement), except that densification is driven by dL/ds, the gradient
 * w.r.t. the uniform ERP screen coordinate s of Eq. 4.  This library takes
 * 3DGS's published method: Adam on raw parameters, the mean of ||dL/ds||
 * over the views where a Gaussian is visible, clone / split / prune, and a
 * periodic opacity reset.
 * ------------------------------------------------------------------------ */

/* Raw (optimised) parameters, device float32, densely packed: the
 * rasterizer sees S = exp(log_scales) and o = sigmoid(logits).  The same
 * struct describes the two Adam moment sets (same shapes). */
typedef struct {
    float *means;      /* [n][3]                                     */
    float *log_scales; /* [n][3]                                     */
    float *quats;      /* [n][4]  raw, normalised by the rasterizer  */
    float *logits;     /* [n]                                        */
    float *sh;         /* [n][sh_coeffs][3]                          */
    int64_t n;
    int32_t sh_degree;
    int32_t sh_coeffs;
} omnigs_params;

/* Adam settings (host).  Learning rates per group: means, SH degree 0, SH
 * degrees >= 1, opacity logits, log-scales, quaternions.  step counts from
 * 1 (bias correction 1 - beta^step). */
typedef struct {
    double lr_means, lr_sh_dc, lr_sh_rest, lr_logits, lr_log_scales, lr_quats;
    double beta1, beta2, eps;
    int32_t step;
} omnigs_adam_settings;

/* Densification statistics (device float32, [n] each). */
typedef struct {
    float *accum;      /* sum of ||dL/ds||_2 over the views where visible */
    float *denom;      /* number of those views                           */
    float *max_radius; /* largest screen radius in pixels seen            */
} omnigs_densify_stats;

/* Densification settings (host).  max_screen <= 0 disables pruning by
 * screen radius and by world size. */
typedef struct {
    double grad_threshold; /* tau: densify where accum / denom >= tau                */
    double percent_dense;  /* clone where max scale <= percent_dense * extent, else split */
    double extent;         /* scene extent (world units)                              */
    double min_opacity;    /* prune where o < min_opacity                             */
    double max_screen;     /* prune where max_radius > max_screen (pixels)            */
    double big_fraction;   /* prune where max scale > big_fraction * extent           */
    double split_shrink;   /* children's scales are the parent's / split_shrink (1.6) */
} omnigs_densify_settings;

/* One Adam step over every parameter (elementwise, float32): the gradients
 * `g` (w.r.t. the activated scales and opacities, as omnigs_backward writes
 * them) are chained through exp and sigmoid; m <- b1 m + (1 - b1) g,
 * v <- b2 v + (1 - b2) g^2, p <- p - lr / (1 - b1^t) m / (sqrt(v) /
 * sqrt(1 - b2^t) + eps).  p, m1, m2 are updated in place.  act (may be NULL)
 * receives the rasterizer's inputs for the new parameters: act->scales =
 * exp(log_scales), act->opacities = sigmoid(logits) (its other pointers are
 * not written).  skip (device int32, may be NULL): when *skip is nonzero on
 * the stream the step writes nothing (pass a forward's overflow flag so that
 * an iteration whose forward overflowed its capacities leaves the
 * parameters, moments and activations as they were).  Errors:
 * OMNIGS_ERR_INVALID for null pointers or mismatched sizes. */
omnigs_status omnigs_adam_step(omnigs_params *p, const omnigs_grads *g, omnigs_params *m1, omnigs_params *m2,
                               const omnigs_adam_settings *s, omnigs_gaussians *act, const int32_t *skip,
                               void *stream);

/* Densification statistics of one view: for every Gaussian the forward
 * `state` saw covering a tile, accum += ||dscreen||_2, denom += 1 and
 * max_radius = max(max_radius, its screen radius in pixels (the larger half
 * extent of the alpha = alpha_min box)).  g->dscreen from omnigs_backward
 * of that view.  skip (device int32, may be NULL): as for omnigs_adam_step. */
omnigs_status omnigs_accumulate_stats(const omnigs_state *state, const omnigs_grads *g,
                                      omnigs_densify_stats *stats, const int32_t *skip, void *stream);

/* Densify and prune (see the section comment; decisions in float32: the
 * averaged gradient by float32 division, scales and opacities compared in
 * log / logit space against thresholds rounded once to float32).  Output
 * order: surviving originals, surviving clones, surviving first children,
 * surviving second children, each in input order.  noise: device [n][2][3]
 * standard normals (children at m + R(q) (S * z)).  The new arrays (p_out,
 * m1_out, m2_out, stats_out; their pointer fields are set by the call) are
 * OMNIGS_MEM_STATE allocations of the caller's allocator; new Gaussians get
 * zero moments, and all statistics start at zero.  *n_out receives the new
 * count (read back: one host synchronisation). */
omnigs_status omnigs_densify(const omnigs_params *p, const omnigs_params *m1, const omnigs_params *m2,
                             const omnigs_densify_stats *stats, const float *noise, const omnigs_densify_settings *s,
                             omnigs_allocator alloc, omnigs_params *p_out, omnigs_params *m1_out,
                             omnigs_params *m2_out, omnigs_densify_stats *stats_out, int64_t *n_out, void *stream);

/* Opacity reset: logits <- min(logits, logit(value)); the logits' Adam
 * moments are zeroed. */
omnigs_status omnigs_reset_opacity(omnigs_params *p, omnigs_params *m1, omnigs_params *m2, double value,
                                   void *stream);

/* Self-test of the failure signalling of the single-pass sort and scan
 * (Sec. 3.3's depth sort and the tile-list binning run on them).  Their
 * decoupled lookback polls the status word of an earlier workgroup until it
 * is published; the poll count is bounded so that a kernel always ends, and
 * a wait that reaches the bound sets a fault bit that the forward calls
 * surface (omnigs_forward and omnigs_forward_batch fail with
 * OMNIGS_ERR_HIP when they read counts back, else set bit 1 (value 2) of
 * *overflow; omnigs_densify fails).  This call runs one primitive on n
 * device-generated keys with the poll bound lowered to max_polls (0: the
 * library's bound; 1: a wait gives up at its first unpublished word),
 * then restores the bound: primitive 0 sorts n 32-bit keys (key, index
 * pairs), 1 scans n values in [0, 15].  *fault (host) receives the fault
 * bits, *correct (host) 1 when the result checked on the host is exact
 * (a wait that gave up leaves a wrong prefix: then normally 0).  Buffers
 * come from `alloc`; the call synchronises `stream`.  Not to be called
 * while other threads launch library work (the bound is process-wide).
 * OMNIGS_ERR_INVALID for primitive not 0 or 1, n outside [1, 2^26] or null
 * outputs. */
omnigs_status omnigs_selftest_lookback(int32_t primitive, int64_t n, uint32_t max_polls, omnigs_allocator alloc,
                                       uint32_t *fault, int32_t *correct, void *stream);

/* Binning path selection, for tests.  The tile binning (Sec. 3.3) takes each
 * (Gaussian, 8x8-tile block) entry's covered tiles from the upper 16 bits of
 * its sort key while a call's images hold at most `blocks` blocks (default
 * and maximum 65536, which keeps the block ids within the lower 16 bits),
 * and from the Gaussians' tile rectangles otherwise; both give the same
 * tile lists.  The same bound (and fewer than 8192 blocks) selects the
 * one-workgroup split of the block lists into chunks over the three-kernel
 * one, again with the same result.  blocks = 0 restores the default, larger
 * values are clamped
 * to it.  Process-wide, like omnigs_selftest_lookback's bound: not to be
 * called while other threads launch library work.  Always OMNIGS_OK. */
omnigs_status omnigs_set_cover_key_blocks(uint32_t blocks);

/* Measured ceilings of the device that `stream` runs on, against which the
 * stages are quoted: the blends are bound by FP32 issue (Sec. 3.3-3.4 do a
 * few dozen scalar operations and one exp per pixel-instance pair), the
 * backward also by the float atomics that merge per-tile gradient sums, the
 * projection, sorting and binning stages by HBM bandwidth.  Each figure is
 * the mean over `repeats` launches (>= 1) of one kernel, after a warm-up
 * launch, timed with HIP events on `stream` (the call synchronises):
 *   fma_tflops   non-packed FP32 FMAs (2 FLOP each), 16 independent chains
 *                per lane, 128 waves per CU;
 *   exp_gops     exp2 results per second (1e9), same shape;
 *   atomic_gops  float atomic adds to hashed addresses spread over
 *                `atomic_words` words (1e9 per second; 0 skips it);
 *   copy_gbps    a float4 copy of `copy_bytes` bytes, read + written bytes
 *                per second (1e9; 0 skips it).
 * Buffers (atomic_words * 4 and 2 * copy_bytes bytes) come from `alloc` as
 * OMNIGS_MEM_SCRATCH.  OMNIGS_ERR_INVALID for repeats < 1, atomic_words
 * >= 2^32 or copy_bytes not a multiple of 16. */
typedef struct {
    double fma_tflops;
    double exp_gops;
    double atomic_gops;
    double copy_gbps;
} omnigs_ceilings;
omnigs_status omnigs_measure_ceilings(int64_t atomic_words, int64_t copy_bytes, int32_t repeats,
                                      omnigs_allocator alloc, omnigs_ceilings *out, void *stream);

/* Thread-local message describing the last non-OK status of this thread. */
const char *omnigs_last_error(void);

/* Stage timing.  Bit k of `stages` enables stage k (0 disables all,
 * OMNIGS_PROFILE_ALL every stage): each enabled stage is bracketed with HIP
 * events on the call's stream and its GPU time is accumulated per stage until
 * omnigs_profile_read (which synchronises the recorded events, then resets
 * the accumulators).  Recording an event costs the stream a few microseconds,
 * so a throughput measurement enables only the stages it reports.  Stages:
 * see omnigs_profile_stage_name. */
#define OMNIGS_PROFILE_ALL 0xffffffffu
omnigs_status omnigs_profile_enable(uint32_t stages);
int32_t omnigs_profile_num_stages(void);
const char *omnigs_profile_stage_name(int32_t stage);
/* ms[k] = total ms of stage k since the last read, launches[k] = number of
 * timed launches; arrays of omnigs_profile_num_stages() entries (host). */
omnigs_status omnigs_profile_read(double *ms, int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* OMNIGS_H */
