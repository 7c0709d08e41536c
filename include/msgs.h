/*
 * msgs.h -- C ABI of libmsgs, a selective multi-scale Gaussian-splatting
 * rasteriser for AMD Instinct MI355X (gfx950).
 *
 * Method: "Multi-Scale 3D Gaussian Splatting for Anti-Aliased Rendering"
 * (Yan, Low, Chen, Lee; CVPR 2024).  A scene of 3D Gaussians, each tagged with
 * a level of detail, is rendered at any resolution by the SelectiveRender
 * procedure (Alg. 2): pixel coverage of every Gaussian (Sec. 4.1), the
 * selection condition with the finest/coarsest exemptions (Sec. 4.1 on selective rendering), an
 * optional range update of S^max/S^min (Sec. 4.1 on selective rendering), then the tile rasteriser of
 * Sec. 3.1 (EWA splatting, 16x16 tiles, depth-sorted front-to-back blending).
 * The backward pass is the exact adjoint of that forward for fixed discrete
 * decisions.
 *
 * Conventions
 *  - Plain C99.  Every pointer documented as "device" is a HIP device address
 *    on the context's device; "host" pointers are ordinary CPU memory.
 *  - `stream` arguments are hipStream_t values passed as void* (NULL = the
 *    null stream).  Work is enqueued asynchronously on that stream unless the
 *    call says it synchronises.
 *  - Return value: MSGS_OK (0) or a negative MSGS_E_* code.  On error no output
 *    is guaranteed, handles stay valid, and msgs_last_error() describes the
 *    failure.
 *  - Planar layout: a per-Gaussian quantity with c components is stored as c
 *    planes of n floats (component-major), e.g. means[3][n].
 *  - Camera: world->camera rotation R (row-major 3x3) and translation t, OpenCV
 *    axes (x right, y down, z forward), pinhole intrinsics given at full
 *    resolution.  A render at downscale d has W_d = floor(W/d), H_d =
 *    floor(H/d) pixels and intrinsics divided by d; pixel (i, j) is sampled at
 *    (i + 1/2, j + 1/2).
 */
#ifndef MSGS_H_
#define MSGS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MSGS_VERSION 1

#define MSGS_OK 0
#define MSGS_E_INVALID (-1)  /* bad argument: null pointer, n < 0, downscale < 1, empty frame, ... */
#define MSGS_E_NOMEM (-2)    /* device memory or the context's pool budget exhausted */
#define MSGS_E_DEVICE (-3)   /* a HIP call failed; its text is in msgs_last_error() */
#define MSGS_E_CAPACITY (-4) /* a fixed capacity (instances, views) was exceeded */
#define MSGS_E_BUSY (-5)     /* a server queue is full */

typedef struct msgs_context msgs_context;
typedef struct msgs_scene msgs_scene;
typedef struct msgs_frame msgs_frame;
typedef struct msgs_server msgs_server;

/* Scene description (Sec. 3.1 Gaussian record; Sec. 4.1: the level and the
 * stored coverage range of selective rendering).  All arrays have n entries
 * per component:
 *   means[3][n]     centres (world units)
 *   scales[3][n]    per-axis standard deviations, linear, > 0
 *   quats[4][n]     rotation quaternion (w, x, y, z), any non-zero length
 *   opacity[n]      density sigma in [0, 1)
 *   sh[(D+1)^2*3][n] spherical-harmonic colour, plane j*3 + c holds real SH
 *                   coefficient j (j = l*l + l + m, orthonormal, no
 *                   Condon-Shortley phase) of channel c; colour = max(0, sum + 1/2)
 *   level[n]        level of detail, 0 = finest (creation downscale 4^level)
 *   s_max[n], s_min[n]  stored pixel-coverage range (px); (0, +inf) means
 *                   "never updated"
 * n in 0 .. 2^30 - 1 (kernels address a plane's element by a 32-bit byte
 * offset); sh_degree D in 0..3; n_levels L in 1..8 with level < L.
 * ptrs_on_device: 1 if all pointers are device addresses, 0 if host. */
typedef struct {
  int64_t n;
  int sh_degree;
  int n_levels;
  const float* means;
  const float* scales;
  const float* quats;
  const float* opacity;
  const float* sh;
  const uint8_t* level;
  float* s_max;
  float* s_min;
  int ptrs_on_device;
} msgs_scene_desc;

typedef struct {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  int width, height;
} msgs_camera;

/* Render options.
 *   downscale    per-side factor d >= 1
 *   selective    1: apply the selection condition of Sec. 4.1 on selective rendering with the level
 *                exemptions; 0: render every Gaussian in front of the camera
 *                (single-scale rendering)
 *   update_range 1: after selection, apply the range update (decays 0.95 and
 *                1.05, Sec. 4.1 on selective rendering) to Gaussians in front of the camera whose
 *                level l satisfies 4^l == downscale; writes the scene's
 *                s_max/s_min in place
 *   lowpass      screen-space dilation h (px^2) added to the projected
 *                covariance, the merged kernel G_{V+V^h} of Sec. 3.2
 *   near_z       near plane (camera-space z)
 *   bg           background colour
 *   profile      1: record HIP events between the pipeline stages on the
 *                render stream (and on the backward's stream) so that
 *                msgs_frame_stats can report per-stage device time */
typedef struct {
  int downscale;
  int selective;
  int update_range;
  float lowpass;
  float near_z;
  float bg[3];
  int profile;
  int no_prefilter;  /* 1: skip the conservative pre-splat bound (results are
                        identical either way; for checks and measurement) */
  long long instance_capacity; /* 0: exact mode, the tile-instance count is read
                        back once per render (one host synchronisation) to
                        size the tile lists.  > 0: fixed capacity, no host
                        synchronisation, so that the render (and its
                        backward) can be captured in a HIP graph; if the
                        frame needs more instances its image is incomplete
                        and msgs_frame_stats returns MSGS_E_CAPACITY.  Not
                        with profile = 1.  Under capture, device blocks come
                        from those the context cached for the capturing
                        stream, else are made in relaxed capture mode; the
                        blocks the captured calls free are kept for later
                        captures on that stream only (never for eager work)
                        until the context is destroyed, which must come after
                        its graphs are destroyed. */
} msgs_render_opts;

typedef struct {
  int64_t n_gaussians;
  int64_t n_selected;   /* in front and passing selection */
  int64_t n_visible;    /* selected with at least one tile */
  int64_t n_instances;  /* (Gaussian, tile) pairs */
  int64_t n_blends;     /* accumulated contributions over all pixels */
  int64_t n_visits;     /* (pixel, instance) pairs up to each pixel's stop position in
                           its tile list (the work of plain tile compositing) */
  int64_t n_evals;      /* (pixel, instance) evaluations the compositing waves spent:
                           per 8x8 quadrant, the list entries that passed its
                           footprint cull up to the point where all its pixels had
                           stopped, times its pixels inside the frame */
  int width, height, tiles_x, tiles_y;
  /* device time (us) per stage when rendered with profile = 1, else 0:
   * [0] projection + selection + compaction  [1] depth sort  [2] tile-count scan
   * [3] emission  [4] tile sort  [5] tile ranges  [6] blending
   * [7] backward blend replay  [8] backward per-Gaussian sum + chain rule
   * [9] whole forward (first to last stage, excluding the host wait)
   * [10] backward: zeroing of the per-instance partials  [11] whole backward */
  float stage_us[12];
  int64_t n_prefiltered; /* Gaussians the pre-splat bound proved unselected
                            (no rotation load, no EWA projection) */
} msgs_stats;

/* Gradient outputs, caller-owned device planar buffers with the scene's
 * layout: dL/d means, dL/d scales (linear), dL/d quats (raw, un-normalised),
 * dL/d opacity (sigma), dL/d sh.  accumulate = 0: written; Gaussians that do
 * not contribute get 0.  accumulate = 1: this frame's gradient is added to
 * the planes and Gaussians that do not contribute are left untouched (a
 * multi-view step zeroes the planes once and accumulates every view; calls
 * that accumulate into the same planes must be ordered, e.g. on one stream). */
typedef struct {
  float* means;
  float* scales;
  float* quats;
  float* opacity;
  float* sh;
  int accumulate;
} msgs_grads;

int msgs_version(void);
/* Text of the last error on the calling thread; owned by the library. */
const char* msgs_last_error(void);
/* Fill `o` with the defaults: downscale 1, selective 1, update_range 0,
 * lowpass 0.3, near_z 0.2, bg 0, profile 0. */
void msgs_default_opts(msgs_render_opts* o);

/* Context: binds a HIP device and a device-memory budget (pool_bytes, 0 = no
 * budget) shared by every frame it renders.  Destroy only after every scene,
 * frame and server created from it. */
int msgs_context_create(int device, size_t pool_bytes, msgs_context** out);
int msgs_context_destroy(msgs_context* ctx);
/* Bytes of device memory the context's frames and scenes hold right now. */
int msgs_context_bytes_in_use(const msgs_context* ctx, size_t* out);

/* Scene.  copy = 1: the library copies every array into HBM it owns (host or
 * device sources; synchronous).  copy = 0: the device pointers are borrowed and
 * must stay valid and unchanged-in-shape until msgs_scene_destroy; their
 * contents may change between renders (training). */
int msgs_scene_create(msgs_context* ctx, const msgs_scene_desc* d, int copy, msgs_scene** out);
int msgs_scene_destroy(msgs_scene* s);
/* Copy the scene's current s_max/s_min to host arrays of n floats (synchronous). */
int msgs_scene_get_ranges(const msgs_scene* s, float* s_max_host, float* s_min_host);

/* Render one view (Alg. 2 followed by the Sec. 3.1 rasteriser).
 *   rgb_out   device [H_d][W_d][3] fp32, caller-owned
 *   frame_out optional; receives the saved state needed by the backward pass
 *             and the debug getters (release with msgs_frame_release).  The
 *             scene must outlive the frame.
 * The call synchronises `stream` once, to size the tile-instance buffers. */
int msgs_render(msgs_context* ctx, msgs_scene* scene, const msgs_camera* cam,
                const msgs_render_opts* opts, float* rgb_out, msgs_frame** frame_out,
                void* stream);

/* Render several views of one scene in one call (the views of a serving batch,
 * or of a multi-scale training step, Sec. 4.1 on multi-scale training and
 * selective rendering).  The projection, coverage, selection and range update
 * of up to 8 views run in one pass over the scene that reads each Gaussian's
 * geometry once; each view's binning, sorts and compositing follow on one
 * of four streams of the library's own that `stream` forks to after the
 * projection and joins back from before the call returns, so that views
 * overlap on the device (a context keeps such streams for up to 64 caller
 * streams; calls on further streams run every view on `stream`).  The frames
 * belong to `stream` (as after msgs_render on it).  Results (images, frames, statistics, and the scene's s_max/s_min
 * when views update ranges) are bit-identical to msgs_render called on the
 * views in order.  Views in exact mode (instance_capacity = 0) share one host
 * synchronisation; with every view in fixed-capacity mode there is none.
 *   cams, opts  host arrays of nviews entries (opts[i].profile must be 0)
 *   rgb_out     host array of nviews device pointers, [H_d][W_d][3] fp32 each
 *   frames_out  optional host array of nviews; receives the frames (release
 *               each with msgs_frame_release)
 *   nviews      1..64 (else MSGS_E_INVALID) */
int msgs_render_views(msgs_context* ctx, msgs_scene* scene, const msgs_camera* cams,
                      const msgs_render_opts* opts, float* const* rgb_out,
                      msgs_frame** frames_out, int nviews, void* stream);

/* Render without allocating: for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The same render as msgs_render with a fixed tile-list capacity
 * (no host synchronisation, no frame kept), but every temporary buffer lives
 * in one device array of MSGS_NOALLOC_SCRATCH_BYTES (256 MiB) that the library
 * holds on each device it runs on until the process ends; the call itself
 * calls no hipMalloc, hipFree or other allocating routine.
 *   opts->instance_capacity  0: as many tile instances as fit in the scratch
 *                (about (256 MiB - per-Gaussian and per-pixel buffers) / 16
 *                bytes; frames of fewer than 128 tiles also keep replay
 *                checkpoints, 64 bytes per instance, and frames of a scene
 *                with more than 8192 Gaussians per tile 4 bytes); > 0: that
 *                capacity, MSGS_E_CAPACITY if it does not fit
 *   counts_out   optional device u64[3]: drawable Gaussians, tile instances the
 *                frame needs, instances that fit (the image is complete when
 *                the last two are equal)
 * Errors: MSGS_E_CAPACITY when the scene (about 90 bytes per Gaussian) and
 * frame (12 bytes per pixel) buffers do not fit in the scratch, or the
 * requested capacity does not; MSGS_E_INVALID as msgs_render, and for
 * profile = 1.  Every call on a device shares that device's scratch and
 * leaves its contents behind: calls whose work overlaps on one device race and
 * must be ordered by the caller (e.g. issued on one stream). */
#define MSGS_NOALLOC_SCRATCH_BYTES (256ull << 20)
int msgs_render_noalloc(msgs_context* ctx, msgs_scene* scene, const msgs_camera* cam,
                        const msgs_render_opts* opts, float* rgb_out,
                        unsigned long long* counts_out, void* stream);

/* Adjoint of msgs_render for the decisions taken in `frame` (selection, tiles,
 * contributor lists, alpha and colour clamps, termination).
 *   dL_drgb  device [H_d][W_d][3] fp32
 *   out      device gradient planes (see msgs_grads)
 * The scene's parameters must not have changed since the render.  The per-tile
 * partial sums are reduced per Gaussian without atomics (deterministic).
 * Stream order: `stream` may differ from the stream the frame was rendered on;
 * the backward then waits for the render's work on the frame's stream, and
 * the frame's stream waits for the backward, so msgs_frame_release may be
 * called right after this call returns (the frame's buffers go back to the
 * context only once the backward has read them).  dL_drgb and the gradient
 * planes are ordered by `stream` alone. */
int msgs_render_backward(msgs_context* ctx, const msgs_frame* frame, const float* dL_drgb,
                         const msgs_grads* out, void* stream);

/* Backward of several renders of one scene (a multi-scale training step, Sec. 4.1,
 * paragraph on multi-scale training and selective rendering:
 * the loss is a sum over views, so the parameter gradients are the sum of the
 * per-view adjoints).  Equivalent to msgs_render_backward on frames[0] with
 * out->accumulate as given, then on frames[1..nviews-1] with accumulate = 1,
 * with bit-identical results: the views' contributions are added in view
 * order in fp32.  The per-view compositing adjoints and partial sums run on
 * four streams of the library's own (view i on stream i mod 4) that `stream`
 * forks to and joins back from (the same streams, and the same limit of 64
 * caller streams, as msgs_render_views); the chain rule then runs on `stream`, reading
 * each Gaussian's parameters and writing its gradients once for up to eight
 * views (more views take further passes).
 *   frames   host array of nviews frames of the same scene and context
 *   dL_drgb  host array of nviews device pointers, [H_d][W_d][3] fp32 each
 *   nviews   >= 1 (else MSGS_E_INVALID)
 * Temporary device memory: 48 bytes per Gaussian per view, and for each of
 * the min(nviews, 4) streams 4 bytes per Gaussian and 36 bytes plus one bit
 * per tile instance of the largest frame that stream takes.  Stream
 * order as for msgs_render_backward, for every frame. */
int msgs_render_backward_views(msgs_context* ctx, const msgs_frame* const* frames,
                               const float* const* dL_drgb, int nviews, const msgs_grads* out,
                               void* stream);

/* Planar Gaussians produced by the library (caller-owned device arrays with
 * room for `cap` Gaussians, same layout as msgs_scene_desc with n = cap). */
typedef struct {
  float* means;    /* [3][cap] */
  float* scales;   /* [3][cap] linear */
  float* quats;    /* [4][cap] unit (w, x, y, z) */
  float* opacity;  /* [cap] */
  float* sh;       /* [3 (D+1)^2][cap] */
  int64_t cap;
} msgs_gaussians;

/* Coarse-level aggregation (Alg. 1 for one target level; supplementary
 * section on the details of Gaussian aggregation):
 *   every Gaussian of a level below `level` is projected with every camera of
 *   `cams` at downscale 4^level; its pixel coverage counts for a camera that
 *   draws it (in front, non-empty level set, at least one tile); Gaussians whose
 *   smallest such coverage is below s_thresh (S_T) are binned by their
 *   normalised position (x / extent inside the cube of half side `extent`,
 *   (2 - extent / m) x / m outside, m the max-norm) on a grid of `grid` voxels
 *   per axis over [-2, 2]^3; each occupied voxel yields one Gaussian: the mean
 *   position, unit rotation, linear scale, opacity and SH of its members, the
 *   scale multiplied by s_thresh / (mean coverage of the members).
 * Defaults (pass 0): s_thresh = 2 px (S_T of Sec. 4.1); extent = the half side
 * of the origin-centred cube holding every camera centre (the extent of the
 * training cameras); grid = floor(400 / (level + 1)) (the paper's (400/l_m)^3
 * grid with 1-based l_m).
 * The new Gaussians are written in ascending voxel order to `out`; *n_out
 * receives their number.  Synchronous.  Errors: MSGS_E_INVALID (level outside
 * [1, n_levels - 1], grid outside [1, 255], negative or NaN threshold, extent
 * or grid, no camera), MSGS_E_CAPACITY (more than out->cap Gaussians: *n_out
 * holds the number needed and nothing is written). */
int msgs_aggregate_level(msgs_context* ctx, msgs_scene* scene, const msgs_camera* cams,
                         int ncams, int level, float s_thresh, float extent, int grid,
                         const msgs_gaussians* out, int64_t* n_out, void* stream);

/* A whole scene as caller-owned device planes of pitch `cap` (room for cap
 * Gaussians): the scene_desc arrays, writable. */
typedef struct {
  float* means;    /* [3][cap] */
  float* scales;   /* [3][cap] */
  float* quats;    /* [4][cap] */
  float* opacity;  /* [cap] */
  float* sh;       /* [3 (D+1)^2][cap] */
  uint8_t* level;  /* [cap] */
  float* s_max;    /* [cap] */
  float* s_min;    /* [cap] */
  int64_t cap;
} msgs_scene_out;

/* Alg. 1 over every coarse level: the base Gaussians (normally all of level
 * 0; host or device arrays, base->ptrs_on_device) are copied to `out`, then for
 * l = 1 .. n_levels - 1 the Gaussians of the levels below l built so far are
 * aggregated as msgs_aggregate_level does (threshold s_thresh, 0 = 2 px; the
 * cameras' extent; floor(400 / (l + 1)) voxels per axis) and appended as level
 * l with the uncalibrated range (s_max 0, s_min +inf).  *n_out receives the
 * scene's size, added[l - 1] the Gaussians level l received (n_levels - 1
 * entries).  Synchronous.  MSGS_E_CAPACITY when `out` cannot hold the scene:
 * *n_out then holds the size needed up to the level that did not fit (a larger
 * out may need more for later levels). */
int msgs_build_levels(msgs_context* ctx, const msgs_scene_desc* base, const msgs_camera* cams,
                      int ncams, int n_levels, float s_thresh, const msgs_scene_out* out,
                      int64_t* n_out, int64_t* added, void* stream);

/* Release a frame (its device memory is returned on the frame's stream). */
int msgs_frame_release(msgs_frame* f);
/* Statistics of a frame (synchronises the frame's stream). */
int msgs_frame_stats(const msgs_frame* f, msgs_stats* out);

/* Debug getters (synchronous, host outputs, caller-owned).
 * selection: mask_host[n] = 1 for Gaussians in front and passing selection.
 * keys: the sorted instance list, key = tile_id * 2^32 + IEEE bits of the
 *   view-space depth, value = Gaussian index; ascending key, ties in ascending
 *   index.  *n receives the count; arrays are filled only if cap >= count.
 * state: per pixel [H_d][W_d] final transmittance and number of accumulated
 *   contributions.
 * ranges: per tile [tiles][2] half-open range in the sorted list, (0,0) when
 *   empty; filled only if cap >= tiles. */
int msgs_frame_get_selection(const msgs_frame* f, uint8_t* mask_host);
int msgs_frame_get_keys(const msgs_frame* f, uint64_t* keys, uint32_t* vals, size_t cap,
                        size_t* n);
int msgs_frame_get_state(const msgs_frame* f, float* T_final, uint32_t* n_contrib);
int msgs_frame_get_ranges(const msgs_frame* f, uint32_t* ranges, size_t cap, size_t* n);

/* ------------------------------------------------------------------ serving
 * Continuous-batching server over one resident scene.  max_inflight slots,
 * each a host worker thread with its own HIP stream, take queued requests in
 * FIFO order as soon as they are free, so requests that arrive while others
 * are on the GPU run concurrently with them.  Admission is by device memory:
 * a request's frame allocates from the context budget (per-Gaussian buffers,
 * then its tile lists once their length is known) and waits for other
 * requests to return memory when it does not fit; if all in-flight requests
 * wait, all but the oldest release theirs and go back to the head of the
 * queue.  A request that cannot fit alone completes with MSGS_E_NOMEM.  Range
 * updates are not allowed through the server (results would depend on the
 * interleaving).  The scene and the output buffers must stay valid until the
 * request completes.  Times are host steady-clock microseconds since the
 * server was created. */
typedef struct {
  uint64_t req_id;
  int status;          /* MSGS_OK or the request's error code */
  double t_submit_us;  /* msgs_server_submit returned */
  double t_admit_us;   /* per-Gaussian buffers allocated, first kernels enqueued */
  double t_start_us;   /* a slot took the request */
  double t_done_us;    /* output complete on the device, observed by the slot */
  int64_t n_blends;
} msgs_completion;

int msgs_server_create(msgs_context* ctx, msgs_scene* scene, int max_inflight,
                       msgs_server** out);
/* Queue one render into rgb_out (device [H_d][W_d][3]); MSGS_E_BUSY when the
 * queue (65536 requests) is full, MSGS_E_INVALID for a bad camera/options. */
int msgs_server_submit(msgs_server* s, const msgs_camera* cam, const msgs_render_opts* opts,
                       float* rgb_out, uint64_t req_id);
/* Up to `max` completions; waits up to timeout_us for the first one. */
int msgs_server_poll(msgs_server* s, msgs_completion* out, int max, int* n, int timeout_us);
/* Requests waiting in the queue and requests being rendered. */
int msgs_server_pending(msgs_server* s, int* queued, int* inflight);
/* Finishes the in-flight requests, drops the queued ones, joins the slots. */
int msgs_server_destroy(msgs_server* s);

/* Device evaluation of the library's fp32 exp (domain [-5.6, 0]) and log
 * (domain (1, 256)) used by selection and blending, on device arrays of n
 * floats.  For verification of the numerics contract. */
int msgs_debug_exp(const float* x, float* y, int64_t n, void* stream);
int msgs_debug_log(const float* x, float* y, int64_t n, void* stream);
/* The library's stable LSD radix sort of (u32 key, u32 value) pairs by key
 * bits [begin_bit, end_bit), in place on device arrays of nmax entries.  Sorts
 * the first min(*d_n, nmax) entries when d_n (device u32) is non-null, else
 * all nmax; entries past the count are left unspecified.  The sort that orders
 * Gaussians by depth and tile instances by tile (Sec. 3.1); for verification.
 * Temporary memory comes from the context.  Synchronises `stream`. */
int msgs_debug_sort_pairs(msgs_context* ctx, uint32_t* keys, uint32_t* vals, const uint32_t* d_n,
                          int64_t nmax, int begin_bit, int end_bit, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* MSGS_H_ */
