/*
 * mvp.h - C ABI of the MI355X ray marcher for mixtures of volumetric primitives.
 *
 * The library renders images of a set of oriented voxel primitives
 * (Lombardi et al., "Mixture of Volumetric Primitives for Efficient Neural
 * Rendering", ACM TOG 40(4), 2021) and differentiates them:
 *
 *   - a primitive k is {t_k, R_k, s_k, V_k}: position, rotation, per-axis scale
 *     and an RGBA payload grid of M^3 voxels; t, R and s form its
 *     model-to-world transform (Sec. 3.1.2);
 *   - a pixel ray r(t) = o + t d is marched at fixed world-space steps, only
 *     against the primitives it intersects, between the first entry and the
 *     last exit (Sec. 3.2.1);
 *   - colour and opacity are accumulated front to back with the additive,
 *     clamped rule I = int V_col dT, T = min(int V_alpha, 1), A = T(t_max),
 *     stopping once T > 1 - eps_early (Sec. 3.2.2).
 *
 * Conventions (all calls):
 *   - Pointers are DEVICE pointers unless marked "host".  The caller owns every
 *     buffer it passes; the library never frees them.  The library owns
 *     contexts, acceleration structures and resident serving scenes.
 *   - Work is enqueued on the given HIP stream (hipStream_t passed as void*;
 *     NULL is the null stream) and returns without waiting, except where a
 *     call says it blocks.
 *   - Argument errors return MVP_ERR_INVALID synchronously and enqueue nothing.
 *     A failed HIP call returns MVP_ERR_DEVICE; out-of-memory returns
 *     MVP_ERR_OOM.  mvp_last_error() then holds a message.  No C++ exception
 *     crosses this boundary.
 *   - Preconditions not checked on the device: payload values finite with
 *     opacity >= 0, scales > 0, rotations finite.
 */
#ifndef MVP_H
#define MVP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MVP_OK = 0,
  MVP_ERR_INVALID = 1,   /* bad argument, unknown handle or ticket            */
  MVP_ERR_OOM = 2,       /* device memory or the serving budget is exhausted   */
  MVP_ERR_DEVICE = 3,    /* a HIP call failed                                  */
  MVP_ERR_BUSY = 4,      /* resource still in use by in-flight work            */
  MVP_ERR_NOT_READY = 5  /* result not available yet                          */
} mvp_status;

typedef enum { MVP_F32 = 0, MVP_BF16 = 1 } mvp_dtype;

typedef struct mvp_ctx mvp_ctx;       /* device, memory cache, serving scheduler */
typedef struct mvp_accel mvp_accel;   /* per-frame culling lists and ray/primitive intervals */

/* The primitives {t_k, R_k, s_k, V_k} (Sec. 3.1.2).  All device pointers.
 *   pos     [N,3]        float32  t_k, world position of the box centre
 *   rot     [N,3,3]      float32  R_k row-major, local-to-world: x = R diag(s) y + t,
 *                                 y in the closed local box [-1,1]^3
 *   scale   [N,3]        float32  s_k > 0, half extent of the box along each local axis
 *   payload [N,M,M,M,4]  float32 or bf16 (payload_dtype), index [k][iz][iy][ix][c],
 *                                 c = (R,G,B,opacity density); voxel i of an axis sits
 *                                 at local coordinate -1 + 2i/(M-1); 16-byte aligned
 *                                 (8-byte for bf16).
 * n_prim == 0 is legal and renders an empty image. */
typedef struct {
  int32_t n_prim;
  int32_t M;               /* >= 2 */
  int32_t payload_dtype;   /* mvp_dtype */
  int32_t reserved;
  const float *pos;
  const float *rot;
  const float *scale;
  const void *payload;
} mvp_prims;

/* Pinhole camera (Sec. 4.1), a HOST struct.  The ray of pixel (px, py) starts at
 * origin and points along pix2dir @ (px + 0.5, py + 0.5, 1), normalised to unit
 * length so that t is world distance. */
typedef struct {
  int32_t width, height;
  float origin[3];
  float pix2dir[9];        /* row-major 3x3 */
} mvp_camera;

/* March parameters: sample j sits at t = j * step (step > 0); the march stops
 * after a sample once the accumulated opacity exceeds 1 - eps_early
 * (0 <= eps_early < 1, Sec. 3.2.2); only t >= t_near >= 0 is integrated.
 * fade_alpha > 0 multiplies every voxel's opacity by the fade window of
 * Sec. 3.1.3, W = exp(-fade_alpha (|x|^b + |y|^b + |z|^b)), b = fade_beta > 0,
 * (x, y, z) the voxel's normalised coordinates in [-1,1]^3 (the paper uses
 * alpha = beta = 8); gradients are then with respect to the stored payload.
 * fade_alpha = 0 disables it.
 * combine chooses how the primitives containing one sample are merged
 * (Sec. 3.2.2): MVP_COMBINE_SUM adds their opacities and opacity-weighted
 * colours into one global field sample before the clamp step;
 * MVP_COMBINE_SEQUENTIAL takes them one after another in increasing primitive
 * id, each with its own clamp step, as a fixed traversal order would.  The two
 * agree on every sample that does not saturate; at the saturating sample the
 * sequential rule gives the clamp to the first primitive that crosses 1.  Any
 * other value is MVP_ERR_INVALID. */
typedef enum { MVP_COMBINE_SUM = 0, MVP_COMBINE_SEQUENTIAL = 1 } mvp_combine;

typedef struct {
  float step;
  float eps_early;
  float t_near;
  float fade_alpha;
  float fade_beta;
  int32_t combine;         /* mvp_combine */
} mvp_march_params;

/* Per-ray state the forward leaves for the backward: the index of the last
 * sample processed (-1 if the ray met no sample) and, if the clamp
 * T = min(., 1) was hit at that sample, the opacity just before it (else -1). */
typedef struct {
  int32_t j_end;
  float t_prev;
} mvp_ray_aux;

/* Sizes of an acceleration structure (host struct). */
typedef struct {
  int32_t n_views, width, height, n_prim;
  int64_t n_tile_pairs;    /* (tile, primitive) entries of the culling lists           */
  int64_t n_ray_pairs;     /* (ray, primitive) pairs with at least one sample           */
  int64_t device_bytes;    /* device memory held by the structure                       */
  int32_t pairs_in_forward; /* 1: the first forward builds the per-ray lists, tile by tile;
                             * 0: the build's pairs kernel did                            */
  int32_t reserved;
} mvp_accel_info;

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device`. */
mvp_status mvp_create(int device, mvp_ctx **out);
/* Destroy a context.  Waits for its serving work; fails with MVP_ERR_BUSY if an
 * acceleration structure created from it is still alive. */
mvp_status mvp_destroy(mvp_ctx *ctx);
/* Message of the last failed call on this thread; never NULL. */
const char *mvp_last_error(void);
/* Library version string; never NULL. */
const char *mvp_version(void);

/* ---- rendering (Sec. 3.2) ------------------------------------------------- */

/* Per-frame acceleration structure for n_views cameras of one resolution:
 * screen-tile culling lists of the primitives (the role the paper's per-frame
 * BVH plays, Sec. 3.2.1), then for every ray the primitives it intersects and
 * the fixed-step sample interval inside each (the ray-specific lists and
 * domain of integration of Sec. 3.2.1).  cams is a HOST array of n_views.
 * Reads prims->pos/rot/scale; the payload is not read.  BLOCKS until the list
 * sizes are known (one stream synchronisation).  The per-ray lists are built
 * on the device by the first mvp_render_fwd* on the structure (each workgroup
 * builds its screen tile's lists and then marches them), or by the first
 * backward if it comes first; the lists the backward reads per primitive are
 * built on the context's second stream after that first forward.  Calls on one
 * structure must be ordered on the caller's streams.  *out must be released
 * with mvp_accel_destroy. */
mvp_status mvp_build_accel(mvp_ctx *ctx, const mvp_prims *prims, const mvp_camera *cams,
                           int32_t n_views, const mvp_march_params *params,
                           mvp_accel **out, void *stream);
/* The same for a subset of the rays: the training mode of Sec. 3.3, where each
 * iteration samples rays from the images.  rays is a DEVICE array of n_rays
 * pixel ids, id = (view * height + py) * width + px, in any order (the library
 * keeps a copy); a pixel may appear more than once as long as no 16x16 tile
 * receives more than 256 rays.  Forward and backward then read and write
 * per-ray arrays in the order of `rays`: rgba [n_rays,4], aux [n_rays],
 * grad_rgba [n_rays,4].  Out-of-range ids fail with MVP_ERR_INVALID.  rays may
 * be NULL only when n_rays == 0 (an empty subset).  BLOCKS like
 * mvp_build_accel. */
mvp_status mvp_build_accel_rays(mvp_ctx *ctx, const mvp_prims *prims, const mvp_camera *cams,
                                int32_t n_views, const mvp_march_params *params, const int64_t *rays,
                                int64_t n_rays, mvp_accel **out, void *stream);
/* Release an acceleration structure.  Its memory is recycled only after the
 * work already enqueued on `stream` has finished. */
mvp_status mvp_accel_destroy(mvp_ctx *ctx, mvp_accel *accel, void *stream);
/* Sizes of a structure.  n_ray_pairs is counted on the device by the pass
 * that builds the per-ray lists (the first forward or backward): it is -1
 * until that pass has been enqueued, and the first call after it BLOCKS until
 * it has finished. */
mvp_status mvp_accel_get_info(const mvp_accel *accel, mvp_accel_info *info);

/* Forward march (Sec. 3.2.2).  prims must be the primitives the structure was
 * built from (payload may differ).  Writes, per ray (per pixel, or per entry of
 * the ray subset):
 *   rgba [n_views,H,W,4] float32: premultiplied colour I and alpha A per pixel,
 *   aux  [n_views,H,W]   mvp_ray_aux (may be NULL if no backward follows).
 * Deterministic: each pixel is written by one thread in a fixed order. */
mvp_status mvp_render_fwd(mvp_ctx *ctx, const mvp_accel *accel, const mvp_prims *prims,
                          float *rgba, mvp_ray_aux *aux, void *stream);

/* Backward of mvp_render_fwd (Sec. 3.2.2, differentiable volumetric
 * aggregation: the additive accumulation makes the ray's final state enough to
 * differentiate it, without storing per-sample values) for L with dL/drgba = grad_rgba [n_views,H,W,4] float32, using the
 * aux of the same forward: each (ray, primitive) pair is replayed from the
 * ray's stored last sample and pre-clamp opacity.  ACCUMULATES (+=) into
 *   grad_payload [N,M,M,M,4] float32 (also for bf16 payloads),
 *   grad_pos [N,3], grad_rot [N,3,3], grad_scale [N,3] float32;
 * any of the four may be NULL to skip it.  A primitive's payload gradient is
 * summed per work item (up to 64 screen tiles of one primitive) in on-chip
 * memory as 64-bit fixed point, with a scale chosen per item from a bound on
 * what any one of its (ray, primitive) pairs contributes, so that no sum
 * overflows and the integer sums do not depend on the order of the additions;
 * each item's sum is then added
 * to grad_payload with FP32 device atomics, as are the pose gradients, so the
 * order of those floating-point additions (not the math) varies between runs.
 * grad_rgba must be finite (a work item whose bound is not finite writes NaN
 * into its primitive's payload gradient).  Scratch device memory of 24 bytes
 * per ray comes from the context's memory cache. */
mvp_status mvp_render_bwd(mvp_ctx *ctx, const mvp_accel *accel, const mvp_prims *prims,
                          const mvp_ray_aux *aux, const float *grad_rgba,
                          float *grad_payload, float *grad_pos, float *grad_rot,
                          float *grad_scale, void *stream);

/* Largest number of rays (pixels of all views, or entries of a ray subset) of
 * one mvp_render_bwd_noalloc call: one 1024x1024 view. */
#define MVP_NOALLOC_MAX_RAYS 1048576

/* mvp_render_bwd for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving or training loops, harnesses that forbid
 * hipMalloc.  Same arguments, results and errors as mvp_render_bwd, but the
 * 24 bytes per ray of scratch come from a fixed library-owned device array
 * (24 MiB on every device the library runs on, held until the process ends)
 * instead of the context's memory cache, so the call allocates nothing.
 * A structure with more than MVP_NOALLOC_MAX_RAYS rays fails with
 * MVP_ERR_INVALID and enqueues nothing.  All calls on one device share that
 * array: calls that may overlap on one device (different streams or threads,
 * or different contexts) race and must be serialised by the caller; calls on
 * one stream are ordered and safe.  Nothing in the array needs to survive a
 * call, and the call clears what it needs cleared with kernels (no memset). */
mvp_status mvp_render_bwd_noalloc(mvp_ctx *ctx, const mvp_accel *accel, const mvp_prims *prims,
                                  const mvp_ray_aux *aux, const float *grad_rgba,
                                  float *grad_payload, float *grad_pos, float *grad_rot,
                                  float *grad_scale, void *stream);

/* The same forward composited over a background (the alpha compositing of
 * Sec. 3.1.4 with the premultiplied colour): rgba = (I + (1 - A) B, A) with
 * background B [rays,3] float32 (rays ordered like rgba). */
mvp_status mvp_render_fwd_bg(mvp_ctx *ctx, const mvp_accel *accel, const mvp_prims *prims,
                             const float *background, float *rgba, mvp_ray_aux *aux, void *stream);

/* Backward of mvp_render_fwd_bg: needs its background and output rgba (for
 * A); additionally ACCUMULATES dL/dB = (1 - A) dL/dcolour into
 * grad_background [rays,3] (may be NULL). */
mvp_status mvp_render_bwd_bg(mvp_ctx *ctx, const mvp_accel *accel, const mvp_prims *prims,
                             const float *background, const float *rgba, const mvp_ray_aux *aux,
                             const float *grad_rgba, float *grad_payload, float *grad_pos,
                             float *grad_rot, float *grad_scale, float *grad_background, void *stream);

/* Sample counts of the most recent forward on this structure (BLOCKS on
 * `stream`): ray-samples (samples inside >= 1 intersected primitive, up to the
 * early stop) and prim-samples ((sample, primitive) pairs, i.e. trilinear
 * payload fetches). */
mvp_status mvp_accel_counts(mvp_ctx *ctx, const mvp_accel *accel, uint64_t *ray_samples,
                            uint64_t *prim_samples, void *stream);

/* Load counts of the most recent forward and backward on this structure
 * (BLOCKS on `stream`), written to the HOST array out[9]:
 *   [0] ray-samples, [1] prim-samples (as mvp_accel_counts);
 *   forward: [2] voxel-corner sets loaded (8 corners each), [3] pair-record
 *   loads (16 B each), [4] culling-entry frames read from device memory
 *   (52 B each; a tile's frames are staged once per tile when they fit);
 *   backward: [5] pairs visited by its ordering pass, [6] pairs replayed,
 *   [7] cell runs (one voxel-corner set loaded each), [8] non-zero payload
 *   gradient values added to grad_payload.
 * The forward's sequential-combine walk over a saturating sample's primitives
 * is not counted.  Used to express the march kernels' memory traffic in
 * bytes. */
mvp_status mvp_accel_load_counts(mvp_ctx *ctx, const mvp_accel *accel, uint64_t *out, void *stream);

/* Hit sets for testing: for every ray, the ids of the primitives its ray
 * intersects (slab test only, including hits with no sample), ascending.
 * offsets [n_rays+1] int64 and ids [ids_cap] int32 are device buffers; if the
 * total exceeds ids_cap, *n_total is set and MVP_ERR_OOM returned (offsets are
 * still written).  BLOCKS on `stream`. */
mvp_status mvp_debug_hits(mvp_ctx *ctx, const mvp_accel *accel, const mvp_prims *prims,
                          int64_t *offsets, int32_t *ids, int64_t ids_cap, int64_t *n_total,
                          void *stream);

/* Kernel timing for benchmarks: from mvp_timing_start on, every forward
 * (MVP_KERNEL_FWD_MARCH: the forward march kernel) and backward
 * (MVP_KERNEL_BWD_MARCH: the per-pair backward kernel, without the per-ray
 * constants kernel before it) records a pair of HIP events around that kernel
 * on the stream it is launched on, for the first `capacity` launches of each.
 * mvp_timing_read BLOCKS until the recorded launches have finished and writes
 * their durations in milliseconds to the HOST array ms [capacity], launch
 * order, and their number to *n.  mvp_timing_stop ends recording and frees
 * the events.  Requests of the serving scheduler are not recorded. */
typedef enum { MVP_KERNEL_FWD_MARCH = 0, MVP_KERNEL_BWD_MARCH = 1 } mvp_kernel;
mvp_status mvp_timing_start(mvp_ctx *ctx, int32_t capacity);
mvp_status mvp_timing_read(mvp_ctx *ctx, int32_t kernel, float *ms, int32_t *n);
mvp_status mvp_timing_stop(mvp_ctx *ctx);

/* ---- serving: resident scenes and continuous batching ----------------------- */

/* Configure the serving scheduler: device memory budget (resident scenes plus
 * in-flight request scratch) and number of concurrent request slots (each
 * with its own stream).  Must be called before the first scene is created. */
mvp_status mvp_serve_configure(mvp_ctx *ctx, size_t budget_bytes, int32_t n_slots);

/* Copy a scene (device pointers in *src) into library-owned device memory that
 * stays resident until released.  Counts against the budget (MVP_ERR_OOM). */
mvp_status mvp_scene_create(mvp_ctx *ctx, const mvp_prims *src, uint64_t *scene_id);
/* Release a resident scene; MVP_ERR_BUSY while requests on it are pending. */
mvp_status mvp_scene_release(mvp_ctx *ctx, uint64_t scene_id);

/* One render request: a resident scene seen from one camera.  rgba_out is a
 * caller-owned device buffer [H,W,4] float32 that must stay valid until the
 * request completes. */
typedef struct {
  uint64_t scene_id;
  mvp_camera cam;
  mvp_march_params params;
  float *rgba_out;
} mvp_request;

/* Queue a request; never blocks.  The scheduler admits queued requests in
 * arrival order as soon as a slot is free; each slot's worker thread builds
 * the request's culling structure and launches its forward on the slot's
 * stream, so builds and marches of different requests overlap on the device.
 * Scratch memory is reserved against the budget as the build sizes it; a
 * build that does not fit waits for running requests to finish, and a request
 * larger than the whole budget fails. */
mvp_status mvp_submit(mvp_ctx *ctx, const mvp_request *req, uint64_t *ticket);

/* Request state: *state = 0 queued, 1 running, 2 done, 3 failed.  Times are
 * seconds on the library's monotonic clock (mvp_clock): submission, and
 * completion of the GPU work (0 until done).  A done/failed ticket stays
 * queryable until mvp_ticket_release.  Unknown ticket: MVP_ERR_INVALID. */
mvp_status mvp_poll(mvp_ctx *ctx, uint64_t ticket, int32_t *state, double *t_submit,
                    double *t_done);
/* The three stamps of a ticket on the mvp_clock clock: submission, the moment
 * a slot worker began enqueuing the request's culling build on its slot stream
 * (0 while queued; a request that gave way to an older one for memory is
 * stamped again when it restarts), and completion of its forward on the
 * device (0 until done).  Any pointer may be NULL. */
mvp_status mvp_ticket_times(mvp_ctx *ctx, uint64_t ticket, double *t_submit, double *t_start,
                            double *t_done);
/* Ray-samples and prim-samples (as mvp_accel_counts) that a done request's
 * forward evaluated; either pointer may be NULL.  Unknown ticket:
 * MVP_ERR_INVALID; queued, running or failed: MVP_ERR_NOT_READY.  (Both are 0
 * if the library could not allocate the pinned block it copies them through.) */
mvp_status mvp_ticket_samples(mvp_ctx *ctx, uint64_t ticket, uint64_t *ray_samples, uint64_t *prim_samples);
/* The monotonic clock (seconds) of the serving stamps, so that a client can
 * measure latency from its own arrival times. */
double mvp_clock(void);
/* Block until the ticket is done or failed, or timeout_s elapses
 * (MVP_ERR_NOT_READY). */
mvp_status mvp_wait(mvp_ctx *ctx, uint64_t ticket, double timeout_s);
mvp_status mvp_ticket_release(mvp_ctx *ctx, uint64_t ticket);

#ifdef __cplusplus
}
#endif
#endif /* MVP_H */
