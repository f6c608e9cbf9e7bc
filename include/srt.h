/*
 * srt.h - C ABI of libsrt: stochastic ray tracing of transparent 3D Gaussians
 * on AMD MI355X (gfx950).
 *
 * Method: Sun, Georgiev, Fei, Hasan, "Stochastic Ray Tracing of Transparent
 * 3D Gaussians" (EGSR 2025). A ray traverses a bounding volume hierarchy over
 * the Gaussians' k-sigma bounds (Sec. 3.2) once, tests each Gaussian whose
 * bound it crosses (Alg. "intersect"), accepts it with probability alpha
 * (eqn "rr"), keeps the closest accepted hit per sample (eqn "cloest"), runs N
 * samples in one traversal (eqn "multisample") and shades the result once.
 *
 * Conventions for every entry point:
 *  - Pointers named "device" are HIP device pointers; the caller owns them
 *    and keeps them alive until the work on `stream` has finished. Nothing in
 *    this library allocates or frees caller memory.
 *  - All calls are asynchronous on `stream` (a hipStream_t; NULL = the null
 *    stream) except srt_build_bvh, srt_refit_bvh and srt_batch_plan_create,
 *    which synchronise `stream` before returning.
 *  - Errors are status codes; nothing throws across the ABI. Arguments are
 *    validated on the host before anything is launched; on an error no work
 *    has been enqueued and outputs are untouched.
 *  - Geometry arrays are FP32, row-major, contiguous.
 *  - Acceptance numbers: Philox4x32-10 (Salmon et al., SC'11) with key
 *    (seed low 32 bits, seed high 32 bits) and counter
 *    (ray id, sample / 4, Gaussian id, purpose); u = (word[sample % 4] >> 8)
 *    * 2^-24. A candidate is accepted iff u < alpha.
 *  - A candidate is valid iff its depth t (by default the mean t* of the 1D
 *    Gaussian the ray cuts through it, Sec. 3.1; see depth_mode) satisfies
 *    tmin < t < tmax and its squared Mahalanobis distance q at t* satisfies
 *    q <= s^2 = 8 (eqn "cuboid", s = 2 sqrt 2); alpha = opacity * exp(-q / 2).
 *    The depth key is t rounded to FP32; keys compare as (t, Gaussian id).
 */
#ifndef SRT_H
#define SRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SRT_OK = 0,
    SRT_ERR_INVALID_ARG = 1,   /* a null pointer, size or option out of range */
    SRT_ERR_OOM = 2,           /* a device allocation failed */
    SRT_ERR_HIP = 3,           /* a HIP runtime call or launch failed */
    SRT_ERR_UNSUPPORTED = 4,   /* a valid but unimplemented combination */
    SRT_ERR_WORKSPACE = 5      /* the workspace is smaller than required */
} srt_status;

/* Human-readable name of a status code (static storage). */
const char* srt_status_str(srt_status s);

/* ABI version: major * 10000 + minor * 100 + patch. */
int32_t srt_version(void);

/* ------------------------------------------------------------------------
 * Scene: raw Gaussian parameters as a training pipeline keeps them
 * (eqn "gaussian": G(x) = exp(-(x-mu)^T Sigma^-1 (x-mu) / 2)).
 *   means          [G,3] device  mu
 *   log_scales     [G,3] device  per-axis log standard deviation (S = diag(exp))
 *   quats          [G,4] device  rotation as an unnormalised (w, x, y, z)
 *                                quaternion; R = R(q / |q|) maps the
 *                                Gaussian's frame to the world and
 *                                Sigma = R S^2 R^T
 *   opacity_logits [G]   device  opacity o = 1 / (1 + exp(-logit))
 *   sh             [G,(deg+1)^2,3] device  real SH colour coefficients; the
 *                                colour seen along unit direction d is
 *                                max(0, 0.5 + sum_lm k_lm Y_lm(d)) per channel
 *   sh_degree      0..3
 * ------------------------------------------------------------------------ */
typedef struct {
    int64_t num_gaussians;
    int32_t sh_degree;
    const float* means;
    const float* log_scales;
    const float* quats;
    const float* opacity_logits;
    const float* sh;
} srt_scene;

/* ------------------------------------------------------------------------
 * Acceleration structure (Sec. 3.2: a BVH over per-Gaussian bounds).
 * width 2, 4 or 8 children per node; leaf_size 1..8 Gaussians per leaf;
 * size_split 0..16: 0 orders Gaussians by the Morton code of their box
 * centres; k > 0 first groups them by size class
 * floor(log2(scene extent / box extent) / k), so Gaussians whose sizes differ
 * by more than 2^k get subtrees of their own (large ones stop inflating the
 * boxes around small ones). Results never depend on these options.
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t width;
    int32_t leaf_size;
    int32_t size_split;
} srt_build_opts;

typedef struct srt_bvh srt_bvh; /* opaque, library-owned */

typedef struct {
    int64_t num_gaussians;
    int64_t num_nodes;
    int32_t width;
    int32_t leaf_size;
    int32_t depth;          /* levels of wide nodes */
    int32_t sh_degree;
    int64_t device_bytes;   /* memory held by the handle */
} srt_bvh_info;

/* Derive each Gaussian's canonical record (whitening matrix M = S^-1 R^T
 * computed in FP64 and rounded to FP32, opacity, conservative FP32 box of the
 * k-sigma ellipsoid) and build a `width`-wide BVH with at most `leaf_size`
 * Gaussians per leaf. The scene's SH buffer is referenced, not copied: it
 * must stay alive and unchanged while the handle is used. Synchronises
 * `stream`. On success *out receives a handle for srt_destroy_bvh.
 * Errors: INVALID_ARG (null pointers with num_gaussians > 0, negative count,
 * sh_degree outside 0..3, width not in {2,4,8}, leaf_size outside 1..8,
 * size_split outside 0..16, more than 2^28 Gaussians), OOM, HIP. */
srt_status srt_build_bvh(const srt_scene* scene, const srt_build_opts* opts, void* stream,
                         srt_bvh** out);

/* Cap the device memory the library holds in use for BVH handles and build
 * temporaries (bytes; 0 removes the cap). An allocation that would exceed
 * it fails with SRT_ERR_OOM before anything is enqueued, as a failed
 * hipMalloc does; memory already held is not freed. Blocks the library
 * keeps for reuse (up to 8 GiB, per device and size class) do not count.
 * Batch plans and caller workspaces are not covered. Process-wide.
 * Errors: INVALID_ARG (bytes < 0). */
srt_status srt_set_memory_limit(int64_t bytes);

/* Bytes the library holds in use (handles and running builds) and keeps
 * for reuse; either pointer may be null, not both (INVALID_ARG). */
srt_status srt_memory_stats(int64_t* in_use, int64_t* cached);

/* Refit a handle to new parameters of the same Gaussians (an optimisation
 * step, Sec. 7's differentiable-rendering use): the records and Gaussian
 * boxes are recomputed from `scene` exactly as srt_build_bvh computes them,
 * and every node box is refilled bottom-up; the topology and leaf order are
 * kept. Trace results do not depend on the tree, so they equal those of a
 * fresh build of `scene` bit for bit; only the traversal cost can grow as
 * Gaussians move away from their build positions. The handle then references
 * `scene`'s SH buffer. No work on the handle may be pending; synchronises
 * `stream`. Errors: INVALID_ARG (null pointers, num_gaussians or sh_degree
 * different from the build's), HIP. */
srt_status srt_refit_bvh(srt_bvh* bvh, const srt_scene* scene, void* stream);

/* Free a handle (null is ignored). No work on the handle may be pending. */
void srt_destroy_bvh(srt_bvh* bvh);

srt_status srt_bvh_get_info(const srt_bvh* bvh, srt_bvh_info* info);

/* Copy the canonical records out, in Gaussian-id order, for validation:
 * mu [G,3], M [G,9] (row-major), opacity [G], box_lo/box_hi [G,3]; all
 * device, any may be null. Asynchronous on `stream`. */
srt_status srt_bvh_records(const srt_bvh* bvh, float* mu, float* M, float* opacity,
                           float* box_lo, float* box_hi, void* stream);

/* Copy the wide-node array out (device, srt_bvh_info.num_nodes nodes of
 * 32 * width bytes: lo_x[W] lo_y[W] lo_z[W] hi_x[W] hi_y[W] hi_z[W] as FP32
 * then child[W] as int32, padded; child >= 0 is a node index, child < 0 a
 * leaf ~((first << 3) | (count - 1)) over the leaf-ordered Gaussians) and
 * the leaf order (device int32 [G]: Gaussian id at each leaf position).
 * Either pointer may be null. */
srt_status srt_bvh_nodes(const srt_bvh* bvh, void* nodes, int32_t* leaf_order, void* stream);

/* ------------------------------------------------------------------------
 * Rays. origins/dirs [R,3] device (dirs need not be unit length; SH colour
 * uses the normalised direction). tmin/tmax [R] device or null (0, +inf).
 * ignore_gid [R] device or null: a Gaussian id the ray never hits (-1 none).
 * ray_ids [R] device or null (the ray index): Philox counter word 0.
 * sample_ids [R] device or null: the sample index of the ray's first sample
 * (added to srt_trace_opts.sample_offset). purpose: Philox counter word 3
 * (0 camera, 2 shadow, 3 mirror, 4 incoherent by convention).
 * ------------------------------------------------------------------------ */
typedef struct {
    int64_t count;
    const float* origins;
    const float* dirs;
    const float* tmin;
    const float* tmax;
    const int32_t* ignore_gid;
    const uint32_t* ray_ids;
    const uint32_t* sample_ids;
    uint32_t purpose;
} srt_rays;

/* Trace options.
 * seed            Philox key.
 * spp             samples per ray (>= 1); the pixel value is their mean
 *                 (eqn "multisample").
 * n_per_traversal samples resolved in one traversal: 1, 2, 4 or 8; samples
 *                 pass*N + k, so results do not depend on N.
 * sample_offset   added to every sample index.
 * bg              colour of a sample that accepts nothing.
 * any_hit         1: terminate at the first accepted hit (shadow rays); the
 *                 sample's "colour" is visibility (1 unoccluded, 0 occluded)
 *                 in all three channels and hit_gid is any accepted id.
 *                 Requires n_per_traversal == 1.
 * stack_limit     0 = default; otherwise caps the on-chip traversal stack
 *                 (testing: forces the deep-stack path in the forward, and
 *                 the global-memory part of the stacks in the backward).
 * depth_mode      0: a candidate's depth is the mean of the 1D Gaussian along
 *                 the ray (Sec. 3.1). 1: the Gaussian centre projected onto
 *                 depth_axis, as the ray parameter of the same depth along
 *                 the axis, t = ((mu - o) . a) / (d . a) (Sec. 4.1; the
 *                 rasterizer-compatible depth); depth_axis (0,0,0) means each
 *                 ray's own direction. Opacity stays at the 1D peak; the
 *                 range test and the depth key use this depth.
 * image_width     0: rays are independent (lane i traces ray i). > 0: the
 *                 rays are the pixels of a row-major image of this width
 *                 (count must be a multiple of it, else SRT_ERR_INVALID_ARG)
 *                 and each wave traces one 8x8 pixel tile (with wave-shared
 *                 walks and 2 or 4 passes per pixel: 8x4 or 4x4 pixels, one
 *                 lane per pass), which keeps its lanes on neighbouring
 *                 rays. Results do not depend on it.
 * persistent      0: one lane per ray. 1: work-stealing waves (one wave per
 *                 workgroup, as many as fit on the GPU) loop over the rays; a
 *                 lane runs all passes of its ray, and once refill_threshold
 *                 lanes of a wave are idle the wave takes that many new rays
 *                 with one atomic, so short walks do not wait for the
 *                 longest walk of their wave. Results do not depend on it.
 * refill_threshold idle lanes (1..64) that trigger a refill; 0 = 16.
 * estimator       backward only. 0: per sample, every valid candidate k in
 *                 front of the result a gets <g, c_k - X> / (1 - alpha_k) on
 *                 its alpha (X = c_a, bg on a miss). 1: the same terms
 *                 averaged over each candidate's own acceptance number:
 *                 k in front of a gets <g, c_k - c_a>, and a gets
 *                 <g, c_a - c_a2>, a2 the sample's next accepted candidate
 *                 behind a (bg if none; the walk goes on to find it). Both are
 *                 unbiased for the exact composite's gradient; 1 has no larger
 *                 variance (Rao-Blackwell). Colour gradients are the same.
 * rng             0: Philox numbers as described above. 1: the paper's
 *                 stateless trigonometric hash (Sec. 4.2, eqns "hash" and
 *                 "rng") of the candidate's hit position p = o + t* d, in
 *                 FP32, moved by the sample index s along (1,1,1) so the N
 *                 samples of one walk differ; frame-to-frame variation comes
 *                 from jittered camera rays (srt_camera.jitter). Results are
 *                 then a different realisation, correct in expectation only.
 *                 seed and purpose are not used by the hash.
 * walk            0: automatic (2 where it is supported, else 1).
 *                 1: every lane walks the BVH for its own ray.
 *                 2: the 64 rays of a wave (an 8x8 tile of an image launch,
 *                 else 64 consecutive rays) walk it together, one node at a
 *                 time (a lane takes part in the nodes and leaves its own
 *                 walk would reach); forward: Philox numbers and
 *                 persistent = 0; backward: image launches; else
 *                 SRT_ERR_UNSUPPORTED. Automatic: image launches of
 *                 closest-hit rays. Results do not depend on it, except
 *                 which accepted id an any-hit ray reports and the order of
 *                 the backward's FP32 atomic additions. In srt_trace_pathmix
 *                 it applies to the camera rays.                           */
typedef struct {
    uint64_t seed;
    int32_t spp;
    int32_t n_per_traversal;
    uint32_t sample_offset;
    float bg[3];
    int32_t any_hit;
    int32_t stack_limit;
    int32_t depth_mode;
    float depth_axis[3];
    int32_t image_width;
    int32_t persistent;
    int32_t refill_threshold;
    int32_t estimator;
    int32_t rng;
    int32_t walk;
} srt_trace_opts;

/* Counters accumulated (+=) into a device uint64 array of SRT_NUM_COUNTERS
 * when a non-null pointer is passed. */
enum {
    SRT_CNT_TRAVERSALS = 0, /* ray traversals started */
    SRT_CNT_NODES = 1,      /* wide nodes visited */
    SRT_CNT_PRIMS = 2,      /* Gaussians tested in leaves */
    SRT_CNT_CANDIDATES = 3, /* valid candidates (passed range + ellipsoid) */
    SRT_CNT_PHILOX = 4,     /* Philox4x32-10 evaluations */
    SRT_CNT_DEEP = 5,       /* traversals rerun with the deep stack */
    SRT_CNT_RAY_SAMPLES = 6,/* ray-samples resolved */
    SRT_CNT_LOST = 7,       /* rays left unresolved (deep stack or step bound
                               exceeded); zero for every tree this library builds */
    SRT_NUM_COUNTERS = 8
};

/* Bytes of device workspace srt_trace_forward / srt_trace_backward need for
 * `num_rays` rays. */
size_t srt_trace_workspace_size(const srt_bvh* bvh, int64_t num_rays);

/* Forward trace (Alg. "intersect" applied to every Gaussian whose box the ray
 * crosses; eqns "rr", "cloest", "multisample").
 * rgb      [R,3] device or null: mean over samples of the shaded colour.
 * hit_gid  [R,spp] device int32 or null: accepted Gaussian id, -1 on a miss.
 * hit_t    [R,spp] device FP32 or null: its depth key, +inf on a miss.
 * counters device uint64[SRT_NUM_COUNTERS] or null.
 * workspace / workspace_bytes: device scratch of srt_trace_workspace_size.
 * The scene must be the one the handle was built from (its sh is read).
 * Errors: INVALID_ARG, WORKSPACE, HIP. */
srt_status srt_trace_forward(const srt_bvh* bvh, const srt_rays* rays,
                             const srt_trace_opts* opts, float* rgb, int32_t* hit_gid,
                             float* hit_t, uint64_t* counters, void* workspace,
                             size_t workspace_bytes, void* stream);

/* Bytes of the per-device scratch array behind srt_trace_forward_noalloc. */
#define SRT_NOALLOC_SCRATCH_BYTES (64u << 20)

/* srt_trace_forward without a workspace argument, for callers that cannot
 * allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid allocation): the same kernels and results, with the
 * scratch taken from a static device array of SRT_NOALLOC_SCRATCH_BYTES
 * (64 MiB) that each GPU holds until the process ends. Nothing is allocated
 * or freed by this call. The array's address on a device is looked up once,
 * at the first call whose stream runs on that device.
 * Limit: srt_trace_workspace_size(bvh, rays->count) must not exceed
 * SRT_NOALLOC_SCRATCH_BYTES (about 15M rays on a 1M-Gaussian BVH), else
 * SRT_ERR_WORKSPACE and nothing is enqueued. Every call on one GPU shares
 * that GPU's array: calls that overlap on one GPU (different streams, or
 * threads without ordering) race and give undefined results; calls ordered
 * on one stream are safe. What must start at zero is cleared by each call.
 * Arguments and other errors as srt_trace_forward. */
srt_status srt_trace_forward_noalloc(const srt_bvh* bvh, const srt_rays* rays,
                                     const srt_trace_opts* opts, float* rgb, int32_t* hit_gid,
                                     float* hit_t, uint64_t* counters, void* stream);

/* ------------------------------------------------------------------------
 * Backward: gradients of the expected colour (the exact composite of eqn
 * "accumulated") with respect to the raw parameters. The paper names
 * differentiable rendering as future work (Sec. 7); the estimator here is,
 * per sample with result a (colour X, or bg on a miss): every valid candidate
 * k in front of a receives <g, c_k - X> / (1 - alpha_k) on alpha_k, and a
 * receives the colour gradient g, each weighted 1/spp; its expectation is the
 * exact gradient T_k (c_k - B_k) on alpha_k and T_k alpha_k on c_k. Each ray
 * is re-traversed once per pass of N samples; no hit lists are stored.
 * ------------------------------------------------------------------------ */

/* Bytes of device workspace srt_trace_backward needs for `num_rays` rays. */
size_t srt_backward_workspace_size(const srt_bvh* bvh, int64_t num_rays);

/* scene     the scene the handle was built from (log_scales and quats are read).
 * rays/opts as for the forward call whose result is being differentiated
 *           (same seed, spp, sample offset; any_hit must be 0).
 * grad_rgb  [R,3] device: d loss / d rgb of each ray's pixel value.
 * hit_gid, hit_t [R,spp] device: the forward's per-sample results; both null
 *           to recompute them inside the kernel.
 * g_*       device gradient buffers shaped like the scene arrays; gradients
 *           are ADDED (+=), so zero them first. g_sh receives the colour
 *           gradient, the others the opacity gradient chained through
 *           alpha = o exp(-q/2) at the 1D mean (envelope: dq/dt = 0).
 * Atomic FP32 accumulation: results are reproducible up to summation order.
 * Errors: INVALID_ARG (mismatched scene, N not in {1,2,4,8}, any_hit, one of
 * hit_gid/hit_t null), WORKSPACE, HIP. */
srt_status srt_trace_backward(const srt_bvh* bvh, const srt_scene* scene, const srt_rays* rays,
                              const srt_trace_opts* opts, const float* grad_rgb,
                              const int32_t* hit_gid, const float* hit_t, float* g_means,
                              float* g_log_scales, float* g_quats, float* g_opacity_logits,
                              float* g_sh, uint64_t* counters, void* workspace,
                              size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Cameras: pinhole rays through pixel centres, row 0 at the top, FP32 with
 * single correctly rounded operations in this order (no contraction):
 *   px = (x + 0.5) / W; sx = ((px * 2) - 1) * tan_half * (W / H)
 *   py = (y + 0.5) / H; sy = (1 - (py * 2)) * tan_half
 *   v = (forward + sx * right) + sy * up; d = v / sqrt((vx^2 + vy^2) + vz^2)
 * The basis (forward, right, up) and tan_half are data, not re-derived.
 * ------------------------------------------------------------------------ */
typedef struct {
    float eye[3];
    float forward[3];
    float right[3];
    float up[3];
    float tan_half;
    int32_t width;
    int32_t height;
    float jitter[2]; /* sub-pixel offset from the pixel centre, in pixels, in
                        [-0.5, 0.5) (0, 0 = centres); a frame's camera
                        perturbation (Sec. 4.2) */
} srt_camera;

/* Write width*height camera rays (pixel y*width + x): origins, dirs [R,3]
 * device. */
srt_status srt_camera_rays(const srt_camera* cam, float* origins, float* dirs, void* stream);

/* ------------------------------------------------------------------------
 * Path-tracer mix: Gaussians inside a renderer (Sec. 1, Sec. 5: secondary
 * rays use the same traversal). Per camera sample the shading point P is the
 * nearer of the accepted Gaussian and the plane y = plane_y; P spawns an
 * any-hit shadow ray to `light` (Philox purpose 2) and, on the plane, a mirror
 * ray (purpose 3), both reusing the camera ray id and sample index. In FP32,
 * single rounded operations: P_i = o_i + (t * d_i) (plane: P_y = plane_y);
 * v = light - P; len = sqrt((vx^2 + vy^2) + vz^2); l = v / len; the shadow
 * ray is (P, l, tmin_secondary, len, ignoring the spawning Gaussian); the
 * mirror ray is (P, (dx, -dy, dz), tmin_secondary, +inf). Colour: Gaussian
 * c * (0.3 + 0.7 V); plane 0.5 V max(0, l_y) + 0.5 Lm with Lm the mirror
 * hit's colour (bg on a miss); nothing hit: bg.
 * ------------------------------------------------------------------------ */
typedef struct {
    float light[3];
    float plane_y;
    float tmin_secondary;
    int32_t stages;  /* 0: the whole mix; else the stages to run, a mask of
                        SRT_PATHMIX_* below. Stages hand their results on
                        through the workspace: running each stage alone, in
                        order, with the same arguments and workspace gives
                        the whole mix's outputs (to time or overlap them). */
} srt_pathmix_opts;

enum {
    SRT_PATHMIX_CAMERA = 1,  /* camera rays, their trace, secondary-ray spawning */
    SRT_PATHMIX_SHADOW = 2,  /* the any-hit shadow rays */
    SRT_PATHMIX_MIRROR = 4,  /* the mirror rays */
    SRT_PATHMIX_COMPOSE = 8  /* shading and the outputs */
};

size_t srt_pathmix_workspace_size(const srt_bvh* bvh, const srt_camera* cam, int32_t spp);

/* Render one camera's path-tracer mix. Camera ray ids are ray_id_base + pixel.
 * The shadow rays of one pixel whose shading points coincide (the samples
 * that accepted the same Gaussian, or that all reached the plane) are
 * identical but for their sample index; with Philox numbers and spp <= 64
 * each such group is resolved by one walk (a sample is occluded iff one of
 * the walk's candidates accepts its own number), which gives every sample
 * the visibility of its own any-hit walk.
 * rgb [H*W,3] device; cam_gid/cam_t [H*W,spp], shadow_vis (uint8: 1 lit,
 * 0 occluded, 255 no shadow ray) [H*W,spp], mirror_gid (-2 no mirror ray,
 * -1 miss) [H*W,spp]: device or null. counters as srt_trace_forward; its
 * SRT_CNT_RAY_SAMPLES entry counts camera samples plus secondary rays.
 * opts->any_hit must be 0. Camera rays are traced as an image (8x8 tiles,
 * wave-shared walks unless opts->walk is 1); the any-hit shadow rays always
 * run on work-stealing waves (see srt_trace_opts.persistent); camera and
 * mirror rays follow opts->persistent.
 * Errors: INVALID_ARG (also pm->stages outside 0..15), WORKSPACE, HIP. */
srt_status srt_trace_pathmix(const srt_bvh* bvh, const srt_camera* cam, uint32_t ray_id_base,
                             const srt_trace_opts* opts, const srt_pathmix_opts* pm,
                             float* rgb, int32_t* cam_gid, float* cam_t, uint8_t* shadow_vis,
                             int32_t* mirror_gid, uint64_t* counters, void* workspace,
                             size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Batched forward: many views with uneven samples per pixel plus extra rays
 * (e.g. incoherent secondary rays) in one graph-captured launch. The
 * per-sample results equal srt_trace_forward's on the same rays, ray ids and
 * samples (N samples per traversal, Philox keyed as above).
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t num_views;
    const srt_camera* cameras;  /* host [num_views]; copied at plan creation */
    const int32_t* spp;         /* host [num_views]: samples per pixel of each view */
    srt_rays extra;             /* device arrays (count may be 0); ignore_gid and
                                   sample_ids must be null; ray_ids null means
                                   ray_id_base + row */
    int32_t extra_spp;          /* samples per extra ray (>= 1 when extra.count > 0) */
    uint32_t ray_id_base;       /* camera ray id = ray_id_base + output row */
} srt_batch;

/* Launch shape. persistent = 1: the work-stealing kernel (a grid of
 * waves_per_cu one-wave workgroups per compute unit, capped at the number
 * the kernel keeps resident; a wave claims new items once at least
 * refill_threshold of its 64 lanes are idle, and the records of the leaves
 * its lanes reach are tested one per lane from a queue in LDS);
 * persistent = 0: the plain kernel, one lane per ray. With opts->walk != 1
 * the views' pixels use wave-shared walks of 8x8 tiles instead: persistent,
 * the extra rays run first on the work-stealing kernel, then a second
 * persistent grid claims one (tile, pass) group of 64 items per atomic;
 * plain, one wave per tile. The extra rays always walk one lane per ray.
 * Results do not depend on the choice (colours up to the order of the
 * persistent kernels' FP32 atomic additions). */
typedef struct {
    int32_t persistent;
    int32_t refill_threshold;  /* 1..64 */
    int32_t waves_per_cu;      /* >= 1 */
    int32_t lds_stack;         /* work-stealing lane kernel: stack entries per lane
                                  kept in LDS, 1..24, 0 = 24; deeper entries live in
                                  global memory (smaller values test that part) */
} srt_tuning;

typedef struct srt_batch_plan srt_batch_plan; /* opaque, library-owned */

/* Output rows: the views' pixels (view by view, y*W + x), then the extra
 * rays. Per-sample outputs follow the same order, spp entries per row.
 * opts->n_per_traversal may also be 16 here: the views' pixels then take 16
 * samples per traversal on wave-shared walks (opts->walk != 1), while lane
 * walks (the extra rays, and the views with walk = 1) take at most 8; the
 * per-sample results do not depend on it.
 * Copies the view table to the device and allocates the plan's work counter,
 * overflow queue and deep stacks (persistent plans: also the global-memory
 * part of the lane stacks, 4 B per entry beyond those kept in LDS, for
 * every lane of the largest resident grid); synchronises `stream`. The handle and the
 * extra-ray arrays must outlive the plan. Errors: INVALID_ARG, OOM, HIP. */
srt_status srt_batch_plan_create(const srt_bvh* bvh, const srt_batch* batch,
                                 const srt_trace_opts* opts, const srt_tuning* tuning,
                                 void* stream, srt_batch_plan** out);

void srt_batch_plan_destroy(srt_batch_plan* plan);

/* rows: output rows; samples: per-sample outputs; items: work items (passes
 * of N samples for the persistent kernel, rays for the plain one). */
srt_status srt_batch_plan_info(const srt_batch_plan* plan, int64_t* rows, int64_t* samples,
                               int64_t* items);

/* Run the plan: rgb [rows,3] device (mean over each row's samples),
 * hit_gid [samples] device or null, counters as srt_trace_forward. The first
 * call (and any call with different output pointers) captures the launch
 * sequence into a HIP graph on a private stream; every call then launches
 * the graph on `stream`. Calls on one plan must not overlap. */
srt_status srt_batch_plan_execute(srt_batch_plan* plan, float* rgb, int32_t* hit_gid,
                                  uint64_t* counters, void* stream);

/* The same launch sequence without the graph (for checking graph replays). */
srt_status srt_batch_plan_execute_eager(srt_batch_plan* plan, float* rgb, int32_t* hit_gid,
                                        uint64_t* counters, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SRT_H */
