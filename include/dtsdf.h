/*
 * dtsdf.h -- C ABI of the Directional-TSDF library for AMD Instinct MI355X (gfx950).
 *
 * The library fuses depth (+colour) frames into a Directional TSDF, renders depth, vertex,
 * normal and colour images from it by ray marching, and registers depth frames against the
 * rendered views with point-to-plane ICP in SE(3) or Sim(3).  Every step runs in the
 * library's own HIP kernels; the caller provides device buffers and a HIP stream.
 *
 * References are to Splietker & Behnke, "Rendering the Directional TSDF for Tracking and
 * Multi-Sensor Registration with Point-To-Plane Scale ICP" (RAS 2023).
 *
 * Conventions shared by every call
 *   - Units are metres.  Cameras are pinhole with OpenCV axes (x right, y down, z forward);
 *     pixel (u, v) has its centre at integer coordinates.
 *   - Poses are host double[16], row-major 4x4; T_world_cam maps camera to world.
 *   - Images are dense row-major device arrays of width x height.  Three-component images
 *     (vertex, normal) are stored as three planes: x plane, then y plane, then z plane.
 *   - `stream` is a hipStream_t passed as void* (NULL: the default stream).  Calls enqueue
 *     work on it and return; device buffers must stay alive until the stream has finished.
 *     Calls that return host results (statistics, icp_step) synchronise the stream.
 *   - Every call returns a dtsdf_status; nothing throws across the ABI.  Output parameters
 *     are written only on DTSDF_OK unless stated otherwise.
 *   - World voxel (i, j, k) sits at (i, j, k) * voxel_size; block (bx, by, bz) holds voxels
 *     8 bx .. 8 bx + 7 per axis.  Directions are ordered X+, X-, Y+, Y-, Z+, Z- (Sec. 3).
 */
#ifndef DTSDF_H_
#define DTSDF_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dtsdf_map dtsdf_map; /* opaque, owned by the library */

typedef enum {
  DTSDF_OK = 0,
  DTSDF_E_INVAL = 1,      /* bad argument: null pointer, size, format or parameter range */
  DTSDF_E_NOMEM = 2,      /* device or host allocation failed */
  DTSDF_E_CAPACITY = 3,   /* brick pool or hash table full; see dtsdf_integrate */
  DTSDF_E_HIP = 4,        /* a HIP runtime call failed */
  DTSDF_E_DEGENERATE = 5, /* icp_step: too few inliers or the normal matrix is not PD */
  DTSDF_E_BUSY = 6        /* resource in use */
} dtsdf_status;

/* Storage of the per-voxel signed distance and weight (Sec. 3: voxel tuple (d, w_d, c, w_c)). */
typedef enum {
  DTSDF_SDF_F32 = 0, /* float32 normalised distance */
  DTSDF_SDF_F16 = 1, /* float16, round to nearest even */
  DTSDF_SDF_I16 = 2  /* int16 q = round(d * 32767), distance scaled by the truncation */
} dtsdf_sdf_fmt;

typedef enum {
  DTSDF_W_F32 = 0, /* float32 weight */
  DTSDF_W_U8 = 1   /* uint8 code q = round(sqrt(1024 w)), w = q^2 / 1024 (at most 63.5) */
} dtsdf_w_fmt;

typedef struct {
  int32_t width, height;
  float fx, fy, cx, cy;
} dtsdf_intrinsics;

/* Map parameters.  theta is the angular threshold of Sec. 3 (eq. angular_threshold), in
 * (pi/4, pi/2].  Values the paper leaves open have these suggested defaults:
 * theta = pi/3, w_carve = 0.1 (free-space weight, Sec. 3), w_max = 63.75 (weight cap),
 * w_min = 1e-4 (updates with a smaller fusion weight are skipped), lattice_step =
 * 0.5 * voxel_size (ray-march probing interval, Sec. 4). */
typedef struct {
  float voxel_size;        /* metres */
  float truncation;        /* tau, metres */
  float theta;             /* radians */
  float w_carve, w_max, w_min;
  float lattice_step;      /* metres */
  int32_t sdf_fmt;         /* dtsdf_sdf_fmt */
  int32_t w_fmt;           /* dtsdf_w_fmt */
  int32_t with_color;      /* 1: keep per-direction rgb + colour weight */
  uint32_t brick_capacity; /* number of 8^3 brick-directions the pool holds */
  uint32_t hash_buckets;   /* power of two, at least 2 * number of blocks expected */
  int32_t dense;           /* 1: allocate the block range below in all six directions and
                              never allocate outside it */
  int32_t dense_lo[3], dense_hi[3]; /* inclusive block range of a dense map */
} dtsdf_params;

typedef struct {
  int64_t bricks;          /* brick-directions in use */
  int64_t capacity;        /* brick_capacity */
  int64_t blocks;          /* distinct blocks (hash entries) */
  int64_t hash_buckets;
  int64_t dropped;         /* brick requests refused for lack of capacity, cumulative */
  int64_t device_bytes;    /* device memory held by the map */
} dtsdf_info;

/* Render outputs; every pointer is a device buffer or NULL (not produced).
 * The trace_* arrays serve traffic accounting: when given, the caller zeroes them and the
 * render sets to 1 the entry of every brick whose (sdf, w) a sample read (trace_bricks,
 * brick_capacity bytes), every brick whose colour an output read (trace_color, same size)
 * and every hash entry whose brick indices a lookup read (trace_slots, hash_buckets bytes);
 * trace_counts (4 int32 per pixel) receives the number of evaluations at lattice points that
 * may end a crossing, evaluations of a skipped positive point that precedes such a point,
 * jumps over absent space, and refinement evaluations.  A traced render marches every ray
 * alone (as with DTSDF_RENDER_ALONE), so that the counts and sets are those of the ray.
 * flags: DTSDF_RENDER_ALONE marches every ray alone; by default lanes of a wave whose ray
 * has finished evaluate lattice points of the rays still marching.  The images are the same
 * either way (the values at lattice points, hence the hit, do not depend on who evaluates
 * them); the flag serves tests and comparisons. */
#define DTSDF_RENDER_ALONE 1
typedef struct {
  float* depth;   /* H*W camera-frame z of the hit, 0 where nothing was hit */
  float* vertex;  /* 3*H*W planes, camera-frame hit point */
  float* normal;  /* 3*H*W planes, camera-frame unit normal facing the camera */
  uint8_t* rgba;  /* H*W*4, colour of the hit, alpha 255 where a colour is defined */
  uint8_t* mask;  /* H*W, 1 where the ray hit a surface */
  uint8_t* trace_bricks;
  uint8_t* trace_color;
  uint8_t* trace_slots;
  int32_t* trace_counts;
  int32_t flags;  /* 0 or DTSDF_RENDER_ALONE */
} dtsdf_render_out;

/* Host-side map image used for checkpoints and exact map transfer.  Bricks are listed in
 * ascending (bx, by, bz, D) order; voxel l of a brick has local coordinates
 * (l % 8, (l / 8) % 8, l / 64).  Arrays are host memory owned by the caller. */
typedef struct {
  int64_t n_bricks; /* in/out: number of bricks (capacity of the arrays on export) */
  int32_t* keys;    /* n_bricks x 4: bx, by, bz, D */
  float* sdf;       /* n_bricks x 512 normalised distance */
  float* w;         /* n_bricks x 512 weight */
  uint8_t* rgb;     /* n_bricks x 512 x 3, or NULL */
  float* wc;        /* n_bricks x 512 colour weight, or NULL */
} dtsdf_blob;

/* Create an empty map (dense maps start with their whole block range allocated).
 * Errors: DTSDF_E_INVAL on a bad parameter (hash_buckets not a power of two, theta outside
 * (pi/4, pi/2], non-positive sizes, unsupported format), DTSDF_E_NOMEM. */
dtsdf_status dtsdf_create(const dtsdf_params* params, dtsdf_map** out);

/* Free a map and its device memory (synchronises the device). NULL is accepted. */
dtsdf_status dtsdf_destroy(dtsdf_map* map);

dtsdf_status dtsdf_get_info(const dtsdf_map* map, dtsdf_info* out);

typedef struct {
  int64_t new_bricks;      /* brick-directions allocated by this call */
  int64_t dropped;         /* requests refused for lack of capacity by this call */
  int64_t bricks;          /* brick-directions in use after the call */
  int64_t visited_bricks;  /* bricks the fusion visited (frustum test passed) */
  int64_t updated_voxels;  /* voxels whose distance and weight were updated */
  int64_t color_voxels;    /* voxels whose colour was updated */
} dtsdf_integrate_stats;

/* Fuse one depth (+ colour) frame with known pose (Sec. 3).
 *   depth: device H*W float32 metres (multiplied by depth_scale), 0 = no measurement.
 *   rgb:   device H*W*3 uint8, or NULL.
 * Steps: cross-product normals of the frame (Sec. 7); allocation of every block on the
 * segment p +/- tau r for each direction D with w_dir(n) > 0 (Sec. 7: blocks keyed by
 * (x, y, z, D)); voxel-projection fusion (Sec. 3) of every allocated voxel with the point-to-
 * plane distance (eq. point-to-plane), fusion weight (eq. combined_fusion_weight), colour
 * weight (eq. color_weight) and free-space carving.
 * stats may be NULL (then the call does not synchronise).  When the pool is full the
 * requests that fit are allocated, the others are dropped, every allocated voxel is still
 * fused, and DTSDF_E_CAPACITY is returned with stats filled in; the map stays consistent. */
dtsdf_status dtsdf_integrate(dtsdf_map* map, const float* depth, const uint8_t* rgb,
                             const dtsdf_intrinsics* intr, const double T_world_cam[16],
                             float depth_scale, void* stream, dtsdf_integrate_stats* stats);

/* dtsdf_integrate with the frame's normals given by the caller instead of the cross-product
 * normals computed from the depth, so that filtered normals (Sec. 7: the cross-product
 * normals are processed by a bilateral filter, see dtsdf_normal_filter) steer allocation,
 * direction weights and fusion weights.  normal: device planar (3, H, W) float32 unit
 * normals in the camera frame facing the camera, all zero = no normal; a pixel without
 * depth contributes nothing whatever its normal.  DTSDF_E_INVAL if normal is NULL. */
dtsdf_status dtsdf_integrate_normals(dtsdf_map* map, const float* depth, const float* normal,
                                     const uint8_t* rgb, const dtsdf_intrinsics* intr,
                                     const double T_world_cam[16], float depth_scale,
                                     void* stream, dtsdf_integrate_stats* stats);

/* Render a view of the map (Sec. 4): per pixel, the combined SDF of the six directions
 * (eq. combine_weight, fallback eq. combine_tsdf_weight) is probed at t0 + k * lattice_step
 * from z_near to z_far along the ray; the first step from a positive to a non-positive value
 * is refined inside its bracket and the outputs are written.  Read-only on the map:
 * concurrent renders of one map are allowed. */
dtsdf_status dtsdf_render(const dtsdf_map* map, const dtsdf_intrinsics* intr,
                          const double T_world_cam[16], float z_near, float z_far,
                          const dtsdf_render_out* out, void* stream);

/* One view of a batched render. */
typedef struct {
  dtsdf_intrinsics intr;
  double T_world_cam[16];
  float z_near, z_far;
  dtsdf_render_out out;
} dtsdf_render_req;

/* Render n views (any sizes, any poses) of one map in a single persistent launch that hands
 * (view, work tile of 64 pixels) items to waves as they free up (8x8 tiles; a batch of at
 * most 9000 such tiles uses the interleaved work tiles of a single-view launch).  Every pixel
 * is computed exactly as by dtsdf_render, so each view is bitwise identical to rendering it
 * alone.  Serves many
 * sensors at once (continuous batching of render requests).  Enqueues on `stream`. */
dtsdf_status dtsdf_render_batch(const dtsdf_map* map, int32_t n, const dtsdf_render_req* reqs,
                                void* stream);

/* Copy the map to host arrays.  With blob->keys == NULL only blob->n_bricks is set.
 * Otherwise blob->n_bricks must be at least the number of bricks (DTSDF_E_INVAL if not);
 * it is set to the number written.  Synchronises. */
dtsdf_status dtsdf_export(const dtsdf_map* map, dtsdf_blob* blob);

/* Replace the map contents with a blob (keys in any order, no duplicates).  rgb and wc may
 * be NULL (colour cleared).  DTSDF_E_CAPACITY if the blob does not fit.  Synchronises. */
dtsdf_status dtsdf_import(dtsdf_map* map, const dtsdf_blob* blob);

/* Recycle bricks that hold no surface (Sec. 3: voxels allocated in error that repeated
 * carving turned into free space go back to the pool): every (block, D) brick whose observed
 * voxels (w > 0) all hold values >= t_free (truncation units; carving drives values towards
 * 1), or that has no observed voxel, is removed from the map, reset and put on a free list
 * that later allocations use before the pool grows.  *recycled (nullable) receives the
 * number removed.  Meant to run every few frames, on the stream of the map's other calls;
 * synchronises it.  DTSDF_E_INVAL for dense or combined-volume maps or t_free <= 0. */
dtsdf_status dtsdf_recycle(dtsdf_map* map, float t_free, int64_t* recycled, void* stream);

/* Camera-frame points (Sec. 6, eq. reprojection) and cross-product normals (Sec. 7) of a
 * depth image: vertex/normal are 3*H*W planes; the normal of a pixel without depth in
 * itself or one of its four neighbours is written as (0, 0, 0), as is its vertex when the
 * pixel has no depth.  Normals face the camera. */
dtsdf_status dtsdf_vertex_normal(const float* depth, const dtsdf_intrinsics* intr,
                                 float depth_scale, float* vertex, float* normal,
                                 void* stream);

/* Halve a depth image: output pixel = mean of its 2x2 input block if all four are valid,
 * else 0.  Output size (width / 2) x (height / 2). */
dtsdf_status dtsdf_depth_downsample(const float* depth_in, int32_t width, int32_t height,
                                    float* depth_out, void* stream);

/* One frame of a registration problem at one pyramid level. */
typedef struct {
  const float* vertex;   /* 3*H*W planes, camera frame */
  const float* normal;   /* 3*H*W planes; (0,0,0) marks an invalid pixel */
  const uint8_t* mask;   /* H*W hit mask of a rendered model image, or NULL */
  dtsdf_intrinsics intr;
} dtsdf_image;

typedef enum { DTSDF_ICP_W_CONST = 0, DTSDF_ICP_W_DEPTH = 1 } dtsdf_icp_weight;

typedef struct {
  float max_dist;          /* reject ||q - y|| above this [m] (0.10) */
  float max_angle_deg;     /* reject normal angle above this (20) */
  int32_t weight;          /* dtsdf_icp_weight; DEPTH is eq. ICP_weight with z_min */
  float z_min;
  int32_t min_inliers_per_dim; /* fewer than this * dim inliers -> DTSDF_E_DEGENERATE (64) */
  int32_t compensated;     /* 1: float32 sums with Neumaier compensation per thread and
                              TwoSum merges across the reduction tree */
} dtsdf_icp_params;

typedef struct {
  double xi[7];        /* solved increment (nu, omega[, sigma]) */
  double H[49];        /* dim x dim normal matrix, row-major (sum w J J^T) */
  double g[7];         /* sum w J r */
  double error;        /* sum w r^2 */
  int64_t inliers;
  double step_norm;    /* ||xi||_2 */
  int32_t status;      /* DTSDF_OK or DTSDF_E_DEGENERATE */
  int32_t photometric; /* photometric terms in the sums (icp_step_rgb), else 0 */
} dtsdf_icp_result;

/* One Gauss-Newton step of point-to-plane ICP (Sec. 5, eq. geometric_ICP .. deltaT_update;
 * Sim(3): Sec. 6, eq. sim3_derivative).  dim = 6 (SE(3)) or 7 (Sim(3)).
 * T_model_live (host, in/out) maps live camera coordinates to model camera coordinates.
 * Every live pixel with a valid normal is transformed by T_model_live, projected into the
 * model image (nearest pixel, must be a hit), and rejected beyond max_dist or
 * max_angle_deg; the residuals r = <q - y, n> and Jacobians J = (-n, -(y x n)[, -<n, y>])
 * are reduced in a fixed order (bitwise run-to-run reproducible), the system H xi = -g is
 * solved by Cholesky in float64 on the device and T_model_live <- exp(xi) T_model_live.
 * DTSDF_E_DEGENERATE (T unchanged, result filled in) if there are too few inliers or H is
 * not positive definite.  Synchronises the stream. */
dtsdf_status icp_step(const dtsdf_image* live, const dtsdf_image* model, int32_t dim,
                      const dtsdf_icp_params* params, double T_model_live[16],
                      dtsdf_icp_result* result, void* stream);

/* Photometric term of combined ICP (Sec. 5.2, eq. combined_icp; Sec. 5.3, eq. keyframe_icp).
 * For every live pixel with depth, its model-frame point y = T_model_live p is taken to the
 * reference camera by T_ref_model, projected with ref_intr to (u, v) in [1, W - 2] x
 * [1, H - 2], and r = I_live(pixel) - I_ref(u, v) (bilinear) enters the sums if
 * |r| <= max_error, with Jacobian -grad I_ref(u, v) . d(u, v)/da . R(T_ref_model) [I | -y^]
 * (eq. keyframe_icp_derivative; grad I_ref = bilinear central differences, zero on the
 * border pixels; Sim(3) scale column -grad I . d(u, v)/da . R y) and weight lambda times the
 * pixel's depth weight.  Grey values are in [0, 1] (dtsdf_intensity). */
typedef struct {
  const float* live_intensity;  /* device, live width x height (the live level's size) */
  const float* ref_intensity;   /* device, ref_intr.width x ref_intr.height */
  dtsdf_intrinsics ref_intr;
  double T_ref_model[16];       /* model camera -> reference camera; the identity for
                                   frame-to-frame and frame-to-render, T_kf^-1 T_model for a
                                   keyframe at T_kf */
  float lambda;                 /* weight of the photometric energy (0.1) */
  float max_error;              /* intensity outlier threshold (0.05 fine, 0.175 coarse) */
} dtsdf_photo;

/* icp_step with the photometric term of `photo` added to the same fixed-order sums
 * (photo == NULL: icp_step).  The degenerate test counts geometric inliers. */
dtsdf_status icp_step_rgb(const dtsdf_image* live, const dtsdf_image* model,
                          const dtsdf_photo* photo, int32_t dim,
                          const dtsdf_icp_params* params, double T_model_live[16],
                          dtsdf_icp_result* result, void* stream);

/* Levenberg-Marquardt state of one registration run (Sec. 7: LM with the damping scheme of
 * Madsen, Nielsen and Tingleff).  The caller sets T (the prior), tau (mu starts at tau times
 * the largest diagonal entry of the first H; 1e-3 suggested) and started = 0; every
 * icp_step_lm reduces at T, accepts or rejects it by the gain ratio
 * rho = (F_acc - F) / (h^T (mu h - g_acc)) (rho > 0: accept, mu *= max(1/3, 1 - (2 rho - 1)^3),
 * nu = 2; else mu *= nu, nu *= 2), solves (H_acc + mu I) h = -g_acc and sets T = exp(h) T_acc.
 * The result of the run is T_acc. */
typedef struct {
  double T[16];        /* candidate pose (model <- live) the next call evaluates */
  double T_acc[16];    /* last accepted pose */
  double H[49];        /* normal equations at T_acc, dim x dim row-major */
  double g[7];
  double F;            /* sum w r^2 at T_acc */
  double h[7];         /* last step */
  double mu, nu, tau;
  int32_t started;
  int32_t accepted;    /* out: the last call accepted its candidate */
} dtsdf_lm_state;

/* One Levenberg-Marquardt iteration (geometric, or combined with `photo`); see
 * dtsdf_lm_state.  DTSDF_E_DEGENERATE (state unchanged) if there are too few inliers or the
 * damped system is not positive definite.  Synchronises the stream. */
dtsdf_status icp_step_lm(const dtsdf_image* live, const dtsdf_image* model,
                         const dtsdf_photo* photo, int32_t dim,
                         const dtsdf_icp_params* params, dtsdf_lm_state* state,
                         dtsdf_icp_result* result, void* stream);

/* Grey values (0.299 R + 0.587 G + 0.114 B) / 255 of a device H*W*3 uint8 image. */
dtsdf_status dtsdf_intensity(const uint8_t* rgb, int32_t width, int32_t height, float* out,
                             void* stream);

/* Halve a grey image: output pixel = mean of its 2x2 input block. */
dtsdf_status dtsdf_intensity_downsample(const float* in, int32_t width, int32_t height,
                                        float* out, void* stream);

/* One registration request of a batch; pose, flag and result live in device memory so that
 * a serving loop can run many iterations without host round-trips. */
typedef struct {
  dtsdf_image live, model;
  int32_t dim;                 /* 6 or 7 */
  dtsdf_icp_params params;
  double* pose;                /* device double[16], T_model_live, updated in place */
  int32_t* active;             /* device flag or NULL: the step runs only while *active != 0,
                                  and clears it when ||xi|| < min_step or the system is
                                  degenerate (then the pose is left unchanged) */
  double min_step;
  dtsdf_icp_result* result;    /* device or NULL */
  const dtsdf_photo* photo;    /* host, or NULL: geometric terms only */
} dtsdf_icp_req;

/* One Gauss-Newton step for each of n requests (any sizes, SE(3) or Sim(3)) in two launches
 * (reduction over (request, chunk) workgroups, then one solve workgroup per request).  The
 * per-request reduction order is the same as icp_step's, so every request's pose is bitwise
 * identical to stepping it alone.  Enqueues on `stream`; does not synchronise. */
dtsdf_status icp_step_batch(int32_t n, const dtsdf_icp_req* reqs, void* stream);

/* `iterations` steps of icp_step_batch enqueued from one upload of the requests: every step
 * continues from the poses the previous one wrote in device memory, and a request whose
 * flag dropped to 0 (converged or degenerate) is skipped on the device, so a coarse-to-fine
 * level runs with no host wait (Sec. 5: the iterations of one pyramid level).  Equal, per
 * request, to that many icp_step_batch calls.  1 <= iterations <= 1000. */
dtsdf_status icp_step_batch_iters(int32_t n, const dtsdf_icp_req* reqs, int32_t iterations,
                                  void* stream);

/* Intrinsics of pyramid level `level` of a camera (Sec. 5, the pyramid of registration):
 * width and height halved `level` times, f / 2^level and c_l = (c + 0.5) / 2^level - 0.5
 * (pixel centres at integer coordinates, each level pixel the mean of a 2x2 block), computed
 * in double and rounded to float.  0 <= level <= 15; a level with no pixels is
 * DTSDF_E_INVAL.  Host function. */
dtsdf_status dtsdf_level_intrinsics(const dtsdf_intrinsics* in, int32_t level,
                                    dtsdf_intrinsics* out);

/* Coarse-to-fine registration of one request on the device (Sec. 5: the levels of the
 * pyramid, coarsest first): reqs[l] describes level l (0 finest; live and model images and
 * intrinsics of that level) and all levels share one device pose and carry a device
 * convergence flag.  For l = levels-1 .. 0 the flag is raised and iterations[l] steps of
 * icp_step_batch_iters run (a converged or degenerate level skips its remaining steps on the
 * device; 0 skips the level).  Enqueues on `stream` with no host wait; the pose is
 * T_model_live after the finest level.  DTSDF_E_INVAL if the levels do not share one pose,
 * a flag is missing, or a count is outside 0..1000. */
dtsdf_status dtsdf_icp_pyramid(int32_t levels, const dtsdf_icp_req* reqs,
                               const int32_t* iterations, void* stream);

/* icp_step_batch_iters for callers that cannot allocate memory: code under HIP graph
 * capture, tight serving loops and harnesses that forbid allocation.  Same arguments,
 * semantics and results as icp_step_batch_iters, for at most DTSDF_NOALLOC_MAX_REQUESTS
 * requests (more: DTSDF_E_INVAL).  The request descriptors reach the device as kernel
 * arguments and the partial sums use a fixed device array of the library (under 1 MB per
 * GPU, held until the process ends); the call allocates no host or device memory and keeps
 * no pointer to `reqs`.  Every call on one GPU uses that same array: calls that overlap on
 * one GPU (different streams, or host threads without ordering) race, so the caller
 * serialises them on that GPU. */
#define DTSDF_NOALLOC_MAX_REQUESTS 16
dtsdf_status icp_step_batch_iters_noalloc(int32_t n, const dtsdf_icp_req* reqs,
                                          int32_t iterations, void* stream);

/* ---- View-dependent combined ("rendering") TSDF (Sec. 4) -------------------------------
 * For a fixed camera position the six directional TSDFs can be merged into one conflict-free
 * regular TSDF (Sec. 4, Lemma positional_unambiguity); ray casting that volume from (near)
 * that position reads one volume instead of six.  A volume is a map whose direction slot 0
 * holds, per voxel, the combined SDF (weight 1; weight 0 = no value) and the combined colour
 * (colour weight 1 where defined).  dtsdf_render / dtsdf_render_batch on a volume march it
 * like the direct path (same lattice, hit test, refinement and outputs) with the
 * interpolated value as f, its gradient as normal and its colour as colour.  dtsdf_export /
 * dtsdf_import work on volumes (keys with D = 0 only); dtsdf_integrate refuses them. */

/* Create an empty volume for combining `src` (its voxel size, truncation, theta, lattice
 * step and colour setting; float32 storage).  brick_capacity bricks (one per block of src:
 * at least src's block count) and hash_buckets (power of two) as in dtsdf_create.
 * Errors: DTSDF_E_INVAL (src is itself a volume, bad sizes), DTSDF_E_NOMEM. */
dtsdf_status dtsdf_volume_create(const dtsdf_map* src, uint32_t brick_capacity,
                                 uint32_t hash_buckets, dtsdf_map** out);

/* Combine `src` into `vol` (Sec. 4, precomputed combined TSDF; Sec. 7, integer positions).
 * First every block of src gets its brick in vol (only when src gained blocks since the
 * last call; this step synchronises the stream).  Then, for every voxel centre x of src's
 * blocks that lies in front of the camera of T_frustum and projects into its image widened
 * by `margin` times the width / height on every side (pixel centres at integer coordinates):
 *   f(x) = sum_D w_D Phi^D(x) / sum_D w_D,  w_D = w_dir(n^D) max(0, <n^D, -r>) W^D(x)
 * (eq. combine_weight) over the directions observed at x (W^D > 0), with r the unit ray from
 * the camera centre of T_center to x and n^D the normalised central difference of Phi^D over
 * the six axis neighbours, usable only if all six are observed in D and |grad| s >= 1e-6;
 * if these weights sum to zero, w_D = W^D max(0, <v^D, -r>) (eq. combine_tsdf_weight); no
 * value if that sum is zero too.  Colour: the directions' voxel colours blended with
 * w_dir(n^D) max(0, <n^D, -r>) W_c^D, else with the combination weights; 8-bit codes
 * rounded half to even.
 *   only_missing == 0 (recombination, margin 1/8 in Sec. 4): every voxel outside that
 *     frustum is left with no value, so the volume is valid for ray casting from T_center.
 *   only_missing != 0: only voxels inside the frustum that hold no value are evaluated
 *     (voxels seen for the first time, Sec. 4; pass the frame's pose as T_frustum, the last
 *     recombination's pose as T_center and margin 0); the others keep their values.
 * Poses are host double[16] (camera to world).  Enqueues on `stream`.
 * Errors: DTSDF_E_INVAL (src is a volume, vol is not, voxel size or theta differ, bad
 * intrinsics or margin outside [0, 4]), DTSDF_E_CAPACITY (vol cannot hold src's blocks; vol
 * keeps what fits and nothing is combined). */
dtsdf_status dtsdf_combine(const dtsdf_map* src, dtsdf_map* vol, const double T_center[16],
                           const double T_frustum[16], const dtsdf_intrinsics* intr,
                           float margin, int32_t only_missing, void* stream);

/* Conditional recombination (Sec. 4, eq. condition_1 .. condition_4).  The caller sets the
 * four limits (suggested 5, 50, 0.05 m, 0.05 pi / 2 rad) and zeroes the rest. */
typedef struct {
  int32_t boot_frames;     /* frames 0 .. boot_frames - 1 always recombine */
  int32_t stale_frames;    /* recombine once more than this many frames have passed */
  double max_translation;  /* metres between the pose and the last recombination's pose */
  double max_angle;        /* radians of the relative rotation (geodesic angle) */
  int64_t frames;          /* frames decided so far */
  int64_t since;           /* frames since the last recombination, this one included */
  double last_pose[16];    /* pose of the last recombination */
  int32_t has_pose;
  int32_t reserved;
} dtsdf_recombine_state;

/* Decide for the next frame with pose T_world_cam whether to recombine (then record T as the
 * new reference); *recombine = 1 or 0.  Host only, no device work. */
dtsdf_status dtsdf_recombine_decide(dtsdf_recombine_state* state, const double T_world_cam[16],
                                    int32_t* recombine);

/* ---- Input preprocessing (Sec. 7; parameters of Sec. 8) and the post-fusion error ---- */

typedef struct {
  float support_rel;    /* a neighbour q supports pixel p if |D(q) - D(p)| <= support_rel * D(p)
                           (suggested 0.02) */
  int32_t min_support;  /* p keeps its depth only with >= min_support supporting pixels among
                           its eight neighbours (Sec. 7: 2); 0 switches the test off; <= 8 */
  float sigma_d;        /* bilateral depth filter: spatial sigma [px] (Sec. 8: 5.0) */
  float sigma_r;        /* range sigma [m] (Sec. 8: 0.025) */
  int32_t radius;       /* window half-size [px], 0..8 (Sec. 8: 5); 0 switches the bilateral
                           filter off */
} dtsdf_depth_filter_params;

/* Depth outlier (support) filter followed by the bilateral depth filter: out(p) = 0 where p
 * has no depth or too little support, else the mean of the supported depths q of the window
 * weighted by exp(-|q - p|^2 / (2 sigma_d^2)) exp(-(D(q) - D(p))^2 / (2 sigma_r^2)).  Device
 * H*W float32 images, depth_in != depth_out.  DTSDF_E_INVAL for bad sizes or parameters. */
dtsdf_status dtsdf_depth_filter(const float* depth_in, int32_t width, int32_t height,
                                const dtsdf_depth_filter_params* params, float* depth_out,
                                void* stream);

/* Bilateral normal filter (Sec. 7; Sec. 8: sigma_d 2.5 px, sigma_r 5.0 degrees, radius 5):
 * normalised sum of the window's normals weighted by exp(-|q - p|^2 / (2 sigma_d^2))
 * exp(-angle(n_q, n_p)^2 / (2 sigma_r^2)), the angle in degrees.  Device planar (3, H, W)
 * float32 maps as written by dtsdf_vertex_normal (zero = no normal, stays zero), in != out,
 * radius 0..8. */
dtsdf_status dtsdf_normal_filter(const float* normal_in, int32_t width, int32_t height,
                                 float sigma_d, float sigma_r_deg, int32_t radius,
                                 float* normal_out, void* stream);

/* Post-fusion error (Sec. 8): out[0] = sum |rendered - measured| and out[1] = the number of
 * pixels where both depths are > 0 (device float64[2]); the mean absolute error is
 * out[0] / out[1].  Deterministic (fixed summation order). */
dtsdf_status dtsdf_depth_error(const float* rendered, const float* measured, int32_t width,
                               int32_t height, double* out, void* stream);

const char* dtsdf_status_string(dtsdf_status status);

#ifdef __cplusplus
}
#endif

#endif /* DTSDF_H_ */
