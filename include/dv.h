/*
 * dv.h - C ABI of the compositional multi-octree sparse-voxel renderer.
 *
 * The renderer follows DrivingVoxels (arXiv 2606.23031): a static
 * world-frame octree O_bg plus one local-frame octree O_i per rigid actor
 * (Sec. 3.1-3.2) are rendered in a single pass (Sec. 3, overview).  Each
 * camera ray is split by the actors' box intervals into background and
 * asset segments (Sec. 3.4, App. A, Alg. 1), every segment is integrated
 * with trilinear raw density, exp-linear activation and alpha compositing,
 * and the result is composited over the sky (Eq. 2): a constant colour or
 * a bilinearly sampled environment map (Sec. 3.1, sky modelling).
 *
 * Conventions used by every call:
 *  - "device" pointers are HIP device memory of the context's GPU; "host"
 *    pointers are ordinary CPU memory.  No call takes ownership of a caller
 *    pointer; caller arrays must stay alive as long as the object that
 *    references them (scene, forward state, request).
 *  - Every call returns dv_status; no C++ exception crosses this boundary.
 *    On failure dv_last_error() returns a message for the calling thread.
 *  - Work is enqueued on the caller's HIP stream (passed as void*; NULL is
 *    the default stream).  Results are valid when that stream completes.
 *  - Arrays are structure-of-arrays: ijk is [3][N], corner_idx is [8][N],
 *    sh is [S][3][N] with S = (degree+1)^2; images are planar [C][h][w].
 */
#ifndef DV_H
#define DV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dv_status;
#define DV_OK 0
#define DV_PENDING 1            /* serving: request not finished yet      */
#define DV_ERR_INVALID (-1)     /* malformed argument                     */
#define DV_ERR_OOM (-2)         /* device or host allocation failed       */
#define DV_ERR_DEVICE (-3)      /* HIP error; the context is poisoned     */
#define DV_ERR_OVERLAP (-4)     /* two leaves of one octree overlap       */
#define DV_ERR_RANGE (-5)       /* level / index / corner out of range    */
#define DV_ERR_LIMIT (-6)       /* a size exceeds a documented limit      */
#define DV_ERR_TICKET (-7)      /* unknown serving ticket                 */
#define DV_ERR_SHUTDOWN (-8)    /* server is shutting down                */

/* Output selection (dv_render_opts.out_mask). */
#define DV_OUT_RGB 1u
#define DV_OUT_DEPTH 2u
#define DV_OUT_NORMAL 4u
#define DV_OUT_T 8u

/* Documented limits. */
#define DV_MAX_LEVEL 16         /* octree depth                           */
#define DV_MAX_SH_DEGREE 3
#define DV_MAX_OCTREES 4096     /* background + actors                    */
#define DV_MAX_TILE_ACTORS 255  /* actor boxes binned to one 16x16 tile   */
#define DV_MAX_K 16             /* midpoint samples per piece             */

typedef struct dv_ctx dv_ctx;
typedef struct dv_scene dv_scene;
typedef struct dv_fwd_state dv_fwd_state;
typedef struct dv_server dv_server;

/* One octree (Sec. 3.1 static background, Sec. 3.2 actor asset).
 * Only leaves are stored: leaf v at level[v] with integer cell ijk[:,v]
 * in [0, 2^level)^3 occupies root_min + ijk*h .. root_min + (ijk+1)*h,
 * h = root_size / 2^level, in the octree's own frame.  Corner m of a leaf
 * (m = mx + 2*my + 4*mz) holds raw density corner_density[corner_idx[m][v]]
 * (shared between leaves when indices coincide).  SH coefficients give the
 * view-dependent colour.  Leaves must not overlap.  For actors, the box
 * [box_min, box_max] (local frame) bounds the asset interval along rays;
 * with has_box = 0 the root cube is used (Sec. 3.3 'Assets'). */
typedef struct {
  double root_min[3];
  double root_size;             /* cube side, > 0                         */
  int32_t n_voxels;             /* N >= 0                                  */
  int32_t max_level;            /* all levels <= max_level <= 16           */
  int32_t n_corners;            /* Nc                                      */
  int32_t sh_degree;            /* 0..3                                    */
  const uint8_t* level;         /* device [N]                              */
  const int32_t* ijk;           /* device [3][N]                           */
  const int32_t* corner_idx;    /* device [8][N], values in [0, Nc)        */
  const float* corner_density;  /* device [Nc]; may change between calls   */
  const float* sh;              /* device [S][3][N]; may change            */
  int32_t has_box;
  double box_min[3];
  double box_max[3];
} dv_octree_desc;

/* Track of actor i (Sec. 3.2: rigid T_t^i from tracking).  Reading used
 * for the synthetic tracks: yaw about world +z and translation, each
 * linear in t between keyframes; the actor is active iff
 * t[0] <= t <= t[n_keys-1].  x_world = R(yaw) x_local + trans.
 * Host arrays; copied by dv_build_scene. */
typedef struct {
  int32_t n_keys;               /* >= 1, t strictly increasing             */
  const double* t;              /* host [n_keys]                           */
  const double* yaw;            /* host [n_keys] radians                   */
  const double* trans;          /* host [n_keys][3]                        */
} dv_track_desc;

/* Pinhole camera, OpenCV axes (x right, y down, z forward).  Rays pass
 * through pixel centres; tau is the Euclidean distance.  Only the window
 * [x0, x0+w) x [y0, y0+h) of the W x H image is rendered; outputs are
 * window-sized.  c2w is the row-major 3x4 camera-to-world matrix. */
typedef struct {
  double fx, fy, cx, cy;
  int32_t W, H;
  int32_t x0, y0, w, h;
  double c2w[12];
  double t;                     /* timestamp used to pose the actors       */
} dv_view;

typedef struct {
  int32_t K;                    /* midpoint samples per piece, 1..16       */
  float eps_stop;               /* stop a ray once T < eps_stop (Alg. 1)   */
  float tau_near;               /* rays start at tau_near >= 0             */
  float bg[3];                  /* constant sky colour C_sky (Eq. 2), used
                                   when sky is NULL                        */
  float explin_c;               /* knee of the exp-linear activation, > 0  */
  uint32_t out_mask;            /* DV_OUT_* bits                           */
  /* Sky environment map (Sec. 3.1; Eq. 2): device float [3][sky_h][sky_w],
   * caller-owned, or NULL for the constant bg.  A ray's world direction d
   * (z up) maps to longitude atan2(d_y, d_x) and colatitude acos(d_z);
   * u = (lon + pi) / (2 pi) sky_w - 1/2, v = colat / pi sky_h - 1/2 (texel
   * (i, j) centred at u = i, v = j), sampled bilinearly with columns
   * wrapping in longitude and rows clamped at the poles.  sky_w, sky_h >= 1
   * when sky is set (DV_ERR_INVALID otherwise). */
  const float* sky;
  int32_t sky_w, sky_h;
  /* Feature accumulation (Sec. 4.3, 3D semantic segmentation: the colour
   * step of the volume rendering replaced by a high-dimensional per-voxel
   * feature).  feat: NULL for the colour render, else a host array
   * [n_octrees] of device pointers, octree k's features [feat_dim][N_k]
   * (caller-owned, f32).  A feature render composites, in place of each
   * leaf's SH colour, its channels 3 feat_group .. 3 feat_group + 2
   * (channels >= feat_dim count as 0; no clamp, no view dependence) with
   * the same weights as the colour render, over a zero background (bg and
   * sky are ignored): out.rgb receives sum_i w_i f_i for those 3 channels.
   * Depth, normal and T are as in the colour render.  Its backward adds
   * dL/dfeature into dv_octree_grads.feat (and corner and pose gradients as
   * usual; features carry no SH term).  feat_dim >= 1 and
   * 0 <= 3 feat_group < feat_dim when feat is set (DV_ERR_INVALID
   * otherwise). */
  const float* const* feat;
  int32_t feat_dim;
  int32_t feat_group;
} dv_render_opts;

/* Per-view device output planes (window-sized, float).  Entries not in
 * out_mask may be NULL. */
typedef struct {
  float* rgb;                   /* [3][h][w]  C_voxels + T * C_sky         */
  float* depth;                 /* [h][w]     sum w_i (a_i + b_i) / 2      */
  float* normal;                /* [3][h][w]  sum w_i R n_i (world frame)  */
  float* T;                     /* [h][w]     final transmittance          */
} dv_outputs;

/* Per-view upstream gradients (device, same layout as dv_outputs); a
 * NULL plane counts as zero. */
typedef struct {
  const float* rgb;
  const float* depth;
  const float* normal;
  const float* T;
} dv_out_grads;

/* Gradient accumulators of one octree (device; results are ADDED). */
typedef struct {
  float* corner;                /* [Nc] or NULL                            */
  float* sh;                    /* [S][3][N] or NULL (colour renders)      */
  float* feat;                  /* [feat_dim][N] or NULL (feature renders:
                                   the render's 3 channels are added)     */
} dv_octree_grads;

typedef struct {
  const dv_octree_grads* octrees; /* host array [n_octrees]                */
  float* pose;                  /* device [n_views][n_actors][12] or NULL:
                                   dL/dR row-major (9) then dL/dp (3)      */
  float* sky;                   /* device [3][sky_h][sky_w] or NULL: dL/dsky
                                   added (atomics); ignored without a map  */
} dv_param_grads;

typedef struct {
  int32_t n_views;
  int64_t n_visible;            /* (view, leaf) records after culling      */
  int64_t n_pairs;              /* (leaf, tile) pairs                      */
  int64_t n_actor_pairs;        /* (actor box, tile) pairs                 */
  int64_t n_tiles;              /* 16x16 tiles over all windows            */
  int32_t key_bits;             /* bits of the record sort key             */
  int32_t tile_bits;            /* bits of the pair sort key               */
  int64_t n_items;              /* compositing work items: one per tile,
                                   several for a tile whose background list
                                   is split into chunks                    */
  int64_t n_chunk_slots;        /* chunks of the split tiles               */
  int64_t n_actor_items;        /* asset work items: one per (tile, actor)
                                   list, several for a split list          */
  int64_t n_actor_chunk_slots;  /* chunks of the split (tile, actor) lists */
} dv_state_info;

/* ---------------------------------------------------------------- context */
/* Device memory provider of a context.  The library keeps a caching pool of
 * device blocks for its per-call buffers (records, pairs, sort ping-pong,
 * per-pixel state) and for a scene's packed tables; the pool takes its
 * backing blocks from alloc and gives them back through free.
 *  - alloc(user, bytes, device, stream): `bytes` of device memory of
 *    `device` (the context's), usable in stream order on `stream` (a
 *    hipStream_t, NULL for the default stream); NULL if none is available
 *    (the pool then returns idle blocks through free and asks once more).
 *    Called from the thread of the library call that needs memory (for a
 *    server, its scheduler threads).
 *  - free(user, ptr, bytes, device, stream): gives back a block from alloc
 *    (same bytes); the device is idle when it is called, so the block may
 *    be reused at once on any stream.
 * With torch as the provider (torch.cuda.caching_allocator_alloc / _delete)
 * the library's scratch is torch's memory, counted by torch and shared with
 * its caching allocator. */
typedef struct {
  void* (*alloc)(void* user, size_t bytes, int32_t device, void* stream);
  void (*free)(void* user, void* ptr, size_t bytes, int32_t device,
               void* stream);
  void* user;
} dv_allocator;

/* Create a context on HIP device `hip_device`.  alloc: the device memory
 * provider (copied; its callbacks must stay valid until dv_ctx_destroy
 * returns), or NULL for hipMalloc / hipFree.  Work runs on the caller's
 * streams.  *out is set on success.  Errors: DV_ERR_INVALID (bad device,
 * alloc with a NULL callback), DV_ERR_OOM, DV_ERR_DEVICE. */
dv_status dv_ctx_create(int32_t hip_device, const dv_allocator* alloc,
                        dv_ctx** out);
/* Synchronise the device, then free every block (calls alloc's free). */
void dv_ctx_destroy(dv_ctx* ctx);
/* Wait for released forward states and hand every idle pool block back to
 * the provider (synchronises the device).  Blocks held by live scenes and
 * forward states stay. */
dv_status dv_ctx_trim(dv_ctx* ctx);
/* Bytes of pool blocks in use (scenes, forward states, calls in flight)
 * and cached (idle, kept for reuse); either pointer may be NULL. */
dv_status dv_ctx_memory(dv_ctx* ctx, int64_t* in_use, int64_t* cached);
/* Message of the last failing call on this thread ("" if none). */
const char* dv_last_error(void);
/* Library version string. */
const char* dv_version(void);

/* Per-stage device timing (HIP events on the caller's stream) and work
 * counters of the compositing kernels.  Enable with
 * dv_ctx_set_profiling(ctx, flags): bit 0 records events around every
 * stage, bit 1 counts the (pixel, list entry) tests and pieces composited
 * by the walks (one wave-reduced atomic per wave; costs a few percent, so
 * time without it).  dv_ctx_stage_times synchronises the recorded events,
 * adds their durations and optionally resets. */
#define DV_PROFILE_EVENTS 1
#define DV_PROFILE_COUNTERS 2
#define DV_NUM_STAGES 14
typedef struct {
  double ms[DV_NUM_STAGES];     /* summed device time per stage            */
  int64_t calls[DV_NUM_STAGES]; /* number of timed intervals               */
  int64_t entries_fwd;          /* (pixel, entry) slab tests, background
                                   walk, forward                           */
  int64_t pieces_fwd;           /* pieces composited, same                 */
  int64_t entries_bwd;          /* same, backward re-walk                  */
  int64_t pieces_bwd;
  int64_t entries_actor_fwd;    /* slab tests of asset-segment walks       */
  int64_t pieces_actor_fwd;
  int64_t entries_actor_bwd;
  int64_t pieces_actor_bwd;
  int64_t wave_entries_fwd;     /* list entries walked by a wave in the
                                   background walk's straight-line
                                   iteration, forward                      */
  int64_t wave_hits_fwd;        /* those where some lane had a chord       */
  int64_t wave_entries_bwd;     /* same, backward re-walk                  */
  int64_t wave_hits_bwd;
} dv_stage_times;
#define DV_NUM_COUNTERS 12
dv_status dv_ctx_set_profiling(dv_ctx* ctx, int32_t flags);
dv_status dv_ctx_stage_times(dv_ctx* ctx, dv_stage_times* out, int32_t reset);
/* Name of stage i (0 <= i < DV_NUM_STAGES), e.g. "composite_fwd". */
const char* dv_stage_name(int32_t i);

/* ---------------------------------------------------------------- scene */
/* Validate and index a scene: octrees[0] is the background O_bg,
 * octrees[1..] are actors with tracks[i-1] (Sec. 3.1-3.2; App. A inputs).
 * Copies leaf structure to the host for validation (no overlapping or
 * duplicate leaves, levels <= max_level <= 16, cells inside the root,
 * corner indices in range, SH degree 0..3) and builds packed device
 * geometry tables.  corner_density and sh stay caller-owned and are read
 * at every render.  Errors: DV_ERR_INVALID, DV_ERR_RANGE, DV_ERR_OVERLAP,
 * DV_ERR_LIMIT, DV_ERR_OOM, DV_ERR_DEVICE. */
dv_status dv_build_scene(dv_ctx* ctx, const dv_octree_desc* octrees,
                         int32_t n_octrees, const dv_track_desc* tracks,
                         dv_scene** out);
void dv_scene_destroy(dv_scene* scene);

/* Host-only validation of one octree's leaf structure (the checks of
 * dv_build_scene).  All pointers are host arrays.  Writes a message into
 * msg (capacity msg_len) on failure. */
dv_status dv_validate_octree_host(const uint8_t* level, const int32_t* ijk,
                                  const int32_t* corner_idx, int32_t n,
                                  int32_t max_level, int32_t n_corners,
                                  int32_t sh_degree, char* msg,
                                  int32_t msg_len);

/* Actor pose at time t from a track (host, FP64): R row-major 3x3 and p.
 * Returns 1 if the actor is active at t, else 0. */
int32_t dv_track_pose(const dv_track_desc* track, double t, double R[9],
                      double p[3]);

/* ---------------------------------------------------------------- render */
/* Render n_views views of the scene in one pass (Sec. 3.4; Alg. 1):
 * per-view leaf preprocessing (culling, tile rectangle, depth rank, SH
 * colour), tile binning, device radix sort, per-tile directories, and
 * the per-pixel compositing walk over the background and actor octrees.
 * pose_override: NULL (poses from tracks at view.t) or a host array
 * [n_views][n_actors][12] (R row-major, then p; all actors active).
 * keep: NULL, or receives a forward state that dv_render_backward needs;
 * release it with dv_fwd_state_release.  Synchronises the stream once, to
 * read the record and pair counts that size the record, pair and sort
 * arrays.  Errors: DV_ERR_INVALID, DV_ERR_LIMIT, DV_ERR_OOM,
 * DV_ERR_DEVICE. */
dv_status dv_render(dv_ctx* ctx, const dv_scene* scene, const dv_view* views,
                    int32_t n_views, const double* pose_override,
                    const dv_render_opts* opts, const dv_outputs* outs,
                    dv_fwd_state** keep, void* stream);

/* Reverse pass of dv_render (Sec. 3.4: gradients flow through each
 * segment; pose gradients go beyond the paper, which keeps tracks fixed).
 * Re-walks every pixel's pieces in forward order with identical FP32
 * arithmetic, accumulating gradients of corner densities, SH coefficients
 * and actor poses (R, p) into `acc`.  Poses use wave-reduced atomics.
 * Corner and SH gradients are added per record (SH by one kernel launch
 * per view, in which every leaf has at most one record, with plain
 * read-modify-write; corners by atomics), or, when the launch holds more
 * than 1.5 records per leaf (several views), per leaf after summing its
 * records over the views (one SH read-modify-write and 8 corner atomics
 * per leaf).  Either way the SH accumulators of different octrees must
 * not overlap.  g: host array [n_views] of device gradient planes.
 * Corner/SH/pose values must be those used by the forward call. */
dv_status dv_render_backward(dv_ctx* ctx, const dv_scene* scene,
                             const dv_fwd_state* state,
                             const dv_out_grads* g, const dv_param_grads* acc,
                             void* stream);

/* dv_render without any allocation, for callers that cannot allocate
 * device memory inside the call (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Same arguments and
 * results as dv_render with keep = NULL (no backward).  Every per-call
 * buffer (records, pairs, sort ping-pong, scan partials, per-pixel state)
 * is carved from one static device workspace of dv_noalloc_capacity()
 * bytes (128 MiB) per GPU, held from the library's first use on that GPU
 * until the process ends; host staging comes from a pinned block made by
 * dv_ctx_create.  The call allocates no device or pinned memory (host-side
 * bookkeeping uses the C++ heap).  A render whose buffers exceed the
 * workspace fails with DV_ERR_LIMIT and a message naming the need; kernels
 * enqueued before the failure may have written into the workspace, and the
 * outputs are then unspecified.  Calls on the same GPU share the one
 * workspace: calls on one stream are ordered, calls that overlap on
 * different streams race (serialise them).  Synchronises the stream once,
 * as dv_render does; profiling timers are not recorded for it. */
dv_status dv_render_noalloc(dv_ctx* ctx, const dv_scene* scene,
                            const dv_view* views, int32_t n_views,
                            const double* pose_override,
                            const dv_render_opts* opts, const dv_outputs* outs,
                            void* stream);
/* Size in bytes of the static workspace of dv_render_noalloc. */
int64_t dv_noalloc_capacity(void);

void dv_fwd_state_release(dv_fwd_state* state);
dv_status dv_fwd_state_info(const dv_fwd_state* state, dv_state_info* info);
/* Copy the sorted tile lists of one view to the host (synchronises):
 * tile_start [n_tiles_of_view + 1] and, for each entry, its octree and
 * leaf index; capacity = length of entry arrays.  Actor lists likewise
 * into actor_start [n_tiles_of_view + 1] / actor_oct (may be NULL). */
dv_status dv_fwd_state_export_lists(const dv_fwd_state* state, int32_t view,
                                    int64_t* tile_start, int32_t* entry_oct,
                                    int32_t* entry_leaf, int64_t capacity,
                                    int64_t* actor_start, int32_t* actor_oct,
                                    int64_t actor_capacity);

/* ---------------------------------------------------------------- training */
/* Training losses (Supp. 'Optimization Details', Training Losses), per
 * view, with the gradient planes of the rendered outputs written for
 * dv_render_backward:
 *   L = color ((1 - ssim) mean|C - C_gt| + ssim (1 - SSIM(C, C_gt)))
 *     + depth mean_{D_lidar > 0} |D - D_lidar|
 *     + normal mean_{|N_pseudo| > 0} (1 - cos(N, N_pseudo))
 *     + sky mean_{sky_mask > 0} (T_final - 1)^2.
 * Readings: the printed colour term is garbled; an L1 pixel loss and an
 * SSIM term are combined with weight `ssim` on SSIM.  SSIM uses an 11 x 11
 * Gaussian window (sigma 1.5), C1 = 0.01^2, C2 = 0.03^2, zero padding at
 * the border, the mean over pixels and channels.  cos = N.Np /
 * (max(|N|, 1e-8) |Np|).  Means over empty pixel sets are 0. */
typedef struct {
  int32_t h, w;                 /* image size (the render's window)        */
  const float* rgb;             /* rendered [3][h][w] (device), or NULL    */
  const float* depth;           /* [h][w] or NULL                          */
  const float* normal;          /* [3][h][w] or NULL                       */
  const float* T;               /* [h][w] or NULL                          */
  const float* rgb_gt;          /* target [3][h][w]; NULL: no colour term  */
  const float* depth_lidar;     /* sparse depth [h][w], 0 = no return      */
  const float* normal_pseudo;   /* [3][h][w], 0 vector = no normal         */
  const float* sky_mask;        /* [h][w], > 0 = sky                       */
  float* g_rgb;                 /* gradient planes, written (overwritten); */
  float* g_depth;               /* a term's plane is required when the term */
  float* g_normal;              /* has both its inputs (g_rgb), else may    */
  float* g_T;                   /* be NULL (the term's gradient is skipped) */
} dv_loss_view;

typedef struct {
  float color, ssim, depth, normal, sky;   /* the loss weights             */
} dv_loss_weights;

/* Losses of n_views views.  terms: device double [n_views][8], written:
 * total, colour term, L1, SSIM, depth, normal, sky, 0.  Enqueued on the
 * stream; allocates scratch from the context's pool.  Errors:
 * DV_ERR_INVALID (empty image, a colour term without g_rgb). */
dv_status dv_loss(dv_ctx* ctx, const dv_loss_view* views, int32_t n_views,
                  const dv_loss_weights* w, double* terms, void* stream);

/* One Adam step over structure-of-arrays parameters (corner densities, SH
 * coefficients, sky map, poses): for each element
 *   m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
 *   p -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps),
 * all tensors of the call in one launch.  All pointers device f32 of n
 * elements; p, m, v updated in place. */
typedef struct {
  float* p;
  const float* g;
  float* m;
  float* v;
  int64_t n;
} dv_adam_param;

typedef struct {
  double lr, beta1, beta2, eps; /* b1, 1 - b1, b2, 1 - b2 and the bias     */
                                /* corrections are formed in double, then  */
                                /* rounded to FP32 for the update          */
  int32_t step;                 /* >= 1 (bias correction)                  */
} dv_adam_opts;

dv_status dv_adam(dv_ctx* ctx, const dv_adam_param* params, int32_t n_params,
                  const dv_adam_opts* opts, void* stream);

/* ---------------------------------------------------------------- structure */
/* LiDAR-guided initialisation of the background octree (Sec. 3.3,
 * 'Initialization': proximity-based voxel subdivision and the soft density
 * prior, Eq. 1) and the structure edits of training (Sec. 3.1: adaptive
 * pruning and progressive subdivision; Supp. 'Adaptive Optimization
 * Schedule').  Points are device FP64 [3][n] (x row, y row, z row); every
 * call enqueues on the stream and synchronises it to read a few counts. */
typedef struct dv_edit dv_edit;

#define DV_EDIT_SUBDIVIDE 0
#define DV_EDIT_PRUNE 1

/* Exact Euclidean distance from each query ([3][n_queries] FP64) to its
 * nearest point, written to dist [n_queries] (FP64, device) when it is
 * below r_max, +inf otherwise (also for non-finite queries and when there
 * are no points).  Points hashed into a grid of r_max / 2 cells.  Errors:
 * DV_ERR_INVALID (r_max <= 0, non-finite points), DV_ERR_LIMIT (point
 * extent above 2^21 cells, 2^32 points). */
dv_status dv_nearest_distance(dv_ctx* ctx, const double* points, int64_t n_points,
                              const double* queries, int64_t n_queries,
                              double r_max, double* dist, void* stream);

/* Soft density prior (Eq. 1): every corner of the octree (leaf geometry
 * and corner_idx of `octree`; its densities and SH are not read) gets
 *   v = v_far + (v_close - v_far) exp(-2 d^2 / s^2),
 * d the distance from the corner's world position (root_min + finest-grid
 * position * root_size / 2^max_level) to the nearest point, written as
 * float to density [n_corners] (device).  Corners farther than r_cut from
 * every point, and corners no leaf uses, get v_far: with r_cut = 3 s the
 * omitted term is below |v_close - v_far| e^-18 (1.2e-7 for the paper's
 * v_close = -2, v_far = -10, under the float spacing at 10).  The paper
 * takes s as the minimum voxel size.  Errors: DV_ERR_INVALID, DV_ERR_RANGE
 * (a level, cell or corner index out of range), those of
 * dv_nearest_distance. */
dv_status dv_corner_prior(dv_ctx* ctx, const dv_octree_desc* octree,
                          const double* points, int64_t n_points, double s,
                          double v_close, double v_far, double r_cut,
                          float* density, void* stream);

/* Proximity rule of the initialisation's subdivision rounds: flags[v]
 * (device uint8 [n_voxels]) = 1 iff some point lies within ratio * h_v of
 * leaf v's closed box (Euclidean point-to-box distance, FP64; the paper
 * names a distance threshold without a value, reading: proportional to
 * the leaf side).  Errors: DV_ERR_INVALID, DV_ERR_RANGE. */
dv_status dv_proximity_flags(dv_ctx* ctx, const dv_octree_desc* octree,
                             const double* points, int64_t n_points, double ratio,
                             uint8_t* flags, void* stream);

/* Structure edit, planned on the device: op DV_EDIT_SUBDIVIDE splits the
 * leaves with flags[v] != 0 into their 8 children (DV_ERR_RANGE if one is
 * at max_level), DV_EDIT_PRUNE keeps only the leaves with flags[v] != 0.
 * New leaf order: the leaves that stay, in order, then the children of the
 * split leaves, parent by parent, child m = mx + 2 my + 4 mz.  New corner
 * table: one corner per distinct finest-grid position of the new leaves'
 * corners, in (i, j, k) lexicographic order.  A position held by an old
 * corner keeps its density; a new position (inside a split leaf) takes the
 * parent's trilinear field there (FP64, rounded to float), so the field
 * inside a split leaf is unchanged unless a finer neighbour already holds
 * a corner at a child corner position.  Positions are assumed to name one
 * old corner each (which survives is unspecified otherwise).  Children
 * take their parent's SH.  *n_leaves and *n_corners receive the new sizes;
 * *out the plan, which keeps device copies of the new tables until
 * dv_edit_release.  `octree`'s arrays (and its SH, read by dv_edit_apply)
 * must stay valid until dv_edit_apply's work has run.  Synchronises the
 * stream twice. */
dv_status dv_edit_plan(dv_ctx* ctx, const dv_octree_desc* octree,
                       const uint8_t* flags, int32_t op, dv_edit** out,
                       int64_t* n_leaves, int64_t* n_corners, void* stream);

/* Proximity-based subdivision rounds (initialisation step 2): while the
 * finest leaf is not below min_size, split the leaves (below max_level)
 * within ratio * h of a point; stop early when a round splits none or
 * after max_rounds.  The corner table is canonical (as dv_edit_plan's) even
 * after zero rounds.  Sources and densities as dv_edit_plan's, relative to
 * the input; each round interpolates the previous round's densities as
 * stored (float), as a sequence of dv_edit_plan calls would.  *rounds
 * receives the rounds done. */
dv_status dv_refine_plan(dv_ctx* ctx, const dv_octree_desc* octree,
                         const double* points, int64_t n_points, double ratio,
                         double min_size, int32_t max_rounds, dv_edit** out,
                         int64_t* n_leaves, int64_t* n_corners, int32_t* rounds,
                         void* stream);

/* Caller-allocated device outputs of a plan (sizes from the plan). */
typedef struct {
  uint8_t* level;               /* [n_leaves]                              */
  int32_t* ijk;                 /* [3][n_leaves]                           */
  int32_t* corner_idx;          /* [8][n_leaves]                           */
  float* corner_density;        /* [n_corners]                             */
  float* sh;                    /* [S][3][n_leaves] or NULL: gathered from
                                   the input's SH by leaf_src              */
  int32_t* leaf_src;            /* [n_leaves] or NULL: the input leaf each
                                   new leaf comes from (itself or parent)  */
  int32_t* corner_src;          /* [n_corners] or NULL: the input corner at
                                   the same position, -1 for a new one     */
} dv_edit_out;

/* Write a plan's tables into caller buffers (enqueued copies and one SH
 * gather).  May be called more than once. */
dv_status dv_edit_apply(dv_edit* edit, const dv_edit_out* out, void* stream);
void dv_edit_release(dv_edit* edit);

/* ---------------------------------------------------------------- serving */
/* Sensor simulation (Sec. 1: the reconstructed scene is rendered for new
 * cameras, timestamps and actor configurations): the scene and actor tracks
 * stay resident in HBM while render requests arrive; each request is one
 * view of the render above (camera, timestamp, resolution). */
typedef struct {
  int32_t max_inflight;         /* requests admitted at once (slots)       */
  int64_t mem_budget;           /* device bytes for in-flight requests     */
  int32_t batched;              /* 1: continuous batching (up to max_batch
                                   queued requests per multi-view launch,
                                   two launches in flight), 0: one launch
                                   per request in FIFO order (same two
                                   streams), 2: persistent drain kernel,
                                   refused (DV_ERR_INVALID) in this build  */
  int32_t max_batch;            /* requests per batched launch             */
  dv_render_opts opts;
} dv_serve_opts;

typedef struct {
  dv_view view;                 /* camera, resolution/window, timestamp    */
  dv_outputs out;               /* caller-owned device planes; must stay
                                   valid until poll returns DV_OK          */
} dv_request;

typedef struct {
  dv_status status;             /* DV_OK, DV_PENDING or an error           */
  double t_submit;              /* seconds, monotonic clock                */
  double t_admit;
  double t_done;
} dv_result;

/* Start a serving loop on `scene` (kept resident; the scene must outlive
 * the server).  Two worker threads admit queued requests while slots and
 * memory allow, render them in batched launches that overlap on the
 * device, and mark them done.  Errors: DV_ERR_INVALID, DV_ERR_OOM. */
dv_status dv_serve_create(dv_ctx* ctx, const dv_scene* scene,
                          const dv_serve_opts* opts, dv_server** out);
/* Queue a request (thread-safe); *ticket identifies it.  A malformed
 * request still gets a ticket whose poll reports DV_ERR_INVALID. */
dv_status dv_serve_submit(dv_server* srv, const dv_request* req,
                          uint64_t* ticket);
/* Status of a ticket, waiting up to wait_us microseconds (0: no wait,
 * <0: wait until finished).  Returns the request's status (DV_OK,
 * DV_PENDING or its error) and fills *res.  A finished ticket is
 * forgotten after its final status has been returned once. */
dv_status dv_serve_poll(dv_server* srv, uint64_t ticket, int32_t wait_us,
                        dv_result* res);
/* Drain, stop and free the server. */
dv_status dv_serve_destroy(dv_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* DV_H */
