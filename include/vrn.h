/*
 * vrn.h -- C ABI of the MI355X-native VR-NeRF renderer hot path
 * (Xu et al., "VR-NeRF: High-Fidelity Virtualized Walkable Spaces",
 * SIGGRAPH Asia 2023, arXiv 2311.02542).
 *
 * The library renders an instant-NGP-style radiance field ray by ray:
 *   occupancy-bitfield lattice march (Sec. 4.3, binary occupancy grid),
 *   multiresolution hash encoding with LOD mip-mapping (Sec. 4.2.1, Eq. 3;
 *   dense coarse levels and skipped fine levels, App. D),
 *   density MLP (1 hidden layer of 64) and color MLP (2 hidden layers of 64,
 *   sigmoid in PQ units) (Sec. 5 and Sec. 6; Sec. 4.1),
 *   front-to-back alpha compositing with early termination into an HDR
 *   framebuffer of PQ values (Sec. 4.1, Eq. 1-2), optionally decoded to
 *   linear HDR (linear 1.0 = 100 cd/m^2).
 *
 * Conventions
 *   - Every pointer marked "host" is read during the call only; the library
 *     keeps its own copies.  Pointers marked "device" are HIP device memory
 *     owned by the caller.  hip_stream is a hipStream_t (NULL = default
 *     stream).  Work is enqueued asynchronously on that stream; the caller
 *     synchronises it before reading outputs.
 *   - All functions return vrn_status.  Arguments are validated on the host
 *     before anything is enqueued; on failure nothing is enqueued and
 *     vrn_last_error() describes the problem.  Device faults surface as
 *     VRN_ERR_DEVICE on the same or a later call.
 *   - A context is guarded by one internal mutex; calls on one context from
 *     several threads are serialised.  Renders that overlap on the device
 *     (different streams) must use different workspaces.
 *   - Sizes are in elements unless the name says bytes.
 */
#ifndef VRN_H
#define VRN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vrn_ctx vrn_ctx;
typedef uint32_t vrn_field_id;

typedef enum {
  VRN_OK = 0,
  VRN_ERR_INVALID_ARG = -1,   /* NULL / NaN / degenerate / out-of-range argument */
  VRN_ERR_UNSUPPORTED = -2,   /* valid but not implemented (e.g. F != 2, L > 16) */
  VRN_ERR_OUT_OF_MEMORY = -3, /* hipMalloc failed */
  VRN_ERR_BUDGET = -4,        /* would exceed the context's HBM budget */
  VRN_ERR_DEVICE = -5,        /* no usable GPU, or a HIP runtime error */
  VRN_ERR_NOT_FOUND = -6,     /* unknown field id */
  VRN_ERR_BUSY = -7,          /* field still in use; request not finished */
  VRN_ERR_TIMEOUT = -8,       /* serving: the request passed its deadline */
  VRN_ERR_CANCELLED = -9      /* serving: the request was cancelled */
} vrn_status;

/* MLP arithmetic (and table storage: VRN_F32 or VRN_F16).  VRN_F32X is FP32
 * arithmetic computed on the BF16 matrix cores: each FP32 operand is split
 * exactly into three BF16 parts and six of the nine part products are
 * accumulated in FP32 (the dropped ones are about 2^-26 of the product,
 * below FP32 rounding); encoding, transmittance and compositing are FP32 as
 * in VRN_F32. */
typedef enum { VRN_F32 = 0, VRN_F16 = 1, VRN_BF16 = 2, VRN_F32X = 3 } vrn_dtype;

/* Everything that defines a field.  Host pointers; copied by vrn_load_field. */
typedef struct {
  uint32_t n_levels;          /* L, 1..16 hash-grid levels */
  uint32_t log2_T;            /* table size T = 2^log2_T entries per level, 4..24 */
  uint32_t n_feat;            /* F, must be 2 */
  const uint32_t* level_res;  /* host [L]: integer lattice resolution N_l >= 1
                                 (lattice of N_l + 1 points per axis; a level is
                                 stored densely when (N_l + 1)^3 <= T) */
  uint32_t hash_primes[3];    /* spatial hash (c0*p0 ^ c1*p1 ^ c2*p2) mod T */
  float base_res;             /* s: LOD level-0 resolution (Sec. 4.2.1) */
  float growth;               /* f: per-level scale factor, > 1 when lod_enable */
  int32_t table_dtype;        /* a vrn_dtype: VRN_F32 or VRN_F16 (int32_t, so that any value a
                                 caller stores is well defined to read; others are refused) */
  const void* tables;         /* host [L][T][F], feature fastest, finite values */
  uint32_t mlp_in;            /* density MLP input width, must be 2 * L */
  uint32_t mlp_hidden;        /* must be 64 */
  uint32_t geo_out;           /* density MLP output width, must be 16 (sigma + 15) */
  uint32_t sh_bands;          /* direction SH bands, 1..4 (bands^2 coefficients) */
  const float* weights;       /* host, concatenated row-major [in][out]:
                                 W1[2L][64] b1[64] W2[64][16] b2[16]
                                 W3[15+bands^2][64] b3[64] W4[64][64] b4[64]
                                 W5[64][3] b5[3] */
  uint32_t occ_res;           /* G, 1..1024 */
  const uint32_t* occ_bits;   /* host, G^3 bits, bit i = x + G*(y + G*z), LSB first */
  float aabb_min[3];          /* the field occupies the cube [aabb_min, aabb_min + extent] */
  float extent;               /* > 0 */
  float dt;                   /* lattice step: samples at t_k = (k + 1/2) dt, > 0 */
  uint32_t max_samples;       /* cap on evaluated (occupied) samples per ray, >= 1 */
  float t_min;                /* early termination once transmittance < t_min, [0, 1) */
  int32_t lod_enable;         /* 0: all levels weight 1; 1: Eq. 3 weights */
  float lod_bias;             /* Delta L added to L* (Sec. 4.2.2) */
  float lod_radius_scale;     /* r = scale * distance of adjacent unit-distance ray points */
  /* unbounded scenes (Sec. 4: L-infinity cubic contraction) and the
   * exponential sample schedule (Sec. 6: exponential distances) */
  int32_t contraction;        /* 0: bounded cube; 1: u = (x - center) / radius,
                                 C(u) = u if |u|inf <= 1 else (2 - 1/|u|inf) u / |u|inf;
                                 then aabb_min must be -2 and extent 4 */
  float center[3];
  float radius;               /* > 0 when contraction = 1 */
  float step_growth;          /* 0: uniform t_k = (k + 1/2) dt; > 0: FP32 table
                                 t_0 = dt/2, t_{k+1} = t_k + max(dt, growth t_k);
                                 contraction requires a table */
  uint32_t max_lattice;       /* table length, 1..65536, when a table is used */
} vrn_field_desc;

/* One pinhole camera.  c2w is row-major 3x4 camera-to-world with OpenCV axes
 * (+x right, +y down, +z forward); pixel centres at +0.5.  Only rows
 * [row_begin, row_end) are rendered (one GPU's share of a frame); the
 * framebuffer is still addressed as the full image. */
typedef struct {
  float c2w[12];
  float fx, fy, cx, cy;
  uint32_t row_begin, row_end;
} vrn_camera;

typedef enum {
  VRN_OUT_PQ = 0,             /* PQ RGB as composited (Sec. 4.1) */
  VRN_OUT_LINEAR = 1,         /* linear HDR: 100 * PQ^-1 per channel (linear 1 = 100 cd/m^2) */
  VRN_OUT_SRGB = 2            /* display: sRGB transfer of clip(2^exposure_ev * linear, 0, 1)
                                 (render-time exposure, Fig. exposure-swipe) */
} vrn_output;

typedef struct {
  int32_t compute;            /* a vrn_dtype, the MLP arithmetic: VRN_F32 (FP32 MFMA), VRN_F32X
                                 (FP32 by split BF16 MFMA), VRN_F16 or
                                 VRN_BF16 (MFMA, FP32 accumulate); march,
                                 transmittance and compositing are FP32 always.
                                 VRN_F16 needs hidden activations within the FP16
                                 range (|x| <= 65504); beyond it they overflow */
  int32_t output;             /* vrn_output; alpha is 1 - T in every mode */
  uint32_t march_budget;      /* lattice steps per march round, 0 = default */
  float exposure_ev;          /* exposure in stops for VRN_OUT_SRGB */
} vrn_render_opts;

/* Work counters accumulated in a workspace by every render. */
typedef struct {
  uint64_t rays;              /* rays finished (pixels written) */
  uint64_t samples;           /* evaluated samples composited */
  uint64_t level_fetches;     /* hash levels gathered (8 corners each) */
  uint64_t march_steps;       /* canonical lattice tests + block skips */
  uint64_t rounds;            /* wave rounds (march, then encode + MLP of the samples found) */
  uint64_t tiles;             /* 16-sample MLP tiles evaluated */
} vrn_stats;

#define VRN_MAX_CAMS 16

/* Open device `device` (HIP ordinal).  hbm_budget_bytes bounds the memory of
 * resident fields (0 = no bound).  VRN_ERR_DEVICE when no GPU is usable. */
vrn_status vrn_create(int device, uint64_t hbm_budget_bytes, vrn_ctx** out);

/* Free every field and internal buffer; waits for the device. NULL is a no-op. */
void vrn_destroy(vrn_ctx* ctx);

/* Thread-local description of the last failure on this thread. */
const char* vrn_last_error(void);

/* Validate a field -- the multiresolution hash grid of Sec. 4 (after iNGP),
 * the density and color MLPs of Sec. 6 and the binary occupancy grid of
 * Sec. 4.3 -- and copy it into library-owned device memory (tables as given,
 * occupancy bits plus a coarse block mip, MLP weights re-laid out for MFMA in
 * FP32, FP16 and BF16).  The field stays resident until unloaded. */
vrn_status vrn_load_field(vrn_ctx* ctx, const vrn_field_desc* desc, vrn_field_id* out);

/* Free a field.  VRN_ERR_BUSY while renders that use it are still running,
 * or while a serving engine holds output buffers (and their graphs) for it
 * (vrn_server_evict, vrn_server_destroy).  Renders enqueued under the
 * caller's own HIP graph capture are not tracked: the caller keeps the field
 * loaded while a graph that renders it can still be replayed. */
vrn_status vrn_unload_field(vrn_ctx* ctx, vrn_field_id field);

/* Device bytes held by a resident field. */
vrn_status vrn_field_bytes(vrn_ctx* ctx, vrn_field_id field, uint64_t* out);

/* Bytes of device workspace one render needs (counters, cameras, stats). */
vrn_status vrn_workspace_bytes(vrn_ctx* ctx, uint64_t* out);

/* Device bytes one render of n_cams cameras of W x H pixels of `field`
 * needs beyond the resident field, for admission against an HBM budget: a
 * workspace plus the caller's RGBA framebuffer ([n_cams][H][W][4] float) and
 * sample counts ([n_cams][H][W] uint32).  No device work.  VRN_ERR_INVALID_ARG
 * for sizes no render accepts, VRN_ERR_NOT_FOUND for an unknown field. */
vrn_status vrn_render_bytes(vrn_ctx* ctx, vrn_field_id field, uint32_t n_cams, uint32_t W, uint32_t H,
                            const vrn_render_opts* opts, uint64_t* out);

/* Zero a caller-owned workspace with a kernel on hip_stream (safe inside
 * graph capture).  Required once before a workspace's first render; a render
 * leaves its counters at zero again, and the stats keep accumulating. */
vrn_status vrn_workspace_init(vrn_ctx* ctx, void* d_workspace, uint64_t workspace_bytes,
                              void* hip_stream);

/* Render n_cams (1..VRN_MAX_CAMS) cameras of W x H pixels: per ray the
 * occupancy march (Sec. 4.3), the hash encoding with LOD weights (Sec. 4.2.1,
 * Eq. 3; App. D), the density and color MLPs (Sec. 6) and front-to-back
 * compositing with early termination into PQ color (Sec. 4.1, Eq. 1-2), all
 * in one kernel launch (the single-kernel interleave of Sec. 5).
 *   cams        host [n_cams]; validated (finite, det(R) != 0, fx, fy > 0,
 *               row_begin < row_end <= H); copied into the workspace.
 *   d_rgba      device [n_cams][H][W][4] float: PQ (or linear) RGB, alpha = 1 - T.
 *   d_nsamples  device [n_cams][H][W] uint32 evaluated samples per pixel, or NULL.
 *   d_workspace device, >= vrn_workspace_bytes, initialised once by
 *               vrn_workspace_init; NULL uses the context's own workspace
 *               (then renders on one context must not overlap).
 * Only pixels in each camera's row share are written. */
vrn_status vrn_render(vrn_ctx* ctx, vrn_field_id field, const vrn_camera* cams, uint32_t n_cams,
                      uint32_t W, uint32_t H, const vrn_render_opts* opts, float* d_rgba,
                      uint32_t* d_nsamples, void* d_workspace, uint64_t workspace_bytes,
                      void* hip_stream);

/* As vrn_render (same passages), but the cameras are already in device memory (d_cams,
 * [n_cams] vrn_camera) and are NOT validated here (use vrn_check_cameras on
 * the host copy).  Enqueues kernels only, so it can be captured in a HIP
 * graph and replayed with new camera contents. */
vrn_status vrn_render_device_cams(vrn_ctx* ctx, vrn_field_id field, const vrn_camera* d_cams,
                                  uint32_t n_cams, uint32_t W, uint32_t H,
                                  const vrn_render_opts* opts, float* d_rgba, uint32_t* d_nsamples,
                                  void* d_workspace, uint64_t workspace_bytes, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): as
 * vrn_render_device_cams, but the render's queue, completion and statistics
 * counters live in a static scratch array of the library (1 KiB per device,
 * held until the process ends) instead of a workspace.  The call allocates
 * nothing: no hipMalloc, no hipFree, no event creation (the field's tracking
 * event is made when the field is loaded).  It enqueues a fill kernel that
 * clears the counters, then the render kernel, on hip_stream.
 *   d_cams      device [n_cams] vrn_camera, NOT validated (vrn_check_cameras).
 *   d_rgba, d_nsamples as in vrn_render.
 * Limits: n_cams 1..VRN_MAX_CAMS, W and H 1..16384, n_cams*W*H <= 2^31;
 * anything beyond is VRN_ERR_INVALID_ARG before any device work.  Every call
 * on one GPU shares that GPU's scratch: calls that overlap on the device (on
 * different streams without ordering) race and give wrong images, so keep
 * them on one stream or order them.  The stats the scratch accumulates are
 * those of the last call and are not readable through vrn_read_stats. */
vrn_status vrn_render_noalloc(vrn_ctx* ctx, vrn_field_id field, const vrn_camera* d_cams,
                              uint32_t n_cams, uint32_t W, uint32_t H, const vrn_render_opts* opts,
                              float* d_rgba, uint32_t* d_nsamples, void* hip_stream);

/* Host-side camera validation used by vrn_render (no device work). */
vrn_status vrn_check_cameras(const vrn_camera* cams, uint32_t n_cams, uint32_t W, uint32_t H);

/* Read (synchronously) the stats a workspace has accumulated. */
vrn_status vrn_read_stats(vrn_ctx* ctx, const void* d_workspace, vrn_stats* out, void* hip_stream);

/* ---- stage entry points: the same device code as vrn_render, one stage at
 *      a time, for parity tests and profiling.  vrn_rays and vrn_march copy
 *      their cameras into the context's own workspace, so they must not
 *      overlap on the device with renders that use it. ---- */

/* Canonical FP32 rays of every pixel of every camera, pixel order
 * (cam, row, col): d_o, d_d device [n][3] float, d_r device [n] float cone
 * pitch at unit distance (Sec. 4.2.1).  Cameras: host, validated. */
vrn_status vrn_rays(vrn_ctx* ctx, const vrn_camera* cams, uint32_t n_cams, uint32_t W, uint32_t H,
                    float lod_radius_scale, float* d_o, float* d_d, float* d_r, void* hip_stream);

/* Occupancy march without compositing (Sec. 4.3): for every pixel (cam, row,
 * col) the evaluated lattice indices k in increasing order, capped at the
 * field's max_samples and at max_k.  d_klist device [n][max_k] uint32,
 * d_count device [n] uint32 (the uncapped-by-max_k count). */
vrn_status vrn_march(vrn_ctx* ctx, vrn_field_id field, const vrn_camera* cams, uint32_t n_cams,
                     uint32_t W, uint32_t H, uint32_t* d_klist, uint32_t max_k, uint32_t* d_count,
                     void* hip_stream);

/* Hash encoding with LOD (Sec. 4.2.1, App. D) of n world points d_xyz
 * [n][3] at ray distance d_t [n] with cone pitch d_r [n] (both ignored when
 * LOD is off): d_feat device [n][2L] float, level-major, feature fastest. */
vrn_status vrn_encode(vrn_ctx* ctx, vrn_field_id field, const float* d_xyz, const float* d_t,
                      const float* d_r, uint32_t n, float* d_feat, void* hip_stream);

/* Density + color MLPs (Sec. 6: one hidden layer of 64 for density, two for
 * color; sigmoid in PQ units, Sec. 4.1) on MFMA in the requested dtype for n samples:
 * d_feat [n][2L], d_dir [n][3] unit view directions -> d_sigma [n]
 * (exp of density output 0), d_rgb [n][3] (sigmoid, PQ units). */
vrn_status vrn_mlp(vrn_ctx* ctx, vrn_field_id field, const float* d_feat, const float* d_dir,
                   uint32_t n, vrn_dtype compute, float* d_sigma, float* d_rgb, void* hip_stream);

/* ---- occupancy maintenance ---- */

/* Grid-based occupancy pruning (Sec. 4.3, the grid half of its joint
 * pruning; App. C: 4 evenly placed points per voxel).  For every occupied
 * voxel of the resident field, the density MLP (all hash levels, no LOD) is
 * evaluated at points_per_voxel points -- 4: the alternating corners of the
 * voxel's 2x2x2 sub-lattice at offsets {1/4, 3/4}; 1, 8, 27, 64: a p^3 grid
 * at (i + 1/2) / p -- and the voxel is kept iff the worst-case opacity
 * 1 - exp(-sigma_max dt) >= alpha.  Pruning only clears bits.
 *   d_bits_out     device, ceil(G^3 / 32) uint32 words, bit i = x + G*(y + G*z).
 *   d_max_opacity  device [G^3] float (NaN for unoccupied voxels) or NULL.
 * The resident field is not modified (see vrn_set_occupancy). */
vrn_status vrn_prune_grid(vrn_ctx* ctx, vrn_field_id field, float alpha, uint32_t points_per_voxel,
                          vrn_dtype compute, uint32_t* d_bits_out, float* d_max_opacity, void* hip_stream);

/* Replace a resident field's occupancy grid (Sec. 4.3) with device bits (same layout as
 * vrn_field_desc.occ_bits), rebuilding its bricks and coarse grids on
 * hip_stream.  Renders of this field on other streams must be ordered by
 * the caller. */
vrn_status vrn_set_occupancy(vrn_ctx* ctx, vrn_field_id field, const uint32_t* d_bits, void* hip_stream);

/* ---- serving engine: continuous batching of render requests ----
 *
 * A serving loop around the single-kernel renderer of Sec. 5, whose
 * latency percentiles matter because the p99 frame rate is the quality
 * measure of the performance evaluation (Sec. 6): requests of mixed
 * resolutions over the resident fields of one context are queued and
 * launched as slots free up, and a finished request's result stays in
 * device memory until the client releases it.
 *
 *   - A slot is a HIP stream of default priority with its own workspace
 *     and camera buffers; up to n_slots renders run at once.
 *   - When a slot is free, the oldest pending request is launched together
 *     with the single-camera requests of the same field and size queued
 *     behind it, up to max_batch cameras in one launch.
 *   - A bucket is (field, W, H, cameras in the launch).  Each slot keeps,
 *     per bucket, a ring of output buffers carved from one device arena;
 *     with use_graphs each buffer has a captured HIP graph (camera upload
 *     from the slot's pinned buffer, then the render into that buffer), so
 *     a launch is a host memcpy and one graph launch.
 *   - Admission is the arena: every ring buffer, held by a client or free,
 *     lives in it; free buffers are evicted least-recently-used when a new
 *     one does not fit, and a request that fits only once held results are
 *     released waits for them.  A request larger than the arena is refused
 *     at submission.
 *   - A request may carry a deadline: still queued at its deadline it is
 *     never launched; finished after it, its result is discarded.
 *   - One scheduler thread per engine makes every device call of serving;
 *     the vrn_server_* calls below are thread-safe.  Times are seconds on
 *     vrn_server_clock() (a monotonic clock).
 */
typedef struct vrn_server vrn_server;

typedef struct {
  uint32_t n_slots;           /* concurrent renders, 1..16 */
  uint32_t max_batch;         /* cameras per launch when requests merge, 1..VRN_MAX_CAMS */
  int32_t use_graphs;         /* 1: one captured HIP graph per ring buffer; 0: eager launches */
  vrn_render_opts render;     /* every render of the engine (compute, output, ...) */
  void* d_arena;              /* device memory for results, owned by the caller and
                                 untouched by the engine outside its ring buffers;
                                 NULL: the engine allocates arena_bytes itself */
  uint64_t arena_bytes;       /* >= 256 */
} vrn_server_opts;

#define VRN_SERVE_RELEASE_ON_DONE 1u  /* latency-only client: the buffer returns to its ring
                                         at completion (the record stays until release) */

typedef struct {
  double t_arrival;           /* arrival on vrn_server_clock(); <= 0: the time of the call */
  double timeout_s;           /* arrival-to-completion bound; 0: none */
  uint32_t flags;             /* VRN_SERVE_* */
} vrn_request_opts;

typedef struct {
  int32_t status;             /* VRN_OK, VRN_ERR_TIMEOUT, VRN_ERR_CANCELLED, VRN_ERR_BUDGET
                                 (could never be admitted), VRN_ERR_NOT_FOUND (field
                                 unloaded), VRN_ERR_DEVICE; VRN_ERR_BUSY: not finished */
  vrn_field_id field;
  uint32_t n_cams, W, H;
  float* d_rgba;              /* device [n_cams][H][W][4] in the arena, valid until
                                 vrn_server_release; NULL unless status is VRN_OK and
                                 the result is held */
  uint32_t* d_nsamples;       /* device [n_cams][H][W] evaluated samples, as d_rgba */
  double t_arrival, t_launch, t_done;  /* t_launch = 0: never launched */
} vrn_served;

typedef struct {
  uint64_t arena_bytes, used_bytes, held_bytes, largest_free_bytes;
  uint64_t pending, running, requests;  /* queued; in flight; submitted and not released */
  uint64_t buffers, buckets;  /* ring buffers; distinct (slot, bucket) rings */
  uint64_t launches, graph_launches, merged_requests, captures, evictions;
  uint64_t completed, failed;
} vrn_serve_stats;

/* Create an engine over ctx's resident fields.  The engine starts held (no
 * launches) until vrn_server_hold(sv, 0).  VRN_ERR_INVALID_ARG for options
 * out of range, VRN_ERR_OUT_OF_MEMORY / VRN_ERR_DEVICE when its streams,
 * workspaces or arena cannot be made.  ctx must outlive the engine. */
vrn_status vrn_server_create(vrn_ctx* ctx, const vrn_server_opts* opts, vrn_server** out);

/* Stop the scheduler, wait for renders in flight, free every buffer and
 * graph, and unpin the fields.  Results not yet released become invalid.
 * NULL is a no-op. */
void vrn_server_destroy(vrn_server* sv);

/* hold != 0: launch nothing new (completions, deadlines and cancellations
 * are still processed); hold = 0: serve. */
vrn_status vrn_server_hold(vrn_server* sv, int hold);

/* Allocate (and with use_graphs capture) one ring buffer per slot for the
 * bucket (field, W, H, n_cams) if the slot has none, so that serving does
 * not capture.  Waits for the slot's render in flight, if any.
 * VRN_ERR_BUDGET when the buffer does not fit the arena's free space. */
vrn_status vrn_server_prepare(vrn_server* sv, vrn_field_id field, uint32_t n_cams, uint32_t W, uint32_t H);

/* Queue a request of n_cams host cameras (validated as in vrn_render,
 * copied) of W x H pixels of `field`; opts may be NULL.  *id names it in
 * the calls below.  VRN_ERR_BUDGET if its outputs exceed the arena,
 * VRN_ERR_NOT_FOUND for an unknown field. */
vrn_status vrn_server_submit(vrn_server* sv, vrn_field_id field, const vrn_camera* cams, uint32_t n_cams,
                             uint32_t W, uint32_t H, const vrn_request_opts* opts, uint64_t* id);

/* Wait up to max_wait_s (0: do not wait) for request id, then describe it
 * in *out.  VRN_OK once the request has finished (its outcome is
 * out->status); VRN_ERR_BUSY if it has not; VRN_ERR_NOT_FOUND for an
 * unknown or released id. */
vrn_status vrn_server_wait(vrn_server* sv, uint64_t id, double max_wait_s, vrn_served* out);

/* Forget a finished request and return its output buffer to its ring; its
 * d_rgba / d_nsamples must no longer be read.  VRN_ERR_BUSY while it has
 * not finished (cancel it first). */
vrn_status vrn_server_release(vrn_server* sv, uint64_t id);

/* Cancel a request: a queued one finishes at once with VRN_ERR_CANCELLED;
 * a running one does so when its render completes (the result is
 * discarded).  VRN_ERR_BUSY when it has already finished. */
vrn_status vrn_server_cancel(vrn_server* sv, uint64_t id);

/* Wait up to max_wait_s until nothing is queued or running.  VRN_ERR_BUSY
 * if that does not happen in time. */
vrn_status vrn_server_drain(vrn_server* sv, double max_wait_s);

/* Free the free ring buffers (and graphs) of `field`, or of every field
 * when field is 0, and unpin fields left without buffers.  VRN_ERR_BUSY if
 * buffers of it remain because they are held or in flight. */
vrn_status vrn_server_evict(vrn_server* sv, vrn_field_id field);

/* Counters and memory of the engine; VRN_ERR_DEVICE (with the counters
 * filled) once a HIP error has been seen in serving. */
vrn_status vrn_server_stats(vrn_server* sv, vrn_serve_stats* out);

/* The engine's clock: seconds, monotonic. */
double vrn_server_clock(void);

/* ---- debugging ---- */

/* Counters of a library built with -DVRN_DEBUG_CHECKS (synchronises the
 * device first): out[0] hash-table offsets outside their level, out[1]
 * brick and out[2] coarse-grid indices outside the grid, out[3] framebuffer
 * writes outside the frame, out[4] NaN encoded features, out[5] NaN MLP
 * outputs.  The kernels count instead of trapping.  reset != 0 zeroes the
 * counters after reading.  VRN_ERR_UNSUPPORTED in release builds. */
vrn_status vrn_debug_counters(vrn_ctx* ctx, uint64_t out[6], int reset);

/* Where render waves spend their time, in a library built with
 * -DVRN_PHASE_TIMING (synchronises the device first): shader clocks
 * (s_memtime) summed over the waves of every render since the last reset,
 * per step of a wave's round -- out[0] refill (new rays and their set-up),
 * out[1] march (with the compaction of the samples found), out[2] encode
 * (gathering each tile's samples and the hash-grid encode), out[3] MLP,
 * out[4] return of the MLP results to the rays' lanes, out[5] compositing
 * (and, once per wave, the block's set-up).  reset != 0 zeroes the sums
 * after reading.  VRN_ERR_UNSUPPORTED in other builds. */
vrn_status vrn_phase_cycles(vrn_ctx* ctx, uint64_t out[6], int reset);

#ifdef __cplusplus
}
#endif

#endif /* VRN_H */
