/*
 * nvgs.h -- C ABI of the NVGS per-frame renderer for composed 3D Gaussian
 * Splatting scenes on AMD Instinct MI355X (gfx950).
 *
 * The method ("NVGS: Neural Visibility for Occlusion Culling in 3D Gaussian
 * Splatting", Sec. 3.3) stores every asset once together with a list of
 * instance transforms.  Per frame and per camera it
 *   1. frustum-culls every Gaussian of every instance on its mean,
 *   2. queries a small per-asset visibility MLP for every in-frustum
 *      (instance, Gaussian) pair, with the camera moved into the asset frame
 *      and corrected for FoV and instance scale (Eq. 2),
 *   3. instantiates only the surviving pairs,
 *   4. projects them to 2D (EWA splatting, as in original 3DGS),
 *   5. bins them into screen tiles ordered by (tile, depth, id), and
 *   6. composites front to back, skipping alpha < 1/255 and stopping before
 *      transmittance would fall below 1e-4 (Sec. 4.1).
 * The MLP is trained per asset on visibility labels, where a Gaussian is
 * visible from a view if its contribution alpha*T to some pixel is non-zero
 * (Sec. 3.1, 3.2).
 *
 * Conventions
 *  - All entry points return nvgs_status and never throw.  On a non-OK
 *    status nvgs_last_error() describes the failure.
 *  - "device" pointers are HIP device memory of the context's device,
 *    "host" pointers are ordinary host memory.  Device inputs are borrowed:
 *    asset arrays until the next nvgs_load_assets / nvgs_destroy, per-call
 *    inputs and outputs until the call's work on the context stream is done.
 *  - Work is enqueued on the context stream; a call synchronises only where
 *    its comment says so.
 *  - A context is not thread-safe; use one context per stream.
 *  - Cameras: world -> camera rotation R with rows (right, down, forward),
 *    the camera looks along +z_cam, fovy is the vertical field of view in
 *    radians, square pixels, principal point (W/2, H/2), pixel centres at
 *    integer + 0.5.
 */
#ifndef NVGS_H_
#define NVGS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t nvgs_status;
#define NVGS_OK 0
#define NVGS_E_INVALID 1  /* bad argument: null pointer, n <= 0, bad enum, non-finite value ... */
#define NVGS_E_STATE 2    /* call order: render before load_assets / set_instances, ... */
#define NVGS_E_NOMEM 3    /* device allocation failed */
#define NVGS_E_CAPACITY 4 /* a planned capacity was exceeded; outputs undefined; call again */
#define NVGS_E_DEVICE 5   /* HIP runtime error (text in nvgs_last_error) */

#define NVGS_PREC_FP32 0 /* MLP operands in FP32, FP32 accumulation */
#define NVGS_PREC_BF16 1 /* MLP operands in BF16 (round to nearest even), FP32 accumulation */
#define NVGS_PREC_FP8 2  /* MLP operands in OCP FP8 E4M3 with per-layer scales, FP32 accumulation */
/* FP32 MLP on BF16 matrix cores: every FP32 operand x of the hidden layers is
 * split into x_hi = bf16(x) and x_lo = bf16(x - x_hi), and each product is
 * formed as a_hi b_hi + a_hi b_lo + a_lo b_hi with FP32 accumulation (the
 * dropped a_lo b_lo and the split's residuals are below 2^-16 relative); layer
 * 1 and the output layer stay in FP32.  Logits meet the FP32 contract (1e-5
 * relative to the logit scale).  Frequency form only. */
#define NVGS_PREC_FP32_SPLIT 3

#define NVGS_RENDER_RECORD_CONTRIB 1u /* write per-pair max alpha*T into opts->contrib */
#define NVGS_RENDER_KEEP_DEBUG 2u     /* keep per-splat debug arrays (nvgs_debug_buffers) */
#define NVGS_RENDER_GRAPH 4u          /* persistent frame: see nvgs_render */
#define NVGS_RENDER_NO_TEST_COUNT 8u  /* with stats: leave blend_tests uncounted (-1), so that the compositing
                                         kernels are the ones a frame without stats runs (stage timing) */

typedef struct nvgs_ctx nvgs_ctx;

/* Device memory provider.  alloc returns device memory (>= 256-byte aligned)
 * or NULL; free releases it.  With alloc == NULL the library uses hipMalloc. */
typedef struct nvgs_allocator {
  void* (*alloc)(size_t bytes, void* user);
  void (*free)(void* ptr, void* user);
  void* user;
} nvgs_allocator;

typedef struct nvgs_create_info {
  int32_t device;           /* HIP device ordinal */
  void* stream;             /* hipStream_t the context enqueues on (NULL = null stream) */
  nvgs_allocator allocator; /* scratch memory provider */
} nvgs_create_info;

/* Visibility MLP of one asset (Sec. 3.2; hidden layers fixed at 3 here).
 * params: device, FP32, packed row-major W1[width][12*bands], b1[width],
 * W2[width][width], b2, W3[width][width], b3, wo[width], bo[1].
 * Input x = (mean_scale * mu, cam_scale * c_local) with c_local the camera
 * position in the asset frame, scaled by train_focal / f_render (Eq. 2 with
 * focal lengths in pixels, f = (height / 2) / tan(fovy / 2), so a render at
 * another resolution or field of view maps onto the training views) and
 * clamped to length d_max when d_max > 0;
 * features sin(2^k pi x_j), cos(2^k pi x_j), k < bands, for the six scalars
 * in order.  A pair is kept iff the logit is >= 0.  If |c_local| < d_min
 * the MLP is not queried and every in-frustum Gaussian is kept (Sec. 3.3). */
typedef struct nvgs_mlp {
  int32_t width; /* 64 or 128 (kind 0); 32 (kind 1) */
  int32_t bands; /* 6 (kind 0); ignored (kind 1) */
  const float* params;
  float mean_scale, cam_scale, train_focal, d_min, d_max;
  int32_t kind;  /* 0: the frequency-encoded MLP above.  1: the paper's compact form
                    (Sec. 3.2, 3.3, 4.1): params = visibility W1[32][16], b1[32],
                    W2[32][32], b2[32], wo[32], bo, then embedding E1[32][8], e1[32],
                    E2[32][32], e2[32], E3[6][32], e3[6] (3175 floats); the embedding
                    MLP maps (opacity, ln scale x3, unit quaternion with w >= 0) of each
                    Gaussian to 6 values once at load time; the visibility inputs are
                    (mean_scale * mu, unit direction camera -> Gaussian, distance
                    |mu - c_local| * train_focal / f_render mapped linearly from
                    [d_min, d_max] to [-1, 1] and clamped, camera forward in the asset
                    frame, embedding), ReLU hidden layers; requires d_max > d_min >= 0;
                    cam_scale is unused; FP32 and BF16 only.  All assets of a context
                    share the kind. */
} nvgs_mlp;

/* One asset, float32 structure-of-arrays in device memory (borrowed). */
typedef struct nvgs_asset {
  int64_t n;            /* Gaussians, 1 <= n < 2^31 */
  int32_t sh_degree;    /* 0..3 */
  const float* mean;    /* [3][n] asset frame */
  const float* scale;   /* [3][n] linear standard deviations */
  const float* quat;    /* [4][n] (w, x, y, z), normalised on use */
  const float* opacity; /* [n] activated, in (0, 1] */
  const float* sh;      /* [(sh_degree+1)^2 * 3][n], plane c*3 + channel,
                           real SH (l-major, m = -l..l); colour =
                           max(0, 0.5 + sum_c Y_c(dir) sh_c), dir = unit
                           vector from camera to Gaussian in the asset frame */
  nvgs_mlp mlp;
} nvgs_asset;

/* Instance: world = s * R * mu + t (R row-major, asset -> world). */
typedef struct nvgs_instance {
  int32_t asset;
  float R[9];
  float s;
  float t[3];
} nvgs_instance;

typedef struct nvgs_camera {
  float pos[3];
  float R[9]; /* world -> camera, rows right, down, forward */
  float fovy;
  int32_t width, height;
  float near_plane; /* frustum: z > near, |x| <= 1.3 tan(fovx/2) z, |y| <= 1.3 tan(fovy/2) z */
} nvgs_camera;

typedef struct nvgs_render_opts {
  int32_t tile;      /* screen tile edge: 8, 16 or 32 (the image does not depend on it) */
  int32_t use_mlp;   /* 0: frustum culling only (the unculled reference) */
  int32_t precision; /* NVGS_PREC_* for the MLP */
  float bg[3];       /* background colour */
  uint32_t flags;    /* NVGS_RENDER_* */
  float* contrib;    /* device [C][P] (P = pairs per camera, instance-major) or NULL;
                        with RECORD_CONTRIB the max alpha*T of every blended fragment
                        of each pair is max-accumulated into it (caller zero-fills);
                        a fragment tested with alpha >= 1/255 whose blend would take T
                        below 1e-4 (the stop, Sec. 4.1) is reached but not blended and
                        records the smallest positive float (bit pattern 1), so
                        contrib > 0 marks exactly the pairs reached before the stop */
  int32_t split_len; /* tile lists longer than this are composited in chunks of at most
                        this many entries by separate work-groups, which equals the
                        sequential composite up to rounding (the association of the
                        transmittance products and colour sums); 0: default, a length
                        set by the frame on the device: max(256, ceil(entries / D)), D =
                        2 x compute units x 2048 / threads per compositing work-group
                        (64 for 8x8 tiles, else 256), i.e. about two chunks per
                        work-group the launch keeps resident; < 0: never split
                        (bit-identical across tile sizes); else >= 64, fixed */
  float det_clip;    /* radius clipping (Sec. 4.3 ablation): a splat whose 2D covariance
                        (after the 0.3 px^2 dilation) has a determinant below det_clip
                        (px^4; the 1-sigma ellipse area is pi sqrt(det)) is not binned;
                        0: off.  Must be finite and >= 0. */
} nvgs_render_opts;

/* Stages timed with HIP events on the context stream (ms_stage index). */
#define NVGS_STAGE_SETUP 0      /* per (camera, instance) transforms and MLP layer-1 camera half */
#define NVGS_STAGE_CULL_MLP 1   /* frustum cull + visibility MLP */
#define NVGS_STAGE_COMPACT 2    /* scan of the per-chunk keep counts */
#define NVGS_STAGE_PROJECT 3    /* compaction + EWA projection + SH + footprint */
#define NVGS_STAGE_DEPTH_SORT 4 /* radix sort of the splats by depth */
#define NVGS_STAGE_BIN 5        /* tile counts in depth order + scan + emission */
#define NVGS_STAGE_TILE_SORT 6  /* stable radix sort by tile + tile ranges */
#define NVGS_STAGE_BLEND 7      /* front-to-back compositing */
#define NVGS_NUM_STAGES 8

typedef struct nvgs_frame_stats {
  int64_t pairs;      /* C * P */
  int64_t in_frustum; /* pairs inside the frustum */
  int64_t queried;    /* pairs the MLP was evaluated for */
  int64_t kept;       /* instantiated splats (survived frustum + MLP) */
  int64_t duplicates; /* (splat, tile) entries sorted */
  int64_t blend_tests; /* (pixel, tile-list entry) pairs examined before each pixel stopped
                          (-1 with NVGS_RENDER_NO_TEST_COUNT) */
  int64_t workspace_bytes;
  float ms_total;     /* frame wall time on the stream (first to last event) */
  float ms_stage[NVGS_NUM_STAGES]; /* per-stage kernel time (HIP events) */
  int64_t blend_items; /* compositing work items: one per tile list, plus one per extra chunk
                          of a split list */
  int32_t chunk_len;   /* entries per chunk of a split list in this frame (0: not split) */
  int32_t reserved;
} nvgs_frame_stats;

/* Borrowed views of the last frame's device buffers (valid until the next
 * render / destroy); arrays are indexed by splat id = position in the
 * (camera, instance, Gaussian)-ordered list of survivors. */
typedef struct nvgs_debug_view {
  int64_t n_splats, n_dup;
  const uint32_t* pair;    /* [n_splats] index into [C][P] of the splat's pair (KEEP_DEBUG only) */
  const float* rec_a;      /* [n_splats][4]: u, v, conic xx, conic xy (pixels; KEEP_DEBUG only) */
  const float* rec_b;      /* [n_splats][4]: conic yy, opacity, r, g (KEEP_DEBUG only) */
  const float* rec_c;      /* [n_splats][4]: b, depth, ex, ey (footprint half extents, pixels; KEEP_DEBUG only) */
  const uint32_t* rect;    /* [n_splats][4]: x0 | y0 << 16, x1 | y1 << 16 (tile coords), cam, tiles */
  const uint32_t* sorted_key; /* [n_dup] cam * n_tiles + tile, ascending */
  const uint32_t* sorted_id;  /* [n_dup] splat id, (depth, id) order within a tile */
  const uint32_t* ranges;  /* [C * n_tiles][2] start, end into the sorted arrays */
  int32_t tiles_x, tiles_y;
  const float* rec_d;      /* [n_splats][2]: low-order parts of u and v (the centre is u + u_lo; KEEP_DEBUG only) */
} nvgs_debug_view;

/* Block shape of the cull + visibility-MLP kernel.  A work-group covers 256
 * consecutive Gaussians of one asset (256 / gaussians_per_wave waves) and
 * loops over up to segments_per_group (camera, instance) pairs of that asset,
 * reusing the Gaussian half of layer 1 (Sec. 3.3 factorisation of the camera
 * and Gaussian inputs). */
typedef struct nvgs_mlp_shape {
  int32_t gaussians_per_wave; /* 32, 64 or 128 (128 not with FP8 operands: falls back to 64) */
  int32_t segments_per_group; /* 1 .. 1024 */
} nvgs_mlp_shape;

/* One autotuner measurement: median milliseconds of the culling + MLP stage
 * (shape sweep) or of the whole frame (tile sweep). */
typedef struct nvgs_tune_entry {
  int32_t tile;
  int32_t gaussians_per_wave;
  int32_t segments_per_group;
  float ms;
} nvgs_tune_entry;

typedef struct nvgs_train_opts {
  int64_t batch;      /* (Gaussian, view) pairs per step, >= 1 */
  int32_t steps;      /* >= 1 */
  int32_t precision;  /* NVGS_PREC_FP32 or NVGS_PREC_BF16 */
  float lr, beta1, beta2, eps; /* Adam */
  uint64_t seed;      /* SplitMix64 seed of the batch draws */
  float threshold;    /* labels made internally: contribution > threshold */
  int32_t tile;       /* labels made internally: tile edge of the label renders */
  int32_t weighting;  /* 0: mean BCE; 1: each sample weighted by B / (2 n_class), n_class the
                         count of its label in the batch (Sec. 4.1 frequency weighting) */
  int32_t schedule;   /* 0: constant lr; 1 (Sec. 4.1): cosine warm-up from 0 to lr over the first
                         20 % of the steps, then exponential decay reaching lr_final at the last step */
  float lr_final;     /* schedule 1: final learning rate (> 0) */
} nvgs_train_opts;

/* Create a context on a device / stream.  Host call, no GPU work. */
nvgs_status nvgs_create(const nvgs_create_info* info, nvgs_ctx** out);
/* Destroy a context, releasing its scratch memory (synchronises its stream). */
void nvgs_destroy(nvgs_ctx* ctx);
/* Message of the last non-OK status of this context ("" if none). */
const char* nvgs_last_error(const nvgs_ctx* ctx);

/* Register the asset store (each asset stored once, Sec. 3.3).  Arrays are
 * borrowed (the means are read by every frame's culling).  Validates shapes;
 * copies the MLP weights into the kernels' operand layouts and the Gaussians
 * into library-owned per-Gaussian projection records (48 bytes of geometry
 * plus 3 (d+1)^2 SH floats rounded up to a multiple of 4, i.e. 240 bytes per
 * SH-3 Gaussian), asynchronously.  Invalidates the instance list. */
nvgs_status nvgs_load_assets(nvgs_ctx* ctx, const nvgs_asset* assets, int32_t n);

/* Copy the instance list (host array).  Synchronous host->device copy.
 * E_INVALID for an asset index out of range, s <= 0 or non-finite values. */
nvgs_status nvgs_set_instances(nvgs_ctx* ctx, const nvgs_instance* inst, int32_t n);

/* Steps 1-2 only.  state: device [C][P] bytes (0 frustum-culled, 1 culled by
 * the MLP, 2 kept); logits: device [C][P] float or NULL (NaN where the MLP was
 * not queried).  P = sum over instances of their asset's n. */
nvgs_status nvgs_query_visibility(nvgs_ctx* ctx, const nvgs_camera* cams, int32_t C, int32_t precision,
                                  uint8_t* state, float* logits);

/* The whole frame (steps 1-6, Sec. 3.3 and 4.1) for C cameras of equal size,
 * all cameras in one launch sequence: the tile key is camera * n_tiles + tile.
 * rgb: device [C][H][W][3].  stats (host, nullable): filled after a stream
 * synchronisation; E_CAPACITY if a capacity was exceeded (then the image is
 * undefined and stats hold the sizes needed).
 * Without NVGS_RENDER_GRAPH the call reads the splat and entry counts back
 * to size its buffers (two synchronisations) and times every stage.
 * With NVGS_RENDER_GRAPH (persistent frame) the call never synchronises
 * unless stats is given: every launch is bounded by the capacities from
 * nvgs_reserve or earlier frames (E_STATE if there are none), kernels clamp
 * to them and raise an overflow flag, and the launch sequence is captured
 * once into a HIP graph that later calls replay after uploading the cameras.
 * It is captured again when anything it was captured for changes (camera
 * count, image size, options, output pointers, buffers, MLP shape, assets,
 * instances).  ms_stage is zero for graph frames. */
nvgs_status nvgs_render(nvgs_ctx* ctx, const nvgs_camera* cams, int32_t C, const nvgs_render_opts* opts,
                        float* rgb, nvgs_frame_stats* stats);

/* Capacities for persistent frames: at least max_splats splats and
 * max_duplicates (splat, tile) entries per frame (both < 2^32).  Grow-only;
 * allocates (synchronises if a buffer moves). */
nvgs_status nvgs_reserve(nvgs_ctx* ctx, int64_t max_splats, int64_t max_duplicates);

/* Largest splat and entry counts of any frame since creation or the last
 * reset, and whether any frame overflowed its capacities.  Synchronises.
 * reset != 0 clears them afterwards.  A frame whose splats overflowed counts
 * the entries of the splats that fit only: grow and render again. */
nvgs_status nvgs_frame_watermarks(nvgs_ctx* ctx, int64_t* max_splats, int64_t* max_duplicates, int32_t* overflowed,
                                  int32_t reset);

/* Set / read the cull + MLP block shape used by later frames and queries
 * (default 32 Gaussians per wave, 64 segments per work-group, the autotuner's
 * choice on the composed 1080p scene for the FP32 and split-FP32 forms). */
/* Device memory the context holds, by what it is sized by (bytes).  Frame
 * buffers grow to the largest frame seen (or nvgs_reserve) and are kept. */
typedef struct nvgs_workspace {
  int64_t total;    /* every buffer: nvgs_frame_stats.workspace_bytes */
  int64_t assets;   /* per asset and instance: projection and MLP operand images, embeddings, tables */
  int64_t pairs;    /* per (camera, instance) segment and 256-pair chunk: keep masks, chunk counts and
                       offsets, segment records, layer-1 camera halves, cameras */
  int64_t splats;   /* per kept splat: compositing record (64 B), 8-byte tile rectangle in projection
                       and depth order, depth key, id, tile count / entry offset (92 B) */
  int64_t entries;  /* per (splat, tile) entry: tile key and id, the radix sort's ping-pong pair (which
                       the depth sort of the splats uses first) and its histograms */
  int64_t tiles;    /* per tile and compositing item: ranges, launch order, split-list records */
  int64_t debug;    /* per splat, KEEP_DEBUG / RECORD_CONTRIB frames only: debug records (60 B) */
  int64_t other;    /* frame counters, nvgs_sort_pairs' buffers, buffers of a call in progress */
  int64_t splat_capacity, entry_capacity;  /* splats and entries the frame buffers hold */
} nvgs_workspace;
nvgs_status nvgs_workspace_info(nvgs_ctx* ctx, nvgs_workspace* out);

/* Stable LSD radix sort, in place, of n (key, value) pairs held in device
 * arrays keys[n] and vals[n] (caller-owned), by key bits [begin_bit, end_bit)
 * (0 <= begin_bit <= end_bit <= 32; 8-bit digits, one pass each): pairs with
 * equal key bits keep their input order.  It is the sort behind the frame's
 * depth order and (tile, depth, id) order of the tile lists (Sec. 3.3, the
 * binning of original 3DGS), exposed for checking and reuse.  Runs on the
 * context stream and synchronises it; the context keeps a grow-only
 * workspace of about 8.5 n bytes.  E_INVALID for n outside [0, 2^32),
 * a bad bit range or null arrays with n > 0. */
nvgs_status nvgs_sort_pairs(nvgs_ctx* ctx, uint32_t* keys, uint32_t* vals, int64_t n, int32_t begin_bit,
                            int32_t end_bit);

nvgs_status nvgs_set_mlp_shape(nvgs_ctx* ctx, const nvgs_mlp_shape* shape);
nvgs_status nvgs_get_mlp_shape(nvgs_ctx* ctx, nvgs_mlp_shape* shape);

/* Autotuner.  Renders the given cameras without NVGS_RENDER_GRAPH: first every
 * supported MLP block shape (gaussians_per_wave 32/64/128 x segments_per_group
 * 4/8/16/32/64) at opts->tile, scored by the median culling + MLP stage time
 * over `reps` frames; then tiles 8, 16 and 32 with the best shape, scored by
 * the median frame time.  Keeps the best shape in the context and writes the
 * best tile into opts->tile.  table (host, nullable, table_cap entries)
 * receives the measurements, n_entries their count.  Synchronises. */
nvgs_status nvgs_autotune(nvgs_ctx* ctx, const nvgs_camera* cams, int32_t C, nvgs_render_opts* opts, float* rgb,
                          int32_t reps, nvgs_tune_entry* table, int32_t table_cap, int32_t* n_entries);

/* Views of the last frame's intermediate buffers (for tests and tools). */
nvgs_status nvgs_debug_buffers(nvgs_ctx* ctx, nvgs_debug_view* out);

/* Visibility labels of one asset from the renderer itself (Sec. 3.1): each
 * view renders a single identity instance of the asset with frustum culling
 * only and records, per Gaussian, the largest contribution alpha*T of its
 * blended fragments; the label is contribution > threshold (1/255 for a
 * non-zero 8-bit contribution; threshold must exceed the smallest normal
 * float, below which the "reached but not blended" marker of RECORD_CONTRIB
 * lies).  views: host [V], equal sizes.
 * labels: device [V][ceil(n/32)] bit words (bit g%32 of word g/32), written.
 * With aux > 0 (at most 64) each view also renders `aux` auxiliary views:
 * the view rotated rigidly about the asset centre by aux_angle (radians)
 * around the axes k_j = cos(phi_j) e1 + sin(phi_j) e2, phi_j = 2 pi j / aux,
 * with d the unit direction from the centre to the view, e1 its right axis
 * made orthogonal to d and e2 = d x e1.  The auxiliary cameras lie at the
 * view's distance on the cone of half-angle aux_angle around d (Sec. 3.1,
 * robustness against popping); a Gaussian is labelled visible for the view
 * if it is visible in any of its 1 + aux renders.
 * The instance list is restored afterwards.  Synchronises. */
nvgs_status nvgs_make_labels(nvgs_ctx* ctx, int32_t asset, const nvgs_camera* views, int32_t V, float threshold,
                             int32_t tile, int32_t aux, float aux_angle, uint32_t* labels);

/* Train the visibility MLP of one asset (Sec. 3.2) on (Gaussian,
 * view) pairs drawn uniformly with replacement: pair i of step s comes from
 * r = SplitMix64(opts->seed, s * batch + i), Gaussian ((r mod 2^32) n) >> 32,
 * view ((r >> 32) V) >> 32.  Loss: mean BCE with logits against the labels
 * (labels == NULL: made here with opts->threshold and opts->tile).  Adam
 * (beta1, beta2, eps, bias-corrected, lr per opts->schedule) on FP32 master weights.
 * precision NVGS_PREC_BF16 runs every GEMM of the forward and backward pass
 * on BF16 operands with FP32 accumulation (BF16 matrix cores for the
 * frequency form); NVGS_PREC_FP32 keeps FP32.
 * Frequency-encoded assets (nvgs_mlp.kind 0) have width 64 or 128.  Compact assets
 * (kind 1, Sec. 3.2, 3.3, 4.1) train the embedding MLP and the visibility MLP
 * jointly (all 3175 parameters): each pair's inputs are those of the query
 * with the view as camera of an identity instance, the embedding computed
 * from the Gaussian's (opacity, log scales, unit quaternion) in the same pass.
 * params: device FP32 packed parameters (layout of nvgs_mlp.params), read as
 * the initial weights and updated in place (reload the asset to render with
 * them).  loss_curve: host [steps] (mean batch loss before each update) or
 * NULL.  Synchronises. */
nvgs_status nvgs_train_visibility(nvgs_ctx* ctx, int32_t asset, const nvgs_camera* views, int32_t V,
                                  const uint32_t* labels, const nvgs_train_opts* opts, float* params,
                                  float* loss_curve);

/* MLP on encoded inputs, for automatic differentiation frameworks (width 64
 * or 128).  X: device [B][72] encoded inputs; logits: device [B].  precision
 * as in nvgs_train_visibility. */
nvgs_status nvgs_mlp_forward(nvgs_ctx* ctx, const float* params, int32_t width, const float* X, int64_t B,
                             int32_t precision, float* logits);
/* Vector-Jacobian product: dparams[p] = sum_b dlogits[b] dz_b/dparams[p]
 * (device [13057] at width 64, [42497] at width 128, overwritten) and, if
 * dX != NULL, dX[b][k] = dlogits[b]
 * dz_b/dX[b][k] (device [B][72]).  The sum over b runs in a fixed order. */
nvgs_status nvgs_mlp_backward(nvgs_ctx* ctx, const float* params, int32_t width, const float* X, int64_t B,
                              const float* dlogits, int32_t precision, float* dparams, float* dX);

/* nvgs_mlp_backward without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, kernels and results (bit-identical) as
 * nvgs_mlp_backward; the per-work-group gradient partials live in a fixed
 * 16 MiB device workspace that each GPU holds from library load until the
 * process ends.  B must be <= NVGS_NOALLOC_MAX_BATCH at width 64 and
 * <= NVGS_NOALLOC_MAX_BATCH_W128 at width 128 (E_INVALID otherwise).
 * Every call on a device shares that device's workspace: calls that overlap
 * in time on one device (other streams or contexts) race and give undefined
 * results; calls on one stream are ordered and safe.  The workspace keeps the
 * last call's contents; nothing in it needs clearing between calls. */
#define NVGS_NOALLOC_MAX_BATCH 65536
#define NVGS_NOALLOC_MAX_BATCH_W128 16896
nvgs_status nvgs_mlp_backward_noalloc(nvgs_ctx* ctx, const float* params, int32_t width, const float* X, int64_t B,
                                      const float* dlogits, int32_t precision, float* dparams, float* dX);

/* The compact model (Sec. 3.2, 3.3, 4.1) as one function of its raw inputs,
 * for automatic differentiation frameworks.  X: device [B][18]: the ten
 * per-pair visibility inputs (mean_scale * mu, unit direction camera ->
 * Gaussian, normalised distance, camera forward), then the eight embedding
 * inputs (opacity, log scales, unit quaternion with w >= 0); the embedding
 * MLP's six outputs complete the sixteen visibility inputs.  params: device
 * [3175] (layout of nvgs_mlp.params for kind 1).  logits: device [B].
 * precision: NVGS_PREC_FP32 or NVGS_PREC_BF16 (GEMM operands rounded). */
nvgs_status nvgs_cmlp_forward(nvgs_ctx* ctx, const float* params, const float* X, int64_t B, int32_t precision,
                              float* logits);
/* Vector-Jacobian product over the parameters: dparams[p] = sum_b dlogits[b]
 * dz_b/dparams[p] (device [3175], overwritten); the sum over b runs in a
 * fixed order. */
nvgs_status nvgs_cmlp_backward(nvgs_ctx* ctx, const float* params, const float* X, int64_t B, const float* dlogits,
                               int32_t precision, float* dparams);

#ifdef __cplusplus
}
#endif
#endif /* NVGS_H_ */
