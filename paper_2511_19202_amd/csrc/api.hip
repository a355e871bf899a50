// C ABI of the NVGS renderer: context, asset store, instance list, and the
// per-frame launch sequence (declared in include/nvgs.h).
#include <algorithm>
#include <initializer_list>
#include <cfloat>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

using namespace nvgs;

namespace {

struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
};

constexpr int kCounters = 24;       // u32 words of the frame counters

}  // namespace

struct nvgs_ctx {
  int device = 0;
  int n_cu = 256;  // compute units of the device
  hipStream_t stream = nullptr;
  nvgs_allocator alloc{};
  std::string err;
  size_t workspace = 0;

  // asset store
  std::vector<nvgs_asset> assets;
  std::vector<AssetDev> adev;
  std::vector<Buf> op_bufs;
  Buf assets_dev;
  int width = 0;
  int kind = 0;  // MLP kind shared by the assets

  // instances
  std::vector<nvgs_instance> inst;
  std::vector<int64_t> inst_off;
  int64_t P = 0;
  Buf inst_dev, inst_off_dev;

  // plan (depends on the camera count and the MLP block shape)
  int planC = -1, plan_segs = -1;
  int mlp_nb = 1, mlp_segs = 64;  // Gaussians per wave / 32, (camera, instance) segments per work-group
  uint64_t gen = 1;               // changes whenever a device buffer moves or the plan is rebuilt
  int64_t n_words = 0, n_chunks = 0;
  std::vector<int64_t> seg_word_base, seg_chunk_base;
  std::vector<WorkItem> items;
  std::vector<int32_t> seglist;
  Buf seg_word_dev, seg_chunk_dev, items_dev, seglist_dev, segs_dev, c1_dev;
  Buf mask, chunk_cnt, chunk_off, scan_part;

  // cameras: pinned staging ring, one completion event per slot
  static constexpr int kRing = 4;
  nvgs_camera* ring[kRing] = {};
  hipEvent_t ring_ev[kRing] = {};
  bool ring_used[kRing] = {};
  int ring_cap = 0, ring_next = 0;
  Buf cam_dev;

  // splats and sort buffers
  int64_t cap_splats = 0, cap_dup = 0;
  // per splat: compositing record, 8-byte tile rectangle (projection order and
  // depth order), depth key, ids, tile count (scanned in place into entry
  // offsets); debug frames add rec_* , rect_dbg and pair_of
  Buf splat, rec_a, rec_b, rec_c, rec_d, rect_dbg, rect, rect_sorted, depth_key, ids, pair_of, cnt;
  // per entry: tile key and splat id, and the radix sort's ping-pong pair,
  // which the depth sort of the splats uses first (sized for both)
  Buf keys, vals, keys_tmp, vals_tmp, hist, hist_part, ranges, tord;  // tord: tile order (4 arrays)
  Buf tsplit, citems, prodb, partb;  // long-list split: per-position counts and offsets, items, chunk products / records
  Buf sort_tmp, sort_ws;             // nvgs_sort_pairs: ping-pong pairs and workspace
  int64_t cap_items = 0, cap_split_px = 0;  // items; split slots x pixels per tile
  // largest compositing-item and split-slot counts of the eager frames seen,
  // per tile size (8, 16, 32): the sizes of the persistent frame's buffers
  int64_t wm_items[3] = {}, wm_split[3] = {};
  int64_t cap_keys = 0;  // tile keys (cameras x tiles) the range buffers hold
  int64_t cap_hist = 0;  // longest list the sort histograms and scan partials cover
  int64_t cap_debug = 0; // splats the debug arrays hold
  // every cap_* is set only once all of its buffers exist at that size and is
  // reset to 0 when an allocation fails, so no launch sees a missing buffer
  // u32 [0] n_splats, [1] n_dup, [2] overflow flags (1 splats, 2 entries, 4 entry offsets wrapped,
  // 8 compositing items); u64 at [4] in-frustum, [6] queried, [8] blend tests; [16] compositing items,
  // [17] split-chunk slots (written by their scans every frame)
  // (reset by every frame); across frames: [12] max splats, [13] max tile entries, [14] OR of overflow flags
  Buf counters;
  uint32_t* counters_host = nullptr;

  // persistent frame: captured launch sequence and what it was captured for
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<uint64_t> gkey;
  hipEvent_t gev[2] = {};

  // last frame (debug view)
  int64_t last_splats = 0, last_dup = 0;
  const uint32_t* last_sorted_key = nullptr;
  const uint32_t* last_sorted_id = nullptr;
  int last_tiles_x = 0, last_tiles_y = 0;
  bool last_debug = false;

  hipEvent_t ev[2 * NVGS_NUM_STAGES] = {};
};

namespace {

nvgs_status fail(nvgs_ctx* c, nvgs_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

#define CK(call)                                                                         \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(ctx, NVGS_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

void* dev_alloc(nvgs_ctx* ctx, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (ctx->alloc.alloc) return ctx->alloc.alloc(bytes, ctx->alloc.user);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  return p;
}

void dev_free(nvgs_ctx* ctx, void* p) {
  if (!p) return;
  if (ctx->alloc.alloc) {
    if (ctx->alloc.free) ctx->alloc.free(p, ctx->alloc.user);
  } else {
    (void)hipFree(p);
  }
}

void release(nvgs_ctx* ctx, Buf& b) {
  if (b.p) {
    dev_free(ctx, b.p);
    ctx->workspace -= b.bytes;
  }
  b.p = nullptr;
  b.bytes = 0;
}

// grow-only device buffer
bool ensure(nvgs_ctx* ctx, Buf& b, size_t bytes) {
  if (b.p && b.bytes >= bytes) return true;
  if (b.p) {
    (void)hipStreamSynchronize(ctx->stream);  // the old buffer may still be in use
    release(ctx, b);
  }
  ++ctx->gen;
  size_t want = std::max<size_t>(bytes, 256);
  b.p = dev_alloc(ctx, want);
  if (!b.p) return false;
  b.bytes = want;
  ctx->workspace += want;
  return true;
}

template <class T>
T* P_(Buf& b) {
  return reinterpret_cast<T*>(b.p);
}

bool finite_f(float x) { return std::isfinite(x); }

nvgs_status check_cams(nvgs_ctx* ctx, const nvgs_camera* cams, int32_t C) {
  if (!cams || C <= 0) return fail(ctx, NVGS_E_INVALID, "cameras: null pointer or C <= 0");
  for (int k = 0; k < C; ++k) {
    const nvgs_camera& c = cams[k];
    if (c.width <= 0 || c.height <= 0 || c.width > 32768 || c.height > 32768)
      return fail(ctx, NVGS_E_INVALID, "camera: width/height out of range");
    if (c.width != cams[0].width || c.height != cams[0].height)
      return fail(ctx, NVGS_E_INVALID, "cameras of one call must share width and height");
    if (!(c.fovy > 0.f && c.fovy < 3.1f) || !(c.near_plane > 0.f))
      return fail(ctx, NVGS_E_INVALID, "camera: fovy must be in (0, pi) and near > 0");
    for (int q = 0; q < 3; ++q)
      if (!finite_f(c.pos[q])) return fail(ctx, NVGS_E_INVALID, "camera: non-finite position");
    for (int q = 0; q < 9; ++q)
      if (!finite_f(c.R[q])) return fail(ctx, NVGS_E_INVALID, "camera: non-finite rotation");
  }
  return NVGS_OK;
}

// Build the per-camera-count plan: segment bases, work items, buffers.
nvgs_status plan(nvgs_ctx* ctx, int C) {
  if (ctx->planC == C && ctx->plan_segs == ctx->mlp_segs) return NVGS_OK;
  ++ctx->gen;
  const int NI = (int)ctx->inst.size();
  const int S = C * NI;
  ctx->seg_word_base.assign(S + 1, 0);
  ctx->seg_chunk_base.assign(S + 1, 0);
  int64_t w = 0, ch = 0;
  for (int s = 0; s < S; ++s) {
    const int64_t n = ctx->assets[ctx->inst[s % NI].asset].n;
    ctx->seg_word_base[s] = w;
    ctx->seg_chunk_base[s] = ch;
    w += (n + 31) / 32;
    ch += (n + kChunk - 1) / kChunk;
  }
  ctx->seg_word_base[S] = w;
  ctx->seg_chunk_base[S] = ch;
  ctx->n_words = w;
  ctx->n_chunks = ch;
  if (ch >= (int64_t)1 << 31 || (int64_t)C * ctx->P >= ((int64_t)1 << 32))
    return fail(ctx, NVGS_E_INVALID, "more than 2^32 (camera, instance, Gaussian) pairs in one frame");
  // work items: chunk x run of up to G segments of the same asset
  ctx->items.clear();
  ctx->seglist.clear();
  const int G = ctx->mlp_segs;
  for (int a = 0; a < (int)ctx->assets.size(); ++a) {
    const int base = (int)ctx->seglist.size();
    for (int s = 0; s < S; ++s)
      if (ctx->inst[s % NI].asset == a) ctx->seglist.push_back(s);
    const int ns = (int)ctx->seglist.size() - base;
    if (ns == 0) continue;
    const int64_t chunks = (ctx->assets[a].n + kChunk - 1) / kChunk;
    for (int64_t c = 0; c < chunks; ++c)
      for (int sb = 0; sb < ns; sb += G) ctx->items.push_back({a, (int32_t)c, base + sb, base + std::min(ns, sb + G)});
  }
  if (!ensure(ctx, ctx->seg_word_dev, sizeof(int64_t) * (S + 1)) ||
      !ensure(ctx, ctx->seg_chunk_dev, sizeof(int64_t) * (S + 1)) ||
      !ensure(ctx, ctx->items_dev, sizeof(WorkItem) * std::max<size_t>(1, ctx->items.size())) ||
      !ensure(ctx, ctx->seglist_dev, sizeof(int32_t) * std::max<size_t>(1, ctx->seglist.size())) ||
      !ensure(ctx, ctx->segs_dev, sizeof(SegRec) * S) || !ensure(ctx, ctx->c1_dev, sizeof(float) * 128 * S) ||
      !ensure(ctx, ctx->mask, sizeof(uint32_t) * (w + 1)) || !ensure(ctx, ctx->chunk_cnt, sizeof(uint32_t) * (ch + 1)) ||
      !ensure(ctx, ctx->chunk_off, sizeof(uint32_t) * (ch + 1)) ||
      !ensure(ctx, ctx->scan_part, sizeof(uint32_t) * scan_partials_needed(ch + 1)) ||
      !ensure(ctx, ctx->cam_dev, sizeof(nvgs_camera) * C))
    return fail(ctx, NVGS_E_NOMEM, "device allocation failed (plan)");
  CK(hipMemcpy(ctx->seg_word_dev.p, ctx->seg_word_base.data(), sizeof(int64_t) * (S + 1), hipMemcpyHostToDevice));
  CK(hipMemcpy(ctx->seg_chunk_dev.p, ctx->seg_chunk_base.data(), sizeof(int64_t) * (S + 1), hipMemcpyHostToDevice));
  if (!ctx->items.empty())
    CK(hipMemcpy(ctx->items_dev.p, ctx->items.data(), sizeof(WorkItem) * ctx->items.size(), hipMemcpyHostToDevice));
  if (!ctx->seglist.empty())
    CK(hipMemcpy(ctx->seglist_dev.p, ctx->seglist.data(), sizeof(int32_t) * ctx->seglist.size(),
                 hipMemcpyHostToDevice));
  ctx->planC = C;
  ctx->plan_segs = ctx->mlp_segs;
  return NVGS_OK;
}

// Copy the cameras through the next slot of the pinned ring; a slot is only
// rewritten once the copy that last read it has completed.
nvgs_status upload_cams(nvgs_ctx* ctx, const nvgs_camera* cams, int C) {
  if (ctx->ring_cap < C) {
    CK(hipStreamSynchronize(ctx->stream));
    for (int j = 0; j < nvgs_ctx::kRing; ++j) {
      if (ctx->ring[j]) (void)hipHostFree(ctx->ring[j]);
      ctx->ring[j] = nullptr;
      ctx->ring_used[j] = false;
    }
    ctx->ring_cap = 0;
    for (int j = 0; j < nvgs_ctx::kRing; ++j)
      CK(hipHostMalloc(reinterpret_cast<void**>(&ctx->ring[j]), sizeof(nvgs_camera) * C, hipHostMallocDefault));
    ctx->ring_cap = C;
  }
  const int j = ctx->ring_next;
  ctx->ring_next = (j + 1) % nvgs_ctx::kRing;
  if (ctx->ring_used[j]) CK(hipEventSynchronize(ctx->ring_ev[j]));
  std::memcpy(ctx->ring[j], cams, sizeof(nvgs_camera) * C);
  CK(hipMemcpyAsync(ctx->cam_dev.p, ctx->ring[j], sizeof(nvgs_camera) * C, hipMemcpyHostToDevice, ctx->stream));
  CK(hipEventRecord(ctx->ring_ev[j], ctx->stream));
  ctx->ring_used[j] = true;
  return NVGS_OK;
}

nvgs_status read_counters(nvgs_ctx* ctx) {
  CK(hipMemcpyAsync(ctx->counters_host, ctx->counters.p, sizeof(uint32_t) * kCounters, hipMemcpyDeviceToHost,
                    ctx->stream));
  CK(hipStreamSynchronize(ctx->stream));
  return NVGS_OK;
}

nvgs_status ready(nvgs_ctx* ctx) {
  if (ctx->assets.empty()) return fail(ctx, NVGS_E_STATE, "no assets loaded");
  if (ctx->inst.empty()) return fail(ctx, NVGS_E_STATE, "no instances set");
  return NVGS_OK;
}

// the configured Gaussians-per-wave, or 2 where that shape is not built for this precision
int shape_nb(const nvgs_ctx* ctx, int precision) {
  return mlp_shape_supported(ctx->width, precision, ctx->mlp_nb) ? ctx->mlp_nb : 2;
}

// cull + visibility query of every (camera, instance, Gaussian) pair with the
// context's MLP kind (mode 1 also writes per-pair state and logits)
hipError_t launch_query(nvgs_ctx* ctx, int precision, int mode, uint8_t* state, float* logits,
                        unsigned long long* counts, hipStream_t st) {
  // the query kernels add their per-wave kept counts into the chunk counts
  hipError_t e = launch_fill_u32(P_<uint32_t>(ctx->chunk_cnt), 0u, ctx->n_chunks, st);
  if (e != hipSuccess) return e;
  if (ctx->kind == 1)
    return launch_cull_cmlp(P_<AssetDev>(ctx->assets_dev), P_<WorkItem>(ctx->items_dev), (int64_t)ctx->items.size(),
                            P_<int32_t>(ctx->seglist_dev), P_<SegRec>(ctx->segs_dev), P_<float>(ctx->c1_dev), 128,
                            precision, mode, P_<uint32_t>(ctx->mask), P_<uint32_t>(ctx->chunk_cnt), state, logits,
                            counts, st);
  return launch_cull_mlp(P_<AssetDev>(ctx->assets_dev), P_<WorkItem>(ctx->items_dev), (int64_t)ctx->items.size(),
                         P_<int32_t>(ctx->seglist_dev), P_<SegRec>(ctx->segs_dev), P_<float>(ctx->c1_dev), 128,
                         ctx->width, precision, shape_nb(ctx, precision), mode, P_<uint32_t>(ctx->mask),
                         P_<uint32_t>(ctx->chunk_cnt), state, logits, counts, st);
}

int bits_for(int64_t v) {
  int b = 0;
  while (((int64_t)1 << b) < v) ++b;
  return b;
}

}  // namespace

extern "C" {

nvgs_status nvgs_create(const nvgs_create_info* info, nvgs_ctx** out) {
  if (!info || !out) return NVGS_E_INVALID;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return NVGS_E_DEVICE;
  if (info->device < 0 || info->device >= ndev) return NVGS_E_INVALID;
  if ((info->allocator.alloc == nullptr) != (info->allocator.free == nullptr)) return NVGS_E_INVALID;
  if (hipSetDevice(info->device) != hipSuccess) return NVGS_E_DEVICE;
  // address of this device's fixed workspace (allocation-free backward)
  if (static_scratch_init(info->device) != hipSuccess) return NVGS_E_DEVICE;
  nvgs_ctx* ctx = new nvgs_ctx();
  ctx->device = info->device;
  if (hipDeviceGetAttribute(&ctx->n_cu, hipDeviceAttributeMultiprocessorCount, info->device) != hipSuccess ||
      ctx->n_cu < 1)
    ctx->n_cu = 256;
  ctx->stream = reinterpret_cast<hipStream_t>(info->stream);
  ctx->alloc = info->allocator;
  bool ok = hipHostMalloc(reinterpret_cast<void**>(&ctx->counters_host), kCounters * sizeof(uint32_t),
                          hipHostMallocDefault) == hipSuccess;
  for (int e = 0; e < 2 * NVGS_NUM_STAGES && ok; ++e) ok = hipEventCreate(&ctx->ev[e]) == hipSuccess;
  for (int e = 0; e < 2 && ok; ++e) ok = hipEventCreate(&ctx->gev[e]) == hipSuccess;
  for (int e = 0; e < nvgs_ctx::kRing && ok; ++e)
    ok = hipEventCreateWithFlags(&ctx->ring_ev[e], hipEventDisableTiming) == hipSuccess;
  ok = ok && hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) == hipSuccess;
  ok = ok && ensure(ctx, ctx->counters, kCounters * sizeof(uint32_t)) &&
       launch_fill_u32(P_<uint32_t>(ctx->counters), 0u, kCounters, ctx->stream) == hipSuccess;
  if (!ok) {
    nvgs_destroy(ctx);
    return NVGS_E_DEVICE;
  }
  *out = ctx;
  return NVGS_OK;
}

void nvgs_destroy(nvgs_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  Buf* all[] = {&ctx->assets_dev, &ctx->inst_dev, &ctx->inst_off_dev, &ctx->seg_word_dev, &ctx->seg_chunk_dev,
                &ctx->items_dev, &ctx->seglist_dev, &ctx->segs_dev, &ctx->c1_dev, &ctx->mask, &ctx->chunk_cnt,
                &ctx->chunk_off, &ctx->scan_part, &ctx->cam_dev, &ctx->splat, &ctx->rect_sorted, &ctx->rec_a, &ctx->rec_b, &ctx->rec_c, &ctx->rec_d, &ctx->rect,
                &ctx->rect_dbg, &ctx->depth_key, &ctx->ids, &ctx->pair_of, &ctx->cnt,
                &ctx->keys, &ctx->vals, &ctx->keys_tmp, &ctx->vals_tmp, &ctx->hist, &ctx->hist_part, &ctx->ranges, &ctx->tord,
                &ctx->tsplit, &ctx->citems, &ctx->prodb, &ctx->partb, &ctx->sort_tmp, &ctx->sort_ws,
                &ctx->counters};
  for (Buf* b : all) release(ctx, *b);
  for (Buf& b : ctx->op_bufs) release(ctx, b);
  if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  for (nvgs_camera* r : ctx->ring)
    if (r) (void)hipHostFree(r);
  if (ctx->counters_host) (void)hipHostFree(ctx->counters_host);
  for (hipEvent_t e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : ctx->gev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : ctx->ring_ev)
    if (e) (void)hipEventDestroy(e);
  delete ctx;
}

const char* nvgs_last_error(const nvgs_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

nvgs_status nvgs_load_assets(nvgs_ctx* ctx, const nvgs_asset* a, int32_t n) {
  if (!ctx) return NVGS_E_INVALID;
  if (!a || n <= 0) return fail(ctx, NVGS_E_INVALID, "assets: null pointer or n <= 0");
  int width = a[0].mlp.width;
  const int kind = a[0].mlp.kind;
  if (kind != 0 && kind != 1) return fail(ctx, NVGS_E_INVALID, "asset: MLP kind must be 0 or 1");
  for (int j = 0; j < n; ++j) {
    const nvgs_asset& x = a[j];
    if (x.mlp.kind != kind) return fail(ctx, NVGS_E_INVALID, "assets of one context must share the MLP kind");
    if (x.n <= 0 || x.n >= ((int64_t)1 << 31)) return fail(ctx, NVGS_E_INVALID, "asset: n out of range");
    if (x.sh_degree < 0 || x.sh_degree > 3) return fail(ctx, NVGS_E_INVALID, "asset: sh_degree must be 0..3");
    if (!x.mean || !x.scale || !x.quat || !x.opacity || !x.sh || !x.mlp.params)
      return fail(ctx, NVGS_E_INVALID, "asset: null array");
    if (kind == 0 && x.mlp.width != 64 && x.mlp.width != 128)
      return fail(ctx, NVGS_E_INVALID, "asset: MLP width must be 64 or 128");
    if (kind == 1 && x.mlp.width != 32) return fail(ctx, NVGS_E_INVALID, "asset: compact MLP width must be 32");
    if (x.mlp.width != width) return fail(ctx, NVGS_E_INVALID, "assets of one context must share the MLP width");
    if (kind == 0 && x.mlp.bands != 6) return fail(ctx, NVGS_E_INVALID, "asset: MLP bands must be 6");
    if (kind == 1 && !(x.mlp.d_max > x.mlp.d_min && x.mlp.d_min >= 0.f))
      return fail(ctx, NVGS_E_INVALID, "asset: compact MLP needs d_max > d_min >= 0");
    if (!finite_f(x.mlp.mean_scale) || !finite_f(x.mlp.cam_scale) || !finite_f(x.mlp.train_focal) ||
        !finite_f(x.mlp.d_min) || !finite_f(x.mlp.d_max) || x.mlp.train_focal <= 0.f)
      return fail(ctx, NVGS_E_INVALID, "asset: non-finite MLP metadata");
  }
  CK(hipSetDevice(ctx->device));
  CK(hipStreamSynchronize(ctx->stream));
  for (Buf& b : ctx->op_bufs) release(ctx, b);
  // per asset: FP32, BF16, FP8 operand images, FP8 scales, projection geometry and SH records,
  // compact-form embeddings
  ctx->op_bufs.assign(7 * (size_t)n, Buf{});
  ctx->assets.assign(a, a + n);
  ctx->adev.assign(n, AssetDev{});
  for (int j = 0; j < n; ++j) {
    const nvgs_asset& x = a[j];
    AssetDev& d = ctx->adev[j];
    d.mean = x.mean; d.scale = x.scale; d.quat = x.quat; d.opacity = x.opacity; d.sh = x.sh;
    d.n = x.n; d.sh_degree = x.sh_degree; d.width = x.mlp.width;
    d.mean_scale = x.mlp.mean_scale; d.cam_scale = x.mlp.cam_scale; d.train_focal = x.mlp.train_focal;
    d.d_min = x.mlp.d_min; d.d_max = x.mlp.d_max;
    d.params = x.mlp.params;
    Buf* ob = &ctx->op_bufs[7 * (size_t)j];
    d.kind = kind;
    if (kind == 1) {
      if (!ensure(ctx, ob[0], cmlp_image_floats() * sizeof(float)) || !ensure(ctx, ob[1], 2048 * sizeof(uint16_t)) ||
          !ensure(ctx, ob[6], 8 * sizeof(float) * (size_t)x.n) ||
          !ensure(ctx, ob[4], 3 * sizeof(float4) * (size_t)x.n) ||
          !ensure(ctx, ob[5], sizeof(float) * (size_t)sh_stride_for(x.sh_degree) * (size_t)x.n))
        return fail(ctx, NVGS_E_NOMEM, "operand images");
      d.op_f32 = P_<float>(ob[0]);
      d.op_bf16 = P_<uint16_t>(ob[1]);
      d.op_fp8 = nullptr;
      d.op_split = nullptr;
      d.fp8_scale = nullptr;
      d.emb = P_<float>(ob[6]);
      d.geo = P_<float4>(ob[4]);
      d.shp = P_<float>(ob[5]);
      d.sh_stride = sh_stride_for(x.sh_degree);
      CK(launch_pack_asset(x.mean, x.scale, x.quat, x.opacity, x.sh, x.n, x.sh_degree, P_<float4>(ob[4]),
                           P_<float>(ob[5]), ctx->stream));
      CK(launch_prepare_cmlp(x.mlp.params, P_<float>(ob[0]), P_<uint16_t>(ob[1]), ctx->stream));
      CK(launch_cembed(x.mlp.params, x.scale, x.quat, x.opacity, x.n, P_<float>(ob[6]), ctx->stream));
      continue;
    }
    d.emb = nullptr;
    if (!ensure(ctx, ob[0], mlp_op_f32_floats(width) * sizeof(float)) ||
        !ensure(ctx, ob[1], mlp_op_bf16_elems(width) * sizeof(uint16_t)) ||
        !ensure(ctx, ob[2], mlp_op_fp8_bytes(width)) || !ensure(ctx, ob[3], 16 * sizeof(float)) ||
        !ensure(ctx, ob[6], mlp_op_split_bytes(width)) ||
        !ensure(ctx, ob[4], 3 * sizeof(float4) * (size_t)x.n) ||
        !ensure(ctx, ob[5], sizeof(float) * (size_t)sh_stride_for(x.sh_degree) * (size_t)x.n))
      return fail(ctx, NVGS_E_NOMEM, "operand images");
    d.geo = P_<float4>(ob[4]);
    d.shp = P_<float>(ob[5]);
    d.sh_stride = sh_stride_for(x.sh_degree);
    CK(launch_pack_asset(x.mean, x.scale, x.quat, x.opacity, x.sh, x.n, x.sh_degree, P_<float4>(ob[4]),
                         P_<float>(ob[5]), ctx->stream));
    d.op_f32 = P_<float>(ob[0]);
    d.op_bf16 = P_<uint16_t>(ob[1]);
    d.op_fp8 = P_<uint8_t>(ob[2]);
    d.op_split = P_<uint8_t>(ob[6]);
    d.fp8_scale = P_<float>(ob[3]);
    CK(launch_prepare_mlp(x.mlp.params, width, P_<float>(ob[0]), P_<uint16_t>(ob[1]), P_<uint8_t>(ob[2]),
                          P_<float>(ob[3]), ctx->stream));
    CK(launch_prepare_split(x.mlp.params, width, P_<uint8_t>(ob[6]), ctx->stream));
  }
  if (!ensure(ctx, ctx->assets_dev, sizeof(AssetDev) * n)) return fail(ctx, NVGS_E_NOMEM, "asset table");
  CK(hipMemcpyAsync(ctx->assets_dev.p, ctx->adev.data(), sizeof(AssetDev) * n, hipMemcpyHostToDevice, ctx->stream));
  CK(hipStreamSynchronize(ctx->stream));
  ctx->width = width;
  ctx->kind = kind;
  ctx->inst.clear();
  ctx->planC = -1;
  ++ctx->gen;
  return NVGS_OK;
}

nvgs_status nvgs_set_instances(nvgs_ctx* ctx, const nvgs_instance* h, int32_t n) {
  if (!ctx) return NVGS_E_INVALID;
  if (ctx->assets.empty()) return fail(ctx, NVGS_E_STATE, "set_instances before load_assets");
  if (!h || n <= 0) return fail(ctx, NVGS_E_INVALID, "instances: null pointer or n <= 0");
  std::vector<int64_t> off(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    if (h[i].asset < 0 || h[i].asset >= (int)ctx->assets.size())
      return fail(ctx, NVGS_E_INVALID, "instance: asset index out of range");
    if (!(h[i].s > 0.f) || !finite_f(h[i].s)) return fail(ctx, NVGS_E_INVALID, "instance: scale must be > 0");
    for (int q = 0; q < 9; ++q)
      if (!finite_f(h[i].R[q])) return fail(ctx, NVGS_E_INVALID, "instance: non-finite rotation");
    for (int q = 0; q < 3; ++q)
      if (!finite_f(h[i].t[q])) return fail(ctx, NVGS_E_INVALID, "instance: non-finite translation");
    off[i + 1] = off[i] + ctx->assets[h[i].asset].n;
  }
  if (off[n] >= ((int64_t)1 << 32)) return fail(ctx, NVGS_E_INVALID, "more than 2^32 pairs per camera");
  CK(hipSetDevice(ctx->device));
  CK(hipStreamSynchronize(ctx->stream));
  ctx->inst.assign(h, h + n);
  ctx->inst_off = off;
  ctx->P = off[n];
  if (!ensure(ctx, ctx->inst_dev, sizeof(nvgs_instance) * n) ||
      !ensure(ctx, ctx->inst_off_dev, sizeof(int64_t) * (n + 1)))
    return fail(ctx, NVGS_E_NOMEM, "instance table");
  CK(hipMemcpy(ctx->inst_dev.p, h, sizeof(nvgs_instance) * n, hipMemcpyHostToDevice));
  CK(hipMemcpy(ctx->inst_off_dev.p, off.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice));
  ctx->planC = -1;
  ++ctx->gen;
  return NVGS_OK;
}

nvgs_status nvgs_query_visibility(nvgs_ctx* ctx, const nvgs_camera* cams, int32_t C, int32_t precision,
                                  uint8_t* state, float* logits) {
  if (!ctx) return NVGS_E_INVALID;
  nvgs_status s = ready(ctx);
  if (s) return s;
  if ((s = check_cams(ctx, cams, C))) return s;
  if (!state) return fail(ctx, NVGS_E_INVALID, "state: null pointer");
  if (precision < NVGS_PREC_FP32 || precision > NVGS_PREC_FP32_SPLIT) return fail(ctx, NVGS_E_INVALID, "bad precision");
  if (ctx->kind == 1 && precision >= NVGS_PREC_FP8)
    return fail(ctx, NVGS_E_INVALID, "the compact MLP runs in FP32 or BF16");
  CK(hipSetDevice(ctx->device));
  if ((s = plan(ctx, C))) return s;
  if ((s = upload_cams(ctx, cams, C))) return s;
  const int NI = (int)ctx->inst.size();
  CK(launch_segment_setup(P_<nvgs_camera>(ctx->cam_dev), P_<nvgs_instance>(ctx->inst_dev),
                          P_<AssetDev>(ctx->assets_dev), P_<int64_t>(ctx->inst_off_dev), NI, C, ctx->P, 1,
                          P_<int64_t>(ctx->seg_word_dev), P_<int64_t>(ctx->seg_chunk_dev), P_<SegRec>(ctx->segs_dev),
                          P_<float>(ctx->c1_dev), 128, ctx->stream));
  // logits may be NULL: write them into a scratch buffer then
  Buf scratch;
  float* lg = logits;
  if (!lg) {
    if (!ensure(ctx, scratch, sizeof(float) * (size_t)C * ctx->P)) return fail(ctx, NVGS_E_NOMEM, "logit scratch");
    lg = P_<float>(scratch);
  }
  CK(launch_query(ctx, precision, 1, state, lg, nullptr, ctx->stream));
  if (scratch.p) {
    CK(hipStreamSynchronize(ctx->stream));
    release(ctx, scratch);
  }
  return NVGS_OK;
}

}  // extern "C"

namespace {

// Radix histograms and scan partials for the largest sorted or scanned list.
nvgs_status size_hist(nvgs_ctx* ctx) {
  const int64_t m = std::max({ctx->cap_dup, ctx->cap_splats, ctx->cap_keys, (int64_t)4096});
  if (m <= ctx->cap_hist) return NVGS_OK;
  if (!ensure(ctx, ctx->hist, 4 * radix_hist_words(m)) ||
      !ensure(ctx, ctx->hist_part, 8 * scan_partials_needed(m))) {
    ctx->cap_hist = 0;
    return fail(ctx, NVGS_E_NOMEM, "sort histograms");
  }
  ctx->cap_hist = m;
  return NVGS_OK;
}

// Debug arrays (KEEP_DEBUG / RECORD_CONTRIB frames) for cap_splats splats.
nvgs_status size_debug(nvgs_ctx* ctx) {
  if (ctx->cap_debug >= ctx->cap_splats && ctx->cap_debug > 0) return NVGS_OK;
  const int64_t cap = ctx->cap_splats;
  if (!ensure(ctx, ctx->rec_a, 16 * cap) || !ensure(ctx, ctx->rec_b, 16 * cap) ||
      !ensure(ctx, ctx->rec_c, 16 * cap) || !ensure(ctx, ctx->rec_d, 8 * cap) || !ensure(ctx, ctx->rect_dbg, 16 * cap) ||
      !ensure(ctx, ctx->pair_of, 4 * cap)) {
    ctx->cap_debug = 0;
    return fail(ctx, NVGS_E_NOMEM, "debug buffers");
  }
  ctx->cap_debug = cap;
  return NVGS_OK;
}

// The radix sort's ping-pong pair serves the splats' depth sort and the
// entries' tile sort: after a failed allocation, the capacity it no longer
// covers is dropped as well.
void drop_shared_temps(nvgs_ctx* ctx) {
  const size_t have = std::min(ctx->keys_tmp.bytes, ctx->vals_tmp.bytes);
  if (have < 4 * (size_t)ctx->cap_splats) ctx->cap_splats = 0;
  if (have < 4 * (size_t)ctx->cap_dup) ctx->cap_dup = 0;
}

// Grow-only splat buffers for `need` splats (1/8 headroom when `slack`).
nvgs_status size_splats(nvgs_ctx* ctx, int64_t need, bool slack) {
  if (need <= ctx->cap_splats && ctx->cap_splats > 0) return NVGS_OK;
  const int64_t cap = std::max<int64_t>(slack ? need + need / 8 : need, 4096);
  ctx->cap_splats = 0;
  const bool ok = ensure(ctx, ctx->splat, 64 * cap) && ensure(ctx, ctx->rect, 8 * cap) &&
                  ensure(ctx, ctx->rect_sorted, 8 * cap) && ensure(ctx, ctx->depth_key, 4 * cap) &&
                  ensure(ctx, ctx->ids, 4 * cap) && ensure(ctx, ctx->cnt, 4 * cap) &&
                  ensure(ctx, ctx->keys_tmp, 4 * cap) && ensure(ctx, ctx->vals_tmp, 4 * cap);
  if (!ok) {
    drop_shared_temps(ctx);
    return fail(ctx, NVGS_E_NOMEM, "splat buffers");
  }
  ctx->cap_splats = cap;
  return size_hist(ctx);
}

// Grow-only (tile, splat) entry buffers for `need` entries.
nvgs_status size_dups(nvgs_ctx* ctx, int64_t need, bool slack) {
  if (need <= ctx->cap_dup && ctx->cap_dup > 0) return NVGS_OK;
  const int64_t cap = std::min<int64_t>(std::max<int64_t>(slack ? need + need / 8 : need, 4096), UINT32_MAX);
  ctx->cap_dup = 0;
  const bool ok = ensure(ctx, ctx->keys, 4 * cap) && ensure(ctx, ctx->vals, 4 * cap) &&
                  ensure(ctx, ctx->keys_tmp, 4 * cap) && ensure(ctx, ctx->vals_tmp, 4 * cap);
  if (!ok) {
    drop_shared_temps(ctx);
    return fail(ctx, NVGS_E_NOMEM, "tile entry buffers");
  }
  ctx->cap_dup = cap;
  return size_hist(ctx);
}

// Tile ranges and launch-order buffers for `nkeys` (camera, tile) keys.
nvgs_status size_tiles(nvgs_ctx* ctx, int64_t nkeys) {
  if (nkeys <= ctx->cap_keys) return NVGS_OK;
  ctx->cap_keys = 0;
  if (!ensure(ctx, ctx->ranges, sizeof(uint32_t) * 2 * (size_t)nkeys) ||
      !ensure(ctx, ctx->tord, sizeof(uint32_t) * 4 * (size_t)nkeys) ||
      !ensure(ctx, ctx->tsplit, sizeof(uint32_t) * 4 * (size_t)nkeys))
    return fail(ctx, NVGS_E_NOMEM, "tile ranges");
  ctx->cap_keys = nkeys;
  return size_hist(ctx);
}

int tile_index(int T) { return T == 8 ? 0 : T == 16 ? 1 : 2; }

// Compositing items and split-chunk buffers (grow-only) for a frame of nkeys
// tiles of T x T pixels.  An eager frame passes its own counts (need_items,
// need_split >= 0) and gets them with 1/8 headroom.  A persistent frame
// passes -1: the largest counts of the eager frames seen at this tile size
// plus 1/4, or, before any, the bound for the entry capacity (every list
// longer than the chunk length S splits into at most 2 len / S chunks; with
// the frame-adaptive length S >= n / split_div, so n / S <= split_div).  A
// frame beyond the capacity raises the overflow flag.
nvgs_status size_items(nvgs_ctx* ctx, int64_t nkeys, int T, int split_len, int64_t split_div, int64_t need_items,
                       int64_t need_split) {
  int64_t items, slots;
  const int ti = tile_index(T);
  if (need_items >= 0) {
    items = need_items + need_items / 8;
    slots = need_split + need_split / 8;
  } else if (ctx->wm_items[ti] > 0) {
    items = ctx->wm_items[ti] + ctx->wm_items[ti] / 4 + 256;
    slots = ctx->wm_split[ti] + ctx->wm_split[ti] / 4 + 16;
  } else {
    const int64_t per = split_len > 0 ? ctx->cap_dup / split_len
                        : split_len == kSplitAuto ? std::min<int64_t>(ctx->cap_dup / kSplitMin, split_div) : 0;
    items = nkeys + per + 1;
    slots = 2 * per + 2;
  }
  items = std::max(items, nkeys + 1);
  const int64_t cap_split_px = split_len != 0 ? std::max<int64_t>(slots, 1) * T * T : 0;
  if (items <= ctx->cap_items && cap_split_px <= ctx->cap_split_px) return NVGS_OK;
  items = std::max(items, ctx->cap_items);
  const int64_t px = std::max(cap_split_px, ctx->cap_split_px);
  ctx->cap_items = 0;
  ctx->cap_split_px = 0;
  if (!ensure(ctx, ctx->citems, 8 * (size_t)items) || !ensure(ctx, ctx->prodb, 4 * (size_t)std::max<int64_t>(px, 1)) ||
      !ensure(ctx, ctx->partb, 16 * (size_t)std::max<int64_t>(px, 1)))
    return fail(ctx, NVGS_E_NOMEM, "compositing items");
  ctx->cap_items = items;
  ctx->cap_split_px = px;
  return NVGS_OK;
}

struct Frame {
  int C, W, H, T, tiles_x, tiles_y, n_tiles;
  int split_len;     // 0: no split; kSplitAuto: frame-adaptive
  int64_t split_div; // kSplitAuto: the frame's entries are cut into about this many chunks
  int64_t nkeys;
  bool record, debug, count_tests;
  const nvgs_render_opts* opts;
  float* rgb;
};

// Enqueue one frame on `st`.  eager: the splat and entry counts are read back
// to size the buffers (two host synchronisations) and stage events are
// recorded.  Otherwise the reserved capacities bound every launch, nothing
// is read back and no buffer is allocated, so the sequence can be captured;
// kernels clamp to the capacities and raise overflow flags.
nvgs_status enqueue_frame(nvgs_ctx* ctx, hipStream_t st, const Frame& f, bool eager, float* ms_bin_count,
                          float* ms_tile_count) {
  hipEvent_t* ev = ctx->ev;
#define STAGE_BEGIN(k) \
  if (eager) CK(hipEventRecord(ev[2 * (k)], st))
#define STAGE_END(k) \
  if (eager) CK(hipEventRecord(ev[2 * (k) + 1], st))
  nvgs_status s = NVGS_OK;
  const nvgs_render_opts* opts = f.opts;
  const int C = f.C, NI = (int)ctx->inst.size();
  uint32_t* counters = P_<uint32_t>(ctx->counters);
  unsigned long long* counts64 = reinterpret_cast<unsigned long long*>(counters + 4);
  STAGE_BEGIN(NVGS_STAGE_SETUP);
  CK(launch_fill_u32(counters, 0u, 12, st));
  CK(launch_segment_setup(P_<nvgs_camera>(ctx->cam_dev), P_<nvgs_instance>(ctx->inst_dev),
                          P_<AssetDev>(ctx->assets_dev), P_<int64_t>(ctx->inst_off_dev), NI, C, ctx->P,
                          opts->use_mlp ? 1 : 0, P_<int64_t>(ctx->seg_word_dev), P_<int64_t>(ctx->seg_chunk_dev),
                          P_<SegRec>(ctx->segs_dev), P_<float>(ctx->c1_dev), 128, st));
  STAGE_END(NVGS_STAGE_SETUP);
  STAGE_BEGIN(NVGS_STAGE_CULL_MLP);
  if (opts->use_mlp)
    CK(launch_query(ctx, opts->precision, 0, nullptr, nullptr, counts64, st));
  else
    CK(launch_cull_only(P_<AssetDev>(ctx->assets_dev), P_<WorkItem>(ctx->items_dev), (int64_t)ctx->items.size(),
                        P_<int32_t>(ctx->seglist_dev), P_<SegRec>(ctx->segs_dev), P_<uint32_t>(ctx->mask),
                        P_<uint32_t>(ctx->chunk_cnt), counts64, st));
  STAGE_END(NVGS_STAGE_CULL_MLP);
  STAGE_BEGIN(NVGS_STAGE_COMPACT);
  CK(launch_scan_u32(P_<uint32_t>(ctx->chunk_cnt), P_<uint32_t>(ctx->chunk_off), ctx->n_chunks, counters + 0,
                     P_<uint32_t>(ctx->scan_part), st));
  STAGE_END(NVGS_STAGE_COMPACT);
  int64_t ns_bound = ctx->cap_splats;  // grid bound of the splat-indexed launches
  if (eager) {
    if ((s = read_counters(ctx))) return s;
    ns_bound = ctx->counters_host[0];
    if ((s = size_splats(ctx, ns_bound, true))) return s;
    if (f.debug && (s = size_debug(ctx))) return s;
  }
  const uint32_t* n_splats_dev = counters + 0;
  STAGE_BEGIN(NVGS_STAGE_PROJECT);
  CK(launch_project(P_<AssetDev>(ctx->assets_dev), P_<WorkItem>(ctx->items_dev), (int64_t)ctx->items.size(),
                    P_<int32_t>(ctx->seglist_dev), P_<SegRec>(ctx->segs_dev), P_<uint32_t>(ctx->mask),
                    P_<uint32_t>(ctx->chunk_off), n_splats_dev, ctx->cap_splats, f.T, f.tiles_x, f.n_tiles,
                    f.debug ? 1 : 0, opts->det_clip, P_<float4>(ctx->splat), P_<float4>(ctx->rec_a),
                    P_<float4>(ctx->rec_b), P_<float4>(ctx->rec_c), P_<float2>(ctx->rec_d), P_<uint4>(ctx->rect_dbg),
                    P_<uint2>(ctx->rect), P_<uint32_t>(ctx->depth_key), P_<uint32_t>(ctx->pair_of), counters + 2,
                    st));
  STAGE_END(NVGS_STAGE_PROJECT);
  // depth order of the splats (stable: equal depths keep id order)
  STAGE_BEGIN(NVGS_STAGE_DEPTH_SORT);
  bool in_tmp = false;
  // the sort also writes each splat's tile rectangle and tile count in depth
  // order (the sorted depth keys themselves are not read afterwards)
  const SortGather gather{P_<uint2>(ctx->rect), P_<uint2>(ctx->rect_sorted), P_<uint32_t>(ctx->cnt)};
  CK(launch_radix_sort(P_<uint32_t>(ctx->depth_key), P_<uint32_t>(ctx->ids), P_<uint32_t>(ctx->keys_tmp),
                       P_<uint32_t>(ctx->vals_tmp), n_splats_dev, ns_bound, 0, 32, 1, P_<uint32_t>(ctx->hist),
                       P_<uint32_t>(ctx->hist_part), &in_tmp, st, &gather));
  // four passes: the order ends in ids, and the ping-pong pair, which the
  // entry sizing below may reallocate, is free again for the tile sort
  if (in_tmp) return fail(ctx, NVGS_E_DEVICE, "depth sort: the order must end in the id buffer");
  const uint32_t* depth_ids = P_<uint32_t>(ctx->ids);
  STAGE_END(NVGS_STAGE_DEPTH_SORT);
  STAGE_BEGIN(NVGS_STAGE_BIN);
  // tile counts -> entry offsets, in place
  CK(launch_scan_u32_dev(P_<uint32_t>(ctx->cnt), P_<uint32_t>(ctx->cnt), ns_bound, n_splats_dev, counters + 1,
                         P_<uint32_t>(ctx->hist_part), st, counters + 2));
  STAGE_END(NVGS_STAGE_BIN);
  int64_t nd_bound = ctx->cap_dup;
  if (eager) {
    if ((s = read_counters(ctx))) return s;
    nd_bound = ctx->counters_host[1];
    if (ctx->counters_host[2] & 4u)
      return fail(ctx, NVGS_E_CAPACITY, "more than 2^32 - 1 (splat, tile) entries in one frame");
    if (ms_bin_count) CK(hipEventElapsedTime(ms_bin_count, ev[2 * NVGS_STAGE_BIN], ev[2 * NVGS_STAGE_BIN + 1]));
    if ((s = size_dups(ctx, nd_bound, true))) return s;
    if ((s = size_tiles(ctx, f.nkeys))) return s;
  }
  const uint32_t* n_dup_dev = counters + 1;
  STAGE_BEGIN(NVGS_STAGE_BIN);
  CK(launch_emit(depth_ids, P_<uint2>(ctx->rect_sorted), P_<uint32_t>(ctx->cnt), n_splats_dev, ns_bound, n_dup_dev,
                 ctx->cap_dup, f.tiles_x, f.n_tiles, P_<uint32_t>(ctx->keys), P_<uint32_t>(ctx->vals), counters + 2, st));
  STAGE_END(NVGS_STAGE_BIN);
  STAGE_BEGIN(NVGS_STAGE_TILE_SORT);
  bool in_tmp2 = false;
  CK(launch_radix_sort(P_<uint32_t>(ctx->keys), P_<uint32_t>(ctx->vals), P_<uint32_t>(ctx->keys_tmp),
                       P_<uint32_t>(ctx->vals_tmp), n_dup_dev, nd_bound, 0, bits_for(f.nkeys), 0,
                       P_<uint32_t>(ctx->hist), P_<uint32_t>(ctx->hist_part), &in_tmp2, st));
  const uint32_t* skeys = in_tmp2 ? P_<uint32_t>(ctx->keys_tmp) : P_<uint32_t>(ctx->keys);
  const uint32_t* sids = in_tmp2 ? P_<uint32_t>(ctx->vals_tmp) : P_<uint32_t>(ctx->vals);
  CK(launch_fill_u32(P_<uint32_t>(ctx->ranges), 0u, 2 * f.nkeys, st));
  CK(launch_ranges(skeys, n_dup_dev, nd_bound, f.nkeys, P_<uint32_t>(ctx->ranges), st));
  // launch order of the tiles: longest lists first
  uint32_t* tk = P_<uint32_t>(ctx->tord);
  const int64_t nk = f.nkeys;
  CK(launch_tile_keys(P_<uint32_t>(ctx->ranges), nk, tk, tk + nk, st));
  bool in_tmp3 = false;
  CK(launch_radix_sort(tk, tk + nk, tk + 2 * nk, tk + 3 * nk, nullptr, nk, 0, 5, 0, P_<uint32_t>(ctx->hist),
                       P_<uint32_t>(ctx->hist_part), &in_tmp3, st));
  const uint32_t* tile_order = in_tmp3 ? tk + 3 * nk : tk + nk;
  // compositing items: long lists split into chunks
  uint32_t* ts = P_<uint32_t>(ctx->tsplit);
  CK(launch_split_count(P_<uint32_t>(ctx->ranges), tile_order, nk, f.split_len, n_dup_dev, nd_bound, f.split_div, ts,
                        ts + nk, ts + 2 * nk, ts + 3 * nk, counters + 16, counters + 17, counters + 18,
                        P_<uint32_t>(ctx->hist_part), st));
  if (eager) {
    // item and split-slot counts of this frame: the buffers are sized from them
    STAGE_END(NVGS_STAGE_TILE_SORT);
    if ((s = read_counters(ctx))) return s;
    if (ms_tile_count)
      CK(hipEventElapsedTime(ms_tile_count, ev[2 * NVGS_STAGE_TILE_SORT], ev[2 * NVGS_STAGE_TILE_SORT + 1]));
    const int64_t n_items = ctx->counters_host[16], n_split = ctx->counters_host[17];
    const int ti = tile_index(f.T);
    ctx->wm_items[ti] = std::max(ctx->wm_items[ti], n_items);
    ctx->wm_split[ti] = std::max(ctx->wm_split[ti], n_split);
    if ((s = size_items(ctx, nk, f.T, f.split_len, f.split_div, n_items, n_split))) return s;
    STAGE_BEGIN(NVGS_STAGE_TILE_SORT);
  }
  const int64_t cap_split = f.split_len != 0 ? ctx->cap_split_px / ((int64_t)f.T * f.T) : 0;
  CK(launch_split_expand(ts, ts + 2 * nk, nk, P_<uint2>(ctx->citems), ctx->cap_items, counters + 17, cap_split,
                         counters + 2, st));
  STAGE_END(NVGS_STAGE_TILE_SORT);
  STAGE_BEGIN(NVGS_STAGE_BLEND);
  BlendItems bi{};
  bi.split_len = f.split_len;
  bi.order = tile_order;
  bi.nch = ts;
  bi.split_off = ts + 3 * nk;
  bi.item_off = ts + 2 * nk;
  bi.nkeys = nk;
  bi.items = P_<uint2>(ctx->citems);
  bi.n_items = counters + 16;
  bi.cap_items = ctx->cap_items;
  bi.cap_split = cap_split;
  bi.prod = P_<float>(ctx->prodb);
  bi.part = P_<float4>(ctx->partb);
  CK(launch_blend(bi, P_<uint32_t>(ctx->ranges), sids, P_<float4>(ctx->splat), f.W, f.H, f.T, f.tiles_x,
                  f.tiles_y, opts->bg[0], opts->bg[1], opts->bg[2], f.rgb, f.record ? opts->contrib : nullptr,
                  f.count_tests ? reinterpret_cast<unsigned long long*>(counters + 8) : nullptr, st));
  STAGE_END(NVGS_STAGE_BLEND);
  CK(launch_watermark(counters, st));
#undef STAGE_BEGIN
#undef STAGE_END
  ctx->last_splats = eager ? ns_bound : -1;
  ctx->last_dup = eager ? nd_bound : -1;
  ctx->last_sorted_key = skeys;
  ctx->last_sorted_id = sids;
  ctx->last_tiles_x = f.tiles_x;
  ctx->last_tiles_y = f.tiles_y;
  ctx->last_debug = f.debug;
  return NVGS_OK;
}

void fill_stats(nvgs_ctx* ctx, const Frame& f, nvgs_frame_stats* stats) {
  const unsigned long long* c64 = reinterpret_cast<const unsigned long long*>(ctx->counters_host + 4);
  stats->pairs = (int64_t)f.C * ctx->P;
  stats->in_frustum = (int64_t)c64[0];
  stats->queried = (int64_t)c64[1];
  stats->blend_tests = f.count_tests ? (int64_t)c64[2] : -1;
  stats->kept = ctx->counters_host[0];
  stats->duplicates = ctx->counters_host[1];
  stats->workspace_bytes = (int64_t)ctx->workspace;
  stats->blend_items = ctx->counters_host[16];
  stats->chunk_len = f.split_len != 0 ? (int32_t)ctx->counters_host[18] : 0;
  stats->reserved = 0;
}

}  // namespace

extern "C" {

nvgs_status nvgs_render(nvgs_ctx* ctx, const nvgs_camera* cams, int32_t C, const nvgs_render_opts* opts, float* rgb,
                        nvgs_frame_stats* stats) {
  if (!ctx) return NVGS_E_INVALID;
  nvgs_status s = ready(ctx);
  if (s) return s;
  if ((s = check_cams(ctx, cams, C))) return s;
  if (!opts || !rgb) return fail(ctx, NVGS_E_INVALID, "render: null opts or rgb");
  const int T = opts->tile;
  if (T != 8 && T != 16 && T != 32) return fail(ctx, NVGS_E_INVALID, "tile must be 8, 16 or 32");
  if (opts->precision < NVGS_PREC_FP32 || opts->precision > NVGS_PREC_FP32_SPLIT)
    return fail(ctx, NVGS_E_INVALID, "bad precision");
  if (ctx->kind == 1 && opts->use_mlp && opts->precision >= NVGS_PREC_FP8)
    return fail(ctx, NVGS_E_INVALID, "the compact MLP runs in FP32 or BF16");
  if (opts->split_len > 0 && opts->split_len < 64) return fail(ctx, NVGS_E_INVALID, "split_len must be 0, < 0 or >= 64");
  if (!(opts->det_clip >= 0.f) || !finite_f(opts->det_clip))
    return fail(ctx, NVGS_E_INVALID, "det_clip must be finite and >= 0");
  const bool record = (opts->flags & NVGS_RENDER_RECORD_CONTRIB) != 0;
  if (record && !opts->contrib) return fail(ctx, NVGS_E_INVALID, "RECORD_CONTRIB needs opts->contrib");
  const bool graph = (opts->flags & NVGS_RENDER_GRAPH) != 0;
  for (int q = 0; q < 3; ++q)
    if (!finite_f(opts->bg[q])) return fail(ctx, NVGS_E_INVALID, "non-finite background");
  CK(hipSetDevice(ctx->device));
  if ((s = plan(ctx, C))) return s;
  Frame f{};
  f.C = C;
  f.W = cams[0].width;
  f.H = cams[0].height;
  f.T = T;
  f.tiles_x = (f.W + T - 1) / T;
  f.tiles_y = (f.H + T - 1) / T;
  f.n_tiles = f.tiles_x * f.tiles_y;
  f.nkeys = (int64_t)C * f.n_tiles;
  if (f.nkeys >= ((int64_t)1 << 31)) return fail(ctx, NVGS_E_INVALID, "too many tiles");
  f.record = record;
  f.split_len = opts->split_len == 0 ? kSplitAuto : (opts->split_len < 0 ? 0 : opts->split_len);
  // about two chunks per work-group the compositing launch keeps resident
  // (2048 threads per compute unit; 64 threads per 8x8 tile, 256 otherwise)
  f.split_div = 2 * (int64_t)ctx->n_cu * 2048 / (T == 8 ? 64 : 256);
  f.debug = record || (opts->flags & NVGS_RENDER_KEEP_DEBUG);
  f.count_tests = stats != nullptr && !(opts->flags & NVGS_RENDER_NO_TEST_COUNT);
  f.opts = opts;
  f.rgb = rgb;
  hipStream_t st = ctx->stream;
  if (!graph) {
    if ((s = upload_cams(ctx, cams, C))) return s;
    float ms_bin_count = 0.f, ms_tile_count = 0.f;
    if ((s = enqueue_frame(ctx, st, f, true, &ms_bin_count, &ms_tile_count))) return s;
    if (stats) {
      if ((s = read_counters(ctx))) return s;
      float ms = 0.f;
      CK(hipEventElapsedTime(&ms, ctx->ev[2 * NVGS_STAGE_SETUP], ctx->ev[2 * NVGS_STAGE_BLEND + 1]));
      for (int k = 0; k < NVGS_NUM_STAGES; ++k) {
        float m = 0.f;
        CK(hipEventElapsedTime(&m, ctx->ev[2 * k], ctx->ev[2 * k + 1]));
        stats->ms_stage[k] = m;
      }
      stats->ms_stage[NVGS_STAGE_BIN] += ms_bin_count;
      stats->ms_stage[NVGS_STAGE_TILE_SORT] += ms_tile_count;
      stats->ms_total = ms;
      fill_stats(ctx, f, stats);
      if (ctx->counters_host[2]) return fail(ctx, NVGS_E_CAPACITY, "capacity exceeded");
    }
    return NVGS_OK;
  }
  // persistent frame
  if (ctx->cap_splats <= 0 || ctx->cap_dup <= 0)
    return fail(ctx, NVGS_E_STATE, "GRAPH frames need capacities: nvgs_reserve, or one frame without NVGS_RENDER_GRAPH");
  if ((s = size_tiles(ctx, f.nkeys)) || (s = size_hist(ctx)) ||
      (s = size_items(ctx, f.nkeys, f.T, f.split_len, f.split_div, -1, -1)))
    return s;
  if (f.debug && (s = size_debug(ctx))) return s;
  if (ctx->cap_keys < f.nkeys || ctx->cap_hist < std::max({ctx->cap_dup, ctx->cap_splats, ctx->cap_keys}) ||
      (f.debug && ctx->cap_debug < ctx->cap_splats))
    return fail(ctx, NVGS_E_STATE, "frame buffers are incomplete after a failed allocation");
  const std::vector<uint64_t> key = {
      (uint64_t)C, (uint64_t)f.W, (uint64_t)f.H, (uint64_t)T, (uint64_t)opts->use_mlp, (uint64_t)opts->precision,
      (uint64_t)opts->flags, (uint64_t)reinterpret_cast<uintptr_t>(rgb),
      (uint64_t)reinterpret_cast<uintptr_t>(record ? opts->contrib : nullptr), (uint64_t)(stats != nullptr),
      ctx->gen, (uint64_t)shape_nb(ctx, opts->precision), (uint64_t)ctx->mlp_segs,
      (uint64_t)ctx->cap_splats, (uint64_t)ctx->cap_dup, (uint64_t)(int64_t)f.split_len,
      (uint64_t)__builtin_bit_cast(uint32_t, opts->det_clip),
      ((uint64_t)__builtin_bit_cast(uint32_t, opts->bg[0]) << 32) | __builtin_bit_cast(uint32_t, opts->bg[1]),
      (uint64_t)__builtin_bit_cast(uint32_t, opts->bg[2])};
  if (!ctx->gexec || key != ctx->gkey) {
    if (ctx->gexec) {
      CK(hipStreamSynchronize(st));
      (void)hipGraphExecDestroy(ctx->gexec);
      ctx->gexec = nullptr;
    }
    CK(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
    s = enqueue_frame(ctx, ctx->cap_stream, f, false, nullptr, nullptr);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(ctx->cap_stream, &g);
    if (s || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return s ? s : fail(ctx, NVGS_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    }
    const hipError_t ei = hipGraphInstantiate(&ctx->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
      ctx->gexec = nullptr;
      return fail(ctx, NVGS_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
    }
    ctx->gkey = key;
  }
  if ((s = upload_cams(ctx, cams, C))) return s;
  if (stats) CK(hipEventRecord(ctx->gev[0], st));
  CK(hipGraphLaunch(ctx->gexec, st));
  if (stats) {
    CK(hipEventRecord(ctx->gev[1], st));
    if ((s = read_counters(ctx))) return s;
    float ms = 0.f;
    CK(hipEventElapsedTime(&ms, ctx->gev[0], ctx->gev[1]));
    for (int k = 0; k < NVGS_NUM_STAGES; ++k) stats->ms_stage[k] = 0.f;
    stats->ms_total = ms;
    fill_stats(ctx, f, stats);
    if (ctx->counters_host[2]) return fail(ctx, NVGS_E_CAPACITY, "capacity exceeded");
  }
  return NVGS_OK;
}

nvgs_status nvgs_reserve(nvgs_ctx* ctx, int64_t max_splats, int64_t max_duplicates) {
  if (!ctx) return NVGS_E_INVALID;
  if (max_splats < 0 || max_duplicates < 0 || max_splats >= ((int64_t)1 << 32) ||
      max_duplicates >= ((int64_t)1 << 32))
    return fail(ctx, NVGS_E_INVALID, "reserve: sizes must be in [0, 2^32)");
  CK(hipSetDevice(ctx->device));
  nvgs_status s = size_splats(ctx, max_splats, false);
  if (!s) s = size_dups(ctx, max_duplicates, false);
  return s;
}

nvgs_status nvgs_frame_watermarks(nvgs_ctx* ctx, int64_t* max_splats, int64_t* max_duplicates, int32_t* overflowed,
                                  int32_t reset) {
  if (!ctx) return NVGS_E_INVALID;
  CK(hipSetDevice(ctx->device));
  nvgs_status s = read_counters(ctx);
  if (s) return s;
  if (max_splats) *max_splats = ctx->counters_host[12];
  if (max_duplicates) *max_duplicates = ctx->counters_host[13];
  if (overflowed) *overflowed = ctx->counters_host[14] != 0;
  if (reset) {
    CK(launch_fill_u32(P_<uint32_t>(ctx->counters) + 12, 0u, 3, ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
  }
  return NVGS_OK;
}

nvgs_status nvgs_workspace_info(nvgs_ctx* ctx, nvgs_workspace* out) {
  if (!ctx) return NVGS_E_INVALID;
  if (!out) return fail(ctx, NVGS_E_INVALID, "workspace_info: null out");
  auto sum = [](std::initializer_list<const Buf*> l) {
    int64_t t = 0;
    for (const Buf* b : l) t += (int64_t)b->bytes;
    return t;
  };
  nvgs_workspace w{};
  w.total = (int64_t)ctx->workspace;
  w.assets = sum({&ctx->assets_dev, &ctx->inst_dev, &ctx->inst_off_dev});
  for (const Buf& b : ctx->op_bufs) w.assets += (int64_t)b.bytes;
  w.pairs = sum({&ctx->seg_word_dev, &ctx->seg_chunk_dev, &ctx->items_dev, &ctx->seglist_dev, &ctx->segs_dev,
                 &ctx->c1_dev, &ctx->mask, &ctx->chunk_cnt, &ctx->chunk_off, &ctx->scan_part, &ctx->cam_dev});
  w.splats = sum({&ctx->splat, &ctx->rect, &ctx->rect_sorted, &ctx->depth_key, &ctx->ids, &ctx->cnt});
  w.entries = sum({&ctx->keys, &ctx->vals, &ctx->keys_tmp, &ctx->vals_tmp, &ctx->hist, &ctx->hist_part});
  w.tiles = sum({&ctx->ranges, &ctx->tord, &ctx->tsplit, &ctx->citems, &ctx->prodb, &ctx->partb});
  w.debug = sum({&ctx->rec_a, &ctx->rec_b, &ctx->rec_c, &ctx->rec_d, &ctx->rect_dbg, &ctx->pair_of});
  w.other = w.total - (w.assets + w.pairs + w.splats + w.entries + w.tiles + w.debug);
  w.splat_capacity = ctx->cap_splats;
  w.entry_capacity = ctx->cap_dup;
  *out = w;
  return NVGS_OK;
}

nvgs_status nvgs_sort_pairs(nvgs_ctx* ctx, uint32_t* keys, uint32_t* vals, int64_t n, int32_t begin_bit,
                            int32_t end_bit) {
  if (!ctx) return NVGS_E_INVALID;
  if (n < 0 || n >= ((int64_t)1 << 32)) return fail(ctx, NVGS_E_INVALID, "sort_pairs: n must be in [0, 2^32)");
  if (begin_bit < 0 || end_bit > 32 || begin_bit > end_bit)
    return fail(ctx, NVGS_E_INVALID, "sort_pairs: need 0 <= begin_bit <= end_bit <= 32");
  if (n > 0 && (!keys || !vals)) return fail(ctx, NVGS_E_INVALID, "sort_pairs: null keys or vals");
  if (n == 0 || begin_bit == end_bit) return NVGS_OK;
  CK(hipSetDevice(ctx->device));
  if (!ensure(ctx, ctx->sort_tmp, 8 * (size_t)n) || !ensure(ctx, ctx->sort_ws, 4 * radix_hist_words(n)))
    return fail(ctx, NVGS_E_NOMEM, "sort_pairs: workspace");
  hipStream_t st = ctx->stream;
  uint32_t* kt = P_<uint32_t>(ctx->sort_tmp);
  bool in_tmp = false;
  CK(launch_radix_sort(keys, vals, kt, kt + n, nullptr, n, begin_bit, end_bit, 0, P_<uint32_t>(ctx->sort_ws), nullptr,
                       &in_tmp, st));
  if (in_tmp) {
    CK(hipMemcpyAsync(keys, kt, 4 * (size_t)n, hipMemcpyDeviceToDevice, st));
    CK(hipMemcpyAsync(vals, kt + n, 4 * (size_t)n, hipMemcpyDeviceToDevice, st));
  }
  CK(hipStreamSynchronize(st));
  return NVGS_OK;
}

nvgs_status nvgs_set_mlp_shape(nvgs_ctx* ctx, const nvgs_mlp_shape* shape) {
  if (!ctx) return NVGS_E_INVALID;
  if (!shape) return fail(ctx, NVGS_E_INVALID, "null shape");
  if (shape->gaussians_per_wave != 32 && shape->gaussians_per_wave != 64 && shape->gaussians_per_wave != 128)
    return fail(ctx, NVGS_E_INVALID, "gaussians_per_wave must be 32, 64 or 128");
  if (shape->segments_per_group < 1 || shape->segments_per_group > 1024)
    return fail(ctx, NVGS_E_INVALID, "segments_per_group must be in [1, 1024]");
  ctx->mlp_nb = shape->gaussians_per_wave / 32;
  ctx->mlp_segs = shape->segments_per_group;
  return NVGS_OK;
}

nvgs_status nvgs_get_mlp_shape(nvgs_ctx* ctx, nvgs_mlp_shape* shape) {
  if (!ctx) return NVGS_E_INVALID;
  if (!shape) return fail(ctx, NVGS_E_INVALID, "null shape");
  shape->gaussians_per_wave = 32 * ctx->mlp_nb;
  shape->segments_per_group = ctx->mlp_segs;
  return NVGS_OK;
}

nvgs_status nvgs_autotune(nvgs_ctx* ctx, const nvgs_camera* cams, int32_t C, nvgs_render_opts* opts, float* rgb,
                          int32_t reps, nvgs_tune_entry* table, int32_t table_cap, int32_t* n_entries) {
  if (!ctx) return NVGS_E_INVALID;
  if (!opts || !rgb) return fail(ctx, NVGS_E_INVALID, "autotune: null opts or rgb");
  if (reps < 1 || reps > 1000) return fail(ctx, NVGS_E_INVALID, "autotune: reps must be in [1, 1000]");
  if (table_cap < 0 || (table_cap > 0 && !table)) return fail(ctx, NVGS_E_INVALID, "autotune: bad table");
  nvgs_status s = ready(ctx);
  if (s) return s;
  nvgs_render_opts o = *opts;
  o.flags &= ~(int32_t)NVGS_RENDER_GRAPH;
  o.flags |= NVGS_RENDER_NO_TEST_COUNT;  // time the kernels of frames without statistics
  if (o.tile != 8 && o.tile != 16 && o.tile != 32) o.tile = 16;
  const int saved_nb = ctx->mlp_nb, saved_segs = ctx->mlp_segs;
  int n = 0;
  auto record = [&](int tile, int nb, int segs, float ms) {
    if (n < table_cap) table[n] = nvgs_tune_entry{tile, 32 * nb, segs, ms};
    ++n;
  };
  // median over `reps` timed frames after one untimed frame; returns the
  // culling + MLP stage time and the whole-frame time
  auto measure = [&](float* cull_ms, float* total_ms) -> nvgs_status {
    nvgs_frame_stats st{};
    nvgs_status r = nvgs_render(ctx, cams, C, &o, rgb, &st);
    if (r) return r;
    std::vector<float> a, b;
    for (int k = 0; k < reps; ++k) {
      if ((r = nvgs_render(ctx, cams, C, &o, rgb, &st))) return r;
      a.push_back(st.ms_stage[NVGS_STAGE_CULL_MLP]);
      b.push_back(st.ms_total);
    }
    std::nth_element(a.begin(), a.begin() + a.size() / 2, a.end());
    std::nth_element(b.begin(), b.begin() + b.size() / 2, b.end());
    *cull_ms = a[a.size() / 2];
    *total_ms = b[b.size() / 2];
    return NVGS_OK;
  };
  // 1. MLP block shape, by the culling + MLP stage time
  int best_nb = saved_nb, best_segs = saved_segs;
  float best_cull = INFINITY;
  for (int nb : {1, 2, 4}) {
    // the compact MLP has one block shape: only the segment grouping varies
    if (ctx->kind == 1 ? nb != saved_nb : !mlp_shape_supported(ctx->width, o.precision, nb)) continue;
    for (int segs : {4, 8, 16, 32, 64}) {
      ctx->mlp_nb = nb;
      ctx->mlp_segs = segs;
      float cm = 0.f, tm = 0.f;
      if ((s = measure(&cm, &tm))) {
        ctx->mlp_nb = saved_nb;
        ctx->mlp_segs = saved_segs;
        return s;
      }
      record(o.tile, nb, segs, cm);
      if (cm < best_cull) best_cull = cm, best_nb = nb, best_segs = segs;
    }
  }
  ctx->mlp_nb = best_nb;
  ctx->mlp_segs = best_segs;
  // 2. tile size, by the whole-frame time with that shape
  int best_tile = o.tile;
  float best_total = INFINITY;
  for (int tile : {8, 16, 32}) {
    o.tile = tile;
    float cm = 0.f, tm = 0.f;
    if ((s = measure(&cm, &tm))) return s;
    record(tile, best_nb, best_segs, tm);
    if (tm < best_total) best_total = tm, best_tile = tile;
  }
  opts->tile = best_tile;
  if (n_entries) *n_entries = n;
  return NVGS_OK;
}

nvgs_status nvgs_debug_buffers(nvgs_ctx* ctx, nvgs_debug_view* out) {
  if (!ctx) return NVGS_E_INVALID;
  if (!out) return fail(ctx, NVGS_E_INVALID, "null output");
  std::memset(out, 0, sizeof(*out));
  if (!ctx->last_sorted_key) return fail(ctx, NVGS_E_STATE, "no frame rendered yet");
  if (ctx->last_splats < 0) {  // graph frame: counts are on the device
    nvgs_status s = read_counters(ctx);
    if (s) return s;
    out->n_splats = std::min<int64_t>(ctx->counters_host[0], ctx->cap_splats);
    out->n_dup = std::min<int64_t>(ctx->counters_host[1], ctx->cap_dup);
  } else {
    out->n_splats = ctx->last_splats;
    out->n_dup = ctx->last_dup;
  }
  out->pair = ctx->last_debug ? P_<uint32_t>(ctx->pair_of) : nullptr;  // debug arrays exist only then
  out->rec_a = ctx->last_debug ? P_<float>(ctx->rec_a) : nullptr;
  out->rec_b = ctx->last_debug ? P_<float>(ctx->rec_b) : nullptr;
  out->rec_c = ctx->last_debug ? P_<float>(ctx->rec_c) : nullptr;
  out->rec_d = ctx->last_debug ? P_<float>(ctx->rec_d) : nullptr;
  out->rect = P_<uint32_t>(ctx->rect_dbg);
  out->sorted_key = ctx->last_sorted_key;
  out->sorted_id = ctx->last_sorted_id;
  out->ranges = P_<uint32_t>(ctx->ranges);
  out->tiles_x = ctx->last_tiles_x;
  out->tiles_y = ctx->last_tiles_y;
  return NVGS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// labels, training and the MLP forward / backward
// ---------------------------------------------------------------------------
namespace {

// temporary device buffer owned by one call
struct Tmp {
  nvgs_ctx* ctx;
  Buf b;
  explicit Tmp(nvgs_ctx* c) : ctx(c) {}
  ~Tmp() {
    if (b.p) {
      (void)hipStreamSynchronize(ctx->stream);
      release(ctx, b);
    }
  }
  template <class T>
  T* get(size_t count) {
    return ensure(ctx, b, count * sizeof(T)) ? reinterpret_cast<T*>(b.p) : nullptr;
  }
};

nvgs_status check_train_prec(nvgs_ctx* ctx, int32_t precision, int32_t width, int32_t kind = 0) {
  if (precision != NVGS_PREC_FP32 && precision != NVGS_PREC_BF16)
    return fail(ctx, NVGS_E_INVALID, "training precision must be FP32 or BF16");
  if (kind == 0 && width != 64 && width != 128) return fail(ctx, NVGS_E_INVALID, "training supports widths 64 and 128");
  if (kind == 1 && width != 32) return fail(ctx, NVGS_E_INVALID, "the compact MLP has width 32");
  return NVGS_OK;
}

// chunks of 128 samples per compact-training work-group: about 512 groups for large batches
int ctrain_chunks(int64_t batch) {
  const int64_t per = ctrain_samples_per_chunk();
  return (int)std::min<int64_t>(16, std::max<int64_t>(1, (batch + per * 512 - 1) / (per * 512)));
}

constexpr int kTrainChunksPerWG = 4;  // 4 x 64 pairs per work-group
constexpr int kPairsPerWG = 64 * kTrainChunksPerWG;

}  // namespace

extern "C" {

// Auxiliary label views of view v: v rotated rigidly (position and
// orientation) about the asset centre, the origin of the asset frame, by
// `angle` around the axes k_j = cos(phi_j) e1 + sin(phi_j) e2, phi_j = 2 pi j / aux,
// where d = pos/|pos|, e1 = v's right axis made orthogonal to d, e2 = d x e1.
// Each auxiliary camera stays at v's distance, on the cone of half-angle
// `angle` around d, and keeps v's framing of the asset.
static std::vector<nvgs_camera> aux_views(const nvgs_camera& v, int aux, double angle) {
  std::vector<nvgs_camera> out;
  double d[3] = {v.pos[0], v.pos[1], v.pos[2]};
  const double dist = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  if (dist <= 0) return out;
  for (double& x : d) x /= dist;
  double e1[3] = {v.R[0], v.R[1], v.R[2]};
  const double rd = e1[0] * d[0] + e1[1] * d[1] + e1[2] * d[2];
  for (int k = 0; k < 3; ++k) e1[k] -= rd * d[k];
  const double l1 = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
  if (!(l1 > 1e-9)) return out;
  for (double& x : e1) x /= l1;
  const double e2[3] = {d[1] * e1[2] - d[2] * e1[1], d[2] * e1[0] - d[0] * e1[2], d[0] * e1[1] - d[1] * e1[0]};
  const double ca = std::cos(angle), sa = std::sin(angle);
  for (int j = 0; j < aux; ++j) {
    const double ph = 2.0 * M_PI * j / aux;
    double k[3];
    for (int q = 0; q < 3; ++q) k[q] = std::cos(ph) * e1[q] + std::sin(ph) * e2[q];
    // Rodrigues: rot(x) = x cos a + (k x x) sin a + k (k.x)(1 - cos a)
    auto rot = [&](const double* x, float* y) {
      const double kx[3] = {k[1] * x[2] - k[2] * x[1], k[2] * x[0] - k[0] * x[2], k[0] * x[1] - k[1] * x[0]};
      const double kd = k[0] * x[0] + k[1] * x[1] + k[2] * x[2];
      for (int q = 0; q < 3; ++q) y[q] = (float)(x[q] * ca + kx[q] * sa + k[q] * kd * (1.0 - ca));
    };
    nvgs_camera cam = v;
    const double p[3] = {v.pos[0], v.pos[1], v.pos[2]};
    rot(p, cam.pos);
    for (int r = 0; r < 3; ++r) {
      const double row[3] = {v.R[3 * r], v.R[3 * r + 1], v.R[3 * r + 2]};
      rot(row, cam.R + 3 * r);
    }
    out.push_back(cam);
  }
  return out;
}

nvgs_status nvgs_make_labels(nvgs_ctx* ctx, int32_t asset, const nvgs_camera* views_in, int32_t V_in, float threshold,
                             int32_t tile, int32_t aux, float aux_angle, uint32_t* labels) {
  if (!ctx) return NVGS_E_INVALID;
  if (aux < 0 || aux > 64 || !std::isfinite(aux_angle)) return fail(ctx, NVGS_E_INVALID, "bad auxiliary views");
  if (!views_in || V_in <= 0) return fail(ctx, NVGS_E_INVALID, "views: null pointer or V <= 0");
  // main views followed, per view, by its auxiliary views: label rows are OR-ed per group
  std::vector<nvgs_camera> all;
  for (int v = 0; v < V_in; ++v) {
    all.push_back(views_in[v]);
    for (const nvgs_camera& c : aux_views(views_in[v], aux, aux_angle)) all.push_back(c);
  }
  const nvgs_camera* views = all.data();
  const int32_t V = (int32_t)all.size();
  const int group = 1 + aux;
  if (ctx->assets.empty()) return fail(ctx, NVGS_E_STATE, "no assets loaded");
  if (asset < 0 || asset >= (int)ctx->assets.size()) return fail(ctx, NVGS_E_INVALID, "asset index out of range");
  if (!labels) return fail(ctx, NVGS_E_INVALID, "labels: null pointer");
  if (!std::isfinite(threshold) || !(threshold >= FLT_MIN))
    return fail(ctx, NVGS_E_INVALID, "threshold must be finite and at least the smallest normal float");
  nvgs_status s = check_cams(ctx, views, V);
  if (s) return s;
  CK(hipSetDevice(ctx->device));
  const int64_t n = ctx->assets[asset].n;
  const int64_t words = (n + 31) / 32;
  // a single identity instance of the asset; the caller's list is restored
  std::vector<nvgs_instance> saved = ctx->inst;
  nvgs_instance id{};
  id.asset = asset;
  id.R[0] = id.R[4] = id.R[8] = 1.f;
  id.s = 1.f;
  if ((s = nvgs_set_instances(ctx, &id, 1))) return s;
  const int VB = std::min(V, 16);
  const int Wd = views[0].width, Ht = views[0].height;
  Tmp contrib(ctx), rgb(ctx), rows(ctx);
  float* cb = contrib.get<float>((size_t)VB * n);
  float* img = rgb.get<float>((size_t)VB * Wd * Ht * 3);
  uint32_t* lab_all = group == 1 ? labels : rows.get<uint32_t>((size_t)V * words);
  if (!cb || !img || !lab_all) s = fail(ctx, NVGS_E_NOMEM, "label buffers");
  for (int v0 = 0; v0 < V && !s; v0 += VB) {
    const int nb = std::min(VB, V - v0);
    if (hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(cb), 0u, (int64_t)nb * n, ctx->stream)) {
      s = fail(ctx, NVGS_E_DEVICE, hipGetErrorString(e));
      break;
    }
    nvgs_render_opts ro{};
    ro.tile = tile;
    ro.use_mlp = 0;
    ro.precision = NVGS_PREC_FP32;
    ro.flags = NVGS_RENDER_RECORD_CONTRIB;
    ro.contrib = cb;
    if ((s = nvgs_render(ctx, views + v0, nb, &ro, img, nullptr))) break;
    if (hipError_t e = launch_label_bits(cb, n, nb, threshold, lab_all + (int64_t)v0 * words, ctx->stream))
      s = fail(ctx, NVGS_E_DEVICE, hipGetErrorString(e));
  }
  if (!s && group > 1)
    if (hipError_t e = launch_or_groups(lab_all, V_in, group, words, labels, ctx->stream))
      s = fail(ctx, NVGS_E_DEVICE, hipGetErrorString(e));
  if (hipStreamSynchronize(ctx->stream) != hipSuccess && !s) s = fail(ctx, NVGS_E_DEVICE, "label renders failed");
  const std::string err = ctx->err;
  nvgs_status s2 = saved.empty() ? NVGS_OK : nvgs_set_instances(ctx, saved.data(), (int)saved.size());
  if (saved.empty()) ctx->inst.clear(), ctx->planC = -1;
  if (s) {
    ctx->err = err;
    return s;
  }
  return s2;
}

// learning rate of step t (0-based) of T: constant, or (Sec. 4.1) a cosine
// warm-up from 0 to lr over the first 20 % of the steps followed by an
// exponential decay from lr to lr_final at the last step
static float step_lr(const nvgs_train_opts* o, int t) {
  if (o->schedule != 1) return o->lr;
  const int T = o->steps, Tw = std::max(1, (int)std::lround(0.2 * T));
  if (t < Tw) return (float)(o->lr * 0.5 * (1.0 - std::cos(M_PI * (t + 1) / Tw)));
  const double u = T - Tw > 1 ? (double)(t - Tw) / (double)(T - Tw - 1) : 1.0;
  return (float)(o->lr * std::pow((double)o->lr_final / o->lr, u));
}

nvgs_status nvgs_train_visibility(nvgs_ctx* ctx, int32_t asset, const nvgs_camera* views, int32_t V,
                                  const uint32_t* labels, const nvgs_train_opts* opts, float* params,
                                  float* loss_curve) {
  if (!ctx) return NVGS_E_INVALID;
  if (ctx->assets.empty()) return fail(ctx, NVGS_E_STATE, "no assets loaded");
  if (asset < 0 || asset >= (int)ctx->assets.size()) return fail(ctx, NVGS_E_INVALID, "asset index out of range");
  if (!opts || !params) return fail(ctx, NVGS_E_INVALID, "null opts or params");
  if (opts->batch < 1 || opts->steps < 1) return fail(ctx, NVGS_E_INVALID, "batch and steps must be >= 1");
  if (opts->schedule != 0 && !(opts->schedule == 1 && opts->lr_final > 0.f && std::isfinite(opts->lr_final)))
    return fail(ctx, NVGS_E_INVALID, "schedule must be 0, or 1 with lr_final > 0");
  if (!(opts->lr > 0.f) || !(opts->beta1 >= 0.f && opts->beta1 < 1.f) || !(opts->beta2 >= 0.f && opts->beta2 < 1.f) ||
      !(opts->eps > 0.f))
    return fail(ctx, NVGS_E_INVALID, "bad Adam hyper-parameters");
  nvgs_status s = check_train_prec(ctx, opts->precision, ctx->assets[asset].mlp.width, ctx->kind);
  if (s) return s;
  if ((s = check_cams(ctx, views, V))) return s;
  CK(hipSetDevice(ctx->device));
  const nvgs_asset& A = ctx->assets[asset];
  const int64_t n = A.n, words = (n + 31) / 32;
  Tmp lab_tmp(ctx);
  if (!labels) {
    uint32_t* lb = lab_tmp.get<uint32_t>((size_t)V * words);
    if (!lb) return fail(ctx, NVGS_E_NOMEM, "labels");
    if ((s = nvgs_make_labels(ctx, asset, views, V, opts->threshold, opts->tile, 0, 0.f, lb))) return s;
    labels = lb;
  }
  const bool compact = ctx->kind == 1;
  const int np = compact ? ctrain_num_params() : train_num_params(A.mlp.width);
  const int cpw = compact ? ctrain_chunks(opts->batch) : kTrainChunksPerWG;
  const int64_t per_wg = compact ? (int64_t)ctrain_samples_per_chunk() * cpw : (int64_t)kPairsPerWG;
  const int nwg = (int)((opts->batch + per_wg - 1) / per_wg);
  if (opts->weighting != 0 && opts->weighting != 1) return fail(ctx, NVGS_E_INVALID, "weighting must be 0 or 1");
  Tmp cams_t(ctx), gam_t(ctx), part_t(ctx), lp_t(ctx), m_t(ctx), v_t(ctx), loss_t(ctx), cnt_t(ctx);
  nvgs_camera* cams_d = cams_t.get<nvgs_camera>(V);
  float* gam = gam_t.get<float>((size_t)V * (compact ? 8 : 36));
  float* part = part_t.get<float>((size_t)nwg * np + reduce_scratch_floats(nwg, np));
  float* lp = lp_t.get<float>(nwg);
  float* m = m_t.get<float>(np);
  float* v = v_t.get<float>(np);
  float* loss = loss_t.get<float>(opts->steps);
  uint32_t* npos = cnt_t.get<uint32_t>(opts->steps);
  if (!cams_d || !gam || !part || !lp || !m || !v || !loss || !npos)
    return fail(ctx, NVGS_E_NOMEM, "training buffers");
  CK(hipMemcpy(cams_d, views, sizeof(nvgs_camera) * V, hipMemcpyHostToDevice));
  CK(launch_fill_u32(reinterpret_cast<uint32_t*>(m), 0u, np, ctx->stream));
  CK(launch_fill_u32(reinterpret_cast<uint32_t*>(v), 0u, np, ctx->stream));
  if (compact)
    CK(launch_cview(cams_d, V, A.mlp.train_focal, A.mlp.d_min, A.mlp.d_max, gam, ctx->stream));
  else
    CK(launch_view_gam(cams_d, V, A.mlp.cam_scale, A.mlp.train_focal, A.mlp.d_max, gam, ctx->stream));
  const bool bf16 = opts->precision == NVGS_PREC_BF16;
  const float inv_b = 1.f / (float)opts->batch;
  const bool weighted = opts->weighting == 1;
  if (weighted) CK(launch_fill_u32(npos, 0u, opts->steps, ctx->stream));
  for (int step = 0; step < opts->steps; ++step) {
    if (weighted)
      CK(launch_count_pos(opts->batch, n, V, labels, opts->seed, step, npos + step, ctx->stream));
    if (compact) {
      const CTrainArgs ca{A.mean, A.scale, A.quat, A.opacity, n, A.mlp.mean_scale, gam, V, labels, opts->seed,
                          step, weighted ? npos + step : nullptr};
      CK(launch_cmlp_train(0, bf16, nwg, cpw, ctx->stream, params, opts->batch, inv_b, ca, nullptr, nullptr, nullptr,
                           part, lp));
    } else {
      CK(launch_mlp_train(0, bf16, A.mlp.width, nwg, ctx->stream, params, opts->batch, inv_b, A.mean, n,
                          A.mlp.mean_scale, gam, V, labels, opts->seed, step, weighted ? npos + step : nullptr,
                          nullptr, nullptr, nullptr, part, lp, nullptr));
    }
    CK(launch_reduce_adam_n(part, nwg, np, params, m, v, nullptr, step_lr(opts, step), opts->beta1, opts->beta2,
                            opts->eps, step + 1, lp, inv_b, loss + step, ctx->stream, part + (size_t)nwg * np));
  }
  CK(hipStreamSynchronize(ctx->stream));
  if (loss_curve) CK(hipMemcpy(loss_curve, loss, sizeof(float) * opts->steps, hipMemcpyDeviceToHost));
  return NVGS_OK;
}

nvgs_status nvgs_mlp_forward(nvgs_ctx* ctx, const float* params, int32_t width, const float* X, int64_t B,
                             int32_t precision, float* logits) {
  if (!ctx) return NVGS_E_INVALID;
  if (!params || !X || !logits || B < 1) return fail(ctx, NVGS_E_INVALID, "mlp_forward: null pointer or B < 1");
  nvgs_status s = check_train_prec(ctx, precision, width);
  if (s) return s;
  CK(hipSetDevice(ctx->device));
  const int nwg = (int)((B + kPairsPerWG - 1) / kPairsPerWG);
  CK(launch_mlp_train(1, precision == NVGS_PREC_BF16, width, nwg, ctx->stream, params, B, 1.f, nullptr,
                      1, 0.f, nullptr, 1, nullptr, 0, 0, nullptr, X, nullptr, logits, nullptr, nullptr, nullptr));
  return NVGS_OK;
}

nvgs_status nvgs_mlp_backward(nvgs_ctx* ctx, const float* params, int32_t width, const float* X, int64_t B,
                              const float* dlogits, int32_t precision, float* dparams, float* dX) {
  if (!ctx) return NVGS_E_INVALID;
  if (!params || !X || !dlogits || !dparams || B < 1)
    return fail(ctx, NVGS_E_INVALID, "mlp_backward: null pointer or B < 1");
  nvgs_status s = check_train_prec(ctx, precision, width);
  if (s) return s;
  CK(hipSetDevice(ctx->device));
  const int nwg = (int)((B + kPairsPerWG - 1) / kPairsPerWG);
  Tmp part_t(ctx);
  const int np = train_num_params(width);
  float* part = part_t.get<float>((size_t)nwg * np + reduce_scratch_floats(nwg, np));
  if (!part) return fail(ctx, NVGS_E_NOMEM, "gradient partials");
  CK(launch_mlp_train(2, precision == NVGS_PREC_BF16, width, nwg, ctx->stream, params, B, 1.f, nullptr,
                      1, 0.f, nullptr, 1, nullptr, 0, 0, nullptr, X, dlogits, nullptr, part, nullptr, dX));
  CK(launch_reduce_adam_n(part, nwg, np, nullptr, nullptr, nullptr, dparams, 0.f, 0.f, 0.f, 1.f, 1, nullptr, 0.f,
                          nullptr, ctx->stream, part + (size_t)nwg * np));
  return NVGS_OK;
}

nvgs_status nvgs_mlp_backward_noalloc(nvgs_ctx* ctx, const float* params, int32_t width, const float* X, int64_t B,
                                      const float* dlogits, int32_t precision, float* dparams, float* dX) {
  if (!ctx) return NVGS_E_INVALID;
  if (!params || !X || !dlogits || !dparams || B < 1)
    return fail(ctx, NVGS_E_INVALID, "mlp_backward_noalloc: null pointer or B < 1");
  if (B > (width == 128 ? NVGS_NOALLOC_MAX_BATCH_W128 : NVGS_NOALLOC_MAX_BATCH))
    return fail(ctx, NVGS_E_INVALID,
                "mlp_backward_noalloc: B exceeds NVGS_NOALLOC_MAX_BATCH (65536; NVGS_NOALLOC_MAX_BATCH_W128 = 16896 "
                "at width 128)");
  nvgs_status s = check_train_prec(ctx, precision, width);
  if (s) return s;
  CK(hipSetDevice(ctx->device));
  size_t cap = 0;
  float* part = static_scratch(ctx->device, &cap);
  if (!part) return fail(ctx, NVGS_E_STATE, "mlp_backward_noalloc: workspace address of this device not looked up");
  // the same partition and kernels as nvgs_mlp_backward, so the results are identical
  const int nwg = (int)((B + kPairsPerWG - 1) / kPairsPerWG);
  const int np = train_num_params(width);
  const size_t need = (size_t)nwg * np + reduce_scratch_floats(nwg, np);
  if (need > cap) return fail(ctx, NVGS_E_INVALID, "mlp_backward_noalloc: batch needs more than the fixed workspace");
  CK(launch_mlp_train(2, precision == NVGS_PREC_BF16, width, nwg, ctx->stream, params, B, 1.f, nullptr,
                      1, 0.f, nullptr, 1, nullptr, 0, 0, nullptr, X, dlogits, nullptr, part, nullptr, dX));
  CK(launch_reduce_adam_n(part, nwg, np, nullptr, nullptr, nullptr, dparams, 0.f, 0.f, 0.f, 1.f, 1, nullptr, 0.f,
                          nullptr, ctx->stream, part + (size_t)nwg * np));
  return NVGS_OK;
}

nvgs_status nvgs_cmlp_forward(nvgs_ctx* ctx, const float* params, const float* X, int64_t B, int32_t precision,
                              float* logits) {
  if (!ctx) return NVGS_E_INVALID;
  if (!params || !X || !logits || B < 1) return fail(ctx, NVGS_E_INVALID, "cmlp_forward: null pointer or B < 1");
  nvgs_status s = check_train_prec(ctx, precision, 32, 1);
  if (s) return s;
  CK(hipSetDevice(ctx->device));
  const int cpw = ctrain_chunks(B);
  const int64_t per_wg = (int64_t)ctrain_samples_per_chunk() * cpw;
  const int nwg = (int)((B + per_wg - 1) / per_wg);
  const CTrainArgs none{};
  CK(launch_cmlp_train(1, precision == NVGS_PREC_BF16, nwg, cpw, ctx->stream, params, B, 1.f, none, X, nullptr,
                       logits, nullptr, nullptr));
  return NVGS_OK;
}

nvgs_status nvgs_cmlp_backward(nvgs_ctx* ctx, const float* params, const float* X, int64_t B, const float* dlogits,
                               int32_t precision, float* dparams) {
  if (!ctx) return NVGS_E_INVALID;
  if (!params || !X || !dlogits || !dparams || B < 1)
    return fail(ctx, NVGS_E_INVALID, "cmlp_backward: null pointer or B < 1");
  nvgs_status s = check_train_prec(ctx, precision, 32, 1);
  if (s) return s;
  CK(hipSetDevice(ctx->device));
  const int cpw = ctrain_chunks(B);
  const int64_t per_wg = (int64_t)ctrain_samples_per_chunk() * cpw;
  const int nwg = (int)((B + per_wg - 1) / per_wg);
  const int np = ctrain_num_params();
  Tmp part_t(ctx);
  float* part = part_t.get<float>((size_t)nwg * np + reduce_scratch_floats(nwg, np));
  if (!part) return fail(ctx, NVGS_E_NOMEM, "gradient partials");
  const CTrainArgs none{};
  CK(launch_cmlp_train(2, precision == NVGS_PREC_BF16, nwg, cpw, ctx->stream, params, B, 1.f, none, X, dlogits,
                       nullptr, part, nullptr));
  CK(launch_reduce_adam_n(part, nwg, np, nullptr, nullptr, nullptr, dparams, 0.f, 0.f, 0.f, 1.f, 1, nullptr, 0.f,
                          nullptr, ctx->stream, part + (size_t)nwg * np));
  return NVGS_OK;
}

}  // extern "C"
