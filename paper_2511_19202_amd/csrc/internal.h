// Internal declarations of the NVGS gfx950 library (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/nvgs.h"

namespace nvgs {

// Compositing constants of original 3DGS (Sec. 4.1): fragments below 1/255
// are skipped, alpha is clamped to 0.99, and the pixel stops before its
// transmittance would drop below 1e-4.
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTMin = 1e-4f;
constexpr float kGuard = 1.3f;   // frustum / Jacobian side guard band
constexpr float kDilate = 0.3f;  // screen-space low-pass added to the 2D covariance

// ReLU as a signed integer max on the bit pattern (negative values and -0
// have the sign bit set): one instruction, where fmaxf on an MFMA result also
// costs a canonicalising max
__device__ __forceinline__ float relu(float x) { return __int_as_float(max(__float_as_int(x), 0)); }

constexpr int kChunk = 256;           // pairs per compaction chunk (one cull/MLP work-group)
constexpr int kSortBlock = 2048;      // keys per radix-sort block
constexpr int kScanBlock = 4096;      // items per scan block

// Per-asset device record (library-owned copy of the borrowed pointers and
// the MLP operands in MFMA register order).
struct AssetDev {
  const float* mean;
  const float* scale;
  const float* quat;
  const float* opacity;
  const float* sh;
  int64_t n;
  int32_t sh_degree;
  int32_t width;
  float mean_scale, cam_scale, train_focal, d_min, d_max;
  const float* params;   // packed FP32 (borrowed)
  const float* op_f32;   // FP32 operand image (library-owned)
  const uint16_t* op_bf16;
  const uint8_t* op_fp8;
  const uint8_t* op_split;  // split-FP32 operand image (frequency form)
  const float* fp8_scale; // per-layer dequantisation scales
  // projection image (library-owned, one record per Gaussian so that the
  // gathers of sparse survivors read whole lines): geo[3g..3g+2] =
  // (mean, opacity), (scale, 0), (qw, qx, qy, qz); shp[g * sh_stride + 3c + ch]
  const float4* geo;
  const float* shp;
  int32_t sh_stride;     // 3 (d+1)^2 rounded up to a multiple of 4
  int32_t kind;          // 0: frequency-encoded MLP; 1: the compact form
  const float* emb;      // compact form: per-Gaussian embedding [n][8] (6 used), library-owned
};

// compact MLP form (16 inputs, 2 x 32 hidden, per-Gaussian 6-D embedding)
constexpr int kCompactVis = 32 * 16 + 32 + 32 * 32 + 32 + 32 + 1;
constexpr int kCompactEmb = 32 * 8 + 32 + 32 * 32 + 32 + 6 * 32 + 6;
size_t cmlp_image_floats();  // FP32 operand image (the BF16 one fits in it)
hipError_t launch_prepare_cmlp(const float* params, float* img_f32, uint16_t* img_bf16, hipStream_t st);
hipError_t launch_cembed(const float* params, const float* scale, const float* quat, const float* opacity, int64_t n,
                         float* emb, hipStream_t st);

int32_t sh_stride_for(int sh_degree);
hipError_t launch_pack_asset(const float* mean, const float* scale, const float* quat, const float* opacity,
                             const float* sh, int64_t n, int sh_degree, float4* geo, float* shp, hipStream_t st);

// Per (camera, instance) segment, built on the device every frame.
struct SegRec {
  float M[12];       // camera-space p = M[:, 0:3] mu + M[:, 3]  (row-major 3x4)
  float Mlo[12];     // M - (double)M: low-order parts, so that M + Mlo carries ~48 bits
  float cl[3];       // camera position in the asset frame (undoes R, t, s)
  float near_plane;
  float tanx_g, tany_g;  // 1.3 * tan(fov/2) in x and y
  float focal;           // pixels
  float focal_lo;        // focal - (double)focal
  float half_w, half_h;
  int32_t asset, inst, cam, n;
  int32_t query;     // 1 = the MLP decides, 0 = every in-frustum Gaussian is kept
  float dn_a, dn_b;  // compact MLP form: distance input = clamp(dn_a |mu - cl| + dn_b, -1, 1)
  int64_t pair_base;   // cam * P + instance offset  (index into [C][P] outputs)
  int64_t word_base;   // first 32-pair mask word of the segment
  int64_t chunk_base;  // first compaction chunk of the segment
};

// One cull/MLP work item: a 256-Gaussian chunk of an asset against a run of
// that asset's segments (indices into the per-asset segment list).
struct WorkItem {
  int32_t asset;
  int32_t chunk;
  int32_t seg_begin;
  int32_t seg_end;
};

// float bits are monotone for non-negative floats
__device__ __forceinline__ uint32_t fbits(float x) { return __float_as_uint(x); }

// feature held by MFMA lane group g in its q-th accumulator value after a
// 32x32 output tile sequence (row = 8*(r/4) + 4*g + r%4 of tile q/16)
__host__ __device__ constexpr int hid_feature(int q, int g) {
  return 32 * (q / 16) + 8 * ((q % 16) / 4) + 4 * g + (q % 4);
}

// ---- launchers (defined in the .hip files) --------------------------------
// operand images of the MLP weights for one asset
hipError_t launch_prepare_mlp(const float* params, int width, float* op_f32, uint16_t* op_bf16, uint8_t* op_fp8,
                              float* fp8_scale, hipStream_t st);
size_t mlp_op_f32_floats(int width);
size_t mlp_op_bf16_elems(int width);
size_t mlp_op_fp8_bytes(int width);
size_t mlp_op_split_bytes(int width);
hipError_t launch_prepare_split(const float* params, int width, uint8_t* op_split, hipStream_t st);

hipError_t launch_segment_setup(const nvgs_camera* cams_dev, const nvgs_instance* inst_dev, const AssetDev* assets,
                                const int64_t* inst_offset, int32_t n_inst, int32_t C, int64_t P, int use_mlp,
                                const int64_t* seg_word_base, const int64_t* seg_chunk_base, SegRec* segs,
                                float* c1perm, int max_width, hipStream_t st);

// mode: 0 = render (mask + chunk counts), 1 = query (state + logits as well).
// nb: Gaussians per wave in units of 32 (the work-group has kChunk / (32 nb)
// waves); supported shapes: mlp_shape_supported().
bool mlp_shape_supported(int width, int precision, int nb);
// frustum culling only (frames rendered without the MLP)
hipError_t launch_cull_only(const AssetDev* assets_dev, const WorkItem* items, int64_t n_items, const int32_t* seglist,
                            const SegRec* segs, uint32_t* mask, uint32_t* chunk_count, unsigned long long* counts,
                            hipStream_t st);
hipError_t launch_cull_mlp(const AssetDev* assets_dev, const WorkItem* items, int64_t n_items, const int32_t* seglist,
                           const SegRec* segs, const float* c1perm, int max_width, int width, int precision, int nb,
                           int mode, uint32_t* mask, uint32_t* chunk_count, uint8_t* state, float* logits,
                           unsigned long long* counts, hipStream_t st);
hipError_t launch_cull_cmlp(const AssetDev* assets, const WorkItem* items, int64_t n_items, const int32_t* seglist,
                            const SegRec* segs, const float* c1perm, int c1_stride, int precision, int mode,
                            uint32_t* mask, uint32_t* chunk_count, uint8_t* state, float* logits,
                            unsigned long long* counts, hipStream_t st);

hipError_t launch_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total, uint32_t* partials,
                           hipStream_t st);
// wrap (nullable): bit value 4 is OR-ed in when the total reaches 2^32
hipError_t launch_scan_u32_dev(const uint32_t* in, uint32_t* out, int64_t n, const uint32_t* n_dev, uint32_t* total,
                               uint32_t* partials, hipStream_t st, uint32_t* wrap);
size_t scan_partials_needed(int64_t n);

hipError_t launch_project(const AssetDev* assets, const WorkItem* items, int64_t n_items, const int32_t* seglist,
                          const SegRec* segs, const uint32_t* mask, const uint32_t* chunk_off, const uint32_t* n_splats,
                          int64_t cap_splats, int tile, int tiles_x, int n_tiles, int keep_debug, float det_clip,
                          float4* splat, float4* rec_a, float4* rec_b, float4* rec_c, float2* rec_d, uint4* rect_dbg,
                          uint2* rect, uint32_t* depth_key, uint32_t* pair_of, uint32_t* overflow, hipStream_t st);

// Optional output of a sort: for each sorted value v (in sorted order),
// rect_out = rect[v] and count_out = the rectangle's width x height (the
// splats' tile rectangles and tile counts in depth order); the sorted keys
// may then be left unwritten.
struct SortGather {
  const uint2* rect;
  uint2* rect_out;
  uint32_t* count_out;
};
hipError_t launch_radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* keys_tmp, uint32_t* vals_tmp,
                             const uint32_t* n_dev, int64_t cap, int begin_bit, int end_bit, int iota_vals,
                             uint32_t* hist, uint32_t* partials, bool* result_in_tmp, hipStream_t st,
                             const SortGather* gather = nullptr);
size_t radix_hist_words(int64_t cap);  // sort workspace (32-bit words) for up to cap keys

hipError_t launch_emit(const uint32_t* sorted_ids, const uint2* rect_sorted, const uint32_t* dup_off, const uint32_t* n_dev,
                       int64_t cap, const uint32_t* n_dup_dev, int64_t cap_dup, int tiles_x, int n_tiles,
                       uint32_t* keys, uint32_t* vals, uint32_t* overflow, hipStream_t st);
hipError_t launch_watermark(uint32_t* counters, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st);
hipError_t launch_ranges(const uint32_t* keys, const uint32_t* n_dev, int64_t cap, int64_t nkeys, uint32_t* ranges,
                         hipStream_t st);
hipError_t launch_tile_keys(const uint32_t* ranges, int64_t n, uint32_t* keys, uint32_t* vals, hipStream_t st);
// Compositing work items (tile lists longer than split_len entries are cut
// into chunks composited by separate work-groups; split_len == 0: never;
// kSplitAuto: the length follows the frame's entry count, see k_split_count).
constexpr int kSplitAuto = -1;
constexpr int kSplitMin = 256;  // shortest chunk of the frame-adaptive length
struct BlendItems {
  int split_len;
  const uint32_t* order;    // tile launch order (positions -> tile keys)
  const uint32_t* nch;      // [nkeys] chunks per position
  const uint32_t* split_off;// [nkeys] first split-chunk slot per position
  const uint2* items;       // [cap_items] (position, chunk)
  const uint32_t* n_items;  // device count of items
  int64_t cap_items;
  int64_t cap_split;        // split-chunk slots (at most 2 cap_dup / split_len + 2 are used)
  float* prod;              // [split slots][T*T]
  float4* part;             // [split slots][T*T]
  const uint32_t* item_off; // [nkeys] first item per position
  int64_t nkeys;            // positions (cameras x tiles)
};
// Builds nch / item_off / split_off and the item list; n_items and n_split
// receive the totals; overflow bit value 8 when cap_items is exceeded.
// split_len == kSplitAuto: chunks of max(kSplitMin, ceil(n_entries / split_div))
// entries, n_entries = min(*n_dev, cap) (the frame's tile-list entries).
hipError_t launch_split_count(const uint32_t* ranges, const uint32_t* order, int64_t nkeys, int split_len,
                              const uint32_t* n_dev, int64_t cap, int64_t split_div, uint32_t* nch, uint32_t* nsp,
                              uint32_t* item_off, uint32_t* split_off, uint32_t* n_items, uint32_t* n_split,
                              uint32_t* chunk_len, uint32_t* partials, hipStream_t st);
hipError_t launch_split_expand(const uint32_t* nch, const uint32_t* item_off, int64_t nkeys, uint2* items,
                               int64_t cap_items, const uint32_t* n_split, int64_t cap_split, uint32_t* overflow,
                               hipStream_t st);
// splat: [n][4] float4 compositing records written by launch_project
hipError_t launch_blend(const BlendItems& bi, const uint32_t* ranges, const uint32_t* ids, const float4* splat, int W,
                        int H, int tile, int tiles_x, int tiles_y, float bg0, float bg1, float bg2, float* rgb,
                        float* contrib, unsigned long long* work, hipStream_t st);

}  // namespace nvgs

namespace nvgs {
// training (k_train.hip)
size_t train_smem_bytes();
int train_num_params(int width = 64);
// modes of the training kernels: sampled pairs with BCE, logits only, vector-Jacobian product
enum { kModeTrainW = 0, kModeForwardW = 1, kModeBackwardW = 2 };
hipError_t launch_view_gam(const nvgs_camera* views, int V, float cam_scale, float train_focal, float d_max,
                           float* gam, hipStream_t st);
hipError_t launch_label_bits(const float* contrib, int64_t n, int V, float thr, uint32_t* bits, hipStream_t st);
// work-groups of 256 pairs (nwg = ceil(batch / 256)); FP32 width 64 on the
// FP32 MFMA kernel, BF16 (widths 64, 128) and FP32 width 128 on k_mlp_train_w
hipError_t launch_mlp_train(int mode, bool bf16, int width, int nwg, hipStream_t st, const float* params,
                            int64_t batch, float inv_batch, const float* mean, int64_t n, float mean_scale,
                            const float* view_gam, int V, const uint32_t* labels, uint64_t seed, int64_t step,
                            const uint32_t* n_pos, const float* X, const float* dlogits, float* logits,
                            float* partial, float* loss_part, float* dX);
hipError_t launch_mlp_train_w(int mode, bool bf16, int width, int nwg, int pairs_per_wg, hipStream_t st,
                              const float* params, int64_t batch, float inv_batch, const float* mean, int64_t n,
                              float mean_scale, const float* view_gam, int V, const uint32_t* labels, uint64_t seed,
                              int64_t step, const uint32_t* n_pos, const float* X, const float* dlogits,
                              float* logits, float* partial, float* loss_part, float* dX);
hipError_t launch_or_groups(const uint32_t* rows, int V, int group, int64_t words, uint32_t* out, hipStream_t st);
hipError_t launch_count_pos(int64_t batch, int64_t n, int V, const uint32_t* labels, uint64_t seed, int64_t step,
                            uint32_t* count, hipStream_t st);
hipError_t launch_reduce_adam(const float* partial, int nwg, float* params, float* m, float* v, float* grad_out,
                              float lr, float b1, float b2, float eps, int64_t t, const float* loss_part,
                              float inv_batch, float* loss_out, hipStream_t st);
// slices (nullable, reduce_scratch_floats(nwg, np) floats) enables a two-level sum
size_t reduce_scratch_floats(int nwg, int np);
hipError_t launch_reduce_adam_n(const float* partial, int nwg, int np, float* params, float* m, float* v,
                                float* grad_out, float lr, float b1, float b2, float eps, int64_t t,
                                const float* loss_part, float inv_batch, float* loss_out, hipStream_t st,
                                float* slices);
// Fixed per-device workspace (16 MiB) of the allocation-free backward: the
// address is looked up once per device (static_scratch_init, with that device
// made current for the lookup); static_scratch returns it (NULL before the
// lookup) and its size in floats.
hipError_t static_scratch_init(int device);
float* static_scratch(int device, size_t* floats);

// training of the compact form (k_ctrain.hip)
struct CTrainArgs {
  const float *mean, *scale, *quat, *opacity;  // asset SoA
  int64_t n;
  float mean_scale;
  const float* vrec;  // [V][8] from launch_cview
  int V;
  const uint32_t* labels;  // [V][ceil(n / 32)] bits
  uint64_t seed;
  int64_t step;
  const uint32_t* n_pos;  // positives of the step's batch (class weighting) or null
};
size_t ctrain_smem_bytes();
int ctrain_num_params();
int ctrain_samples_per_chunk();
hipError_t launch_cview(const nvgs_camera* views, int V, float train_focal, float d_min, float d_max, float* out,
                        hipStream_t st);
// mode 0: train step gradients from sampled (Gaussian, view) pairs; 1: logits of X [B][18];
// 2: parameter-gradient partials of X under dlogits.  Partials: one [3175] row per work-group.
hipError_t launch_cmlp_train(int mode, bool bf16, int nwg, int chunks_per_wg, hipStream_t st, const float* params,
                             int64_t batch, float inv_batch, const CTrainArgs& a, const float* X,
                             const float* dlogits, float* logits, float* partial, float* loss_part);
}  // namespace nvgs
