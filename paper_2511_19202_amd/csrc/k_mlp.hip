// Per-frame steps 1-2 of the NVGS renderer (Sec. 3.3): frustum culling of
// every (camera, instance, Gaussian) pair on the Gaussian mean, and the
// visibility-MLP query for the in-frustum pairs, on gfx950 MFMA.
//
// Design (MI355X-first):
//  * Layer 1 is linear in the 72 encoded inputs, which split into the 36
//    Gaussian features gamma(mu) and the 36 camera features gamma(c).  The
//    camera half W1c gamma(c) + b1 is the same for every Gaussian of a
//    (camera, instance) segment, so a tiny setup kernel computes it once per
//    segment (in FP64).  The Gaussian half U = W1u gamma(mu) does not depend
//    on the instance, so one work-group computes it once for a chunk of 256
//    Gaussians and reuses it, in registers, for every segment of that asset.
//  * Hidden layers run on v_mfma_f32_32x32x2_f32 with the pairs as the N
//    dimension.  The accumulator of one layer is used directly as the B
//    operand of the next: the contraction index is permuted to follow the
//    accumulator register order and the weights are stored pre-permuted in
//    LDS (operand image built once per asset), so activations never leave
//    registers.
//  * Per 32 pairs a wave-uniform ballot skips the MLP when no pair is in the
//    frustum.  The keep decisions are written as 32-pair bit words plus one
//    count per 256-pair chunk for the ordered compaction that follows.
#include "internal.h"

namespace nvgs {

typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kK1 = 18;  // K=2 steps over the 36 Gaussian features of layer 1

// floats in the FP32 operand image of a width-W MLP
__host__ __device__ constexpr int op_f32_size(int W) { return ((36 * W + 2 * W * W + 3 * W + 1) + 3) / 4 * 4; }

size_t mlp_op_f32_floats(int width) { return (size_t)op_f32_size(width); }

// ---------------------------------------------------------------------------
// operand image: W1u [NT][18][64], W2p [NT][KS][64], W3p [NT][KS][64],
// b2p [2][KS], b3p [2][KS], wop [2][KS], bo
// ---------------------------------------------------------------------------
__global__ void k_prepare_f32(const float* __restrict__ P, int W, float* __restrict__ op) {
  const int NT = W / 32, KS = W / 2, in1 = 72;
  const float* W1 = P;
  const float* b1 = W1 + W * in1;
  const float* W2 = b1 + W;
  const float* b2 = W2 + W * W;
  const float* W3 = b2 + W;
  const float* b3 = W3 + W * W;
  const float* wo = b3 + W;
  const float bo = wo[W];
  (void)b1;
  const int total = op_f32_size(W);
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x) {
    float v = 0.f;
    int o = idx;
    if (o < NT * kK1 * 64) {
      int lane = o % 64, s = (o / 64) % kK1, t = o / (64 * kK1);
      v = W1[(32 * t + lane % 32) * in1 + 2 * s + lane / 32];
    } else if ((o -= NT * kK1 * 64) < 2 * NT * KS * 64) {
      const float* Wl = o < NT * KS * 64 ? W2 : W3;
      o %= NT * KS * 64;
      int lane = o % 64, s = (o / 64) % KS, t = o / (64 * KS);
      v = Wl[(32 * t + lane % 32) * W + hid_feature(s, lane / 32)];
    } else if ((o -= 2 * NT * KS * 64) < 6 * KS) {
      int which = o / (2 * KS), r = o % (2 * KS), g = r / KS, q = r % KS;
      const float* vec = which == 0 ? b2 : which == 1 ? b3 : wo;
      v = vec[hid_feature(q, g)];
    } else if (o == 6 * KS) {
      v = bo;
    }
    op[idx] = v;
  }
}

hipError_t launch_prepare_mlp(const float* params, int width, float* op_f32, uint16_t* op_bf16, uint8_t* op_fp8,
                              float* fp8_scale, hipStream_t st) {
  (void)op_bf16; (void)op_fp8; (void)fp8_scale;
  int total = op_f32_size(width);
  hipLaunchKernelGGL(k_prepare_f32, dim3((total + 255) / 256), dim3(256), 0, st, params, width, op_f32);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// per-frame segment setup: one 64-thread group per (camera, instance)
// ---------------------------------------------------------------------------
__global__ void k_segment_setup(const nvgs_camera* __restrict__ cams, const nvgs_instance* __restrict__ insts,
                                const AssetDev* __restrict__ assets, const int64_t* __restrict__ inst_offset,
                                int32_t n_inst, int64_t P, int use_mlp, const int64_t* __restrict__ word_base,
                                const int64_t* __restrict__ chunk_base, SegRec* __restrict__ segs,
                                float* __restrict__ c1perm, int c1_stride) {
  const int seg = blockIdx.x;
  const int k = seg / n_inst, i = seg % n_inst;
  const nvgs_camera& cam = cams[k];
  const nvgs_instance& in = insts[i];
  const AssetDev& A = assets[in.asset];
  __shared__ double s_gam[36];
  __shared__ double s_c1[128];
  __shared__ int s_query;
  // camera in the asset frame: R^T (c - t) / s  (FP64)
  double d[3] = {(double)cam.pos[0] - in.t[0], (double)cam.pos[1] - in.t[1], (double)cam.pos[2] - in.t[2]};
  double cl[3];
  for (int r = 0; r < 3; ++r)
    cl[r] = ((double)in.R[r] * d[0] + (double)in.R[3 + r] * d[1] + (double)in.R[6 + r] * d[2]) / (double)in.s;
  // FoV correction (Eq. 2) and far clamp of the MLP's camera input
  double f_r = 1.0 / tan(0.5 * (double)cam.fovy);
  double fac = (double)A.train_focal / f_r;
  double cm[3] = {cl[0] * fac, cl[1] * fac, cl[2] * fac};
  double len = sqrt(cm[0] * cm[0] + cm[1] * cm[1] + cm[2] * cm[2]);
  if (A.d_max > 0.f && len > (double)A.d_max) {
    double sc = (double)A.d_max / len;
    for (int r = 0; r < 3; ++r) cm[r] *= sc;
    len = (double)A.d_max;
  }
  if (threadIdx.x == 0) s_query = (use_mlp && len >= (double)A.d_min) ? 1 : 0;
  if (threadIdx.x < 36) {
    int j = threadIdx.x / 12, band = (threadIdx.x % 12) / 2, cs = threadIdx.x % 2;
    double a = ldexp(M_PI * ((double)A.cam_scale * cm[j]), band);
    s_gam[threadIdx.x] = cs ? cos(a) : sin(a);
  }
  __syncthreads();
  const int W = A.width;
  const float* W1 = A.params;
  const float* b1 = W1 + (size_t)W * 72;
  for (int r = threadIdx.x; r < W; r += blockDim.x) {
    double s = b1[r];
    for (int q = 0; q < 36; ++q) s += (double)W1[(size_t)r * 72 + 36 + q] * s_gam[q];
    s_c1[r] = s;
  }
  __syncthreads();
  const int KS = W / 2;
  for (int e = threadIdx.x; e < W; e += blockDim.x) {
    int g = e / KS, q = e % KS;
    c1perm[(size_t)seg * c1_stride + e] = (float)s_c1[hid_feature(q, g)];
  }
  if (threadIdx.x == 0) {
    SegRec R;
    // camera-space p = Rc (s Ri mu + t - c) = (s Rc Ri) mu + Rc (t - c)
    double Rc[9], Ri[9];
    for (int q = 0; q < 9; ++q) { Rc[q] = cam.R[q]; Ri[q] = in.R[q]; }
    for (int r = 0; r < 3; ++r) {
      for (int c = 0; c < 3; ++c) {
        double s = 0;
        for (int q = 0; q < 3; ++q) s += Rc[3 * r + q] * Ri[3 * q + c];
        R.M[4 * r + c] = (float)(s * (double)in.s);
      }
      R.M[4 * r + 3] = (float)(Rc[3 * r] * -d[0] + Rc[3 * r + 1] * -d[1] + Rc[3 * r + 2] * -d[2]);
    }
    for (int r = 0; r < 3; ++r) R.cl[r] = (float)cl[r];
    double tany = tan(0.5 * (double)cam.fovy);
    double focal = 0.5 * (double)cam.height / tany;
    double tanx = 0.5 * (double)cam.width / focal;
    R.near_plane = cam.near_plane;
    R.tanx_g = (float)(1.3 * tanx);
    R.tany_g = (float)(1.3 * tany);
    R.focal = (float)focal;
    R.half_w = 0.5f * (float)cam.width;
    R.half_h = 0.5f * (float)cam.height;
    R.asset = in.asset;
    R.inst = i;
    R.cam = k;
    R.n = (int32_t)A.n;
    R.query = s_query;
    R.pad0 = 0;
    R.pair_base = (int64_t)k * P + inst_offset[i];
    R.word_base = word_base[seg];
    R.chunk_base = chunk_base[seg];
    segs[seg] = R;
  }
}

hipError_t launch_segment_setup(const nvgs_camera* cams_dev, const nvgs_instance* inst_dev, const AssetDev* assets,
                                const int64_t* inst_offset, int32_t n_inst, int32_t C, int64_t P, int use_mlp,
                                const int64_t* seg_word_base, const int64_t* seg_chunk_base, SegRec* segs,
                                float* c1perm, int max_width, hipStream_t st) {
  hipLaunchKernelGGL(k_segment_setup, dim3(C * n_inst), dim3(64), 0, st, cams_dev, inst_dev, assets, inst_offset,
                     n_inst, P, use_mlp, seg_word_base, seg_chunk_base, segs, c1perm, max_width);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP32 cull + MLP kernel
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool frustum(const SegRec& R, const float mu[3], float* pz_out) {
  float px = fmaf(R.M[0], mu[0], fmaf(R.M[1], mu[1], fmaf(R.M[2], mu[2], R.M[3])));
  float py = fmaf(R.M[4], mu[0], fmaf(R.M[5], mu[1], fmaf(R.M[6], mu[2], R.M[7])));
  float pz = fmaf(R.M[8], mu[0], fmaf(R.M[9], mu[1], fmaf(R.M[10], mu[2], R.M[11])));
  if (pz_out) *pz_out = pz;
  return pz > R.near_plane && fabsf(px) <= R.tanx_g * pz && fabsf(py) <= R.tany_g * pz;
}

template <int W, int NB>
__device__ __forceinline__ void hidden_f32(const float* __restrict__ Wp, const float* __restrict__ bp,
                                           const float (&h)[NB][W / 2], float (&o)[NB][W / 2], int lane, int grp) {
  constexpr int NT = W / 32, KS = W / 2;
  f32x16 acc[NB][NT];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[b][t] = (f32x16){0};
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    float a[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) a[t] = Wp[(t * KS + s) * 64 + lane];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[b][t] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[t], h[b][s], acc[b][t], 0, 0, 0);
  }
  const float* bg = bp + grp * KS;
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int q = 0; q < KS; ++q) o[b][q] = fmaxf(acc[b][q / 16][q % 16] + bg[q], 0.f);
}

template <int W, int NB, int WAVES, int MODE>
__global__ __launch_bounds__(64 * WAVES) void k_cull_mlp_f32(
    const AssetDev* __restrict__ assets, const WorkItem* __restrict__ items, const int32_t* __restrict__ seglist,
    const SegRec* __restrict__ segs, const float* __restrict__ c1perm, int c1_stride, uint32_t* __restrict__ mask,
    uint32_t* __restrict__ chunk_count, uint8_t* __restrict__ state, float* __restrict__ logits,
    unsigned long long* __restrict__ frame_counts) {
  static_assert(WAVES * NB * 32 == kChunk, "a work-group covers one compaction chunk");
  constexpr int NT = W / 32, KS = W / 2;
  constexpr int OPN = op_f32_size(W);
  __shared__ __attribute__((aligned(16))) float lds[OPN];
  __shared__ uint32_t s_cnt[2];
  __shared__ uint32_t s_tot[2];
  const WorkItem it = items[blockIdx.x];
  const AssetDev* A = assets + it.asset;
  {
    const float4* src = reinterpret_cast<const float4*>(A->op_f32);
    for (int k = threadIdx.x; k < OPN / 4; k += 64 * WAVES) reinterpret_cast<float4*>(lds)[k] = src[k];
  }
  if (threadIdx.x < 2) s_cnt[threadIdx.x] = s_tot[threadIdx.x] = 0;
  const float* W1u = lds;
  const float* W2p = W1u + NT * kK1 * 64;
  const float* W3p = W2p + NT * KS * 64;
  const float* b2p = W3p + NT * KS * 64;
  const float* b3p = b2p + 2 * KS;
  const float* wop = b3p + 2 * KS;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ncol = lane & 31, grp = lane >> 5;
  const int64_t n = A->n;
  const float msc = A->mean_scale;
  const int64_t g0 = (int64_t)it.chunk * kChunk + wave * (32 * NB);
  float mu[NB][3];
  bool valid[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    int64_t g = g0 + 32 * b + ncol;
    valid[b] = g < n;
    for (int j = 0; j < 3; ++j) mu[b][j] = valid[b] ? A->mean[j * n + g] : 0.f;
  }
  __syncthreads();
  const float bo = wop[2 * KS];
  // layer 1, Gaussian half: U = W1u gamma(mean_scale * mu)
  f32x16 U[NB][NT];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int t = 0; t < NT; ++t) U[b][t] = (f32x16){0};
#pragma unroll
  for (int s = 0; s < kK1; ++s) {
    const int j = s / 6, band = s % 6;
    float a[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) a[t] = W1u[(t * kK1 + s) * 64 + lane];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      float x = ldexpf(msc * mu[b][j], band);
      float e = grp ? cospif(x) : sinpif(x);
#pragma unroll
      for (int t = 0; t < NT; ++t) U[b][t] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[t], e, U[b][t], 0, 0, 0);
    }
  }
  int parity = 0;
  uint32_t n_in = 0, n_q = 0;  // in-frustum and queried pairs of this wave
  for (int si = it.seg_begin; si < it.seg_end; ++si, parity ^= 1) {
    const int seg = seglist[si];
    const SegRec& R = segs[seg];
    bool in[NB];
    bool any = false;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      in[b] = valid[b] && frustum(R, mu[b], nullptr);
      any |= in[b];
    }
    const bool wave_any = __ballot(any) != 0;
    const bool query = R.query != 0;
    {
      uint32_t cin = 0;
#pragma unroll
      for (int b = 0; b < NB; ++b) cin += __popc((uint32_t)__ballot(in[b]));
      n_in += cin;
      n_q += query ? cin : 0u;
    }
    float z[NB];
    bool keep[NB];
    if (query && wave_any) {
      const float* c1 = c1perm + (size_t)seg * c1_stride + grp * KS;
      float h[NB][KS], h2[NB][KS];
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int q = 0; q < KS; ++q) h[b][q] = fmaxf(U[b][q / 16][q % 16] + c1[q], 0.f);
      hidden_f32<W, NB>(W2p, b2p, h, h2, lane, grp);
      hidden_f32<W, NB>(W3p, b3p, h2, h, lane, grp);
      const float* wg = wop + grp * KS;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        float part = 0.f;
#pragma unroll
        for (int q = 0; q < KS; ++q) part = fmaf(wg[q], h[b][q], part);
        z[b] = part + __shfl_xor(part, 32) + bo;
        keep[b] = in[b] && z[b] >= 0.f;
      }
    } else {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        z[b] = __builtin_nanf("");
        keep[b] = in[b] && !query;
      }
    }
    uint32_t cnt = 0;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      uint32_t word = (uint32_t)__ballot(keep[b]);
      cnt += __popc(word);
      if (lane == 0 && g0 + 32 * b < n) mask[R.word_base + (g0 >> 5) + b] = word;
    }
    if (lane == 0) atomicAdd(&s_cnt[parity], cnt);
    if (MODE == 1 && grp == 0) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        if (valid[b]) {
          int64_t idx = R.pair_base + g0 + 32 * b + ncol;
          state[idx] = keep[b] ? 2 : (in[b] ? 1 : 0);
          logits[idx] = (in[b] && query) ? z[b] : __builtin_nanf("");
        }
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      chunk_count[R.chunk_base + it.chunk] = s_cnt[parity];
      s_cnt[parity] = 0;
    }
  }
  if (frame_counts) {
    if (lane == 0) {
      atomicAdd(&s_tot[0], n_in);
      atomicAdd(&s_tot[1], n_q);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      atomicAdd(frame_counts + 0, (unsigned long long)s_tot[0]);
      atomicAdd(frame_counts + 1, (unsigned long long)s_tot[1]);
    }
  }
}

template <int W, int NB, int WAVES>
static hipError_t launch_f32(const AssetDev* assets, const WorkItem* items, int64_t n_items, const int32_t* seglist,
                             const SegRec* segs, const float* c1perm, int c1_stride, int mode, uint32_t* mask,
                             uint32_t* chunk_count, uint8_t* state, float* logits, unsigned long long* counts,
                             hipStream_t st) {
  if (mode == 1)
    hipLaunchKernelGGL((k_cull_mlp_f32<W, NB, WAVES, 1>), dim3((unsigned)n_items), dim3(64 * WAVES), 0, st, assets,
                       items, seglist, segs, c1perm, c1_stride, mask, chunk_count, state, logits, counts);
  else
    hipLaunchKernelGGL((k_cull_mlp_f32<W, NB, WAVES, 0>), dim3((unsigned)n_items), dim3(64 * WAVES), 0, st, assets,
                       items, seglist, segs, c1perm, c1_stride, mask, chunk_count, state, logits, counts);
  return hipGetLastError();
}

hipError_t launch_cull_mlp(const AssetDev* assets_dev, const AssetDev* assets_host, int32_t n_assets,
                           const WorkItem* items, int64_t n_items, const int32_t* seglist, const SegRec* segs,
                           const float* c1perm, int max_width, int width, int precision, int mode, uint32_t* mask,
                           uint32_t* chunk_count, uint8_t* state, float* logits, unsigned long long* counts,
                           hipStream_t st) {
  (void)assets_host; (void)n_assets; (void)precision;
  if (n_items == 0) return hipSuccess;
  if (width == 64)
    return launch_f32<64, 2, 4>(assets_dev, items, n_items, seglist, segs, c1perm, max_width, mode, mask,
                                chunk_count, state, logits, counts, st);
  if (width == 128)
    return launch_f32<128, 1, 8>(assets_dev, items, n_items, seglist, segs, c1perm, max_width, mode, mask,
                                 chunk_count, state, logits, counts, st);
  return hipErrorInvalidValue;
}

}  // namespace nvgs
