// Per-frame steps 1-2 of the NVGS renderer (Sec. 3.3): frustum culling of
// every (camera, instance, Gaussian) pair on the Gaussian mean, and the
// visibility-MLP query for the in-frustum pairs, on gfx950 MFMA, with FP32,
// BF16 or FP8 (OCP E4M3) operands and FP32 accumulation.
//
// Design (MI355X-first):
//  * Layer 1 is linear in the 72 encoded inputs, which split into the 36
//    Gaussian features gamma(mu) and the 36 camera features gamma(c).  The
//    camera half W1c gamma(c) + b1 is the same for every Gaussian of a
//    (camera, instance) segment, so a tiny setup kernel computes it once per
//    segment (in FP64).  The Gaussian half U = W1u gamma(mu) does not depend
//    on the instance, so one work-group computes it once for a chunk of 256
//    Gaussians and reuses it, in registers, for every segment of that asset.
//  * Hidden layers run on 32x32 MFMA tiles with the pairs as the N
//    dimension.  The accumulator of one layer is used directly as the B
//    operand of the next: the contraction index is permuted to follow the
//    accumulator register order and the weights are stored pre-permuted in
//    LDS (an operand image built once per asset), so activations never leave
//    registers.
//  * FP8 uses power-of-two per-layer scales: weights by their maximum,
//    activations by a rigorous interval bound derived from the weights
//    (|gamma| <= 1 propagates through |W| row sums), so no value saturates;
//    dequantisation is one multiply in the epilogue.
//  * Per 32 pairs a wave-uniform ballot skips the MLP when no pair is in the
//    frustum.  The keep decisions are written as 32-pair bit words plus one
//    count per 256-pair chunk for the ordered compaction that follows.
#include "internal.h"

namespace nvgs {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
// operand image of a width-W MLP for precision P (bytes):
//   W1u  [NT][KS1][64 lanes][EPL]  Gaussian half of layer 1 (36 of 72 inputs)
//   W2p  [NT][KSH][64][EPL], W3p   hidden layers, contraction index permuted
//   vec  f32: b2p [2][W/2], b3p [2][W/2], wop [2][W/2], bo, scales[8]
// EPL = operand elements per lane per MFMA (1 FP32, 8 BF16, 32 FP8).
// ---------------------------------------------------------------------------
template <int P>
struct Prec;
template <>
struct Prec<NVGS_PREC_FP32> {
  static constexpr int EPL = 1, ESZ = 4, K = 2;
};
template <>
struct Prec<NVGS_PREC_BF16> {
  static constexpr int EPL = 8, ESZ = 2, K = 16;
};
template <>
struct Prec<NVGS_PREC_FP8> {
  static constexpr int EPL = 32, ESZ = 1, K = 64;
};
// split FP32: the hidden layers' operands are BF16 pairs (hi, lo)
template <>
struct Prec<NVGS_PREC_FP32_SPLIT> {
  static constexpr int EPL = 8, ESZ = 2, K = 16;
};

// scale slots of the vec section (FP8 only)
enum { kInvU = 0, kInv2 = 1, kInv3 = 2, kSaH1 = 3, kSaH2 = 4, kSaG = 5, kSw1 = 6, kSw2 = 7, kSw3 = 8, kNumScales = 9 };

__host__ __device__ constexpr int img_ks1(int K) { return (36 + K - 1) / K; }
__host__ __device__ constexpr int img_w1_bytes(int W, int K, int EPL, int ESZ) {
  return (W / 32) * img_ks1(K) * 64 * EPL * ESZ;
}
__host__ __device__ constexpr int img_wh_bytes(int W, int K, int EPL, int ESZ) { return (W / 32) * (W / K) * 64 * EPL * ESZ; }
__host__ __device__ constexpr int img_vec_floats(int W) { return (3 * W + 1 + kNumScales + 3) / 4 * 4; }
__host__ __device__ constexpr int img_bytes(int W, int K, int EPL, int ESZ) {
  return img_w1_bytes(W, K, EPL, ESZ) + 2 * img_wh_bytes(W, K, EPL, ESZ) + 4 * img_vec_floats(W);
}
template <int P, int W>
struct Img {
  using T = Prec<P>;
  static constexpr int NT = W / 32, KS1 = img_ks1(T::K), KSH = W / T::K;
  static constexpr int W1 = 0;
  static constexpr int W2 = img_w1_bytes(W, T::K, T::EPL, T::ESZ);
  static constexpr int W3 = W2 + img_wh_bytes(W, T::K, T::EPL, T::ESZ);
  static constexpr int VEC = W3 + img_wh_bytes(W, T::K, T::EPL, T::ESZ);
  static constexpr int BYTES = img_bytes(W, T::K, T::EPL, T::ESZ);
};

// split FP32: layer 1's Gaussian half in the FP32 layout, then the hidden
// layers' hi and lo BF16 images (W2 hi, W2 lo, W3 hi, W3 lo), then the vectors
template <int W>
struct Img<NVGS_PREC_FP32_SPLIT, W> {
  static constexpr int NT = W / 32, KS1 = img_ks1(2), KSH = W / 16;
  static constexpr int W1 = 0;
  static constexpr int HB = img_wh_bytes(W, 16, 8, 2);
  static constexpr int W2 = img_w1_bytes(W, 2, 1, 4);
  static constexpr int W2L = W2 + HB;
  static constexpr int W3 = W2L + HB;
  static constexpr int W3L = W3 + HB;
  static constexpr int VEC = W3L + HB;
  static constexpr int BYTES = VEC + 4 * img_vec_floats(W);
};
static size_t img_size_split(int W) {
  return img_w1_bytes(W, 2, 1, 4) + 4 * img_wh_bytes(W, 16, 8, 2) + 4 * img_vec_floats(W);
}

static size_t img_size(int P, int W) {
  if (P == NVGS_PREC_FP32_SPLIT) return img_size_split(W);
  if (P == NVGS_PREC_FP32) return img_bytes(W, 2, 1, 4);
  if (P == NVGS_PREC_BF16) return img_bytes(W, 16, 8, 2);
  return img_bytes(W, 64, 32, 1);
}
size_t mlp_op_f32_floats(int width) { return img_size(NVGS_PREC_FP32, width) / 4; }
size_t mlp_op_bf16_elems(int width) { return img_size(NVGS_PREC_BF16, width) / 2; }
size_t mlp_op_fp8_bytes(int width) { return img_size(NVGS_PREC_FP8, width); }
size_t mlp_op_split_bytes(int width) { return img_size(NVGS_PREC_FP32_SPLIT, width); }

__host__ __device__ inline float pow2_floor(float x) {  // largest power of two <= x (x > 0)
  int e;
  frexpf(x, &e);
  return ldexpf(1.f, e - 1);
}

// FP8 scales: weights by max |W| of each MFMA layer, activations by interval
// bounds: |gamma| <= 1, |h1| <= max_r (sum_k |W1[r,k]| + |b1[r]|),
// |h2| <= max_r (sum_k |W2[r,k]| B1 + |b2[r]|).  One 256-thread group.
__global__ void k_mlp_scales(const float* __restrict__ P, int W, float* __restrict__ scales) {
  __shared__ float s_red[256];
  const float* W1 = P;
  const float* b1 = W1 + W * 72;
  const float* W2 = b1 + W;
  const float* b2 = W2 + W * W;
  const float* W3 = b2 + W;
  auto block_max = [&](float v) {
    s_red[threadIdx.x] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) s_red[threadIdx.x] = fmaxf(s_red[threadIdx.x], s_red[threadIdx.x + o]);
      __syncthreads();
    }
    float r = s_red[0];
    __syncthreads();
    return r;
  };
  float m1 = 0.f, m2 = 0.f, m3 = 0.f, r1 = 0.f;
  for (int i = threadIdx.x; i < W * 36; i += blockDim.x) m1 = fmaxf(m1, fabsf(W1[(i / 36) * 72 + i % 36]));
  for (int i = threadIdx.x; i < W * W; i += blockDim.x) {
    m2 = fmaxf(m2, fabsf(W2[i]));
    m3 = fmaxf(m3, fabsf(W3[i]));
  }
  for (int r = threadIdx.x; r < W; r += blockDim.x) {
    float s = fabsf(b1[r]);
    for (int k = 0; k < 72; ++k) s += fabsf(W1[r * 72 + k]);
    r1 = fmaxf(r1, s);
  }
  m1 = block_max(m1);
  m2 = block_max(m2);
  m3 = block_max(m3);
  const float B1 = block_max(r1);
  float r2 = 0.f;
  for (int r = threadIdx.x; r < W; r += blockDim.x) {
    float s = 0.f;
    for (int k = 0; k < W; ++k) s += fabsf(W2[r * W + k]);
    r2 = fmaxf(r2, s * B1 + fabsf(b2[r]));
  }
  const float B2 = block_max(r2);
  if (threadIdx.x == 0) {
    const float sw1 = pow2_floor(448.f / fmaxf(m1, 1e-30f)), sw2 = pow2_floor(448.f / fmaxf(m2, 1e-30f));
    const float sw3 = pow2_floor(448.f / fmaxf(m3, 1e-30f));
    const float sag = pow2_floor(448.f), sa1 = pow2_floor(448.f / fmaxf(B1, 1e-30f));
    const float sa2 = pow2_floor(448.f / fmaxf(B2, 1e-30f));
    scales[kInvU] = 1.f / (sw1 * sag);
    scales[kInv2] = 1.f / (sw2 * sa1);
    scales[kInv3] = 1.f / (sw3 * sa2);
    scales[kSaH1] = sa1;
    scales[kSaH2] = sa2;
    scales[kSaG] = sag;
    scales[kSw1] = sw1;
    scales[kSw2] = sw2;
    scales[kSw3] = sw3;
  }
}

__device__ inline uint8_t to_fp8(float v) {
  return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(v, 0.f, 0, false) & 0xff);
}

template <int P>
__global__ void k_prepare(const float* __restrict__ Pm, int W, const float* __restrict__ scales,
                          uint8_t* __restrict__ img) {
  using T = Prec<P>;
  constexpr int EPL = T::EPL, ESZ = T::ESZ, K = T::K;
  const int NT = W / 32, KS1 = img_ks1(K), KSH = W / K;
  const int in1 = 72;
  const float* W1 = Pm;
  const float* b1 = W1 + W * in1;
  const float* W2 = b1 + W;
  const float* b2 = W2 + W * W;
  const float* W3 = b2 + W;
  const float* b3 = W3 + W * W;
  const float* wo = b3 + W;
  const int n1 = NT * KS1 * 64 * EPL, nh = NT * KSH * 64 * EPL;
  const int nvec = img_vec_floats(W);
  const int total = n1 + 2 * nh + nvec;
  const float sw1 = P == NVGS_PREC_FP8 ? scales[kSw1] : 1.f;
  const float sw2 = P == NVGS_PREC_FP8 ? scales[kSw2] : 1.f;
  const float sw3 = P == NVGS_PREC_FP8 ? scales[kSw3] : 1.f;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x) {
    if (idx < n1 + 2 * nh) {
      float v;
      int o = idx, base = 0;
      if (o < n1) {
        const int j = o % EPL, lane = (o / EPL) % 64, s = (o / (EPL * 64)) % KS1, t = o / (EPL * 64 * KS1);
        const int k = s * 2 * EPL + (lane / 32) * EPL + j;  // Gaussian feature (natural order)
        v = k < 36 ? W1[(32 * t + lane % 32) * in1 + k] * sw1 : 0.f;
      } else {
        o -= n1;
        const bool third = o >= nh;
        o %= nh;
        base = n1 + (third ? nh : 0);
        const int j = o % EPL, lane = (o / EPL) % 64, s = (o / (EPL * 64)) % KSH, t = o / (EPL * 64 * KSH);
        v = (third ? W3 : W2)[(32 * t + lane % 32) * W + hid_feature(s * EPL + j, lane / 32)] * (third ? sw3 : sw2);
      }
      (void)base;
      if (P == NVGS_PREC_FP32) reinterpret_cast<float*>(img)[idx] = v;
      if (P == NVGS_PREC_BF16) reinterpret_cast<__bf16*>(img)[idx] = (__bf16)v;
      if (P == NVGS_PREC_FP8) img[idx] = to_fp8(v);
    } else {
      const int e = idx - (n1 + 2 * nh);
      float v = 0.f;
      const int KQ = W / 2;
      if (e < 6 * KQ) {
        const int which = e / (2 * KQ), r = e % (2 * KQ), g = r / KQ, q = r % KQ;
        const float* vec = which == 0 ? b2 : which == 1 ? b3 : wo;
        v = vec[hid_feature(q, g)];
        // FP8: layer 2's accumulators hold sa2 (W2 h1 + b2) and start from sa2 b2
        // (a power of two: exact); layer 3's hold W3 h2 + b3
        if (P == NVGS_PREC_FP8 && which == 0) v *= scales[kSaH2];
      } else if (e == 6 * KQ) {
        v = wo[W];
      } else if (e - 6 * KQ - 1 < kNumScales) {
        v = P == NVGS_PREC_FP8 ? scales[e - 6 * KQ - 1] : 1.f;
      }
      reinterpret_cast<float*>(img + (size_t)(n1 + 2 * nh) * ESZ)[e] = v;
    }
  }
}

// operand image of the split-FP32 form (layout of Img<NVGS_PREC_FP32_SPLIT, W>)
__global__ void k_prepare_split(const float* __restrict__ Pm, int W, uint8_t* __restrict__ img) {
  const int NT = W / 32, KS1 = img_ks1(2), KSH = W / 16;
  const float* W1 = Pm;
  const float* b1 = W1 + W * 72;
  const float* W2 = b1 + W;
  const float* b2 = W2 + W * W;
  const float* W3 = b2 + W;
  const float* b3 = W3 + W * W;
  const float* wo = b3 + W;
  const int n1 = NT * KS1 * 64, nh = NT * KSH * 64 * 8, nvec = img_vec_floats(W);
  const int total = n1 + 4 * nh + nvec;
  float* f1 = reinterpret_cast<float*>(img);
  __bf16* hb = reinterpret_cast<__bf16*>(img + 4 * (size_t)n1);
  float* vecp = reinterpret_cast<float*>(img + 4 * (size_t)n1 + 2 * (size_t)(4 * nh));
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x) {
    if (idx < n1) {
      const int lane = idx % 64, s = (idx / 64) % KS1, t = idx / (64 * KS1);
      const int k = s * 2 + lane / 32;  // Gaussian feature (natural order)
      f1[idx] = k < 36 ? W1[(32 * t + lane % 32) * 72 + k] : 0.f;
    } else if (idx < n1 + 4 * nh) {
      const int o = idx - n1, which = o / nh, r = o % nh;  // W2 hi, W2 lo, W3 hi, W3 lo
      const int j = r % 8, lane = (r / 8) % 64, s = (r / 512) % KSH, t = r / (512 * KSH);
      const float v = (which < 2 ? W2 : W3)[(32 * t + lane % 32) * W + hid_feature(s * 8 + j, lane / 32)];
      const __bf16 hi = (__bf16)v;
      hb[o] = (which & 1) ? (__bf16)(v - (float)hi) : hi;
    } else {
      const int e = idx - n1 - 4 * nh, KQ = W / 2;
      float v = 0.f;
      if (e < 6 * KQ) {
        const int which = e / (2 * KQ), r = e % (2 * KQ), g = r / KQ, q = r % KQ;
        v = (which == 0 ? b2 : which == 1 ? b3 : wo)[hid_feature(q, g)];
      } else if (e == 6 * KQ) {
        v = wo[W];
      } else if (e - 6 * KQ - 1 < kNumScales) {
        v = 1.f;
      }
      vecp[e] = v;
    }
  }
}

hipError_t launch_prepare_split(const float* params, int width, uint8_t* op_split, hipStream_t st) {
  const size_t n = img_size_split(width) / 2;  // more than enough threads (one per element at most)
  hipLaunchKernelGGL(k_prepare_split, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, params, width, op_split);
  return hipGetLastError();
}

hipError_t launch_prepare_mlp(const float* params, int width, float* op_f32, uint16_t* op_bf16, uint8_t* op_fp8,
                              float* fp8_scale, hipStream_t st) {
  const int W = width;
  auto grid = [](size_t n) { return dim3((unsigned)((n + 255) / 256)); };
  if (op_f32)
    hipLaunchKernelGGL(k_prepare<NVGS_PREC_FP32>, grid(img_size(NVGS_PREC_FP32, W) / 4), dim3(256), 0, st, params, W,
                       (const float*)nullptr, reinterpret_cast<uint8_t*>(op_f32));
  if (op_bf16)
    hipLaunchKernelGGL(k_prepare<NVGS_PREC_BF16>, grid(img_size(NVGS_PREC_BF16, W) / 2), dim3(256), 0, st, params, W,
                       (const float*)nullptr, reinterpret_cast<uint8_t*>(op_bf16));
  if (op_fp8 && fp8_scale) {
    hipLaunchKernelGGL(k_mlp_scales, dim3(1), dim3(256), 0, st, params, W, fp8_scale);
    hipLaunchKernelGGL(k_prepare<NVGS_PREC_FP8>, grid(img_size(NVGS_PREC_FP8, W)), dim3(256), 0, st, params, W,
                       (const float*)fp8_scale, op_fp8);
  }
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
  // Eq. 2 with focal lengths in pixels: f_r = (H / 2) / tan(fovy / 2)
  double f_r = 0.5 * (double)cam.height / tan(0.5 * (double)cam.fovy);
  double fac = (double)A.train_focal / f_r;
  double cm[3] = {cl[0] * fac, cl[1] * fac, cl[2] * fac};
  double len = sqrt(cm[0] * cm[0] + cm[1] * cm[1] + cm[2] * cm[2]);
  if (A.d_max > 0.f && len > (double)A.d_max) {
    double sc = (double)A.d_max / len;
    for (int r = 0; r < 3; ++r) cm[r] *= sc;
    len = (double)A.d_max;
  }
  if (threadIdx.x == 0) s_query = (use_mlp && len >= (double)A.d_min) ? 1 : 0;
  if (A.kind == 1) {
    // compact form: per-segment vector = b1 + W1[:, forward] (R_i^T forward), in the
    // lane order kappa(j, g) = 16 (j / 8) + 8 g + j % 8 of the compact kernel
    double fw[3];
    for (int r = 0; r < 3; ++r)
      fw[r] = (double)in.R[r] * cam.R[6] + (double)in.R[3 + r] * cam.R[7] + (double)in.R[6 + r] * cam.R[8];
    const float* W1 = A.params;
    const float* b1 = W1 + 32 * 16;
    for (int e = threadIdx.x; e < 32; e += blockDim.x) {
      const int gq = e / 16, j = e % 16, kk = 16 * (j / 8) + 8 * gq + (j % 8);
      double s = b1[kk];
      for (int q = 0; q < 3; ++q) s += (double)W1[kk * 16 + 7 + q] * fw[q];
      c1perm[(size_t)seg * c1_stride + e] = (float)s;
    }
  } else if (threadIdx.x < 36) {
    int j = threadIdx.x / 12, band = (threadIdx.x % 12) / 2, cs = threadIdx.x % 2;
    double a = ldexp(M_PI * ((double)A.cam_scale * cm[j]), band);
    s_gam[threadIdx.x] = cs ? cos(a) : sin(a);
  }
  __syncthreads();
  const int W = A.kind == 1 ? 0 : A.width;
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
        const double m = s * (double)in.s;
        R.M[4 * r + c] = (float)m;
        R.Mlo[4 * r + c] = (float)(m - (double)R.M[4 * r + c]);
      }
      const double m = Rc[3 * r] * -d[0] + Rc[3 * r + 1] * -d[1] + Rc[3 * r + 2] * -d[2];
      R.M[4 * r + 3] = (float)m;
      R.Mlo[4 * r + 3] = (float)(m - (double)R.M[4 * r + 3]);
    }
    for (int r = 0; r < 3; ++r) R.cl[r] = (float)cl[r];
    double tany = tan(0.5 * (double)cam.fovy);
    double focal = 0.5 * (double)cam.height / tany;
    double tanx = 0.5 * (double)cam.width / focal;
    R.near_plane = cam.near_plane;
    R.tanx_g = (float)(1.3 * tanx);
    R.tany_g = (float)(1.3 * tany);
    R.focal = (float)focal;
    R.focal_lo = (float)(focal - (double)R.focal);
    R.half_w = 0.5f * (float)cam.width;
    R.half_h = 0.5f * (float)cam.height;
    R.asset = in.asset;
    R.inst = i;
    R.cam = k;
    R.n = (int32_t)A.n;
    R.query = s_query;
    // compact form: distance input = 2 (|mu - cl| f_t / f_r - d_min) / (d_max - d_min) - 1
    const double span = (double)A.d_max - (double)A.d_min;
    R.dn_a = A.kind == 1 ? (float)(2.0 * fac / span) : 0.f;
    R.dn_b = A.kind == 1 ? (float)(-2.0 * (double)A.d_min / span - 1.0) : 0.f;
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
// cull + MLP kernel
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool frustum(const SegRec& R, const float mu[3]) {
  const float px = fmaf(R.M[0], mu[0], fmaf(R.M[1], mu[1], fmaf(R.M[2], mu[2], R.M[3])));
  const float py = fmaf(R.M[4], mu[0], fmaf(R.M[5], mu[1], fmaf(R.M[6], mu[2], R.M[7])));
  const float pz = fmaf(R.M[8], mu[0], fmaf(R.M[9], mu[1], fmaf(R.M[10], mu[2], R.M[11])));
  return pz > R.near_plane && fabsf(px) <= R.tanx_g * pz && fabsf(py) <= R.tany_g * pz;
}

// MFMA operand of one lane for precision P: load from the LDS image, pack
// from FP32 values, multiply-accumulate a 32x32 tile.
template <int P>
struct Mfma;
template <>
struct Mfma<NVGS_PREC_FP32> {
  using Op = float;
  static __device__ __forceinline__ Op load(const uint8_t* p, int idx) {
    return reinterpret_cast<const float*>(p)[idx];
  }
  static __device__ __forceinline__ Op pack(const float* v) { return v[0]; }
  static __device__ __forceinline__ f32x16 mma(Op a, Op b, f32x16 c, int = 127, int = 127) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<NVGS_PREC_BF16> {
  using Op = bf16x8;
  static __device__ __forceinline__ Op load(const uint8_t* p, int idx) {
    return reinterpret_cast<const bf16x8*>(p)[idx];
  }
  static __device__ __forceinline__ Op pack(const float* v) {
    Op r;
#pragma unroll
    for (int j = 0; j < 8; ++j) r[j] = (__bf16)v[j];
    return r;
  }
  static __device__ __forceinline__ f32x16 mma(Op a, Op b, f32x16 c, int = 127, int = 127) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<NVGS_PREC_FP8> {
  using Op = i32x8;
  static __device__ __forceinline__ Op load(const uint8_t* p, int idx) {
    return reinterpret_cast<const i32x8*>(p)[idx];
  }
  static __device__ __forceinline__ Op pack(const float* v) {
    Op r;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      int w = __builtin_amdgcn_cvt_pk_fp8_f32(v[4 * q], v[4 * q + 1], 0, false);
      r[q] = __builtin_amdgcn_cvt_pk_fp8_f32(v[4 * q + 2], v[4 * q + 3], w, true);
    }
    return r;
  }
  // E4M3 x E4M3; ea, eb: E8M0 block scales (2^(e - 127)) of the weights and
  // the activations, the same in every lane: the per-layer dequantisation
  // and the next layer's quantisation scale (powers of two) are applied to
  // every product by the matrix core, not by the epilogue
  static __device__ __forceinline__ f32x16 mma(Op a, Op b, f32x16 c, int ea = 127, int eb = 127) {
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, ea, 0, eb);
  }
};

// E8M0 code of a normal power-of-two float: its biased exponent
__device__ __forceinline__ int e8m0(float s) { return (int)((__float_as_uint(s) >> 23) & 0xffu); }

typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

// Next-layer operands from KQ values per lane in accumulator order, value
// q = relu(scale * (acc[q] + add[q])) (add may be null), rounded to the
// operand precision: FP32 as is, BF16 round-to-nearest-even with ReLU taken
// on the packed 16-bit patterns (a sign-bit test, exact since rounding keeps
// the sign), FP8 E4M3 after the ReLU.
template <int P, int W, int NB, bool ADD>
__device__ __forceinline__ void relu_pack(const f32x16 (&acc)[NB][W / 32], float scale, const float* __restrict__ add,
                                          float add_scale, typename Mfma<P>::Op (&out)[NB][W / Prec<P>::K]) {
  using M = Mfma<P>;
  constexpr int EPL = Prec<P>::EPL, KSH = W / Prec<P>::K;
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int s = 0; s < KSH; ++s) {
      float v[EPL];
#pragma unroll
      for (int j = 0; j < EPL; ++j) {
        const int q = s * EPL + j;
        const float x = ADD ? fmaf(acc[b][q / 16][q % 16], add_scale, add[q]) : acc[b][q / 16][q % 16];
        v[j] = P == NVGS_PREC_BF16 ? x * scale : relu(x * scale);
      }
      if constexpr (P == NVGS_PREC_BF16) {
        // pairs rounded together (one v_cvt_pk_bf16_f32), ReLU as a packed
        // signed 16-bit max with 0 (one v_pk_max_i16)
        i32x4 w;
#pragma unroll
        for (int p2 = 0; p2 < 4; ++p2) {
          const bf16x2 h = __builtin_convertvector((f32x2){v[2 * p2], v[2 * p2 + 1]}, bf16x2);
          const s16x2 m = __builtin_elementwise_max(__builtin_bit_cast(s16x2, h), (s16x2){0, 0});
          w[p2] = __builtin_bit_cast(int, m);
        }
        out[b][s] = __builtin_bit_cast(typename M::Op, w);
      } else {
        out[b][s] = M::pack(v);
      }
    }
}

// Split-FP32 operands of the next layer: v = relu(acc[q] (+ add[q])) in FP32,
// hi = bf16(v) and lo = bf16(v - hi) (v - hi is exact in FP32), packed as
// BF16 operands in accumulator order.
template <int W, int NB, bool ADD>
__device__ __forceinline__ void relu_split(const f32x16 (&acc)[NB][W / 32], const float* __restrict__ add,
                                           bf16x8 (&hi)[NB][W / 16], bf16x8 (&lo)[NB][W / 16]) {
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int s = 0; s < W / 16; ++s) {
      i32x4 wh, wl;
#pragma unroll
      for (int p2 = 0; p2 < 4; ++p2) {
        const int q = s * 8 + 2 * p2;
        const float x0 = ADD ? acc[b][q / 16][q % 16] + add[q] : acc[b][q / 16][q % 16];
        const float x1 = ADD ? acc[b][(q + 1) / 16][(q + 1) % 16] + add[q + 1] : acc[b][(q + 1) / 16][(q + 1) % 16];
        const float v0 = relu(x0), v1 = relu(x1);
        const bf16x2 h = __builtin_convertvector((f32x2){v0, v1}, bf16x2);
        const uint32_t hbits = __builtin_bit_cast(uint32_t, h);
        const float h0 = __uint_as_float(hbits << 16), h1 = __uint_as_float(hbits & 0xffff0000u);
        const bf16x2 l = __builtin_convertvector((f32x2){v0 - h0, v1 - h1}, bf16x2);
        wh[p2] = (int)hbits;
        wl[p2] = __builtin_bit_cast(int, l);
      }
      hi[b][s] = __builtin_bit_cast(bf16x8, wh);
      lo[b][s] = __builtin_bit_cast(bf16x8, wl);
    }
}

// Split-FP32 operands from one 32-unit accumulator tile tt (the K-steps 2 tt
// and 2 tt + 1 of the next layer), as relu_split.
template <int W, int NB, bool ADD>
__device__ __forceinline__ void relu_split_tile(const f32x16 (&acc)[NB][W / 32], int tt, const float* __restrict__ add,
                                                bf16x8 (&hi)[NB][W / 16], bf16x8 (&lo)[NB][W / 16]) {
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int s = 2 * tt; s < 2 * tt + 2; ++s) {
      i32x4 wh, wl;
#pragma unroll
      for (int p2 = 0; p2 < 4; ++p2) {
        const int q = s * 8 + 2 * p2;
        const float x0 = ADD ? acc[b][tt][q % 16] + add[q] : acc[b][tt][q % 16];
        const float x1 = ADD ? acc[b][tt][(q + 1) % 16] + add[q + 1] : acc[b][tt][(q + 1) % 16];
        const float v0 = relu(x0), v1 = relu(x1);
        const bf16x2 h = __builtin_convertvector((f32x2){v0, v1}, bf16x2);
        const uint32_t hbits = __builtin_bit_cast(uint32_t, h);
        const float h0 = __uint_as_float(hbits << 16), h1 = __uint_as_float(hbits & 0xffff0000u);
        const bf16x2 l = __builtin_convertvector((f32x2){v0 - h0, v1 - h1}, bf16x2);
        wh[p2] = (int)hbits;
        wl[p2] = __builtin_bit_cast(int, l);
      }
      hi[b][s] = __builtin_bit_cast(bf16x8, wh);
      lo[b][s] = __builtin_bit_cast(bf16x8, wl);
    }
}

// One split-FP32 layer, pipelined with the previous layer's epilogue: for each
// 32-unit tile tt of the previous activations (prev, + add for layer 1), its
// ReLU and split, then the K-steps 2 tt, 2 tt + 1 of every output tile, so
// that a tile's epilogue can issue while the previous tile's MFMAs run.  Each
// accumulator sees the same sequence of products as in mma_layer_split.
template <int W, int NB, bool ADD>
__device__ __forceinline__ void split_layer_pipelined(const f32x16 (&prev)[NB][W / 32], const float* __restrict__ add,
                                                      const uint8_t* __restrict__ Wh, const uint8_t* __restrict__ Wl,
                                                      const float* __restrict__ binit, f32x16 (&acc)[NB][W / 32],
                                                      int lane) {
  constexpr int NT = W / 32, KSH = W / 16;
  bf16x8 xh[NB][KSH], xl[NB][KSH];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[b][t][r] = binit[16 * t + r];
#pragma unroll
  for (int tt = 0; tt < NT; ++tt) {
    relu_split_tile<W, NB, ADD>(prev, tt, add, xh, xl);
#pragma unroll
    for (int s = 2 * tt; s < 2 * tt + 2; ++s) {
      bf16x8 ah[NT], al[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        ah[t] = reinterpret_cast<const bf16x8*>(Wh)[(t * KSH + s) * 64 + lane];
        al[t] = reinterpret_cast<const bf16x8*>(Wl)[(t * KSH + s) * 64 + lane];
      }
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int t = 0; t < NT; ++t)
          acc[b][t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[t], xh[b][s], acc[b][t], 0, 0, 0);
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int t = 0; t < NT; ++t)
          acc[b][t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[t], xl[b][s], acc[b][t], 0, 0, 0);
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int t = 0; t < NT; ++t)
          acc[b][t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[t], xh[b][s], acc[b][t], 0, 0, 0);
    }
  }
}

// One hidden layer of the split-FP32 form: acc = bias + sum over the depth of
// W_lo x_hi + W_hi x_lo + W_hi x_hi (three BF16 MFMAs per 32x32x16 block,
// FP32 accumulation; the independent tiles of a round are issued between the
// dependent accumulations)
template <int W, int NB>
__device__ __forceinline__ void mma_layer_split(const uint8_t* __restrict__ Wh, const uint8_t* __restrict__ Wl,
                                                const float* __restrict__ binit, const bf16x8 (&xh)[NB][W / 16],
                                                const bf16x8 (&xl)[NB][W / 16], f32x16 (&acc)[NB][W / 32], int lane) {
  constexpr int NT = W / 32, KSH = W / 16;
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[b][t][r] = binit[16 * t + r];
#pragma unroll
  for (int s = 0; s < KSH; ++s) {
    bf16x8 ah[NT], al[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      ah[t] = reinterpret_cast<const bf16x8*>(Wh)[(t * KSH + s) * 64 + lane];
      al[t] = reinterpret_cast<const bf16x8*>(Wl)[(t * KSH + s) * 64 + lane];
    }
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[b][t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[t], xh[b][s], acc[b][t], 0, 0, 0);
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[b][t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[t], xl[b][s], acc[b][t], 0, 0, 0);
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[b][t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[t], xh[b][s], acc[b][t], 0, 0, 0);
  }
}

// One hidden layer on 32x32 MFMA tiles with the pairs as columns: the
// accumulators start from the layer's bias (in accumulator order; for FP8
// stored divided by the layer's dequantisation scale), so the epilogue is a
// scale and the ReLU only.
template <int P, int W, int NB>
__device__ __forceinline__ void mma_layer(const uint8_t* __restrict__ Wp, const float* __restrict__ binit,
                                          const typename Mfma<P>::Op (&in)[NB][W / Prec<P>::K],
                                          f32x16 (&acc)[NB][W / 32], int lane, int ea = 127, int eb = 127) {
  using M = Mfma<P>;
  constexpr int NT = W / 32, KSH = W / Prec<P>::K;
  f32x16 c0[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) c0[t][r] = binit[16 * t + r];
#pragma unroll
  for (int s = 0; s < KSH; ++s) {
    typename M::Op a[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) a[t] = M::load(Wp, (t * KSH + s) * 64 + lane);
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[b][t] = M::mma(a[t], in[b][s], s == 0 ? c0[t] : acc[b][t], ea, eb);
  }
}

template <int P, int W, int NB, int WAVES, int MODE>
__global__ __launch_bounds__(64 * WAVES) void k_cull_mlp(
    const AssetDev* __restrict__ assets, const WorkItem* __restrict__ items, const int32_t* __restrict__ seglist,
    const SegRec* __restrict__ segs, const float* __restrict__ c1perm, int c1_stride, uint32_t* __restrict__ mask,
    uint32_t* __restrict__ chunk_count, uint8_t* __restrict__ state, float* __restrict__ logits,
    unsigned long long* __restrict__ frame_counts) {
  static_assert(WAVES * NB * 32 == kChunk, "a work-group covers one compaction chunk");
  // split FP32: layer 1's Gaussian half on FP32 MFMA, hidden layers on BF16 (hi, lo) pairs
  constexpr bool SPLIT = P == NVGS_PREC_FP32_SPLIT;
  constexpr int P1 = SPLIT ? NVGS_PREC_FP32 : P;
  using M = Mfma<P1>;
  using I = Img<P, W>;
  constexpr int EPL = Prec<P1>::EPL, NT = W / 32, KQ = W / 2, KS1 = I::KS1;
  __shared__ __attribute__((aligned(16))) uint8_t lds[I::BYTES];
  // per wave: the current segment's layer-1 camera half, published from
  // registers that were loaded one segment earlier (so the MFMA chain never
  // waits on its global load)
  __shared__ __attribute__((aligned(16))) float s_c1[WAVES][W];
  __shared__ uint32_t s_tot[2];
  const WorkItem it = items[blockIdx.x];
  const AssetDev* A = assets + it.asset;
  {
    const uint8_t* img = P == NVGS_PREC_FP32 ? reinterpret_cast<const uint8_t*>(A->op_f32)
                         : P == NVGS_PREC_BF16 ? reinterpret_cast<const uint8_t*>(A->op_bf16)
                         : P == NVGS_PREC_FP8  ? A->op_fp8
                                               : A->op_split;
    const uint4* src = reinterpret_cast<const uint4*>(img);
    for (int k = threadIdx.x; k < I::BYTES / 16; k += 64 * WAVES) reinterpret_cast<uint4*>(lds)[k] = src[k];
  }
  if (threadIdx.x < 2) s_tot[threadIdx.x] = 0;
  const uint8_t* W1u = lds + I::W1;
  const uint8_t* W2p = lds + I::W2;
  const uint8_t* W3p = lds + I::W3;
  const float* vec = reinterpret_cast<const float*>(lds + I::VEC);
  const float* b2p = vec;
  const float* b3p = vec + 2 * KQ;
  const float* wop = vec + 4 * KQ;
  const float* scl = vec + 6 * KQ + 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ncol = lane & 31, grp = lane >> 5;
  const int64_t n = A->n;
  const float msc = A->mean_scale;
  const int64_t g0 = (int64_t)it.chunk * kChunk + wave * (32 * NB);
  float mu[NB][3];
  bool valid[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int64_t g = g0 + 32 * b + ncol;
    valid[b] = g < n;
    for (int j = 0; j < 3; ++j) mu[b][j] = valid[b] ? A->mean[j * n + g] : 0.f;
  }
  __syncthreads();
  const float bo = wop[2 * KQ];
  const float invU = P == NVGS_PREC_FP8 ? scl[kInvU] : 1.f;
  const float inv2 = P == NVGS_PREC_FP8 ? scl[kInv2] : 1.f;
  const float inv3 = P == NVGS_PREC_FP8 ? scl[kInv3] : 1.f;
  const float saG = P == NVGS_PREC_FP8 ? scl[kSaG] : 1.f;
  const float saH1 = P == NVGS_PREC_FP8 ? scl[kSaH1] : 1.f;
  const float saH2 = P == NVGS_PREC_FP8 ? scl[kSaH2] : 1.f;
  // FP8: E8M0 scales of the three MFMA stages (weights, activations): U comes
  // out as sa1 (W1u gamma), layer 2 as sa2 (W2 h1 + b2), layer 3 as W3 h2 + b3
  // (the accumulators start from the biases in those units), so the epilogues
  // are an add (layer 1, with the camera half staged as sa1 c1), the ReLU and
  // the conversion
  const int eU_a = e8m0(invU), eU_b = e8m0(saH1), e2_a = e8m0(inv2), e2_b = e8m0(saH2), e3_a = e8m0(inv3);
  // layer 1, Gaussian half: U = W1u gamma(mean_scale * mu), features in the
  // natural order k = s*2*EPL + grp*EPL + j (zero beyond 36)
  f32x16 U[NB][NT];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int t = 0; t < NT; ++t) U[b][t] = (f32x16){0};
#pragma unroll
  for (int s = 0; s < KS1; ++s) {
    typename M::Op a[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) a[t] = M::load(W1u, (t * KS1 + s) * 64 + lane);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      float e[EPL];
#pragma unroll
      for (int j = 0; j < EPL; ++j) {
        const int k = s * 2 * EPL + grp * EPL + j;  // grp is 0/1: the compiler keeps both paths cheap
        const int coord = k / 12, band = (k % 12) / 2;
        const float x = ldexpf(msc * mu[b][min(coord, 2)], band);
        const float v = (k % 2) ? cospif(x) : sinpif(x);
        e[j] = k < 36 ? v * saG : 0.f;
      }
      const typename M::Op eb = M::pack(e);
#pragma unroll
      for (int t = 0; t < NT; ++t) U[b][t] = M::mma(a[t], eb, U[b][t], eU_a, eU_b);
    }
  }
  uint32_t n_in = 0, n_q = 0;  // in-frustum and queried pairs of this wave
  constexpr int CPL = W / 64;  // camera-half values per lane
  float pref[CPL];
  auto fetch_c1 = [&](int s_idx) {
    if (s_idx < it.seg_end) {
      const float* row = c1perm + (size_t)seglist[s_idx] * c1_stride;
#pragma unroll
      for (int q = 0; q < CPL; ++q) pref[q] = row[q * 64 + lane];
    }
  };
  fetch_c1(it.seg_begin);
  // waves proceed through the segments independently: each adds its kept
  // count to the (zero-filled) chunk count
  for (int si = it.seg_begin; si < it.seg_end; ++si) {
    const int seg = seglist[si];
    const SegRec& R = segs[seg];
#pragma unroll
    for (int q = 0; q < CPL; ++q) s_c1[wave][q * 64 + lane] = P == NVGS_PREC_FP8 ? pref[q] * saH1 : pref[q];
    fetch_c1(si + 1);
    bool in[NB];
    bool any = false;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      in[b] = valid[b] && frustum(R, mu[b]);
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
      const float* c1 = &s_c1[wave][grp * KQ];
      f32x16 acc[NB][NT];
      if constexpr (SPLIT) {
        f32x16 acc2[NB][NT];
        split_layer_pipelined<W, NB, true>(U, c1, W2p, lds + I::W2L, b2p + grp * KQ, acc2, lane);
        split_layer_pipelined<W, NB, false>(acc2, nullptr, W3p, lds + I::W3L, b3p + grp * KQ, acc, lane);
      } else {
        constexpr int KSH = W / Prec<P>::K;
        typename Mfma<P>::Op op[NB][KSH];
        // layer 1: h1 = relu(U + c1) as layer 2's operands (FP8: both already in units of sa1)
        relu_pack<P, W, NB, true>(U, 1.f, c1, 1.f, op);
        mma_layer<P, W, NB>(W2p, b2p + grp * KQ, op, acc, lane, e2_a, e2_b);
        relu_pack<P, W, NB, false>(acc, 1.f, nullptr, 1.f, op);
        mma_layer<P, W, NB>(W3p, b3p + grp * KQ, op, acc, lane, e3_a, 127);
      }
      // output layer in FP32 on h3 = relu(acc)
      const float* wg = wop + grp * KQ;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        float part = 0.f;
#pragma unroll
        for (int q = 0; q < KQ; ++q) part = fmaf(wg[q], relu(acc[b][q / 16][q % 16]), part);
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
      const uint32_t word = (uint32_t)__ballot(keep[b]);
      cnt += __popc(word);
      if (lane == 0 && g0 + 32 * b < n) mask[R.word_base + (g0 >> 5) + b] = word;
    }
    if (lane == 0 && cnt) atomicAdd(chunk_count + R.chunk_base + it.chunk, cnt);
    if (MODE == 1 && grp == 0) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        if (valid[b]) {
          const int64_t idx = R.pair_base + g0 + 32 * b + ncol;
          state[idx] = keep[b] ? 2 : (in[b] ? 1 : 0);
          logits[idx] = (in[b] && query) ? z[b] : __builtin_nanf("");
        }
      }
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

// Frustum culling alone (frames without the MLP): the same work items, keep
// bits = in-frustum bits, no weights staged and no MLP evaluated.
__global__ __launch_bounds__(kChunk) void k_cull_only(const AssetDev* __restrict__ assets,
                                                      const WorkItem* __restrict__ items,
                                                      const int32_t* __restrict__ seglist,
                                                      const SegRec* __restrict__ segs, uint32_t* __restrict__ mask,
                                                      uint32_t* __restrict__ chunk_count,
                                                      unsigned long long* __restrict__ frame_counts) {
  __shared__ uint32_t s_cnt[2];
  __shared__ uint32_t s_tot;
  const WorkItem it = items[blockIdx.x];
  const AssetDev* A = assets + it.asset;
  const int lane = threadIdx.x & 63;
  const int64_t n = A->n;
  const int64_t g = (int64_t)it.chunk * kChunk + threadIdx.x;
  const bool valid = g < n;
  float mu[3];
  for (int j = 0; j < 3; ++j) mu[j] = valid ? A->mean[j * n + g] : 0.f;
  if (threadIdx.x < 2) s_cnt[threadIdx.x] = 0;
  if (threadIdx.x == 0) s_tot = 0;
  __syncthreads();
  int parity = 0;
  uint32_t n_in = 0;
  for (int si = it.seg_begin; si < it.seg_end; ++si, parity ^= 1) {
    const int seg = seglist[si];
    const SegRec& R = segs[seg];
    const bool in = valid && frustum(R, mu);
    const uint64_t b = __ballot(in);
    const uint32_t lo = (uint32_t)b, hi = (uint32_t)(b >> 32);
    const int64_t g0 = (int64_t)it.chunk * kChunk + (threadIdx.x & ~63);
    if (lane == 0) {
      if (g0 < n) mask[R.word_base + (g0 >> 5)] = lo;
      if (g0 + 32 < n) mask[R.word_base + (g0 >> 5) + 1] = hi;
      atomicAdd(&s_cnt[parity], (uint32_t)__popcll(b));
    }
    n_in += lane == 0 ? (uint32_t)__popcll(b) : 0u;
    __syncthreads();
    if (threadIdx.x == 0) {
      chunk_count[R.chunk_base + it.chunk] = s_cnt[parity];
      s_cnt[parity] = 0;
    }
  }
  if (frame_counts) {
    if (lane == 0) atomicAdd(&s_tot, n_in);
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(frame_counts + 0, (unsigned long long)s_tot);
  }
}

hipError_t launch_cull_only(const AssetDev* assets_dev, const WorkItem* items, int64_t n_items, const int32_t* seglist,
                            const SegRec* segs, uint32_t* mask, uint32_t* chunk_count, unsigned long long* counts,
                            hipStream_t st) {
  if (n_items == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cull_only, dim3((unsigned)n_items), dim3(kChunk), 0, st, assets_dev, items, seglist, segs, mask,
                     chunk_count, counts);
  return hipGetLastError();
}

template <int P, int W, int NB, int WAVES>
static hipError_t launch_t(const AssetDev* assets, const WorkItem* items, int64_t n_items, const int32_t* seglist,
                           const SegRec* segs, const float* c1perm, int c1_stride, int mode, uint32_t* mask,
                           uint32_t* chunk_count, uint8_t* state, float* logits, unsigned long long* counts,
                           hipStream_t st) {
  if (mode == 1)
    hipLaunchKernelGGL((k_cull_mlp<P, W, NB, WAVES, 1>), dim3((unsigned)n_items), dim3(64 * WAVES), 0, st, assets,
                       items, seglist, segs, c1perm, c1_stride, mask, chunk_count, state, logits, counts);
  else
    hipLaunchKernelGGL((k_cull_mlp<P, W, NB, WAVES, 0>), dim3((unsigned)n_items), dim3(64 * WAVES), 0, st, assets,
                       items, seglist, segs, c1perm, c1_stride, mask, chunk_count, state, logits, counts);
  return hipGetLastError();
}

bool mlp_shape_supported(int width, int precision, int nb) {
  if (width != 64 && width != 128) return false;
  return nb == 1 || nb == 2 || (nb == 4 && width == 64 && precision != NVGS_PREC_FP8);
}

hipError_t launch_cull_mlp(const AssetDev* assets_dev, const WorkItem* items, int64_t n_items, const int32_t* seglist,
                           const SegRec* segs, const float* c1perm, int max_width, int width, int precision, int nb,
                           int mode, uint32_t* mask, uint32_t* chunk_count, uint8_t* state, float* logits,
                           unsigned long long* counts, hipStream_t st) {
  if (n_items == 0) return hipSuccess;
#define NVGS_LAUNCH(P, W, NB)                                                                                  \
  return launch_t<P, W, NB, kChunk / (32 * NB)>(assets_dev, items, n_items, seglist, segs, c1perm, max_width, \
                                                mode, mask, chunk_count, state, logits, counts, st)
#define NVGS_SHAPES(P)                          \
  if (width == 64) {                            \
    if (nb == 1) NVGS_LAUNCH(P, 64, 1);         \
    if (nb == 2) NVGS_LAUNCH(P, 64, 2);         \
  } else if (width == 128) {                    \
    if (nb == 1) NVGS_LAUNCH(P, 128, 1);        \
    if (nb == 2) NVGS_LAUNCH(P, 128, 2);        \
  }
  // four blocks per wave spill with the FP8 operand packing: FP32 and BF16 only
  if (precision == NVGS_PREC_FP32) {
    NVGS_SHAPES(NVGS_PREC_FP32)
    if (width == 64 && nb == 4) NVGS_LAUNCH(NVGS_PREC_FP32, 64, 4);
  } else if (precision == NVGS_PREC_BF16) {
    NVGS_SHAPES(NVGS_PREC_BF16)
    if (width == 64 && nb == 4) NVGS_LAUNCH(NVGS_PREC_BF16, 64, 4);
  } else if (precision == NVGS_PREC_FP8) {
    NVGS_SHAPES(NVGS_PREC_FP8)
  } else if (precision == NVGS_PREC_FP32_SPLIT) {
    NVGS_SHAPES(NVGS_PREC_FP32_SPLIT)
    if (width == 64 && nb == 4) NVGS_LAUNCH(NVGS_PREC_FP32_SPLIT, 64, 4);
  }
#undef NVGS_SHAPES
#undef NVGS_LAUNCH
  return hipErrorInvalidValue;
}

}  // namespace nvgs
