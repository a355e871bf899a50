// The paper's compact visibility-MLP form (Sec. 3.2, 3.3, 4.1) on gfx950:
// a per-Gaussian 6-D embedding from a secondary MLP on (opacity, log scales,
// unit quaternion), computed once per asset at load time, and the visibility
// MLP 16 -> 32 -> 32 -> 1 on (normalised mean, unit view direction, min-max
// camera distance, camera forward, embedding).
//
// Design: the 16 inputs split into a per-Gaussian part (mean, embedding: 9
// inputs), a per-(camera, instance) part (forward vector, folded with the
// bias into one vector by the segment setup) and a per-pair part (direction
// and distance: 4 inputs).  A work-group covers 256 Gaussians of one asset
// (8 waves of 64 lanes, 32 Gaussians each); the two halves of a wave hold the two halves of the hidden
// layer of the same 32 Gaussians, so layer 1 is 4 FMAs per hidden unit per
// pair on top of the per-chunk part, and layer 2 runs on MFMA with the pairs
// as columns (FP32 32x32x2 or BF16 32x32x16), its operands built straight
// from the layer-1 registers.  Hidden unit j of lane group g is
// kappa(j, g) = 16 (j / 8) + 8 g + j % 8 in both precisions.
#include "internal.h"

namespace nvgs {

typedef float f32x16c __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8c __attribute__((ext_vector_type(8)));

__host__ __device__ constexpr int ckappa(int j, int g) { return 16 * (j / 8) + 8 * g + (j % 8); }
__host__ __device__ constexpr int crho(int r, int g) { return 8 * (r / 4) + 4 * g + (r % 4); }

// FP32 image (floats): W2 A operands [16 steps][64 lanes], then the vectors
constexpr int kImW2 = 0;
constexpr int kImW1P = 1024;        // [2][16][4]: W1[kappa][3..6] (direction, distance)
constexpr int kImW1G = 1024 + 128;  // [2][16][9]: W1[kappa][0..2, 10..15] (mean, embedding)
constexpr int kImB2 = kImW1G + 288; // [2][16] b2 in accumulator order
constexpr int kImWo = kImB2 + 32;   // [2][16] wo in accumulator order
constexpr int kImBo = kImWo + 32;
constexpr int kImFloats = (kImBo + 1 + 3) / 4 * 4;

size_t cmlp_image_floats() { return kImFloats; }

__global__ void k_prepare_c(const float* __restrict__ P, float* __restrict__ img, __bf16* __restrict__ img16) {
  const float* W1 = P;
  const float* b1 = W1 + 32 * 16;
  const float* W2 = b1 + 32;
  const float* b2 = W2 + 32 * 32;
  const float* wo = b2 + 32;
  (void)b1;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < kImFloats; e += gridDim.x * blockDim.x) {
    float v = 0.f;
    if (e < kImW1P) {
      const int s = e / 64, l = e % 64;
      v = W2[(l % 32) * 32 + ckappa(s, l / 32)];
    } else if (e < kImW1G) {
      const int q = e - kImW1P, g = q / 64, j = (q / 4) % 16, i = q % 4;
      v = W1[ckappa(j, g) * 16 + 3 + i];
    } else if (e < kImB2) {
      const int q = e - kImW1G, g = q / 144, j = (q / 9) % 16, i = q % 9;
      v = W1[ckappa(j, g) * 16 + (i < 3 ? i : 7 + i)];
    } else if (e < kImWo) {
      const int q = e - kImB2;
      v = b2[crho(q % 16, q / 16)];
    } else if (e < kImBo) {
      const int q = e - kImWo;
      v = wo[crho(q % 16, q / 16)];
    } else if (e == kImBo) {
      v = wo[32];
    }
    img[e] = v;
  }
  // BF16 W2 operands [2 steps][64 lanes][8]: A[row l % 32][k = 16 s + 8 g + i]
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < 2 * 64 * 8; e += gridDim.x * blockDim.x) {
    const int s = e / 512, l = (e / 8) % 64, i = e % 8;
    img16[e] = (__bf16)W2[(l % 32) * 32 + 16 * s + 8 * (l / 32) + i];
  }
}

hipError_t launch_prepare_cmlp(const float* params, float* img_f32, uint16_t* img_bf16, hipStream_t st) {
  hipLaunchKernelGGL(k_prepare_c, dim3(8), dim3(256), 0, st, params, img_f32, reinterpret_cast<__bf16*>(img_bf16));
  return hipGetLastError();
}

// per-Gaussian embedding: 8 -> 32 -> 32 -> 6 in FP32, weights staged in LDS
__global__ __launch_bounds__(256) void k_cembed(const float* __restrict__ P, const float* __restrict__ scale,
                                                const float* __restrict__ quat, const float* __restrict__ opacity,
                                                int64_t n, float* __restrict__ emb) {
  __shared__ float s_p[kCompactEmb];
  for (int e = threadIdx.x; e < kCompactEmb; e += blockDim.x) s_p[e] = P[kCompactVis + e];
  __syncthreads();
  const float* E1 = s_p;
  const float* e1 = E1 + 32 * 8;
  const float* E2 = e1 + 32;
  const float* e2 = E2 + 32 * 32;
  const float* E3 = e2 + 32;
  const float* e3 = E3 + 6 * 32;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x) {
    float x[8];
    x[0] = opacity[g];
    for (int k = 0; k < 3; ++k) x[1 + k] = logf(scale[k * n + g]);
    float q[4];
    for (int k = 0; k < 4; ++k) q[k] = quat[k * n + g];
    const float qn = (q[0] < 0.f ? -1.f : 1.f) / sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int k = 0; k < 4; ++k) x[4 + k] = q[k] * qn;
    float h1[32], h2[32];
    for (int r = 0; r < 32; ++r) {
      float s = e1[r];
      for (int k = 0; k < 8; ++k) s = fmaf(E1[r * 8 + k], x[k], s);
      h1[r] = fmaxf(s, 0.f);
    }
    for (int r = 0; r < 32; ++r) {
      float s = e2[r];
      for (int k = 0; k < 32; ++k) s = fmaf(E2[r * 32 + k], h1[k], s);
      h2[r] = fmaxf(s, 0.f);
    }
    float o[8];
    for (int r = 0; r < 6; ++r) {
      float s = e3[r];
      for (int k = 0; k < 32; ++k) s = fmaf(E3[r * 32 + k], h2[k], s);
      o[r] = s;
    }
    o[6] = o[7] = 0.f;
    float4* dst = reinterpret_cast<float4*>(emb + g * 8);
    dst[0] = make_float4(o[0], o[1], o[2], o[3]);
    dst[1] = make_float4(o[4], o[5], o[6], o[7]);
  }
}

hipError_t launch_cembed(const float* params, const float* scale, const float* quat, const float* opacity, int64_t n,
                         float* emb, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_cembed, dim3(grid), dim3(256), 0, st, params, scale, quat, opacity, n, emb);
  return hipGetLastError();
}

__device__ __forceinline__ bool cfrustum(const SegRec& R, const float mu[3]) {
  const float px = fmaf(R.M[0], mu[0], fmaf(R.M[1], mu[1], fmaf(R.M[2], mu[2], R.M[3])));
  const float py = fmaf(R.M[4], mu[0], fmaf(R.M[5], mu[1], fmaf(R.M[6], mu[2], R.M[7])));
  const float pz = fmaf(R.M[8], mu[0], fmaf(R.M[9], mu[1], fmaf(R.M[10], mu[2], R.M[11])));
  return pz > R.near_plane && fabsf(px) <= R.tanx_g * pz && fabsf(py) <= R.tany_g * pz;
}

constexpr int kCThreads = 2 * kChunk;  // 8 waves, 32 Gaussians each
static_assert(kChunk == 256, "one compact work-group covers a 256-Gaussian chunk in 8 waves");

// Cull + compact MLP.  P: FP32 or BF16 layer-2 operands; MODE 0: keep bits
// and chunk counts, 1: state and logits as well.
template <int P, int MODE>
__global__ __launch_bounds__(kCThreads) void k_cull_cmlp(
    const AssetDev* __restrict__ assets, const WorkItem* __restrict__ items, const int32_t* __restrict__ seglist,
    const SegRec* __restrict__ segs, const float* __restrict__ c1perm, int c1_stride, uint32_t* __restrict__ mask,
    uint32_t* __restrict__ chunk_count, uint8_t* __restrict__ state, float* __restrict__ logits,
    unsigned long long* __restrict__ frame_counts) {
  __shared__ __attribute__((aligned(16))) float s_img[kImFloats];
  __shared__ __attribute__((aligned(16))) __bf16 s_w16[P == NVGS_PREC_BF16 ? 2 * 64 * 8 : 8];
  __shared__ uint32_t s_tot[2];
  const WorkItem it = items[blockIdx.x];
  const AssetDev* A = assets + it.asset;
  for (int e = threadIdx.x; e < kImFloats; e += kCThreads) s_img[e] = A->op_f32[e];
  if (P == NVGS_PREC_BF16)
    for (int e = threadIdx.x; e < 2 * 64 * 8; e += kCThreads) s_w16[e] = reinterpret_cast<const __bf16*>(A->op_bf16)[e];
  if (threadIdx.x < 2) s_tot[threadIdx.x] = 0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 31, grp = lane >> 5;
  const int64_t n = A->n;
  const int64_t g = (int64_t)it.chunk * kChunk + wave * 32 + col;
  const bool valid = g < n;
  float mu[3];
  for (int k = 0; k < 3; ++k) mu[k] = valid ? A->mean[k * n + g] : 0.f;
  float em[6];
  {
    const float4* ep = reinterpret_cast<const float4*>(A->emb + (valid ? g : 0) * 8);
    const float4 e0 = ep[0], e1 = ep[1];
    em[0] = e0.x; em[1] = e0.y; em[2] = e0.z; em[3] = e0.w; em[4] = e1.x; em[5] = e1.y;
  }
  __syncthreads();
  // per-Gaussian part of layer 1 and the per-pair weights of this lane's 16 hidden units
  const float msc = A->mean_scale;
  const float xm[3] = {msc * mu[0], msc * mu[1], msc * mu[2]};
  float G[16], wd[16][4];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const float* w = s_img + kImW1G + (grp * 16 + j) * 9;
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < 3; ++i) s = fmaf(w[i], xm[i], s);
#pragma unroll
    for (int i = 0; i < 6; ++i) s = fmaf(w[3 + i], em[i], s);
    G[j] = s;
    const float* p = s_img + kImW1P + (grp * 16 + j) * 4;
#pragma unroll
    for (int i = 0; i < 4; ++i) wd[j][i] = p[i];
  }
  const float* b2p = s_img + kImB2 + grp * 16;
  const float* wop = s_img + kImWo + grp * 16;
  const float bo = s_img[kImBo];
  uint32_t n_in = 0, n_q = 0;
  // waves proceed through the segments independently: each adds its kept
  // count to the (zero-filled) chunk count
  for (int si = it.seg_begin; si < it.seg_end; ++si) {
    const int seg = seglist[si];
    const SegRec& R = segs[seg];
    const bool in = valid && cfrustum(R, mu);
    const uint64_t bal = __ballot(in);
    const bool query = R.query != 0;
    const uint32_t cin = (uint32_t)__popcll(bal) / 2;  // both lane groups hold the same 32 Gaussians
    n_in += cin;
    n_q += query ? cin : 0u;
    float z = __builtin_nanf("");
    bool keep = in && !query;
    if (query && bal != 0) {
      // per-pair inputs: unit direction camera -> Gaussian and the min-max distance
      const float vx = mu[0] - R.cl[0], vy = mu[1] - R.cl[1], vz = mu[2] - R.cl[2];
      const float len = sqrtf(vx * vx + vy * vy + vz * vz);
      const float il = 1.f / len;
      const float u[4] = {vx * il, vy * il, vz * il, fminf(1.f, fmaxf(-1.f, fmaf(R.dn_a, len, R.dn_b)))};
      const float4* cs = reinterpret_cast<const float4*>(c1perm + (size_t)seg * c1_stride + grp * 16);
      float h[16];
#pragma unroll
      for (int q4 = 0; q4 < 4; ++q4) {
        const float4 c = cs[q4];
        const float cc[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int j = 4 * q4 + t;
          float s = G[j] + cc[t];
#pragma unroll
          for (int i = 0; i < 4; ++i) s = fmaf(wd[j][i], u[i], s);
          h[j] = fmaxf(s, 0.f);
        }
      }
      f32x16c acc;
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[r] = b2p[r];
      if constexpr (P == NVGS_PREC_BF16) {
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          const bf16x8c a = reinterpret_cast<const bf16x8c*>(s_w16)[s * 64 + lane];
          bf16x8c b;
#pragma unroll
          for (int i = 0; i < 8; ++i) b[i] = (__bf16)h[8 * s + i];
          acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
      } else {
#pragma unroll
        for (int s = 0; s < 16; ++s)
          acc = __builtin_amdgcn_mfma_f32_32x32x2f32(s_img[kImW2 + s * 64 + lane], h[s], acc, 0, 0, 0);
      }
      float part = 0.f;
#pragma unroll
      for (int r = 0; r < 16; ++r) part = fmaf(wop[r], relu(acc[r]), part);
      z = part + __shfl_xor(part, 32) + bo;
      keep = in && z >= 0.f;
    }
    const uint32_t word = (uint32_t)__ballot(keep);  // lanes 0..31 (the same in both halves)
    if (lane == 0) {
      const int64_t g0 = (int64_t)it.chunk * kChunk + wave * 32;
      if (g0 < n) mask[R.word_base + (g0 >> 5)] = word;
      if (word) atomicAdd(chunk_count + R.chunk_base + it.chunk, (uint32_t)__popc(word));
    }
    if (MODE == 1 && grp == 0 && valid) {
      const int64_t idx = R.pair_base + g;
      state[idx] = keep ? 2 : (in ? 1 : 0);
      logits[idx] = (in && query) ? z : __builtin_nanf("");
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

hipError_t launch_cull_cmlp(const AssetDev* assets, const WorkItem* items, int64_t n_items, const int32_t* seglist,
                            const SegRec* segs, const float* c1perm, int c1_stride, int precision, int mode,
                            uint32_t* mask, uint32_t* chunk_count, uint8_t* state, float* logits,
                            unsigned long long* counts, hipStream_t st) {
  if (n_items == 0) return hipSuccess;
  const dim3 grid((unsigned)n_items), block(kCThreads);
#define NVGS_C(P, M)                                                                                          \
  hipLaunchKernelGGL((k_cull_cmlp<P, M>), grid, block, 0, st, assets, items, seglist, segs, c1perm, c1_stride, \
                     mask, chunk_count, state, logits, counts)
  if (precision == NVGS_PREC_FP32) {
    if (mode == 1) NVGS_C(NVGS_PREC_FP32, 1); else NVGS_C(NVGS_PREC_FP32, 0);
  } else if (precision == NVGS_PREC_BF16) {
    if (mode == 1) NVGS_C(NVGS_PREC_BF16, 1); else NVGS_C(NVGS_PREC_BF16, 0);
  } else {
    return hipErrorInvalidValue;
  }
#undef NVGS_C
  return hipGetLastError();
}

}  // namespace nvgs
