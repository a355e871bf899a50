// Training of the paper's compact visibility model (Sec. 3.2, 3.3, 4.1): the
// embedding MLP 8 -> 32 -> 32 -> 6 and the visibility MLP 16 -> 32 -> 32 -> 1
// trained jointly, BCE-with-logits loss, a hand-written backward and Adam on
// FP32 master weights (the Adam step is the frequency form's kernel).
//
// One 256-thread work-group processes chunks of 128 samples; wave w owns
// samples 32w .. 32w + 31 of a chunk and every GEMM of its samples runs on
// one 32 x 32 MFMA output tile (FP32 or BF16 operands; outputs x samples in
// the forward pass and for the input deltas, outputs x inputs for the weight
// gradients, which stay in the accumulators across the chunks).  The bias
// gradients of the layers with fewer than 32 inputs ride in the spare
// columns of the weight-gradient tiles (a column of ones); the others are
// lane sums.  At the end the four waves' gradients are summed in LDS into
// one partial per work-group; the reduce kernel adds the partials in a
// fixed order, so runs are deterministic.  With BF16 on, every GEMM operand
// is rounded to BF16 when it is staged and the GEMMs run on
// v_mfma_f32_32x32x16_bf16 (FP32 accumulation).
#include <algorithm>

#include "internal.h"

namespace nvgs {

typedef float f32x16t __attribute__((ext_vector_type(16)));

namespace {

constexpr int kH = 32;        // hidden width of both networks
constexpr int kS = 128;       // samples per chunk
constexpr int kLd = kH + 1;   // row stride of [sample][32] arrays
constexpr int kLdX = 17;      // visibility inputs
constexpr int kLdE = 9;       // embedding inputs / embedding deltas
// packed parameters: visibility W1 b1 W2 b2 wo bo, then embedding E1 e1 E2 e2 E3 e3
constexpr int oW1 = 0, ob1 = oW1 + kH * 16, oW2 = ob1 + kH, ob2 = oW2 + kH * kH, owo = ob2 + kH, obo = owo + kH;
constexpr int oE1 = obo + 1, oe1 = oE1 + kH * 8, oE2 = oe1 + kH, oe2 = oE2 + kH * kH, oE3 = oe2 + kH,
              oe3 = oE3 + 6 * kH;
constexpr int kNP = oe3 + 6;  // 3175
static_assert(kNP == kCompactVis + kCompactEmb, "compact parameter count");

enum { kTrain = 0, kForward = 1, kBackward = 2 };

struct CTrainSmem {
  // weights (row-major [out][in] with padded rows)
  float W1[kH * kLdX];
  float W2[kH * kLd];
  float E1[kH * kLdE];
  float E2[kH * kLd];
  float E3[6 * kLd];
  float b1[kH], b2[kH], wo[kH], e1[kH], e2[kH], e3[8];
  float bo;
  // per sample of the chunk
  float X[kS * kLdX];   // 10 visibility inputs + 6 embedding outputs
  float XE[kS * kLdE];  // 8 embedding inputs
  float act[6 * kS * kLd];  // G1, G2, H1, H2 (activations), DA, DB (deltas): [sample][32] each
  float DE[kS * kLdE];  // embedding output deltas
  float dz[kS];
  float y[kS];
};
// the wave reduction at the end reuses the per-sample arrays
static_assert(4 * kNP <= 6 * kS * kLd, "gradient staging fits in the activation and delta arrays");

__device__ __forceinline__ float rbf(float v) { return (float)(__bf16)v; }

__device__ __forceinline__ uint64_t smix(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

typedef __bf16 bf16x8c __attribute__((ext_vector_type(8)));

// acc[r][c] += sum_k A(r, k) B(k, c) over K, r = lane % 32 for A, c = lane %
// 32 for B.  FP32: v_mfma_f32_32x32x2f32, k = 2 s + lane / 32 (K even).
// BF16: v_mfma_f32_32x32x16_bf16 on operands the caller has rounded to BF16
// (the conversion is exact), lane group g holding k = 16 s + 8 g .. + 7, K
// padded to a multiple of 16 with zeros.
template <bool BF16, class FA, class FB>
__device__ __forceinline__ f32x16t mma(f32x16t acc, int K, FA a_at, FB b_at) {
  const int l = threadIdx.x & 63, r = l & 31, g = l >> 5;
  if constexpr (BF16) {
    for (int k0 = 0; k0 < K; k0 += 16) {
      bf16x8c av, bv;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = k0 + 8 * g + j;
        av[j] = (__bf16)(k < K ? a_at(r, k) : 0.f);
        bv[j] = (__bf16)(k < K ? b_at(k, r) : 0.f);
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
    }
  } else {
#pragma unroll 4
    for (int s = 0; s < K / 2; ++s) {
      const int k = 2 * s + g;
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a_at(r, k), b_at(k, r), acc, 0, 0, 0);
    }
  }
  return acc;
}
__device__ __forceinline__ int arow(int i) { return 8 * (i / 4) + 4 * ((threadIdx.x & 63) >> 5) + (i % 4); }

}  // namespace

// per view: camera position, forward vector (asset frame of an identity
// instance) and the affine map of the camera distance to the [-1, 1] input
__global__ void k_cview(const nvgs_camera* __restrict__ views, int V, float train_focal, float d_min, float d_max,
                        float* __restrict__ out) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  const nvgs_camera& c = views[v];
  const double f_r = 0.5 * (double)c.height / tan(0.5 * (double)c.fovy);
  const double fac = (double)train_focal / f_r, span = (double)d_max - (double)d_min;
  float* o = out + (int64_t)v * 8;
  for (int k = 0; k < 3; ++k) {
    o[k] = c.pos[k];
    o[3 + k] = c.R[6 + k];
  }
  o[6] = (float)(2.0 * fac / span);
  o[7] = (float)(-2.0 * (double)d_min / span - 1.0);
}

template <bool BF16R, int MODE>
__global__ __launch_bounds__(256) void k_cmlp_train(
    const float* __restrict__ params, int64_t batch, int chunks_per_wg, float inv_batch,
    // training inputs
    const float* __restrict__ mean, const float* __restrict__ scale, const float* __restrict__ quat,
    const float* __restrict__ opacity, int64_t n, float mean_scale, const float* __restrict__ vrec, int V,
    const uint32_t* __restrict__ labels, uint64_t seed, int64_t step, const uint32_t* __restrict__ n_pos,
    // forward / backward inputs [B][18]: 10 visibility inputs, 8 embedding inputs
    const float* __restrict__ Xin, const float* __restrict__ dlogits,
    // outputs
    float* __restrict__ logits, float* __restrict__ partial, float* __restrict__ loss_part) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  CTrainSmem& S = *reinterpret_cast<CTrainSmem*>(smem_raw);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, col = lane & 31;
  const int p0 = 32 * wave;  // this wave's samples in the chunk
  auto rnd = [](float v) { return BF16R ? rbf(v) : v; };
  float* const G1 = S.act;
  float* const G2 = G1 + kS * kLd;
  float* const H1 = G2 + kS * kLd;
  float* const H2 = H1 + kS * kLd;
  float* const DA = H2 + kS * kLd;
  float* const DB = DA + kS * kLd;
  for (int i = t; i < kH * 16; i += 256) S.W1[(i / 16) * kLdX + i % 16] = rnd(params[oW1 + i]);
  for (int i = t; i < kH * kH; i += 256) {
    S.W2[(i / kH) * kLd + i % kH] = rnd(params[oW2 + i]);
    S.E2[(i / kH) * kLd + i % kH] = rnd(params[oE2 + i]);
  }
  for (int i = t; i < kH * 8; i += 256) S.E1[(i / 8) * kLdE + i % 8] = rnd(params[oE1 + i]);
  for (int i = t; i < 6 * kH; i += 256) S.E3[(i / kH) * kLd + i % kH] = rnd(params[oE3 + i]);
  if (t < kH) {
    S.b1[t] = params[ob1 + t];
    S.b2[t] = params[ob2 + t];
    S.wo[t] = params[owo + t];
    S.e1[t] = params[oe1 + t];
    S.e2[t] = params[oe2 + t];
  }
  if (t < 8) S.e3[t] = t < 6 ? params[oe3 + t] : 0.f;
  if (t == 0) S.bo = params[obo];
  const f32x16t zero = (f32x16t){0};
  f32x16t gW1 = zero, gW2 = zero, gE1 = zero, gE2 = zero, gE3 = zero;
  float r_db2 = 0.f, r_de2 = 0.f, r_dwo = 0.f, r_de3 = 0.f, r_dbo = 0.f, loss = 0.f;
  __syncthreads();
  for (int ch = 0; ch < chunks_per_wg; ++ch) {
    const int64_t base = ((int64_t)blockIdx.x * chunks_per_wg + ch) * kS;
    // ---- inputs
    if (t < kS) {
      const int64_t gi = base + t;
      float x[10], xe[8];
      if (MODE == kTrain) {
        const uint64_t r = smix(seed, (uint64_t)step * (uint64_t)batch + (uint64_t)gi);
        const int64_t g = (int64_t)(((r & 0xffffffffull) * (uint64_t)n) >> 32);
        const int64_t v = (int64_t)(((r >> 32) * (uint64_t)V) >> 32);
        const float* vr = vrec + v * 8;
        float mu[3], d[3];
        for (int k = 0; k < 3; ++k) {
          mu[k] = mean[k * n + g];
          d[k] = mu[k] - vr[k];
        }
        const float len = sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        const float il = 1.f / len;
        for (int k = 0; k < 3; ++k) {
          x[k] = mean_scale * mu[k];
          x[3 + k] = d[k] * il;
          x[7 + k] = vr[3 + k];
        }
        x[6] = fminf(1.f, fmaxf(-1.f, fmaf(vr[6], len, vr[7])));
        xe[0] = opacity[g];
        for (int k = 0; k < 3; ++k) xe[1 + k] = logf(scale[k * n + g]);
        float q[4];
        for (int k = 0; k < 4; ++k) q[k] = quat[k * n + g];
        const float qn = (q[0] < 0.f ? -1.f : 1.f) / sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        for (int k = 0; k < 4; ++k) xe[4 + k] = q[k] * qn;
        const int64_t words = (n + 31) / 32;
        S.y[t] = (float)((labels[v * words + (g >> 5)] >> (g & 31)) & 1u);
      } else {
        const bool live = gi < batch;
        for (int k = 0; k < 10; ++k) x[k] = live ? Xin[gi * 18 + k] : 0.f;
        for (int k = 0; k < 8; ++k) xe[k] = live ? Xin[gi * 18 + 10 + k] : 0.f;
      }
      for (int k = 0; k < 10; ++k) S.X[t * kLdX + k] = rnd(x[k]);
      for (int k = 0; k < 8; ++k) S.XE[t * kLdE + k] = rnd(xe[k]);
    }
    __syncthreads();
    // ---- forward, per wave on its 32 samples: outputs (rows) x samples (columns)
    {
      f32x16t a = mma<BF16R>(zero, 8, [&](int r, int k) { return S.E1[r * kLdE + k]; },
                      [&](int k, int c) { return S.XE[(p0 + c) * kLdE + k]; });
      for (int i = 0; i < 16; ++i) G1[(p0 + col) * kLd + arow(i)] = rnd(fmaxf(a[i] + S.e1[arow(i)], 0.f));
    }
    __syncthreads();
    {
      f32x16t a = mma<BF16R>(zero, kH, [&](int r, int k) { return S.E2[r * kLd + k]; },
                      [&](int k, int c) { return G1[(p0 + c) * kLd + k]; });
      for (int i = 0; i < 16; ++i) G2[(p0 + col) * kLd + arow(i)] = rnd(fmaxf(a[i] + S.e2[arow(i)], 0.f));
    }
    __syncthreads();
    {
      f32x16t a = mma<BF16R>(zero, kH, [&](int r, int k) { return r < 6 ? S.E3[r * kLd + k] : 0.f; },
                      [&](int k, int c) { return G2[(p0 + c) * kLd + k]; });
      for (int i = 0; i < 16; ++i) {
        const int r = arow(i);
        if (r < 6) S.X[(p0 + col) * kLdX + 10 + r] = rnd(a[i] + S.e3[r]);
      }
    }
    __syncthreads();
    {
      f32x16t a = mma<BF16R>(zero, 16, [&](int r, int k) { return S.W1[r * kLdX + k]; },
                      [&](int k, int c) { return S.X[(p0 + c) * kLdX + k]; });
      for (int i = 0; i < 16; ++i) H1[(p0 + col) * kLd + arow(i)] = rnd(fmaxf(a[i] + S.b1[arow(i)], 0.f));
    }
    __syncthreads();
    {
      f32x16t a = mma<BF16R>(zero, kH, [&](int r, int k) { return S.W2[r * kLd + k]; },
                      [&](int k, int c) { return H1[(p0 + c) * kLd + k]; });
      // FP32: the output layer is a VALU dot
      for (int i = 0; i < 16; ++i) H2[(p0 + col) * kLd + arow(i)] = fmaxf(a[i] + S.b2[arow(i)], 0.f);
    }
    __syncthreads();
    // ---- output, loss, dz
    if (t < kS) {
      float z = S.bo;
      for (int m = 0; m < kH; ++m) z = fmaf(S.wo[m], H2[t * kLd + m], z);
      const int64_t gi = base + t;
      const bool live = gi < batch;
      float d = 0.f;
      if (MODE == kTrain && live) {
        const float y = S.y[t];
        float w = 1.f;  // frequency weighting: B / (2 n_class)
        if (n_pos) {
          const float np_ = (float)*n_pos, nn_ = (float)batch - np_;
          const float wc = y > 0.5f ? np_ : nn_;
          w = wc > 0.f ? 0.5f * (float)batch / wc : 0.f;
        }
        const float sig = 1.f / (1.f + expf(-z));
        loss += w * (fmaxf(z, 0.f) - z * y + log1pf(expf(-fabsf(z))));
        d = w * (sig - y) * inv_batch;
      } else if (MODE == kBackward) {
        d = live ? dlogits[gi] : 0.f;
      } else if (live) {
        logits[gi] = z;
      }
      S.dz[t] = d;
    }
    __syncthreads();
    if (MODE == kForward) continue;
    // ---- D2 = dz wo * 1[H2 > 0]
    for (int e = t; e < kS * kH; e += 256) {
      const int p = e / kH, m = e % kH;
      DA[p * kLd + m] = rnd(H2[p * kLd + m] > 0.f ? S.dz[p] * S.wo[m] : 0.f);
    }
    __syncthreads();
    // lane sums over this wave's samples: db2 (lanes < 32), dwo (lanes >= 32), dbo
    {
      float s = 0.f;
      for (int p = p0; p < p0 + 32; ++p) s += lane < 32 ? DA[p * kLd + col] : S.dz[p] * H2[p * kLd + col];
      if (lane < 32) r_db2 += s; else r_dwo += s;
      if (lane == 0)
        for (int p = p0; p < p0 + 32; ++p) r_dbo += S.dz[p];
    }
    // dW2 += D2' H1 (outputs x inputs, over this wave's samples)
    gW2 = mma<BF16R>(gW2, 32, [&](int r, int k) { return DA[(p0 + k) * kLd + r]; },
              [&](int k, int c) { return H1[(p0 + k) * kLd + c]; });
    // D1 = (W2' D2) * 1[H1 > 0]
    {
      f32x16t a = mma<BF16R>(zero, kH, [&](int r, int k) { return S.W2[k * kLd + r]; },
                      [&](int k, int c) { return DA[(p0 + c) * kLd + k]; });
      for (int i = 0; i < 16; ++i) {
        const int r = arow(i);
        DB[(p0 + col) * kLd + r] = rnd(H1[(p0 + col) * kLd + r] > 0.f ? a[i] : 0.f);
      }
    }
    __syncthreads();
    // dW1 += D1' [X | 1] (the column of ones gives db1); embedding deltas = (W1' D1) rows 10..15
    gW1 = mma<BF16R>(gW1, 32, [&](int r, int k) { return DB[(p0 + k) * kLd + r]; },
              [&](int k, int c) { return c < 16 ? S.X[(p0 + k) * kLdX + c] : (c == 16 ? 1.f : 0.f); });
    {
      f32x16t a = mma<BF16R>(zero, kH, [&](int r, int k) { return r < 16 ? S.W1[k * kLdX + r] : 0.f; },
                      [&](int k, int c) { return DB[(p0 + c) * kLd + k]; });
      for (int i = 0; i < 16; ++i) {
        const int r = arow(i);
        if (r >= 10 && r < 16) S.DE[(p0 + col) * kLdE + r - 10] = rnd(a[i]);
      }
    }
    __syncthreads();
    // dE3 += DE' G2 ; de3 ; DG2 = (E3' DE) * 1[G2 > 0]
    gE3 = mma<BF16R>(gE3, 32, [&](int r, int k) { return r < 6 ? S.DE[(p0 + k) * kLdE + r] : 0.f; },
              [&](int k, int c) { return G2[(p0 + k) * kLd + c]; });
    if (lane >= 32 && lane < 38) {
      float s = 0.f;
      for (int p = p0; p < p0 + 32; ++p) s += S.DE[p * kLdE + lane - 32];
      r_de3 += s;
    }
    {
      f32x16t a = mma<BF16R>(zero, 8, [&](int r, int k) { return k < 6 ? S.E3[k * kLd + r] : 0.f; },
                      [&](int k, int c) { return k < 6 ? S.DE[(p0 + c) * kLdE + k] : 0.f; });
      for (int i = 0; i < 16; ++i) {
        const int r = arow(i);
        DA[(p0 + col) * kLd + r] = rnd(G2[(p0 + col) * kLd + r] > 0.f ? a[i] : 0.f);
      }
    }
    __syncthreads();
    // dE2 += DG2' G1 ; de2 ; DG1 = (E2' DG2) * 1[G1 > 0]
    gE2 = mma<BF16R>(gE2, 32, [&](int r, int k) { return DA[(p0 + k) * kLd + r]; },
              [&](int k, int c) { return G1[(p0 + k) * kLd + c]; });
    if (lane < 32) {
      float s = 0.f;
      for (int p = p0; p < p0 + 32; ++p) s += DA[p * kLd + lane];
      r_de2 += s;
    }
    {
      f32x16t a = mma<BF16R>(zero, kH, [&](int r, int k) { return S.E2[k * kLd + r]; },
                      [&](int k, int c) { return DA[(p0 + c) * kLd + k]; });
      for (int i = 0; i < 16; ++i) {
        const int r = arow(i);
        DB[(p0 + col) * kLd + r] = rnd(G1[(p0 + col) * kLd + r] > 0.f ? a[i] : 0.f);
      }
    }
    __syncthreads();
    // dE1 += DG1' [XE | 1] (the column of ones gives de1)
    gE1 = mma<BF16R>(gE1, 32, [&](int r, int k) { return DB[(p0 + k) * kLd + r]; },
              [&](int k, int c) { return c < 8 ? S.XE[(p0 + k) * kLdE + c] : (c == 8 ? 1.f : 0.f); });
    __syncthreads();
  }
  if (MODE == kForward) return;
  // ---- the four waves' gradients into LDS, summed into one partial
  float* G = S.act;  // 4 x kNP floats over the activation and delta arrays
  float* mine = G + wave * kNP;
  for (int i = 0; i < 16; ++i) {
    const int r = arow(i);
    mine[oW2 + r * kH + col] = gW2[i];
    mine[oE2 + r * kH + col] = gE2[i];
    if (col < 16) mine[oW1 + r * 16 + col] = gW1[i];
    if (col == 16) mine[ob1 + r] = gW1[i];
    if (col < 8) mine[oE1 + r * 8 + col] = gE1[i];
    if (col == 8) mine[oe1 + r] = gE1[i];
    if (r < 6) mine[oE3 + r * kH + col] = gE3[i];
  }
  if (lane < 32) {
    mine[ob2 + lane] = r_db2;
    mine[oe2 + lane] = r_de2;
  } else {
    mine[owo + lane - 32] = r_dwo;
    if (lane < 38) mine[oe3 + lane - 32] = r_de3;
  }
  if (lane == 0) mine[obo] = r_dbo;
  __syncthreads();
  float* out = partial + (int64_t)blockIdx.x * kNP;
  for (int p = t; p < kNP; p += 256) out[p] = (G[p] + G[kNP + p]) + (G[2 * kNP + p] + G[3 * kNP + p]);
  if (MODE == kTrain) {
    float* red = S.DE;  // 256 floats (not part of the gradient staging)
    red[t] = loss;
    __syncthreads();
    if (t == 0) {
      float s = 0.f;
      for (int k = 0; k < 256; ++k) s += red[k];
      loss_part[blockIdx.x] = s;
    }
  }
}

size_t ctrain_smem_bytes() { return sizeof(CTrainSmem); }

hipError_t launch_cview(const nvgs_camera* views, int V, float train_focal, float d_min, float d_max, float* out,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_cview, dim3((V + 63) / 64), dim3(64), 0, st, views, V, train_focal, d_min, d_max, out);
  return hipGetLastError();
}

template <bool B, int M>
static hipError_t launch_ct(int nwg, int cpw, hipStream_t st, const float* params, int64_t batch, float inv_batch,
                            const CTrainArgs& a, const float* X, const float* dlogits, float* logits, float* partial,
                            float* loss_part) {
  auto kern = k_cmlp_train<B, M>;
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(CTrainSmem));
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL(kern, dim3(nwg), dim3(256), sizeof(CTrainSmem), st, params, batch, cpw, inv_batch, a.mean,
                     a.scale, a.quat, a.opacity, a.n, a.mean_scale, a.vrec, a.V, a.labels, a.seed, a.step, a.n_pos,
                     X, dlogits, logits, partial, loss_part);
  return hipGetLastError();
}

hipError_t launch_cmlp_train(int mode, bool bf16, int nwg, int chunks_per_wg, hipStream_t st, const float* params,
                             int64_t batch, float inv_batch, const CTrainArgs& a, const float* X,
                             const float* dlogits, float* logits, float* partial, float* loss_part) {
#define NVGS_CT(B, M) return launch_ct<B, M>(nwg, chunks_per_wg, st, params, batch, inv_batch, a, X, dlogits, \
                                             logits, partial, loss_part)
  if (bf16) {
    if (mode == 0) NVGS_CT(true, 0);
    if (mode == 1) NVGS_CT(true, 1);
    NVGS_CT(true, 2);
  }
  if (mode == 0) NVGS_CT(false, 0);
  if (mode == 1) NVGS_CT(false, 1);
  NVGS_CT(false, 2);
#undef NVGS_CT
}

int ctrain_num_params() { return kNP; }
int ctrain_samples_per_chunk() { return kS; }

}  // namespace nvgs
