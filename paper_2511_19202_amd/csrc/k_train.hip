// Training of the visibility MLP (Sec. 3.1-3.2): labels from the renderer's
// contribution recording, BCE-with-logits loss, a hand-written backward and
// Adam on FP32 master weights.
//
// One 256-thread work-group processes chunks of 64 (Gaussian, view) pairs.
// Per chunk every GEMM of the forward and backward pass runs on
// v_mfma_f32_32x32x2_f32 with operands read from LDS (one 32x32 output tile
// per wave): H1' = W1 G', H2' = W2 H1', H3' = W3 H2'; d3 = dz wo * 1[H3 > 0];
// dW3 += d3' H2; d2 = (W3' d3) * 1[H2 > 0]; dW2 += d2' H1; d1 = (W2' d2) *
// 1[H1 > 0]; dW1 += d1' G.  The weight gradients stay in the MFMA
// accumulators across the chunks of a work-group and are written once as a
// per-group partial; a second kernel sums the partials in a fixed order (so
// runs are deterministic) and applies Adam.  With BF16 rounding on, every
// GEMM operand (inputs, activations, deltas, weights) is rounded to BF16 when
// it is staged, so the FP32 MFMA forms the same exact products as a BF16
// MFMA with FP32 accumulation.
#include <algorithm>
#include <mutex>

#include "internal.h"

// Fixed device workspace of the allocation-free backward entry point: the
// per-work-group gradient partials and the slices of their two-level sum.
// Each device the library runs on holds its own copy until the process ends.
// Host code never passes this name to a kernel (on the host it is only a
// stand-in for the symbol): it uses the address looked up per device below.
static constexpr size_t kStaticScratchFloats = size_t(1) << 22;  // 16 MiB
static __device__ __align__(256) float scratch[kStaticScratchFloats];

namespace nvgs {

typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kTW = 64;      // hidden width supported by the training kernels
constexpr int kTP = 64;      // pairs per chunk
constexpr int kIn = 72;      // encoded inputs
constexpr int kLdW1 = kIn + 1;
constexpr int kLdH = kTW + 1;
constexpr int kNumParams = kIn * kTW + kTW + 2 * (kTW * kTW + kTW) + kTW + 1;  // 13,057

enum { kModeTrain = 0, kModeForward = 1, kModeBackward = 2 };

__device__ __forceinline__ float round_bf16(float v) { return (float)(__bf16)v; }

// SplitMix64 (Steele, Lea, Flood 2014): the i-th output for a seed
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct TrainSmem {
  float W1[kTW * kLdW1];
  float W2[kTW * kLdH];
  float W3[kTW * kLdH];
  float b[4][kTW];  // b1, b2, b3, wo
  float bo;
  float G[kTP * kLdW1];
  float H1[kTP * kLdH];
  float H2[kTP * kLdH];
  float H3[kTP * kLdH];
  float D[kTP * kLdH];
  float D2[kTP * kLdH];
  float dz[kTP];
  float red[256];
};

// acc += A (32 rows at m0) x B (32 cols at n0) over K, operands via accessors
template <class FA, class FB>
__device__ __forceinline__ f32x16 tile_mma(f32x16 acc, int K, FA a_at, FB b_at) {
  const int l = threadIdx.x & 63, r = l & 31, g = l >> 5;
#pragma unroll 4
  for (int s = 0; s < K / 2; ++s) {
    const int k = 2 * s + g;
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a_at(r, k), b_at(k, r), acc, 0, 0, 0);
  }
  return acc;
}
// row of accumulator element i held by this lane
__device__ __forceinline__ int acc_row(int i) { return 8 * (i / 4) + 4 * ((threadIdx.x & 63) >> 5) + (i % 4); }

template <bool BF16R, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_mlp_train(
    const float* __restrict__ params, int64_t batch, int chunks_per_wg, float inv_batch,
    // training inputs
    const float* __restrict__ mean, int64_t n, float mean_scale, const float* __restrict__ view_gam, int V,
    const uint32_t* __restrict__ labels, uint64_t seed, int64_t step, const uint32_t* __restrict__ n_pos,
    // forward / backward inputs
    const float* __restrict__ X, const float* __restrict__ dlogits,
    // outputs
    float* __restrict__ logits, float* __restrict__ partial, float* __restrict__ loss_part, float* __restrict__ dX) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  TrainSmem& S = *reinterpret_cast<TrainSmem*>(smem_raw);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int mt = wave >> 1, nt = wave & 1;  // this wave's 32x32 tile of a 64x64 output
  auto rnd = [](float v) { return BF16R ? round_bf16(v) : v; };
  // weights into LDS
  {
    const float* W1 = params;
    const float* b1 = W1 + kTW * kIn;
    const float* W2 = b1 + kTW;
    const float* b2 = W2 + kTW * kTW;
    const float* W3 = b2 + kTW;
    const float* b3 = W3 + kTW * kTW;
    const float* wo = b3 + kTW;
    for (int i = t; i < kTW * kIn; i += 256) S.W1[(i / kIn) * kLdW1 + i % kIn] = rnd(W1[i]);
    for (int i = t; i < kTW * kTW; i += 256) {
      S.W2[(i / kTW) * kLdH + i % kTW] = rnd(W2[i]);
      S.W3[(i / kTW) * kLdH + i % kTW] = rnd(W3[i]);
    }
    for (int i = t; i < kTW; i += 256) {
      S.b[0][i] = b1[i];
      S.b[1][i] = b2[i];
      S.b[2][i] = b3[i];
      S.b[3][i] = wo[i];
    }
    if (t == 0) S.bo = wo[kTW];
  }
  f32x16 dW1[2], dW2, dW3;
  for (int q = 0; q < 2; ++q) dW1[q] = (f32x16){0};
  dW2 = dW3 = (f32x16){0};
  float db[3] = {0.f, 0.f, 0.f}, dwo = 0.f, dbo = 0.f, loss = 0.f;  // thread t < 64 owns feature t
  __syncthreads();
  for (int ch = 0; ch < chunks_per_wg; ++ch) {
    const int64_t base = ((int64_t)blockIdx.x * chunks_per_wg + ch) * kTP;
    // ---- inputs G [pair][72]
    if (MODE == kModeTrain) {
      __shared__ int s_g[kTP], s_v[kTP];
      if (t < kTP) {
        const uint64_t r = splitmix64(seed, (uint64_t)step * (uint64_t)batch + (uint64_t)(base + t));
        s_g[t] = (int)(((r & 0xffffffffull) * (uint64_t)n) >> 32);
        s_v[t] = (int)(((r >> 32) * (uint64_t)V) >> 32);
      }
      __syncthreads();
      for (int e = t; e < kTP * kIn; e += 256) {
        const int p = e / kIn, c = e % kIn;
        float v;
        if (c < 36) {
          const int j = c / 12, band = (c % 12) / 2;
          const float x = ldexpf(mean_scale * mean[j * n + s_g[p]], band);
          v = (c & 1) ? cospif(x) : sinpif(x);
        } else {
          v = view_gam[(int64_t)s_v[p] * 36 + (c - 36)];
        }
        S.G[p * kLdW1 + c] = rnd(v);
      }
      if (t < kTP) {
        const int g = s_g[t], v = s_v[t];
        const int64_t words = (n + 31) / 32;
        S.dz[t] = (float)((labels[(int64_t)v * words + (g >> 5)] >> (g & 31)) & 1u);  // label y for now
      }
    } else {
      for (int e = t; e < kTP * kIn; e += 256) {
        const int p = e / kIn, c = e % kIn;
        const int64_t gi = base + p;
        S.G[p * kLdW1 + c] = gi < batch ? rnd(X[gi * kIn + c]) : 0.f;
      }
    }
    __syncthreads();
    // ---- forward: H1' = W1 G', H2' = W2 H1', H3' = W3 H2'
    {
      f32x16 a = tile_mma((f32x16){0}, kIn, [&](int r, int k) { return S.W1[(mt * 32 + r) * kLdW1 + k]; },
                          [&](int k, int c) { return S.G[(nt * 32 + c) * kLdW1 + k]; });
      for (int i = 0; i < 16; ++i) {
        const int m = mt * 32 + acc_row(i), p = nt * 32 + (lane & 31);
        S.H1[p * kLdH + m] = rnd(fmaxf(a[i] + S.b[0][m], 0.f));
      }
    }
    __syncthreads();
    {
      f32x16 a = tile_mma((f32x16){0}, kTW, [&](int r, int k) { return S.W2[(mt * 32 + r) * kLdH + k]; },
                          [&](int k, int c) { return S.H1[(nt * 32 + c) * kLdH + k]; });
      for (int i = 0; i < 16; ++i) {
        const int m = mt * 32 + acc_row(i), p = nt * 32 + (lane & 31);
        S.H2[p * kLdH + m] = rnd(fmaxf(a[i] + S.b[1][m], 0.f));
      }
    }
    __syncthreads();
    {
      f32x16 a = tile_mma((f32x16){0}, kTW, [&](int r, int k) { return S.W3[(mt * 32 + r) * kLdH + k]; },
                          [&](int k, int c) { return S.H2[(nt * 32 + c) * kLdH + k]; });
      for (int i = 0; i < 16; ++i) {
        const int m = mt * 32 + acc_row(i), p = nt * 32 + (lane & 31);
        S.H3[p * kLdH + m] = fmaxf(a[i] + S.b[2][m], 0.f);  // FP32: the output layer is a VALU dot
      }
    }
    __syncthreads();
    // ---- output layer, loss, dz
    if (t < kTP) {
      float z = S.bo;
      for (int m = 0; m < kTW; ++m) z = fmaf(S.b[3][m], S.H3[t * kLdH + m], z);
      const int64_t gi = base + t;
      const bool live = gi < batch;
      float d = 0.f;
      if (MODE == kModeTrain && live) {
        const float y = S.dz[t];
        float w = 1.f;  // frequency weighting: B / (2 n_class)
        if (n_pos) {
          const float np_ = (float)*n_pos, nn_ = (float)batch - np_;
          const float wc = y > 0.5f ? np_ : nn_;
          w = wc > 0.f ? 0.5f * (float)batch / wc : 0.f;
        }
        const float sig = 1.f / (1.f + expf(-z));
        loss += w * (fmaxf(z, 0.f) - z * y + log1pf(expf(-fabsf(z))));
        d = w * (sig - y) * inv_batch;
      } else if (MODE == kModeBackward) {
        d = live ? dlogits[gi] : 0.f;
      } else if (live) {
        logits[gi] = z;
      }
      S.dz[t] = d;
    }
    if (MODE == kModeForward) {
      __syncthreads();
      continue;
    }
    __syncthreads();
    // ---- d3 = dz wo * 1[H3 > 0]  (H3 itself is kept in FP32 for dwo)
    for (int e = t; e < kTP * kTW; e += 256) {
      const int p = e / kTW, m = e % kTW;
      const float h = S.H3[p * kLdH + m];
      S.D[p * kLdH + m] = rnd(h > 0.f ? S.dz[p] * S.b[3][m] : 0.f);
    }
    if (t < kTW) {
      float s = 0.f;
      for (int p = 0; p < kTP; ++p) s = fmaf(S.dz[p], S.H3[p * kLdH + t], s);
      dwo += s;
    }
    if (t == 0)
      for (int p = 0; p < kTP; ++p) dbo += S.dz[p];
    __syncthreads();
    // dW3 += d3' H2 ; db3
    dW3 = tile_mma(dW3, kTP, [&](int r, int k) { return S.D[k * kLdH + mt * 32 + r]; },
                   [&](int k, int c) { return S.H2[k * kLdH + nt * 32 + c]; });
    if (t < kTW) {
      float s = 0.f;
      for (int p = 0; p < kTP; ++p) s += S.D[p * kLdH + t];
      db[2] += s;
    }
    // d2 = (W3' d3) * 1[H2 > 0]
    {
      f32x16 a = tile_mma((f32x16){0}, kTW, [&](int r, int k) { return S.W3[k * kLdH + mt * 32 + r]; },
                          [&](int k, int c) { return S.D[(nt * 32 + c) * kLdH + k]; });
      for (int i = 0; i < 16; ++i) {
        const int j = mt * 32 + acc_row(i), p = nt * 32 + (lane & 31);
        S.D2[p * kLdH + j] = rnd(S.H2[p * kLdH + j] > 0.f ? a[i] : 0.f);
      }
    }
    __syncthreads();
    // dW2 += d2' H1 ; db2
    dW2 = tile_mma(dW2, kTP, [&](int r, int k) { return S.D2[k * kLdH + mt * 32 + r]; },
                   [&](int k, int c) { return S.H1[k * kLdH + nt * 32 + c]; });
    if (t < kTW) {
      float s = 0.f;
      for (int p = 0; p < kTP; ++p) s += S.D2[p * kLdH + t];
      db[1] += s;
    }
    // d1 = (W2' d2) * 1[H1 > 0]   (into D: every wave finished reading d3 above)
    {
      f32x16 a = tile_mma((f32x16){0}, kTW, [&](int r, int k) { return S.W2[k * kLdH + mt * 32 + r]; },
                          [&](int k, int c) { return S.D2[(nt * 32 + c) * kLdH + k]; });
      __syncthreads();
      for (int i = 0; i < 16; ++i) {
        const int j = mt * 32 + acc_row(i), p = nt * 32 + (lane & 31);
        S.D[p * kLdH + j] = rnd(S.H1[p * kLdH + j] > 0.f ? a[i] : 0.f);
      }
    }
    __syncthreads();
    // dW1 += d1' G: 2 x 3 tiles of 32 (the last column tile covers 64..71),
    // wave (mt, nt) owns column tiles nt and nt + 2
    for (int u = 0; u < 2; ++u) {
      const int q = nt + 2 * u;
      if (q < 3)
        dW1[u] = tile_mma(dW1[u], kTP, [&](int r, int k) { return S.D[k * kLdH + mt * 32 + r]; },
                          [&](int k, int c) {
                            const int cc = q * 32 + c;
                            return cc < kIn ? S.G[k * kLdW1 + cc] : 0.f;
                          });
    }
    if (t < kTW) {
      float s = 0.f;
      for (int p = 0; p < kTP; ++p) s += S.D[p * kLdH + t];
      db[0] += s;
    }
    // dX = W1' d1 (backward mode only): 3 input tiles x 2 pair tiles, wave
    // (mt, nt) owns input tiles mt and mt + 2 of pair tile nt
    if (MODE == kModeBackward && dX) {
      for (int u = 0; u < 2; ++u) {
        const int q = mt + 2 * u;
        if (q >= 3) continue;
        f32x16 a = tile_mma((f32x16){0}, kTW,
                            [&](int r, int k) {
                              const int c = q * 32 + r;
                              return c < kIn ? S.W1[k * kLdW1 + c] : 0.f;
                            },
                            [&](int k, int c) { return S.D[(nt * 32 + c) * kLdH + k]; });
        for (int i = 0; i < 16; ++i) {
          const int c = q * 32 + acc_row(i);
          const int64_t gi = base + nt * 32 + (lane & 31);
          if (c < kIn && gi < batch) dX[gi * kIn + c] = a[i];
        }
      }
    }
    __syncthreads();
  }
  if (MODE == kModeForward) return;
  // ---- write this work-group's partial gradients
  float* out = partial + (int64_t)blockIdx.x * kNumParams;
  float* oW1 = out;
  float* ob1 = oW1 + kTW * kIn;
  float* oW2 = ob1 + kTW;
  float* ob2 = oW2 + kTW * kTW;
  float* oW3 = ob2 + kTW;
  float* ob3 = oW3 + kTW * kTW;
  float* owo = ob3 + kTW;
  for (int i = 0; i < 16; ++i) {
    const int m = mt * 32 + acc_row(i), c = nt * 32 + (lane & 31);
    oW2[m * kTW + c] = dW2[i];
    oW3[m * kTW + c] = dW3[i];
  }
  // dW1: this wave holds rows mt*32.. of column tiles nt and nt + 2
  for (int u = 0; u < 2; ++u) {
    const int q = nt + 2 * u;
    if (q >= 3) continue;
    for (int i = 0; i < 16; ++i) {
      const int m = mt * 32 + acc_row(i), c = q * 32 + (lane & 31);
      if (c < kIn) oW1[m * kIn + c] = dW1[u][i];
    }
  }
  if (t < kTW) {
    ob1[t] = db[0];
    ob2[t] = db[1];
    ob3[t] = db[2];
    owo[t] = dwo;
  }
  if (t == 0) owo[kTW] = dbo;
  if (MODE == kModeTrain) {
    S.red[t] = loss;
    __syncthreads();
    if (t == 0) {
      float s = 0.f;
      for (int k = 0; k < 256; ++k) s += S.red[k];
      loss_part[blockIdx.x] = s;
    }
  }
}

// first level of the gradient sum: slice s of the work-group partials
// (a fixed contiguous range) summed in order, for every parameter and the loss
__global__ void k_reduce_slices(const float* __restrict__ partial, int nwg, int np, int S,
                                const float* __restrict__ loss_part, float* __restrict__ tmp,
                                float* __restrict__ tmp_loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x, s = blockIdx.y;
  const int w0 = (int)((int64_t)nwg * s / S), w1 = (int)((int64_t)nwg * (s + 1) / S);
  if (p < np) {
    float g = 0.f;
    for (int w = w0; w < w1; ++w) g += partial[(int64_t)w * np + p];
    tmp[(int64_t)s * np + p] = g;
  }
  if (loss_part && blockIdx.x == 0 && threadIdx.x == 0) {
    float l = 0.f;
    for (int w = w0; w < w1; ++w) l += loss_part[w];
    tmp_loss[s] = l;
  }
}

// sum of the per-group partials (fixed order), then Adam or a plain store
__global__ void k_reduce_adam(const float* __restrict__ partial, int nwg, int np, float* __restrict__ params,
                              float* __restrict__ m, float* __restrict__ v, float* __restrict__ grad_out, float lr,
                              float b1, float b2, float eps, float c1, float c2, const float* __restrict__ loss_part,
                              float inv_batch, float* __restrict__ loss_out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < np) {
    float g = 0.f;
    for (int w = 0; w < nwg; ++w) g += partial[(int64_t)w * np + p];
    if (grad_out) {
      grad_out[p] = g;
    } else {
      const float mm = b1 * m[p] + (1.f - b1) * g;
      const float vv = b2 * v[p] + (1.f - b2) * g * g;
      m[p] = mm;
      v[p] = vv;
      params[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    }
  }
  if (loss_out && p == 0) {
    float s = 0.f;
    for (int w = 0; w < nwg; ++w) s += loss_part[w];
    *loss_out = s * inv_batch;
  }
}

// encoded camera features of every view (asset frame = world frame of a
// single identity instance), FP64, layout [V][36]
__global__ void k_view_gam(const nvgs_camera* __restrict__ views, int V, float cam_scale, float train_focal,
                           float d_max, float* __restrict__ gam) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  const nvgs_camera& c = views[v];
  const double f_r = 0.5 * (double)c.height / tan(0.5 * (double)c.fovy);  // pixels
  const double fac = (double)train_focal / f_r;
  double cm[3] = {c.pos[0] * fac, c.pos[1] * fac, c.pos[2] * fac};
  const double len = sqrt(cm[0] * cm[0] + cm[1] * cm[1] + cm[2] * cm[2]);
  if (d_max > 0.f && len > (double)d_max)
    for (int r = 0; r < 3; ++r) cm[r] *= (double)d_max / len;
  for (int j = 0; j < 3; ++j)
    for (int band = 0; band < 6; ++band) {
      const double a = ldexp(M_PI * ((double)cam_scale * cm[j]), band);
      gam[(int64_t)v * 36 + j * 12 + band * 2] = (float)sin(a);
      gam[(int64_t)v * 36 + j * 12 + band * 2 + 1] = (float)cos(a);
    }
}

// label bits: bit g of word (v, g/32) = contribution[v][g] > threshold
__global__ void k_label_bits(const float* __restrict__ contrib, int64_t n, int V, float thr,
                             uint32_t* __restrict__ bits) {
  const int64_t words = (n + 31) / 32;
  for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < (int64_t)V * words;
       w += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = w / words, g0 = (w % words) * 32;
    uint32_t b = 0;
    for (int k = 0; k < 32; ++k)
      if (g0 + k < n && contrib[v * n + g0 + k] > thr) b |= 1u << k;
    bits[w] = b;
  }
}

// number of positive labels among the pairs of one training step
__global__ void k_count_pos(int64_t batch, int64_t n, int V, const uint32_t* __restrict__ labels, uint64_t seed,
                            int64_t step, uint32_t* __restrict__ count) {
  const int64_t words = (n + 31) / 32;
  uint32_t c = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < batch; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t r = splitmix64(seed, (uint64_t)step * (uint64_t)batch + (uint64_t)i);
    const int64_t g = (int64_t)(((r & 0xffffffffull) * (uint64_t)n) >> 32);
    const int64_t v = (int64_t)(((r >> 32) * (uint64_t)V) >> 32);
    c += (labels[v * words + (g >> 5)] >> (g & 31)) & 1u;
  }
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  if ((threadIdx.x & 63) == 0) atomicAdd(count, c);
}

hipError_t launch_count_pos(int64_t batch, int64_t n, int V, const uint32_t* labels, uint64_t seed, int64_t step,
                            uint32_t* count, hipStream_t st) {
  const unsigned grid = (unsigned)std::min<int64_t>((batch + 255) / 256, 1024);
  hipLaunchKernelGGL(k_count_pos, dim3(grid), dim3(256), 0, st, batch, n, V, labels, seed, step, count);
  return hipGetLastError();
}

// labels[v][w] = OR over the `group` rows v*group .. v*group+group-1 of rows
__global__ void k_or_groups(const uint32_t* __restrict__ rows, int V, int group, int64_t words,
                            uint32_t* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)V * words;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = e / words, w = e % words;
    uint32_t b = 0;
    for (int k = 0; k < group; ++k) b |= rows[((int64_t)v * group + k) * words + w];
    out[e] = b;
  }
}

hipError_t launch_or_groups(const uint32_t* rows, int V, int group, int64_t words, uint32_t* out, hipStream_t st) {
  const unsigned grid = (unsigned)std::min<int64_t>(((int64_t)V * words + 255) / 256, 65536);
  hipLaunchKernelGGL(k_or_groups, dim3(grid), dim3(256), 0, st, rows, V, group, words, out);
  return hipGetLastError();
}

size_t train_smem_bytes() { return sizeof(TrainSmem); }
int train_num_params(int width) { return kIn * width + width + 2 * (width * width + width) + width + 1; }

hipError_t launch_view_gam(const nvgs_camera* views, int V, float cam_scale, float train_focal, float d_max,
                           float* gam, hipStream_t st) {
  hipLaunchKernelGGL(k_view_gam, dim3((V + 63) / 64), dim3(64), 0, st, views, V, cam_scale, train_focal, d_max, gam);
  return hipGetLastError();
}

hipError_t launch_label_bits(const float* contrib, int64_t n, int V, float thr, uint32_t* bits, hipStream_t st) {
  const int64_t total = (int64_t)V * ((n + 31) / 32);
  const unsigned grid = (unsigned)std::min<int64_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(k_label_bits, dim3(grid), dim3(256), 0, st, contrib, n, V, thr, bits);
  return hipGetLastError();
}

template <bool BF16R, int MODE>
static hipError_t launch_mlp_t(int nwg, int cpw, hipStream_t st, const float* params, int64_t batch, float inv_batch,
                               const float* mean, int64_t n, float msc, const float* gam, int V, const uint32_t* labels,
                               uint64_t seed, int64_t step, const uint32_t* n_pos, const float* X,
                               const float* dlogits, float* logits, float* partial, float* loss_part, float* dX) {
  auto kern = k_mlp_train<BF16R, MODE>;
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(TrainSmem));
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL(kern, dim3(nwg), dim3(256), sizeof(TrainSmem), st, params, batch, cpw, inv_batch, mean, n, msc,
                     gam, V, labels, seed, step, n_pos, X, dlogits, logits, partial, loss_part, dX);
  return hipGetLastError();
}

// mode: 0 train (sampled pairs, BCE), 1 forward (logits), 2 backward (given dlogits)
hipError_t launch_mlp_train(int mode, bool bf16, int width, int nwg, hipStream_t st, const float* params,
                            int64_t batch, float inv_batch, const float* mean, int64_t n, float mean_scale,
                            const float* view_gam, int V, const uint32_t* labels, uint64_t seed, int64_t step,
                            const uint32_t* n_pos, const float* X, const float* dlogits, float* logits,
                            float* partial, float* loss_part, float* dX) {
  constexpr int kPairsPerWG = 256;
  if (bf16 || width != 64)
    return launch_mlp_train_w(mode, bf16, width, nwg, kPairsPerWG, st, params, batch, inv_batch, mean, n,
                              mean_scale, view_gam, V, labels, seed, step, n_pos, X, dlogits, logits, partial,
                              loss_part, dX);
  const int chunks_per_wg = kPairsPerWG / kTP;
#define NVGS_MLPT(B, M)                                                                                             \
  return launch_mlp_t<B, M>(nwg, chunks_per_wg, st, params, batch, inv_batch, mean, n, mean_scale, view_gam, V,   \
                            labels, seed, step, n_pos, X, dlogits, logits, partial, loss_part, dX)
  if (mode == 0) NVGS_MLPT(false, 0);
  if (mode == 1) NVGS_MLPT(false, 1);
  NVGS_MLPT(false, 2);
#undef NVGS_MLPT
}

constexpr int kSlices = 32;  // first-level slices of a two-level gradient sum

size_t reduce_scratch_floats(int nwg, int np) { return nwg > 2 * kSlices ? (size_t)kSlices * (np + 1) : 0; }

hipError_t launch_reduce_adam_n(const float* partial, int nwg, int np, float* params, float* m, float* v,
                                float* grad_out, float lr, float b1, float b2, float eps, int64_t t,
                                const float* loss_part, float inv_batch, float* loss_out, hipStream_t st,
                                float* slices) {
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  if (slices && reduce_scratch_floats(nwg, np) > 0) {
    // two levels: kSlices contiguous slices of the partials, then the slices in order
    float* tmp = slices;
    float* tmp_loss = slices + (size_t)kSlices * np;
    hipLaunchKernelGGL(k_reduce_slices, dim3((np + 255) / 256, kSlices), dim3(256), 0, st, partial, nwg, np, kSlices,
                       loss_part, tmp, tmp_loss);
    partial = tmp;
    nwg = kSlices;
    loss_part = loss_part ? tmp_loss : nullptr;
  }
  hipLaunchKernelGGL(k_reduce_adam, dim3((np + 255) / 256), dim3(256), 0, st, partial, nwg, np, params, m, v,
                     grad_out, lr, b1, b2, eps, c1, c2, loss_part, inv_batch, loss_out);
  return hipGetLastError();
}

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (cur != device) (void)hipSetDevice(cur);
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = static_cast<float*>(p);
  return hipSuccess;
}

float* static_scratch(int device, size_t* floats) {
  if (floats) *floats = kStaticScratchFloats;
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

hipError_t launch_reduce_adam(const float* partial, int nwg, float* params, float* m, float* v, float* grad_out,
                              float lr, float b1, float b2, float eps, int64_t t, const float* loss_part,
                              float inv_batch, float* loss_out, hipStream_t st) {
  return launch_reduce_adam_n(partial, nwg, kNumParams, params, m, v, grad_out, lr, b1, b2, eps, t, loss_part,
                              inv_batch, loss_out, st, nullptr);
}

}  // namespace nvgs
