// Training of the visibility MLP (Sec. 3.1-3.2) on BF16 matrix cores, at
// widths 64 and 128, and at width 128 in FP32.
//
// The same algorithm as the FP32 width-64 kernel (sampled pairs, frequency
// encoding, BCE with logits, hand-written backward dW = delta^T h and
// delta_prev = (delta W) * relu', per-work-group partial gradients summed in
// a fixed order by the reduction + Adam kernels), with every GEMM of the
// forward and backward pass on v_mfma_f32_32x32x16_bf16 (BF16 operands,
// FP32 accumulation) or v_mfma_f32_32x32x2f32.
//
// Work-group: 256 threads (4 waves) take chunks of P pairs (P = 64 at width
// 64, 32 at width 128 so that the BF16 weights and activations fit in LDS).
// Every output of a GEMM is a set of 32x32 tiles spread over the waves.
// Activations are stored pair-major ([pair][feature]); an MFMA operand whose
// depth runs along a stored row is one 16-byte LDS read per lane, the others
// (the transposed weights of the backward deltas, both operands of the
// weight gradients, whose depth is the pair) are gathered element-wise.
// BF16: weights are rounded to BF16 when staged in LDS; activations and
// deltas when stored; the output layer (a dot product of FP32 h3 with wo),
// the biases and the loss stay FP32.  FP32 at width 128: the weights stay in
// global memory (L2-resident; they do not fit in LDS in FP32).
#include <algorithm>
#include <type_traits>

#include "internal.h"

namespace nvgs {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kInF = 72;  // encoded inputs

__device__ __forceinline__ uint64_t splitmix64_w(uint64_t seed, uint64_t i) {
  // SplitMix64 (Steele, Lea, Flood 2014): the i-th output for a seed
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <int W, bool BF16>
struct Cfg {
  using T = typename std::conditional<BF16, __bf16, float>::type;
  static constexpr int P = W == 128 ? 32 : 64;         // pairs per chunk
  static constexpr int K0 = BF16 ? 80 : kInF;          // input depth padded to the MFMA depth
  static constexpr int KB = BF16 ? 16 : 2;             // MFMA depth
  static constexpr int PAD = BF16 ? 8 : 1;             // row padding (elements) against bank conflicts
  static constexpr int LG = K0 + PAD;                  // row of G and W1
  static constexpr int LH = W + PAD;                   // row of H1, H2, D, D2, W2, W3
  static constexpr int LF = W + 1;                     // row of the FP32 H3
  static constexpr bool WLDS = BF16;                   // weights staged in LDS
  static constexpr int NP = kInF * W + W + 2 * (W * W + W) + W + 1;
  // LDS: T arrays, then FP32 arrays
  static constexpr int nW1 = WLDS ? W * LG : 0;
  static constexpr int nW = WLDS ? W * LH : 0;
  static constexpr int oW1 = 0, oW2 = oW1 + nW1, oW3 = oW2 + nW, oG = oW3 + nW;
  static constexpr int oH1 = oG + P * LG, oH2 = oH1 + P * LH, oD = oH2 + P * LH, oD2 = oD + P * LH;
  static constexpr int nT = oD2 + P * LH;
  static constexpr size_t tbytes = ((size_t)nT * sizeof(T) + 15) & ~(size_t)15;
  static constexpr int fH3 = 0, fB = fH3 + P * LF, fBo = fB + 4 * W, fDz = fBo + 4, fRed = fDz + P;
  static constexpr int nF = fRed + 256;
  static constexpr size_t bytes = tbytes + (size_t)nF * sizeof(float);
  static_assert(bytes <= 160 * 1024, "LDS budget");
};

__device__ __forceinline__ int acc_row_w(int i) { return 8 * (i / 4) + 4 * ((threadIdx.x & 63) >> 5) + (i % 4); }

// acc += A[32 rows][K] B[K][32 cols] for this wave's 32x32 tile: element (m, k)
// of A at a[m * sam + k * sak], element (k, n) of B at b[k * sbk + n * sbn]
// (offsets relative to the tile origin); K a multiple of the MFMA depth.
// ACONT / BCONT: the 8 BF16 depth elements of a lane are contiguous and
// 16-byte aligned (sak == 1 / sbk == 1).
template <bool BF16, bool ACONT, bool BCONT, class TA, class TB>
__device__ __forceinline__ f32x16 mma_tile(f32x16 acc, const TA* __restrict__ a, int sam, int sak,
                                           const TB* __restrict__ b, int sbk, int sbn, int K) {
  const int l = threadIdx.x & 63, r = l & 31, h = l >> 5;
  if constexpr (BF16) {
    for (int k = 0; k < K; k += 16) {
      const TA* pa = a + r * sam + (k + 8 * h) * sak;
      const TB* pb = b + (k + 8 * h) * sbk + r * sbn;
      bf16x8 av, bv;
      if constexpr (ACONT) {
        av = *reinterpret_cast<const bf16x8*>(pa);
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) av[j] = pa[j * sak];
      }
      if constexpr (BCONT) {
        bv = *reinterpret_cast<const bf16x8*>(pb);
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) bv[j] = pb[j * sbk];
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
    }
  } else {
#pragma unroll 4
    for (int k = 0; k < K; k += 2)
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[r * sam + (k + h) * sak], b[(k + h) * sbk + r * sbn], acc, 0, 0,
                                                  0);
  }
  return acc;
}

}  // namespace

template <int W, bool BF16, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_mlp_train_w(
    const float* __restrict__ params, int64_t batch, int chunks_per_wg, float inv_batch,
    const float* __restrict__ mean, int64_t n, float mean_scale, const float* __restrict__ view_gam, int V,
    const uint32_t* __restrict__ labels, uint64_t seed, int64_t step, const uint32_t* __restrict__ n_pos,
    const float* __restrict__ X, const float* __restrict__ dlogits, float* __restrict__ logits,
    float* __restrict__ partial, float* __restrict__ loss_part, float* __restrict__ dX) {
  using C = Cfg<W, BF16>;
  using T = typename C::T;
  constexpr int P = C::P, K0 = C::K0, LG = C::LG, LH = C::LH, LF = C::LF;
  constexpr int MT = W / 32;           // row tiles of a width-W output
  constexpr int PT = P / 32;           // pair tiles
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  T* S = reinterpret_cast<T*>(smem_raw);
  float* F = reinterpret_cast<float*>(smem_raw + C::tbytes);
  float* sH3 = F + C::fH3;
  float* sB = F + C::fB;  // b1, b2, b3, wo
  float* sDz = F + C::fDz;
  T* sG = S + C::oG;
  T* sH1 = S + C::oH1;
  T* sH2 = S + C::oH2;
  T* sD = S + C::oD;
  T* sD2 = S + C::oD2;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const float* gW1 = params;
  const float* gb1 = gW1 + W * kInF;
  const float* gW2 = gb1 + W;
  const float* gb2 = gW2 + W * W;
  const float* gW3 = gb2 + W;
  const float* gb3 = gW3 + W * W;
  const float* gwo = gb3 + W;
  // weights (as the MFMA operands see them): row-major, W1 [W][K0] with zero
  // padding; LDS copies rounded to BF16, or the FP32 parameters in place
  const T* W1;
  const T* W2;
  const T* W3;
  int ldw1, ldw;
  if constexpr (C::WLDS) {
    T* w1 = S + C::oW1;
    T* w2 = S + C::oW2;
    T* w3 = S + C::oW3;
    for (int i = t; i < W * K0; i += 256) {
      const int m = i / K0, k = i % K0;
      w1[m * LG + k] = (T)(k < kInF ? gW1[m * kInF + k] : 0.f);
    }
    for (int i = t; i < W * W; i += 256) {
      w2[(i / W) * LH + i % W] = (T)gW2[i];
      w3[(i / W) * LH + i % W] = (T)gW3[i];
    }
    W1 = w1; W2 = w2; W3 = w3;
    ldw1 = LG; ldw = LH;
  } else {
    W1 = reinterpret_cast<const T*>(gW1);
    W2 = reinterpret_cast<const T*>(gW2);
    W3 = reinterpret_cast<const T*>(gW3);
    ldw1 = kInF; ldw = W;
  }
  for (int i = t; i < W; i += 256) {
    sB[i] = gb1[i];
    sB[W + i] = gb2[i];
    sB[2 * W + i] = gb3[i];
    sB[3 * W + i] = gwo[i];
  }
  const float bo = gwo[W];
  // gradient accumulators (persist across chunks): dW2, dW3 [W][W] in
  // (W/32)^2 tiles, dW1 [W][72] in (W/32) x 3 tiles; tile u of this wave is
  // tile index wave + 4 u
  constexpr int NT2 = MT * MT / 4 > 0 ? MT * MT / 4 : 1;
  constexpr int NT1 = (MT * 3 + 3) / 4;
  f32x16 dW2[NT2], dW3[NT2], dW1[NT1];
#pragma unroll
  for (int u = 0; u < NT2; ++u) dW2[u] = dW3[u] = (f32x16){0};
#pragma unroll
  for (int u = 0; u < NT1; ++u) dW1[u] = (f32x16){0};
  float db1 = 0.f, db2 = 0.f, db3 = 0.f, dwo = 0.f, dbo = 0.f, loss = 0.f;  // thread t < W owns feature t
  __shared__ int s_g[64], s_v[64];
  __syncthreads();

  // one forward layer: H_out[p][m] = relu(Wl[m][:] . H_in[p][:] + b[m]) over
  // the (W/32) x (P/32) output tiles (rows m, columns p)
  auto layer = [&](const T* Wl, int ldwl, const T* Hin, int ldin, int K, const float* bias, T* Hout, float* Hf) {
    for (int tile = wave; tile < MT * PT; tile += 4) {
      const int m0 = (tile / PT) * 32, p0 = (tile % PT) * 32;
      f32x16 a = mma_tile<BF16, true, true>((f32x16){0}, Wl + m0 * ldwl, ldwl, 1, Hin + p0 * ldin, 1, ldin, K);
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int m = m0 + acc_row_w(i), p = p0 + (lane & 31);
        const float h = fmaxf(a[i] + bias[m], 0.f);
        if (Hf) Hf[p * LF + m] = h;
        else Hout[p * LH + m] = (T)h;
      }
    }
  };

  for (int ch = 0; ch < chunks_per_wg; ++ch) {
    const int64_t base = ((int64_t)blockIdx.x * chunks_per_wg + ch) * P;
    // ---- inputs G [pair][K0]
    if (MODE == kModeTrainW) {
      if (t < P) {
        const uint64_t r = splitmix64_w(seed, (uint64_t)step * (uint64_t)batch + (uint64_t)(base + t));
        s_g[t] = (int)(((r & 0xffffffffull) * (uint64_t)n) >> 32);
        s_v[t] = (int)(((r >> 32) * (uint64_t)V) >> 32);
      }
      __syncthreads();
      for (int e = t; e < P * K0; e += 256) {
        const int p = e / K0, c = e % K0;
        float v = 0.f;
        if (c < 36) {
          const int j = c / 12, band = (c % 12) / 2;
          const float x = ldexpf(mean_scale * mean[j * n + s_g[p]], band);
          v = (c & 1) ? cospif(x) : sinpif(x);
        } else if (c < kInF) {
          v = view_gam[(int64_t)s_v[p] * 36 + (c - 36)];
        }
        sG[p * LG + c] = (T)v;
      }
      if (t < P) {
        const int g = s_g[t], v = s_v[t];
        const int64_t words = (n + 31) / 32;
        sDz[t] = (float)((labels[(int64_t)v * words + (g >> 5)] >> (g & 31)) & 1u);  // label y for now
      }
    } else {
      for (int e = t; e < P * K0; e += 256) {
        const int p = e / K0, c = e % K0;
        const int64_t gi = base + p;
        sG[p * LG + c] = (T)(gi < batch && c < kInF ? X[gi * kInF + c] : 0.f);
      }
    }
    __syncthreads();
    // ---- forward
    layer(W1, ldw1, sG, LG, K0, sB, sH1, nullptr);
    __syncthreads();
    layer(W2, ldw, sH1, LH, W, sB + W, sH2, nullptr);
    __syncthreads();
    layer(W3, ldw, sH2, LH, W, sB + 2 * W, nullptr, sH3);
    __syncthreads();
    // ---- output layer, loss, dz
    if (t < P) {
      float z = bo;
      for (int m = 0; m < W; ++m) z = fmaf(sB[3 * W + m], sH3[t * LF + m], z);
      const int64_t gi = base + t;
      const bool live = gi < batch;
      float d = 0.f;
      if (MODE == kModeTrainW && live) {
        const float y = sDz[t];
        float w = 1.f;  // frequency weighting: B / (2 n_class)
        if (n_pos) {
          const float np_ = (float)*n_pos, nn_ = (float)batch - np_;
          const float wc = y > 0.5f ? np_ : nn_;
          w = wc > 0.f ? 0.5f * (float)batch / wc : 0.f;
        }
        const float sig = 1.f / (1.f + expf(-z));
        loss += w * (fmaxf(z, 0.f) - z * y + log1pf(expf(-fabsf(z))));
        d = w * (sig - y) * inv_batch;
      } else if (MODE == kModeBackwardW) {
        d = live ? dlogits[gi] : 0.f;
      } else if (live) {
        logits[gi] = z;
      }
      sDz[t] = d;
    }
    if (MODE == kModeForwardW) {
      __syncthreads();
      continue;
    }
    __syncthreads();
    // ---- d3 = dz wo * 1[h3 > 0]
    for (int e = t; e < P * W; e += 256) {
      const int p = e / W, m = e % W;
      const float h = sH3[p * LF + m];
      sD[p * LH + m] = (T)(h > 0.f ? sDz[p] * sB[3 * W + m] : 0.f);
    }
    if (t < W) {
      float s = 0.f;
      for (int p = 0; p < P; ++p) s = fmaf(sDz[p], sH3[p * LF + t], s);
      dwo += s;
    }
    if (t == 0)
      for (int p = 0; p < P; ++p) dbo += sDz[p];
    __syncthreads();
    // dW3 += d3^T h2 (depth: the pairs); db3
#pragma unroll
    for (int u = 0; u < NT2; ++u) {
      const int tile = wave + 4 * u;
      if (tile >= MT * MT) break;
      const int m0 = (tile / MT) * 32, n0 = (tile % MT) * 32;
      dW3[u] = mma_tile<BF16, false, false>(dW3[u], sD + m0, 1, LH, sH2 + n0, LH, 1, P);
    }
    if (t < W) {
      float s = 0.f;
      for (int p = 0; p < P; ++p) s += (float)sD[p * LH + t];
      db3 += s;
    }
    // d2[p][j] = (sum_m d3[p][m] W3[m][j]) * 1[h2 > 0]: tiles of d2^T (rows j)
    for (int tile = wave; tile < MT * PT; tile += 4) {
      const int j0 = (tile / PT) * 32, p0 = (tile % PT) * 32;
      f32x16 a = mma_tile<BF16, false, true>((f32x16){0}, W3 + j0, 1, ldw, sD + p0 * LH, 1, LH, W);
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int j = j0 + acc_row_w(i), p = p0 + (lane & 31);
        sD2[p * LH + j] = (T)((float)sH2[p * LH + j] > 0.f ? a[i] : 0.f);
      }
    }
    __syncthreads();
    // dW2 += d2^T h1; db2
#pragma unroll
    for (int u = 0; u < NT2; ++u) {
      const int tile = wave + 4 * u;
      if (tile >= MT * MT) break;
      const int m0 = (tile / MT) * 32, n0 = (tile % MT) * 32;
      dW2[u] = mma_tile<BF16, false, false>(dW2[u], sD2 + m0, 1, LH, sH1 + n0, LH, 1, P);
    }
    if (t < W) {
      float s = 0.f;
      for (int p = 0; p < P; ++p) s += (float)sD2[p * LH + t];
      db2 += s;
    }
    // d1 = (d2 W2) * 1[h1 > 0], into sD (d3 is no longer read once every
    // wave is past the barrier below)
    {
      f32x16 acc[(MT * PT + 3) / 4];
#pragma unroll
      for (int u = 0; u < (MT * PT + 3) / 4; ++u) {
        const int tile = wave + 4 * u;
        if (tile >= MT * PT) break;
        const int j0 = (tile / PT) * 32, p0 = (tile % PT) * 32;
        acc[u] = mma_tile<BF16, false, true>((f32x16){0}, W2 + j0, 1, ldw, sD2 + p0 * LH, 1, LH, W);
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < (MT * PT + 3) / 4; ++u) {
        const int tile = wave + 4 * u;
        if (tile >= MT * PT) break;
        const int j0 = (tile / PT) * 32, p0 = (tile % PT) * 32;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int j = j0 + acc_row_w(i), p = p0 + (lane & 31);
          sD[p * LH + j] = (T)((float)sH1[p * LH + j] > 0.f ? acc[u][i] : 0.f);
        }
      }
    }
    __syncthreads();
    // dW1 += d1^T G: columns 0..95 in three tiles (columns >= 72 are not parameters)
#pragma unroll
    for (int u = 0; u < NT1; ++u) {
      const int tile = wave + 4 * u;
      if (tile >= MT * 3) break;
      const int m0 = (tile / 3) * 32, c0 = (tile % 3) * 32;
      if (c0 + 32 <= K0) {
        dW1[u] = mma_tile<BF16, false, false>(dW1[u], sD + m0, 1, LH, sG + c0, LG, 1, P);
      } else {
        // last tile: columns 64..95; beyond K0 the operand reads as zero
        const int c = c0 + (lane & 31);
        const T* gcol = c < K0 ? sG + c0 : sG;  // any in-bounds column; its values are masked below
        if constexpr (BF16) {
          const int h = lane >> 5;
          for (int k = 0; k < P; k += 16) {
            bf16x8 av, bv;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
              av[j] = sD[(k + 8 * h + j) * LH + m0 + (lane & 31)];
              bv[j] = c < K0 ? gcol[(k + 8 * h + j) * LG + (lane & 31)] : (__bf16)0.f;
            }
            dW1[u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, dW1[u], 0, 0, 0);
          }
        } else {
          const int h = lane >> 5;
          for (int k = 0; k < P; k += 2) {
            const float av = sD[(k + h) * LH + m0 + (lane & 31)];
            const float bv = c < K0 ? (float)gcol[(k + h) * LG + (lane & 31)] : 0.f;
            dW1[u] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, dW1[u], 0, 0, 0);
          }
        }
      }
    }
    if (t < W) {
      float s = 0.f;
      for (int p = 0; p < P; ++p) s += (float)sD[p * LH + t];
      db1 += s;
    }
    // dX[p][c] = sum_m d1[p][m] W1[m][c] (backward mode): tiles of dX^T, rows c < 72
    if (MODE == kModeBackwardW && dX) {
      for (int tile = wave; tile < 3 * PT; tile += 4) {
        const int c0 = (tile / PT) * 32, p0 = (tile % PT) * 32;
        const int rows = (c0 + 32 <= K0) ? 32 : K0 - c0;  // A rows beyond K0 read as zero
        f32x16 a = (f32x16){0};
        if constexpr (BF16) {
          const int h = lane >> 5, r = lane & 31;
          for (int k = 0; k < W; k += 16) {
            bf16x8 av, bv;
#pragma unroll
            for (int j = 0; j < 8; ++j) av[j] = r < rows ? W1[(k + 8 * h + j) * ldw1 + c0 + r] : (__bf16)0.f;
            bv = *reinterpret_cast<const bf16x8*>(sD + (p0 + r) * LH + k + 8 * h);
            a = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, a, 0, 0, 0);
          }
        } else {
          const int h = lane >> 5, r = lane & 31;
          for (int k = 0; k < W; k += 2) {
            const float av = r < rows ? (float)W1[(k + h) * ldw1 + c0 + r] : 0.f;
            const float bv = sD[(p0 + r) * LH + k + h];
            a = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, a, 0, 0, 0);
          }
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int c = c0 + acc_row_w(i);
          const int64_t gi = base + p0 + (lane & 31);
          if (c < kInF && gi < batch) dX[gi * kInF + c] = a[i];
        }
      }
    }
    __syncthreads();
  }
  if (MODE == kModeForwardW) return;
  // ---- this work-group's partial gradients, in the parameter layout
  float* out = partial + (int64_t)blockIdx.x * C::NP;
  float* oW1 = out;
  float* ob1 = oW1 + W * kInF;
  float* oW2 = ob1 + W;
  float* ob2 = oW2 + W * W;
  float* oW3 = ob2 + W;
  float* ob3 = oW3 + W * W;
  float* owo = ob3 + W;
#pragma unroll
  for (int u = 0; u < NT2; ++u) {
    const int tile = wave + 4 * u;
    if (tile >= MT * MT) break;
    const int m0 = (tile / MT) * 32, n0 = (tile % MT) * 32;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int m = m0 + acc_row_w(i), c = n0 + (lane & 31);
      oW2[m * W + c] = dW2[u][i];
      oW3[m * W + c] = dW3[u][i];
    }
  }
#pragma unroll
  for (int u = 0; u < NT1; ++u) {
    const int tile = wave + 4 * u;
    if (tile >= MT * 3) break;
    const int m0 = (tile / 3) * 32, c0 = (tile % 3) * 32;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int m = m0 + acc_row_w(i), c = c0 + (lane & 31);
      if (c < kInF) oW1[m * kInF + c] = dW1[u][i];
    }
  }
  if (t < W) {
    ob1[t] = db1;
    ob2[t] = db2;
    ob3[t] = db3;
    owo[t] = dwo;
  }
  if (t == 0) owo[W] = dbo;
  if (MODE == kModeTrainW) {
    float* red = F + C::fRed;
    red[t] = loss;
    __syncthreads();
    if (t == 0) {
      float s = 0.f;
      for (int k = 0; k < 256; ++k) s += red[k];
      loss_part[blockIdx.x] = s;
    }
  }
}

template <int W, bool BF16, int MODE>
static hipError_t launch_w(int nwg, int cpw, hipStream_t st, const float* params, int64_t batch, float inv_batch,
                           const float* mean, int64_t n, float msc, const float* gam, int V, const uint32_t* labels,
                           uint64_t seed, int64_t step, const uint32_t* n_pos, const float* X, const float* dlogits,
                           float* logits, float* partial, float* loss_part, float* dX) {
  using C = Cfg<W, BF16>;
  auto kern = k_mlp_train_w<W, BF16, MODE>;
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)C::bytes);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL(kern, dim3(nwg), dim3(256), C::bytes, st, params, batch, cpw, inv_batch, mean, n, msc, gam, V,
                     labels, seed, step, n_pos, X, dlogits, logits, partial, loss_part, dX);
  return hipGetLastError();
}

int train_pairs_per_chunk(int width, bool bf16) {
  return width == 128 ? Cfg<128, true>::P : (bf16 ? Cfg<64, true>::P : 64);
}

// width 64 BF16, width 128 BF16 and FP32; pairs_per_wg a multiple of 64
hipError_t launch_mlp_train_w(int mode, bool bf16, int width, int nwg, int pairs_per_wg, hipStream_t st,
                              const float* params, int64_t batch, float inv_batch, const float* mean, int64_t n,
                              float mean_scale, const float* view_gam, int V, const uint32_t* labels, uint64_t seed,
                              int64_t step, const uint32_t* n_pos, const float* X, const float* dlogits,
                              float* logits, float* partial, float* loss_part, float* dX) {
  const int cpw = pairs_per_wg / train_pairs_per_chunk(width, bf16);
#define NVGS_W(Wd, B, M)                                                                                           \
  return launch_w<Wd, B, M>(nwg, cpw, st, params, batch, inv_batch, mean, n, mean_scale, view_gam, V, labels,    \
                            seed, step, n_pos, X, dlogits, logits, partial, loss_part, dX)
  if (width == 64 && bf16) {
    if (mode == kModeTrainW) NVGS_W(64, true, kModeTrainW);
    if (mode == kModeForwardW) NVGS_W(64, true, kModeForwardW);
    NVGS_W(64, true, kModeBackwardW);
  }
  if (width == 128 && bf16) {
    if (mode == kModeTrainW) NVGS_W(128, true, kModeTrainW);
    if (mode == kModeForwardW) NVGS_W(128, true, kModeForwardW);
    NVGS_W(128, true, kModeBackwardW);
  }
  if (width == 128) {
    if (mode == kModeTrainW) NVGS_W(128, false, kModeTrainW);
    if (mode == kModeForwardW) NVGS_W(128, false, kModeForwardW);
    NVGS_W(128, false, kModeBackwardW);
  }
#undef NVGS_W
  return hipErrorInvalidValue;
}

}  // namespace nvgs
