// Per-frame steps 3-6 of the NVGS renderer (Sec. 3.3, 4.1): instantiate the
// surviving pairs in (camera, instance, Gaussian) order, project them with
// EWA splatting, bin them into screen tiles, and composite front to back.
//
//  * k_project fuses the ordered compaction with the projection: each
//    256-pair chunk knows its output offset from the exclusive scan of the
//    per-chunk keep counts, and each kept lane's slot is that offset plus the
//    popcount of the keep bits before it.  Only survivors are ever read from
//    the asset store or written as splats.
//  * Footprints are the exact AABB of the alpha = 1/255 level set of the
//    splat (not a 3-sigma box), widened slightly, so the image does not
//    depend on the tile size.
//  * k_blend stages batches of 256 splats in LDS and stops a tile as soon as
//    every pixel of it has stopped.
#include <algorithm>
#include <utility>

#include "internal.h"

namespace nvgs {

// ---------------------------------------------------------------------------
// real spherical harmonics (l <= 3, order l-major, m = -l..l, no Condon-
// Shortley phase) evaluated on a unit direction, accumulated into rgb
// ---------------------------------------------------------------------------
__device__ __forceinline__ void sh_color(const float* __restrict__ sh, int64_t n, int64_t g, int degree, float x,
                                         float y, float z, float rgb[3]) {
  // normalisation constants sqrt((2l+1)/(4pi) (l-m)!/(l+m)!) (x sqrt2 for m != 0)
  constexpr float c0 = 0.28209479177387814f;
  constexpr float c1 = 0.48860251190291992f;
  constexpr float c2a = 1.0925484305920792f;   // 0.5 sqrt(15/pi)
  constexpr float c2b = 0.31539156525252005f;  // 0.25 sqrt(5/pi)
  constexpr float c2c = 0.54627421529603959f;  // 0.25 sqrt(15/pi)
  constexpr float c3a = 0.59004358992664352f;  // 0.25 sqrt(35/(2pi))
  constexpr float c3b = 2.8906114426405538f;   // 0.5 sqrt(105/pi)
  constexpr float c3c = 0.45704579946446572f;  // 0.25 sqrt(21/(2pi))
  constexpr float c3d = 0.37317633259011546f;  // 0.25 sqrt(7/pi)
  constexpr float c3e = 1.4453057213202769f;   // 0.25 sqrt(105/pi)
  float Y[16];
  Y[0] = c0;
  int K = 1;
  if (degree >= 1) {
    Y[1] = c1 * y; Y[2] = c1 * z; Y[3] = c1 * x;
    K = 4;
  }
  if (degree >= 2) {
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = c2a * x * y;
    Y[5] = c2a * y * z;
    Y[6] = c2b * (3.f * zz - 1.f);
    Y[7] = c2a * x * z;
    Y[8] = c2c * (xx - yy);
    K = 9;
    if (degree >= 3) {
      Y[9] = c3a * y * (3.f * xx - yy);
      Y[10] = c3b * x * y * z;
      Y[11] = c3c * y * (5.f * zz - 1.f);
      Y[12] = c3d * z * (5.f * zz - 3.f);
      Y[13] = c3c * x * (5.f * zz - 1.f);
      Y[14] = c3e * z * (xx - yy);
      Y[15] = c3a * x * (xx - 3.f * yy);
      K = 16;
    }
  }
  float r = 0.5f, gg = 0.5f, b = 0.5f;
  for (int k = 0; k < K; ++k) {
    const float* p = sh + (int64_t)(3 * k) * n + g;
    r = fmaf(Y[k], p[0], r);
    gg = fmaf(Y[k], p[n], gg);
    b = fmaf(Y[k], p[2 * n], b);
  }
  rgb[0] = fmaxf(r, 0.f);
  rgb[1] = fmaxf(gg, 0.f);
  rgb[2] = fmaxf(b, 0.f);
}

// pixel-rectangle bound of the alpha >= 1/255 set: centres x + 0.5 within
// u -/+ e, widened by 1e-4 e + 1e-3 px (evaluated without FMA contraction)
__device__ __forceinline__ void pixel_range(float u, float e, int size, int* lo, int* hi) {
#pragma clang fp contract(off)
  const float w = 1e-4f * e + 1e-3f;
  float a = ceilf(((u - e) - 0.5f) - w);
  float b = floorf(((u + e) - 0.5f) + w);
  a = fmaxf(a, 0.f);
  b = fminf(b, (float)(size - 1));
  *lo = (int)a;
  *hi = (int)b;
}

__global__ __launch_bounds__(kChunk) void k_project(
    const AssetDev* __restrict__ assets, const SegRec* __restrict__ segs, int32_t n_segs,
    const int64_t* __restrict__ seg_chunk_base, const uint32_t* __restrict__ mask,
    const uint32_t* __restrict__ chunk_off, int64_t cap, int tile, int tiles_x, int tiles_y, int keep_debug,
    float4* __restrict__ rec_a, float4* __restrict__ rec_b, float4* __restrict__ rec_c, uint4* __restrict__ rect,
    uint32_t* __restrict__ depth_key, uint32_t* __restrict__ pair_of, uint32_t* __restrict__ overflow) {
  const int64_t chunk = blockIdx.x;
  // segment of this chunk: last s with seg_chunk_base[s] <= chunk
  int lo = 0, hi = n_segs - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (seg_chunk_base[mid] <= chunk) lo = mid; else hi = mid - 1;
  }
  const SegRec& R = segs[lo];
  const int64_t c = chunk - seg_chunk_base[lo];
  const int t = threadIdx.x;
  const int64_t g = c * kChunk + t;
  const int64_t n = R.n;
  const int64_t words = (n + 31) >> 5;
  __shared__ uint32_t s_w[kChunk / 32];
  if (t < kChunk / 32) {
    const int64_t wi = c * (kChunk / 32) + t;
    s_w[t] = wi < words ? mask[R.word_base + wi] : 0u;
  }
  __syncthreads();
  const uint32_t word = s_w[t >> 5];
  if (!((word >> (t & 31)) & 1u)) return;
  uint32_t before = __popc(word & ((1u << (t & 31)) - 1u));
  for (int w = 0; w < (t >> 5); ++w) before += __popc(s_w[w]);
  const uint32_t slot = chunk_off[chunk] + before;
  if (slot >= cap) {
    atomicOr(overflow, 1u);
    return;
  }
  const AssetDev& A = assets[R.asset];
  const float mu[3] = {A.mean[g], A.mean[n + g], A.mean[2 * n + g]};
  const float s3[3] = {A.scale[g], A.scale[n + g], A.scale[2 * n + g]};
  float qw = A.quat[g], qx = A.quat[n + g], qy = A.quat[2 * n + g], qz = A.quat[3 * n + g];
  const float o = A.opacity[g];
  // camera space
  const float* M = R.M;
  const float px = fmaf(M[0], mu[0], fmaf(M[1], mu[1], fmaf(M[2], mu[2], M[3])));
  const float py = fmaf(M[4], mu[0], fmaf(M[5], mu[1], fmaf(M[6], mu[2], M[7])));
  const float pz = fmaf(M[8], mu[0], fmaf(M[9], mu[1], fmaf(M[10], mu[2], M[11])));
  const float f = R.focal;
  const float iz = 1.f / pz;
  // perspective Jacobian at the guard-clamped tangent position
  const float txz = fminf(R.tanx_g, fmaxf(-R.tanx_g, px * iz)) * pz;
  const float tyz = fminf(R.tany_g, fmaxf(-R.tany_g, py * iz)) * pz;
  const float j00 = f * iz, j02 = -f * txz * iz * iz;
  const float j11 = f * iz, j12 = -f * tyz * iz * iz;
  // T = J * M3 (M3 = s_i Rc Ri)
  float T0[3], T1[3];
  for (int k = 0; k < 3; ++k) {
    T0[k] = fmaf(j00, M[k], j02 * M[8 + k]);
    T1[k] = fmaf(j11, M[4 + k], j12 * M[8 + k]);
  }
  // rotation of the normalised quaternion, columns scaled by the std devs
  const float qn = rsqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
  qw *= qn; qx *= qn; qy *= qn; qz *= qn;
  const float Rq[9] = {1.f - 2.f * (qy * qy + qz * qz), 2.f * (qx * qy - qw * qz), 2.f * (qx * qz + qw * qy),
                       2.f * (qx * qy + qw * qz), 1.f - 2.f * (qx * qx + qz * qz), 2.f * (qy * qz - qw * qx),
                       2.f * (qx * qz - qw * qy), 2.f * (qy * qz + qw * qx), 1.f - 2.f * (qx * qx + qy * qy)};
  // V = T Rq S, Sigma2D = V V^T + 0.3 I
  float V0[3], V1[3];
  for (int k = 0; k < 3; ++k) {
    V0[k] = (T0[0] * Rq[k] + T0[1] * Rq[3 + k] + T0[2] * Rq[6 + k]) * s3[k];
    V1[k] = (T1[0] * Rq[k] + T1[1] * Rq[3 + k] + T1[2] * Rq[6 + k]) * s3[k];
  }
  const float a0 = V0[0] * V0[0] + V0[1] * V0[1] + V0[2] * V0[2];
  const float c0 = V1[0] * V1[0] + V1[1] * V1[1] + V1[2] * V1[2];
  const float b = V0[0] * V1[0] + V0[1] * V1[1] + V0[2] * V1[2];
  const float a = a0 + kDilate, cc = c0 + kDilate;
  // det(V V^T + 0.3 I) = |V0 x V1|^2 + 0.3 (|V0|^2 + |V1|^2) + 0.09: a sum of
  // non-negative terms (Lagrange identity), free of the cancellation in ac - b^2
  const float x0 = V0[1] * V1[2] - V0[2] * V1[1];
  const float x1 = V0[2] * V1[0] - V0[0] * V1[2];
  const float x2 = V0[0] * V1[1] - V0[1] * V1[0];
  const float det = (x0 * x0 + x1 * x1 + x2 * x2) + kDilate * (a0 + c0) + kDilate * kDilate;
  float ca, cb, cc2;
  if (a * cc > 1024.f * det) {
    // near-degenerate (condition number above 1024): invert in FP64 from the
    // exact products of the FP32 rows
    double v0[3], v1[3];
    for (int k = 0; k < 3; ++k) { v0[k] = V0[k]; v1[k] = V1[k]; }
    const double da = v0[0] * v0[0] + v0[1] * v0[1] + v0[2] * v0[2] + 0.3;
    const double dc = v1[0] * v1[0] + v1[1] * v1[1] + v1[2] * v1[2] + 0.3;
    const double db = v0[0] * v1[0] + v0[1] * v1[1] + v0[2] * v1[2];
    const double dd = da * dc - db * db;
    ca = (float)(dc / dd);
    cb = (float)(-db / dd);
    cc2 = (float)(da / dd);
  } else {
    const float id = 1.f / det;
    ca = cc * id;
    cb = -b * id;
    cc2 = a * id;
  }
  const float u = fmaf(f * px, iz, R.half_w);
  const float v = fmaf(f * py, iz, R.half_h);
  // colour: SH along the camera -> Gaussian direction in the asset frame
  float dx = mu[0] - R.cl[0], dy = mu[1] - R.cl[1], dz = mu[2] - R.cl[2];
  const float dn = rsqrtf(dx * dx + dy * dy + dz * dz);
  float rgb[3];
  sh_color(A.sh, n, g, A.sh_degree, dx * dn, dy * dn, dz * dn, rgb);
  // footprint
  const float k2 = 2.f * logf(255.f * o);
  const int W = (int)(2.f * R.half_w), H = (int)(2.f * R.half_h);
  float ex = 0.f, ey = 0.f;
  uint32_t r0 = 0, r1 = 0, ntiles = 0;
  if (k2 >= 0.f) {
    ex = sqrtf(k2 * a);
    ey = sqrtf(k2 * cc);
    int x0, x1, y0, y1;
    pixel_range(u, ex, W, &x0, &x1);
    pixel_range(v, ey, H, &y0, &y1);
    if (x0 <= x1 && y0 <= y1) {
      const int tx0 = x0 / tile, tx1 = x1 / tile, ty0 = y0 / tile, ty1 = y1 / tile;
      r0 = (uint32_t)tx0 | ((uint32_t)ty0 << 16);
      r1 = (uint32_t)tx1 | ((uint32_t)ty1 << 16);
      ntiles = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
    }
  }
  rec_a[slot] = make_float4(u, v, ca, cb);
  rec_b[slot] = make_float4(cc2, o, rgb[0], rgb[1]);
  rec_c[slot] = make_float4(rgb[2], pz, ex, ey);
  rect[slot] = make_uint4(r0, r1, (uint32_t)R.cam, ntiles);
  depth_key[slot] = fbits(pz);
  if (keep_debug) pair_of[slot] = (uint32_t)(R.pair_base + g);
  (void)tiles_x; (void)tiles_y;
}

hipError_t launch_project(const AssetDev* assets, const SegRec* segs, int32_t n_segs, const int64_t* seg_chunk_base,
                          int64_t n_chunks, const uint32_t* mask, const uint32_t* chunk_off, const uint32_t* n_splats,
                          int64_t cap_splats, int tile, int tiles_x, int tiles_y, int keep_debug, float4* rec_a,
                          float4* rec_b, float4* rec_c, uint4* rect, uint32_t* depth_key, uint32_t* pair_of,
                          uint32_t* overflow, hipStream_t st) {
  (void)n_splats;
  if (n_chunks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_project, dim3((unsigned)n_chunks), dim3(kChunk), 0, st, assets, segs, n_segs, seg_chunk_base,
                     mask, chunk_off, cap_splats, tile, tiles_x, tiles_y, keep_debug, rec_a, rec_b, rec_c, rect,
                     depth_key, pair_of, overflow);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// binning
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t live(const uint32_t* n_dev, int64_t cap) {
  return n_dev ? (int64_t)min((uint64_t)*n_dev, (uint64_t)cap) : cap;
}

__global__ void k_gather_tiles(const uint32_t* __restrict__ ids, const uint4* __restrict__ rect,
                               const uint32_t* __restrict__ n_dev, int64_t cap, uint32_t* __restrict__ out) {
  const int64_t n = live(n_dev, cap);
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
    out[j] = rect[ids[j]].w;
}

hipError_t launch_gather_tiles(const uint32_t* sorted_ids, const uint4* rect, const uint32_t* n_dev, int64_t cap,
                               uint32_t* out, hipStream_t st) {
  if (cap == 0) return hipSuccess;
  unsigned grid = (unsigned)std::min<int64_t>((cap + 255) / 256, 65536);
  hipLaunchKernelGGL(k_gather_tiles, dim3(grid), dim3(256), 0, st, sorted_ids, rect, n_dev, cap, out);
  return hipGetLastError();
}

// one thread per splat in depth order: one (tile key, splat id) entry per
// overlapped tile, written at the splat's exclusive offset
__global__ void k_emit(const uint32_t* __restrict__ ids, const uint4* __restrict__ rect,
                       const uint32_t* __restrict__ off, const uint32_t* __restrict__ n_dev, int64_t cap,
                       const uint32_t* __restrict__ n_dup_dev, int64_t cap_dup, int tiles_x, int n_tiles,
                       uint32_t* __restrict__ keys, uint32_t* __restrict__ vals, uint32_t* __restrict__ overflow) {
  const int64_t n = live(n_dev, cap);
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t s = ids[j];
    const uint4 r = rect[s];
    if (r.w == 0) continue;
    int64_t o = off[j];
    if (o + r.w > cap_dup) {
      atomicOr(overflow, 2u);
      continue;
    }
    const int tx0 = r.x & 0xffff, ty0 = r.x >> 16, tx1 = r.y & 0xffff, ty1 = r.y >> 16;
    const uint32_t kb = r.z * (uint32_t)n_tiles;
    for (int ty = ty0; ty <= ty1; ++ty)
      for (int tx = tx0; tx <= tx1; ++tx) {
        keys[o] = kb + (uint32_t)(ty * tiles_x + tx);
        vals[o] = s;
        ++o;
      }
  }
  (void)n_dup_dev;
}

hipError_t launch_emit(const uint32_t* sorted_ids, const uint4* rect, const uint32_t* dup_off, const uint32_t* n_dev,
                       int64_t cap, const uint32_t* n_dup_dev, int64_t cap_dup, int tiles_x, int n_tiles,
                       uint32_t* keys, uint32_t* vals, uint32_t* overflow, hipStream_t st) {
  if (cap == 0) return hipSuccess;
  unsigned grid = (unsigned)std::min<int64_t>((cap + 255) / 256, 65536);
  hipLaunchKernelGGL(k_emit, dim3(grid), dim3(256), 0, st, sorted_ids, rect, dup_off, n_dev, cap, n_dup_dev, cap_dup,
                     tiles_x, n_tiles, keys, vals, overflow);
  return hipGetLastError();
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, int64_t n) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
    p[j] = v;
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}

// [start, end) of every tile key in the sorted list (ranges pre-filled with 0)
__global__ void k_ranges(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ n_dev, int64_t cap,
                         uint32_t* __restrict__ ranges) {
  const int64_t n = live(n_dev, cap);
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t k = keys[j];
    if (j == 0 || keys[j - 1] != k) ranges[2 * (int64_t)k] = (uint32_t)j;
    if (j == n - 1 || keys[j + 1] != k) ranges[2 * (int64_t)k + 1] = (uint32_t)(j + 1);
  }
}

hipError_t launch_ranges(const uint32_t* keys, const uint32_t* n_dev, int64_t cap, uint32_t* ranges, hipStream_t st) {
  if (cap == 0) return hipSuccess;
  unsigned grid = (unsigned)std::min<int64_t>((cap + 255) / 256, 65536);
  hipLaunchKernelGGL(k_ranges, dim3(grid), dim3(256), 0, st, keys, n_dev, cap, ranges);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// front-to-back compositing, one work-group per (camera, tile)
// ---------------------------------------------------------------------------
template <int T, bool RECORD>
__global__ __launch_bounds__(T == 8 ? 64 : 256) void k_blend(
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ ids, const float4* __restrict__ rec_a,
    const float4* __restrict__ rec_b, const float4* __restrict__ rec_c, const uint32_t* __restrict__ pair_of, int W,
    int H, int tiles_x, int n_tiles, float bg0, float bg1, float bg2, float* __restrict__ rgb,
    uint32_t* __restrict__ contrib) {
  constexpr int NT = T == 8 ? 64 : 256;   // threads
  constexpr int PPT = T * T / NT;         // pixels per thread
  constexpr int BATCH = NT;
  constexpr float kLog2e = 1.4426950408889634f;
  __shared__ float s_u[BATCH], s_v[BATCH], s_A[BATCH], s_B[BATCH], s_C[BATCH], s_o[BATCH];
  __shared__ float s_r[BATCH], s_g[BATCH], s_b[BATCH];
  __shared__ uint32_t s_p[RECORD ? BATCH : 1];
  const int key = blockIdx.x;
  const int cam = key / n_tiles, tile = key % n_tiles;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const uint32_t start = ranges[2 * (int64_t)key], end = ranges[2 * (int64_t)key + 1];
  const int t = threadIdx.x;
  float px[PPT], py[PPT], Tr[PPT], cr[PPT], cg[PPT], cb[PPT];
  bool done[PPT];
  int alive = 0;
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    const int lp = t + j * NT;
    const int x = tx * T + lp % T, y = ty * T + lp / T;
    px[j] = (float)x + 0.5f;
    py[j] = (float)y + 0.5f;
    Tr[j] = 1.f;
    cr[j] = cg[j] = cb[j] = 0.f;
    done[j] = !(x < W && y < H);
    alive += done[j] ? 0 : 1;
  }
  for (uint32_t b0 = start; b0 < end; b0 += BATCH) {
    if (__syncthreads_count(alive > 0) == 0) break;
    const uint32_t cnt = min((uint32_t)BATCH, end - b0);
    if (t < (int)cnt) {
      const uint32_t id = ids[b0 + t];
      const float4 A = rec_a[id], B = rec_b[id];
      const float C = rec_c[id].x;
      s_u[t] = A.x;
      s_v[t] = A.y;
      // exponent in base 2: -q/2 * log2(e) with q = d^T conic d
      s_A[t] = -0.5f * kLog2e * A.z;
      s_B[t] = -kLog2e * A.w;
      s_C[t] = -0.5f * kLog2e * B.x;
      s_o[t] = B.y;
      s_r[t] = B.z;
      s_g[t] = B.w;
      s_b[t] = C;
      if (RECORD) s_p[t] = pair_of[id];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      if (done[j]) continue;
      for (uint32_t k = 0; k < cnt; ++k) {
        const float dx = px[j] - s_u[k], dy = py[j] - s_v[k];
        const float pw = s_A[k] * dx * dx + s_B[k] * dx * dy + s_C[k] * dy * dy;
        if (pw > 0.f) continue;
        const float al = fminf(kAlphaMax, s_o[k] * __builtin_amdgcn_exp2f(pw));
        if (al < kAlphaMin) continue;
        const float Tn = Tr[j] * (1.f - al);
        if (Tn < kTMin) {
          done[j] = true;
          --alive;
          break;
        }
        const float w = al * Tr[j];
        cr[j] = fmaf(w, s_r[k], cr[j]);
        cg[j] = fmaf(w, s_g[k], cg[j]);
        cb[j] = fmaf(w, s_b[k], cb[j]);
        if (RECORD) atomicMax(contrib + s_p[k], __float_as_uint(w));
        Tr[j] = Tn;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    const int lp = t + j * NT;
    const int x = tx * T + lp % T, y = ty * T + lp / T;
    if (x < W && y < H) {
      float* o = rgb + (((int64_t)cam * H + y) * W + x) * 3;
      o[0] = fmaf(Tr[j], bg0, cr[j]);
      o[1] = fmaf(Tr[j], bg1, cg[j]);
      o[2] = fmaf(Tr[j], bg2, cb[j]);
    }
  }
}

template <int T>
static void launch_blend_t(bool record, dim3 grid, hipStream_t st, const uint32_t* ranges, const uint32_t* ids,
                           const float4* ra, const float4* rb, const float4* rc, const uint32_t* pair_of, int W, int H,
                           int tiles_x, int n_tiles, float b0, float b1, float b2, float* rgb, float* contrib) {
  constexpr int NT = T == 8 ? 64 : 256;
  if (record)
    hipLaunchKernelGGL((k_blend<T, true>), grid, dim3(NT), 0, st, ranges, ids, ra, rb, rc, pair_of, W, H, tiles_x,
                       n_tiles, b0, b1, b2, rgb, reinterpret_cast<uint32_t*>(contrib));
  else
    hipLaunchKernelGGL((k_blend<T, false>), grid, dim3(NT), 0, st, ranges, ids, ra, rb, rc, pair_of, W, H, tiles_x,
                       n_tiles, b0, b1, b2, rgb, reinterpret_cast<uint32_t*>(contrib));
}

hipError_t launch_blend(const uint32_t* ranges, const uint32_t* ids, const float4* rec_a, const float4* rec_b,
                        const float4* rec_c, const uint32_t* pair_of, int C, int W, int H, int tile, int tiles_x,
                        int tiles_y, float bg0, float bg1, float bg2, float* rgb, float* contrib, int64_t P,
                        const uint4* rect, hipStream_t st) {
  (void)P; (void)rect;
  const int n_tiles = tiles_x * tiles_y;
  dim3 grid((unsigned)(C * n_tiles));
  const bool record = contrib != nullptr;
  if (tile == 8)
    launch_blend_t<8>(record, grid, st, ranges, ids, rec_a, rec_b, rec_c, pair_of, W, H, tiles_x, n_tiles, bg0, bg1,
                      bg2, rgb, contrib);
  else if (tile == 16)
    launch_blend_t<16>(record, grid, st, ranges, ids, rec_a, rec_b, rec_c, pair_of, W, H, tiles_x, n_tiles, bg0, bg1,
                       bg2, rgb, contrib);
  else if (tile == 32)
    launch_blend_t<32>(record, grid, st, ranges, ids, rec_a, rec_b, rec_c, pair_of, W, H, tiles_x, n_tiles, bg0, bg1,
                       bg2, rgb, contrib);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace nvgs
