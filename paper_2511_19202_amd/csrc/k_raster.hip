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
//  * k_blend stages batches of splats (one per thread) in LDS, fetching the
//    next batch while compositing the current one, and stops a tile as soon
//    as every pixel of it has stopped; an 8x8 tile passes over the splats
//    whose footprint box holds none of its live pixels.
#include <algorithm>
#include <utility>

#include <hip/hip_fp16.h>

#include "internal.h"

namespace nvgs {

// ---------------------------------------------------------------------------
// real spherical harmonics (l <= 3, order l-major, m = -l..l, no Condon-
// Shortley phase) evaluated on a unit direction, accumulated into rgb
// ---------------------------------------------------------------------------
// 16-byte load through the global address space (pointers read from a table
// are generic, which would give flat loads)
typedef float f32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 ld_global(const float4* p, int64_t i) {
  const f32x4_t v = ((const __attribute__((address_space(1))) f32x4_t*)p)[i];
  return make_float4(v.x, v.y, v.z, v.w);
}

template <int D, bool SHARED>
__device__ __forceinline__ void sh_color_t(const float4* __restrict__ row, float x, float y, float z, float rgb[3]) {
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
  constexpr int K = (D + 1) * (D + 1);
  constexpr int N4 = (3 * K + 3) / 4;
  // the Gaussian's whole coefficient row in 16-byte loads
  float c[4 * N4];
#pragma unroll
  for (int q = 0; q < N4; ++q) {
    const float4 v = SHARED ? row[q] : ld_global(row, q);
    c[4 * q] = v.x;
    c[4 * q + 1] = v.y;
    c[4 * q + 2] = v.z;
    c[4 * q + 3] = v.w;
  }
  float Y[K];
  Y[0] = c0;
  if (D >= 1) {
    Y[1] = c1 * y; Y[2] = c1 * z; Y[3] = c1 * x;
  }
  if (D >= 2) {
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = c2a * x * y;
    Y[5] = c2a * y * z;
    Y[6] = c2b * (3.f * zz - 1.f);
    Y[7] = c2a * x * z;
    Y[8] = c2c * (xx - yy);
    if (D >= 3) {
      Y[9] = c3a * y * (3.f * xx - yy);
      Y[10] = c3b * x * y * z;
      Y[11] = c3c * y * (5.f * zz - 1.f);
      Y[12] = c3d * z * (5.f * zz - 3.f);
      Y[13] = c3c * x * (5.f * zz - 1.f);
      Y[14] = c3e * z * (xx - yy);
      Y[15] = c3a * x * (xx - 3.f * yy);
    }
  }
  float r = 0.5f, gg = 0.5f, b = 0.5f;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    r = fmaf(Y[k], c[3 * k], r);
    gg = fmaf(Y[k], c[3 * k + 1], gg);
    b = fmaf(Y[k], c[3 * k + 2], b);
  }
  rgb[0] = fmaxf(r, 0.f);
  rgb[1] = fmaxf(gg, 0.f);
  rgb[2] = fmaxf(b, 0.f);
}

// colour of one Gaussian: real SH up to degree 3 (l-major, m = -l..l, no
// Condon-Shortley phase) on the unit view direction, from its packed row (in
// global memory, or in LDS when SHARED)
template <bool SHARED = false>
__device__ __forceinline__ void sh_color(const float4* __restrict__ row, int degree, float x, float y, float z,
                                         float rgb[3]) {
  switch (degree) {
    case 0: sh_color_t<0, SHARED>(row, x, y, z, rgb); break;
    case 1: sh_color_t<1, SHARED>(row, x, y, z, rgb); break;
    case 2: sh_color_t<2, SHARED>(row, x, y, z, rgb); break;
    default: sh_color_t<3, SHARED>(row, x, y, z, rgb); break;
  }
}

int32_t sh_stride_for(int sh_degree) {
  const int k = 3 * (sh_degree + 1) * (sh_degree + 1);
  return (k + 3) & ~3;
}

// SoA asset arrays -> one geometry record and one SH row per Gaussian
__global__ void k_pack_asset(const float* __restrict__ mean, const float* __restrict__ scale,
                             const float* __restrict__ quat, const float* __restrict__ opacity,
                             const float* __restrict__ sh, int64_t n, int K, int stride, float4* __restrict__ geo,
                             float* __restrict__ shp) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x) {
    geo[3 * g] = make_float4(mean[g], mean[n + g], mean[2 * n + g], opacity[g]);
    geo[3 * g + 1] = make_float4(scale[g], scale[n + g], scale[2 * n + g], 0.f);
    geo[3 * g + 2] = make_float4(quat[g], quat[n + g], quat[2 * n + g], quat[3 * n + g]);
    float* row = shp + g * stride;
    for (int c = 0; c < stride; ++c) row[c] = c < K ? sh[(int64_t)c * n + g] : 0.f;
  }
}

hipError_t launch_pack_asset(const float* mean, const float* scale, const float* quat, const float* opacity,
                             const float* sh, int64_t n, int sh_degree, float4* geo, float* shp, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_pack_asset, dim3(grid), dim3(256), 0, st, mean, scale, quat, opacity, sh, n,
                     3 * (sh_degree + 1) * (sh_degree + 1), sh_stride_for(sh_degree), geo, shp);
  return hipGetLastError();
}

// Error-free transformations of FP32 values (Knuth's TwoSum; TwoProduct with
// one FMA): a + b = s + e and a * b = p + e exactly, so that a quantity can be
// carried as an unevaluated sum hi + lo of two floats (about 48 bits).
__device__ __forceinline__ float two_sum(float a, float b, float* e) {
#pragma clang fp contract(off)
  const float s = a + b;
  const float bb = s - a;
  *e = (a - (s - bb)) + (b - bb);
  return s;
}
__device__ __forceinline__ float two_prod(float a, float b, float* e) {
  const float p = a * b;
  *e = fmaf(a, b, -p);
  return p;
}

// one camera-space coordinate (M + Mlo)[0:3] . mu + (M + Mlo)[3] as hi + lo:
// the 3x4 row is the composite s_i Rc Ri | Rc (t_i - c) of the segment, held
// to ~48 bits, so a centre 30 m away keeps its sub-micrometre position
__device__ __forceinline__ float cam_coord(const float* M, const float* Mlo, float m0, float m1, float m2,
                                           float* lo) {
#pragma clang fp contract(off)
  float e0, e1, e2, e3, e4, e5;
  float s = two_prod(M[0], m0, &e0);
  float t = two_prod(M[1], m1, &e1);
  s = two_sum(s, t, &e2);
  t = two_prod(M[2], m2, &e3);
  s = two_sum(s, t, &e4);
  s = two_sum(M[3], s, &e5);
  const float small = fmaf(Mlo[0], m0, fmaf(Mlo[1], m1, fmaf(Mlo[2], m2, Mlo[3])));
  const float l = ((e0 + e1) + (e2 + e3)) + ((e4 + e5) + small);
  const float h = s + l;
  *lo = l - (h - s);
  return h;
}

// pixel coordinate f p / p_z + c of a camera-space position given as hi + lo
// parts, returned as hi + lo: the quotient's remainder is exact with an FMA,
// and the product with the focal length and the offset are error-free
__device__ __forceinline__ float screen_coord(float ph, float pl, float zh, float zl, float fh, float fl, float c,
                                              float* lo) {
#pragma clang fp contract(off)
  const float qh = ph / zh;
  const float r = fmaf(-qh, zh, ph);  // ph - qh zh, exact
  const float ql = fmaf(-qh, zl, r + pl) / zh;
  float me, ue;
  const float mh = two_prod(fh, qh, &me);
  const float ml = me + fmaf(fh, ql, fl * qh);
  const float uh = two_sum(mh, c, &ue);
  const float ul = ue + ml;
  const float h = uh + ul;
  *lo = ul - (h - uh);
  return h;
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

// Projection of one kept pair (Gaussian g of segment R) into output slot
// `slot`: the compositing record, tile rectangle, depth key and, on debug
// frames, the per-splat debug arrays.
// The Gaussian: its geometry record (g0, g1, g2) and SH row (sh_row, in LDS),
// pair id pid.
__device__ __forceinline__ void project_pair(
    const SegRec& R, float4 g0, float4 g1, float4 g2, const float4* sh_row, int sh_degree, uint32_t pid,
    uint32_t slot, int tile, int tiles_x, int n_tiles, int keep_debug, float det_clip, float4* __restrict__ splat,
    float4* __restrict__ rec_a, float4* __restrict__ rec_b, float4* __restrict__ rec_c, float2* __restrict__ rec_d,
    uint4* __restrict__ rect_dbg, uint2* __restrict__ rect, uint32_t* __restrict__ depth_key,
    uint32_t* __restrict__ pair_of) {
  const float mu[3] = {g0.x, g0.y, g0.z};
  const float s3[3] = {g1.x, g1.y, g1.z};
  float qw = g2.x, qx = g2.y, qy = g2.z, qz = g2.w;
  const float o = g0.w;
  // camera space, each coordinate as hi + lo (the hi parts drive the
  // Jacobian and the depth key; the centre below uses both)
  const float* M = R.M;
  float px_lo, py_lo, pz_lo;
  const float px = cam_coord(M, R.Mlo, mu[0], mu[1], mu[2], &px_lo);
  const float py = cam_coord(M + 4, R.Mlo + 4, mu[0], mu[1], mu[2], &py_lo);
  const float pz = cam_coord(M + 8, R.Mlo + 8, mu[0], mu[1], mu[2], &pz_lo);
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
  // inverse 2D covariance (conic) for the debug record
  const float id = 1.f / det;
  const float ca = cc * id, cb = -b * id, cc2 = a * id;
  // The compositing evaluates the exponent as -|F d|^2 with F's rows along
  // the ellipse axes, F^T F = (log2(e) / 2) conic: a sum of two squares.  The
  // expanded form A dx^2 + 2B dx dy + C dy^2 cancels along the long axis of
  // a thin splat and loses ~kappa * 2^-24 of the exponent to the rounding of
  // A, B, C (kappa = condition number of Sigma2D); the axis form loses
  // ~sqrt(kappa) * 2^-24.  Eigenvalues l1 >= l2 of Sigma2D: l1 = m + r
  // (sums of non-negative terms), l2 = det / l1 with the cancellation-free
  // determinant; l1's eigenvector from the row whose entries do not cancel.
  float f1x, f1y, f2x, f2y;
  {
    constexpr float kS = 0.72134752044448170f;  // log2(e) / 2
    const float hd = 0.5f * (a - cc);
    const float r = sqrtf(hd * hd + b * b);
    const float l1 = 0.5f * (a + cc) + r;
    const float l2 = det / l1;
    float e0 = hd >= 0.f ? hd + r : b, e1 = hd >= 0.f ? b : r - hd;
    float nn = e0 * e0 + e1 * e1;
    if (!(nn > 0.f)) e0 = 1.f, e1 = 0.f, nn = 1.f;  // isotropic: any axes
    const float in = rsqrtf(nn);
    const float s1 = sqrtf(kS / l1) * in, s2 = sqrtf(kS / l2) * in;
    f1x = s1 * e0; f1y = s1 * e1;
    f2x = -s2 * e1; f2y = s2 * e0;
  }
  // the centre to ~48 bits: a 1080p centre rounded to FP32 is off by up to
  // 3e-5 px, and the narrowest splats (dilated variance 0.3 px^2) change alpha
  // by about one part in 1e4 for that, above the pixel tolerance once
  // dozens of fragments are blended; the compositing takes u - tile origin
  // from the two parts
  float u_lo, v_lo;
  const float u = screen_coord(px, px_lo, pz, pz_lo, f, R.focal_lo, R.half_w, &u_lo);
  const float v = screen_coord(py, py_lo, pz, pz_lo, f, R.focal_lo, R.half_h, &v_lo);
  // colour: SH along the camera -> Gaussian direction in the asset frame
  float dx = mu[0] - R.cl[0], dy = mu[1] - R.cl[1], dz = mu[2] - R.cl[2];
  const float dn = rsqrtf(dx * dx + dy * dy + dz * dz);
  float rgb[3];
  sh_color<true>(sh_row, sh_degree, dx * dn, dy * dn, dz * dn, rgb);
  // footprint
  const float k2 = 2.f * logf(255.f * o);
  const int W = (int)(2.f * R.half_w), H = (int)(2.f * R.half_h);
  float ex = 0.f, ey = 0.f;
  uint32_t r0 = 0, r1 = 0, ntiles = 0, key0 = 0, wh = 0;
  if (k2 >= 0.f && !(det < det_clip)) {  // radius clipping: splats of small 2D area are not binned
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
      // the binning's 8-byte form: the tile key of the top-left tile, and
      // the rectangle's width and height in tiles
      key0 = (uint32_t)R.cam * (uint32_t)n_tiles + (uint32_t)ty0 * (uint32_t)tiles_x + (uint32_t)tx0;
      wh = (uint32_t)(tx1 - tx0 + 1) | ((uint32_t)(ty1 - ty0 + 1) << 16);
    }
  }
  // the compositing record: one 64-byte line per splat: the centre (hi
  // parts), the axis rows F (exponent base 2), log2 of the opacity that
  // joins the exponent, the colour, the centre's low parts; then the pair id
  // and the footprint extents (they only pick 8x8 blocks of a larger tile:
  // rounded up to FP16)
  const __half2 exy = __halves2half2(__float2half_ru(ex), __float2half_ru(ey));
  float4* sp = splat + 4 * (int64_t)slot;
  sp[0] = make_float4(u, v, f1x, f1y);
  sp[1] = make_float4(f2x, f2y, __log2f(o), rgb[0]);
  sp[2] = make_float4(rgb[1], rgb[2], u_lo, v_lo);
  sp[3] = make_float4(__uint_as_float(pid), __builtin_bit_cast(float, exy), pz, 0.f);
  rect[slot] = make_uint2(key0, wh);
  depth_key[slot] = fbits(pz);
  if (keep_debug) {
    rec_a[slot] = make_float4(u, v, ca, cb);
    rec_b[slot] = make_float4(cc2, o, rgb[0], rgb[1]);
    rec_c[slot] = make_float4(rgb[2], pz, ex, ey);
    rec_d[slot] = make_float2(u_lo, v_lo);
    rect_dbg[slot] = make_uint4(r0, r1, (uint32_t)R.cam, ntiles);
    pair_of[slot] = pid;
  }

}

// Projection over the cull/MLP work items: a work-group takes one 256-
// Gaussian chunk of an asset and a run of its segments (camera x instance),
// stages half of the chunk's geometry records and SH rows in LDS at a time,
// and projects the kept pairs of all those segments in that half with one
// thread per pair, so that a Gaussian kept by several instances is read from
// memory once and every lane has a pair whatever the keep rate (half chunks
// keep the staging to ~40 KB: four work-groups per compute unit).  A pair's
// output slot is its segment-chunk's offset (exclusive scan of the chunks'
// keep counts) plus its rank among the chunk's kept pairs, as in the ordered
// compaction.
constexpr int kPjSegs = 32;        // segments staged at a time
constexpr int kPjRow = 13;         // float4 per staged SH row (48 floats + padding)
constexpr int kPjHalf = kChunk / 2;  // Gaussians staged at a time
constexpr int kPjWords = kPjHalf / 32;
__global__ __launch_bounds__(256) void k_project(
    const AssetDev* __restrict__ assets, const WorkItem* __restrict__ items, const int32_t* __restrict__ seglist,
    const SegRec* __restrict__ segs, const uint32_t* __restrict__ mask, const uint32_t* __restrict__ chunk_off,
    const uint32_t* __restrict__ n_splats, int64_t cap, int tile, int tiles_x, int n_tiles, int keep_debug,
    float det_clip, float4* __restrict__ splat, float4* __restrict__ rec_a, float4* __restrict__ rec_b,
    float4* __restrict__ rec_c, float2* __restrict__ rec_d, uint4* __restrict__ rect_dbg, uint2* __restrict__ rect,
    uint32_t* __restrict__ depth_key, uint32_t* __restrict__ pair_of, uint32_t* __restrict__ overflow) {
  __shared__ float4 s_geo[3 * kPjHalf];
  __shared__ float4 s_sh[kPjHalf * kPjRow];
  __shared__ SegRec s_seg[kPjSegs];
  __shared__ uint32_t s_mask[kPjSegs][kChunk / 32];
  __shared__ uint32_t s_base[kPjSegs + 1];  // exclusive scan of the segments' kept counts in this half
  __shared__ uint32_t s_slot[kPjSegs];      // output slot of each segment's first kept pair in this half
  const int t = threadIdx.x;
  if (blockIdx.x == 0 && t == 0 && (int64_t)*n_splats > cap) atomicOr(overflow, 1u);
  const WorkItem it = items[blockIdx.x];
  const AssetDev& A = assets[it.asset];
  const int64_t n = A.n;
  const int64_t words = (n + 31) >> 5;
  constexpr int RW = sizeof(SegRec) / 4;
  static_assert(sizeof(SegRec) % 4 == 0, "segment records are copied word by word");
  for (int h = 0; h < 2; ++h) {
    const int64_t g0 = (int64_t)it.chunk * kChunk + h * kPjHalf;
    bool staged = false;
    for (int sb = it.seg_begin; sb < it.seg_end; sb += kPjSegs) {
      const int ns = min(kPjSegs, it.seg_end - sb);
      __syncthreads();  // the previous batch's reads of the segment records and masks are done
      for (int i = t; i < ns * RW; i += 256)
        reinterpret_cast<uint32_t*>(s_seg)[i] = reinterpret_cast<const uint32_t*>(segs + seglist[sb + i / RW])[i % RW];
      for (int i = t; i < ns * (kChunk / 32); i += 256) {
        const int j = i / (kChunk / 32), w = i % (kChunk / 32);
        const int64_t wi = (int64_t)it.chunk * (kChunk / 32) + w;
        s_mask[j][w] = wi < words ? mask[segs[seglist[sb + j]].word_base + wi] : 0u;
      }
      __syncthreads();
      if (t < 64) {  // one wave: kept counts of this half, their scan, the slot bases
        uint32_t c = 0, before = 0;
        if (t < ns) {
          for (int w = 0; w < kPjWords; ++w) c += (uint32_t)__popc(s_mask[t][h * kPjWords + w]);
          for (int w = 0; w < h * kPjWords; ++w) before += (uint32_t)__popc(s_mask[t][w]);
        }
        uint32_t x = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const uint32_t y = __shfl_up(x, o);
          if (t >= o) x += y;
        }
        if (t == 0) s_base[0] = 0;
        if (t < ns) {
          s_base[t + 1] = x;
          s_slot[t] = chunk_off[s_seg[t].chunk_base + it.chunk] + before;
        }
      }
      __syncthreads();
      const uint32_t K = s_base[ns];
      if (K == 0) continue;
      if (!staged) {
        const int q4 = A.sh_stride / 4;
        for (int i = t; i < 3 * kPjHalf; i += 256)
          s_geo[i] = g0 + i / 3 < n ? ld_global(A.geo, 3 * g0 + i) : make_float4(0.f, 0.f, 0.f, 0.f);
        const float4* shp = reinterpret_cast<const float4*>(A.shp);
        for (int i = t; i < kPjHalf * q4; i += 256) {
          const int gi = i / q4, q = i % q4;
          s_sh[gi * kPjRow + q] = g0 + gi < n ? ld_global(shp, (g0 + gi) * q4 + q) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
        staged = true;
        __syncthreads();
      }
      for (uint32_t p = (uint32_t)t; p < K; p += 256) {
        // segment: the last j with s_base[j] <= p
        int j = 0;
#pragma unroll
        for (int step = kPjSegs / 2; step > 0; step >>= 1)
          if (j + step < ns && s_base[j + step] <= p) j += step;
        // rank among the segment's kept pairs of this half -> mask word and bit
        const uint32_t r = p - s_base[j];
        uint32_t cum = 0, below = 0, x = 0;
        int wsel = 0;
        bool found = false;
#pragma unroll
        for (int w = 0; w < kPjWords; ++w) {
          const uint32_t m = s_mask[j][h * kPjWords + w];
          const uint32_t pc = (uint32_t)__popc(m);
          if (!found && r < cum + pc) {
            found = true;
            wsel = w;
            below = cum;
            x = m;
          }
          cum += pc;
        }
        uint32_t rr = r - below;
        int pos = 0;
#pragma unroll
        for (int half = 16; half > 0; half >>= 1) {
          const uint32_t low = (uint32_t)__popc(x & ((1u << half) - 1u));
          if (rr >= low) {
            rr -= low;
            x >>= half;
            pos += half;
          }
        }
        const int gl = wsel * 32 + pos;
        const uint32_t slot = s_slot[j] + r;
        if ((int64_t)slot >= cap) continue;  // flagged above
        const SegRec& R = s_seg[j];
        project_pair(R, s_geo[3 * gl], s_geo[3 * gl + 1], s_geo[3 * gl + 2], s_sh + gl * kPjRow, A.sh_degree,
                     (uint32_t)(R.pair_base + g0 + gl), slot, tile, tiles_x, n_tiles, keep_debug, det_clip, splat,
                     rec_a, rec_b, rec_c, rec_d, rect_dbg, rect, depth_key, pair_of);
      }
    }
  }
}

hipError_t launch_project(const AssetDev* assets, const WorkItem* items, int64_t n_items, const int32_t* seglist,
                          const SegRec* segs, const uint32_t* mask, const uint32_t* chunk_off, const uint32_t* n_splats,
                          int64_t cap_splats, int tile, int tiles_x, int n_tiles, int keep_debug, float det_clip,
                          float4* splat, float4* rec_a, float4* rec_b, float4* rec_c, float2* rec_d, uint4* rect_dbg,
                          uint2* rect, uint32_t* depth_key, uint32_t* pair_of, uint32_t* overflow, hipStream_t st) {
  if (n_items == 0) return hipSuccess;
  hipLaunchKernelGGL(k_project, dim3((unsigned)n_items), dim3(256), 0, st, assets, items, seglist, segs, mask,
                     chunk_off, n_splats, cap_splats, tile, tiles_x, n_tiles, keep_debug, det_clip, splat, rec_a,
                     rec_b, rec_c, rec_d, rect_dbg, rect, depth_key, pair_of, overflow);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// binning
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t live(const uint32_t* n_dev, int64_t cap) {
  return n_dev ? (int64_t)min((uint64_t)*n_dev, (uint64_t)cap) : cap;
}

// One (tile key, splat id) entry per overlapped tile of each splat, in depth
// order: splat j's entries occupy [off[j], off[j] + ntiles_j), its tiles in
// row-major order.  A wave takes 64 consecutive splats and its lanes write
// the group's entries consecutively (coalesced, and a splat over many tiles
// does not hold one lane for all of them): entry e of the group belongs to the
// last lane whose group-relative offset is <= e (binary search over the
// lanes).  Past the entry capacity the overflow flag is raised and only the
// entries below it are written, so every position of [0, cap_dup) still holds
// an entry of this frame (a clipped frame, never stale keys).
__global__ __launch_bounds__(256) void k_emit(const uint32_t* __restrict__ ids, const uint2* __restrict__ rect_sorted,
                                              const uint32_t* __restrict__ off, const uint32_t* __restrict__ n_dev,
                                              int64_t cap, const uint32_t* __restrict__ n_dup_dev, int64_t cap_dup,
                                              int tiles_x, int n_tiles, uint32_t* __restrict__ keys,
                                              uint32_t* __restrict__ vals, uint32_t* __restrict__ overflow) {
  const int lane = threadIdx.x & 63;
  const int64_t n = live(n_dev, cap);
  const int64_t ngroups = (n + 63) / 64;
  const int64_t wstride = (int64_t)gridDim.x * (blockDim.x / 64);
  for (int64_t grp = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); grp < ngroups; grp += wstride) {
    const int64_t j = grp * 64 + lane;
    uint2 r = make_uint2(0u, 0u);  // (tile key of the top-left tile, width | height << 16)
    uint32_t o = 0u, id = 0u;
    if (j < n) {
      r = rect_sorted[j];
      o = off[j];
      id = ids[j];
    }
    const uint32_t start = __shfl(o, 0);  // lane 0's splat is live
    const uint32_t rel = j < n ? o - start : 0xffffffffu;
    uint32_t total = j < n ? rel + (r.y & 0xffffu) * (r.y >> 16) : 0u;
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) total = max(total, __shfl_xor(total, m));
    if (lane == 0 && (int64_t)start + total > cap_dup) atomicOr(overflow, 2u);
    // every lane stays in the loop (the shuffles read all 64 lanes); only the
    // stores are limited to the group's entries
    for (uint32_t e0 = 0; e0 < total; e0 += 64) {
      const uint32_t e = e0 + (uint32_t)lane;
      int src = 0;  // rel of lane 0 is 0 <= e
#pragma unroll
      for (int step = 32; step > 0; step >>= 1)
        if (__shfl(rel, src + step) <= e) src += step;
      const uint32_t q = e - __shfl(rel, src);
      const uint32_t key0 = __shfl(r.x, src), w = __shfl(r.y, src) & 0xffffu, sid = __shfl(id, src);
      const uint32_t dy = q / max(w, 1u), dx = q - dy * w;
      const int64_t pos = (int64_t)start + e;
      if (e < total && pos < cap_dup) {
        keys[pos] = key0 + dy * (uint32_t)tiles_x + dx;
        vals[pos] = sid;
      }
    }
  }
  (void)n_dup_dev;
  (void)n_tiles;
}

hipError_t launch_emit(const uint32_t* sorted_ids, const uint2* rect_sorted, const uint32_t* dup_off, const uint32_t* n_dev,
                       int64_t cap, const uint32_t* n_dup_dev, int64_t cap_dup, int tiles_x, int n_tiles,
                       uint32_t* keys, uint32_t* vals, uint32_t* overflow, hipStream_t st) {
  if (cap == 0) return hipSuccess;
  unsigned grid = (unsigned)std::min<int64_t>((cap + 255) / 256, 65536);
  hipLaunchKernelGGL(k_emit, dim3(grid), dim3(256), 0, st, sorted_ids, rect_sorted, dup_off, n_dev, cap, n_dup_dev, cap_dup,
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

// High-water marks across frames: [12] max splats, [13] max tile entries,
// [14] OR of the overflow flags (word [2] of the per-frame counters).
__global__ void k_watermark(uint32_t* __restrict__ c) {
  if (threadIdx.x == 0) {
    c[12] = max(c[12], c[0]);
    c[13] = (c[2] & 4u) ? 0xffffffffu : max(c[13], c[1]);  // 4: the 32-bit entry offsets wrapped
    c[14] |= c[2];
  }
}

hipError_t launch_watermark(uint32_t* counters, hipStream_t st) {
  hipLaunchKernelGGL(k_watermark, dim3(1), dim3(64), 0, st, counters);
  return hipGetLastError();
}

// [start, end) of every tile key in the sorted list (ranges pre-filled with
// 0).  Each thread takes four consecutive positions with one 16-byte load and
// handles the boundaries after each of them (and before position 0).
__global__ void k_ranges(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ n_dev, int64_t cap,
                         int64_t nkeys, uint32_t* __restrict__ ranges) {
  const int64_t n = live(n_dev, cap);
  const uint32_t kNone = 0xffffffffu;
  for (int64_t j0 = 4 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x); j0 < n;
       j0 += 4 * (int64_t)gridDim.x * blockDim.x) {
    uint32_t k[5];
    if (j0 + 4 <= n) {
      const uint4 q = *reinterpret_cast<const uint4*>(keys + j0);
      k[0] = q.x;
      k[1] = q.y;
      k[2] = q.z;
      k[3] = q.w;
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) k[u] = j0 + u < n ? keys[j0 + u] : kNone;
    }
    k[4] = j0 + 4 < n ? keys[j0 + 4] : kNone;
    if (j0 == 0 && k[0] < nkeys) ranges[2 * (int64_t)k[0]] = 0u;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      // boundary between positions j0 + u and j0 + u + 1
      if (j0 + u < n && k[u] != k[u + 1]) {
        const uint32_t pos = (uint32_t)(j0 + u + 1);
        if (k[u] < nkeys) ranges[2 * (int64_t)k[u] + 1] = pos;
        if (k[u + 1] < nkeys) ranges[2 * (int64_t)k[u + 1]] = pos;
      }
    }
  }
}

hipError_t launch_ranges(const uint32_t* keys, const uint32_t* n_dev, int64_t cap, int64_t nkeys, uint32_t* ranges,
                         hipStream_t st) {
  if (cap == 0) return hipSuccess;
  if (reinterpret_cast<uintptr_t>(keys) % 16 != 0) return hipErrorInvalidValue;  // the 16-byte loads
  unsigned grid = (unsigned)std::min<int64_t>((cap + 1023) / 1024, 65536);
  hipLaunchKernelGGL(k_ranges, dim3(grid), dim3(256), 0, st, keys, n_dev, cap, nkeys, ranges);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// tile order: longest tile lists first (one stable radix pass on a 5-bit
// log2 bucket of the list length), so the heaviest tiles do not start last
// ---------------------------------------------------------------------------
__global__ void k_tile_keys(const uint32_t* __restrict__ ranges, int64_t n, uint32_t* __restrict__ keys,
                            uint32_t* __restrict__ vals) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t len = ranges[2 * j + 1] - ranges[2 * j];
    keys[j] = 31u - (uint32_t)(32 - __clz(len));  // 31 - bit length: longer lists get smaller keys
    vals[j] = (uint32_t)j;
  }
}

hipError_t launch_tile_keys(const uint32_t* ranges, int64_t n, uint32_t* keys, uint32_t* vals, hipStream_t st) {
  if (n == 0) return hipSuccess;
  unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_tile_keys, dim3(grid), dim3(256), 0, st, ranges, n, keys, vals);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// front-to-back compositing, one work-group per (camera, tile)
//
// Each wave owns an 8x8 block of pixels (one lane per pixel; the 32-pixel
// tile gives every lane four blocks).  Splats are staged in LDS 256 at a
// time; the next batch is fetched into registers while the current one is
// composited.  Per (pixel, splat) alpha is one base-2 exponential whose
// argument carries log2 of the opacity.  A wave skips splats whose alpha
// footprint box misses its pixel block.
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// compositing work items.  A tile list longer than split_len entries is cut
// into nch equal chunks composited by nch work-groups: the first chunk is
// composited from T = 1 and stores its per-pixel product, while a product pass
// gives each middle chunk's per-pixel product of (1 - alpha) over its passing
// fragments (no stop rule); chunk j then starts from the product of the chunks
// before it.  Transmittance only falls, so a pixel stopped before chunk j exactly
// when that product is below 1e-4, and chunk j applies the stop rule from
// there.  A combine pass sums the chunks' colours in list order.  The result
// equals the sequential composite up to the association of the products and
// sums (rounding).  Items are (position in the tile launch order, chunk).
// ---------------------------------------------------------------------------
__global__ void k_split_count(const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ order, int64_t nkeys,
                              int split_len, const uint32_t* __restrict__ n_dev, int64_t cap, int64_t split_div,
                              uint32_t* __restrict__ nch, uint32_t* __restrict__ nsp, uint32_t* __restrict__ chunk_len) {
  if (split_len == kSplitAuto) {
    // the frame's entries over split_div chunks (about two per work-group
    // the compositing launch keeps resident): long lists are cut into pieces
    // that balance the launch, short frames keep kSplitMin
    const int64_t n = min((int64_t)*n_dev, cap);
    split_len = (int)max((int64_t)kSplitMin, (n + split_div - 1) / split_div);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *chunk_len = (uint32_t)max(split_len, 0);
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nkeys; p += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t key = order[p];
    const uint32_t len = ranges[2 * (int64_t)key + 1] - ranges[2 * (int64_t)key];
    const uint32_t c = (split_len > 0 && len > (uint32_t)split_len) ? (len + split_len - 1) / split_len : 1u;
    nch[p] = c;
    nsp[p] = c > 1 ? c : 0u;
  }
}

// Items of every launch position; past the item or split-slot capacity the
// overflow flag (8) is raised (such a frame is reported, never used).
__global__ void k_split_expand(const uint32_t* __restrict__ nch, const uint32_t* __restrict__ item_off, int64_t nkeys,
                               int64_t cap_items, uint2* __restrict__ items, const uint32_t* __restrict__ n_split,
                               int64_t cap_split, uint32_t* __restrict__ overflow) {
  if (blockIdx.x == 0 && threadIdx.x == 0 && (int64_t)*n_split > cap_split) atomicOr(overflow, 8u);
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nkeys; p += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t c = nch[p], o = item_off[p];
    for (uint32_t j = 0; j < c; ++j) {
      if ((int64_t)o + j < cap_items)
        items[o + j] = make_uint2((uint32_t)p, j);
      else
        atomicOr(overflow, 8u);
    }
  }
}

struct ItemCtx {
  const uint2* items;
  const uint32_t* n_items;  // device count
  int64_t cap_items;
  int64_t cap_split;        // split-chunk slots of prod / part
  const uint32_t* order;
  const uint32_t* nch;
  const uint32_t* split_off;
  float* prod;              // [split chunk][T*T]
  float4* part;             // [split chunk][T*T]: r, g, b, flag
  const uint32_t* item_off; // [nkeys] first item per position
  int64_t nkeys;            // positions
};

// A pixel that has stopped (or lies outside the image, or stopped in an
// earlier chunk) is moved to x = kFar: every later quadratic form is -inf, so
// it fails the level-set test with no per-pixel flag to keep.
constexpr float kFar = 1e30f;
constexpr float kFarTest = 1e29f;

// One compositing item.  MODE 0: composite; 1: composite and record
// contributions; 2: product pass.  STATS: also count the list entries each
// pixel examined (statistics frames).  FIRST_PROD: composite of a split
// list's first chunk that also stores the chunk's transmittance product
// (0 if the pixel stopped in it), so the product pass can skip that chunk.
template <int T, int MODE, bool STATS, bool FIRST_PROD>
__device__ __forceinline__ void blend_item(
    const ItemCtx& ic, const uint2 it, const uint32_t nch, const uint32_t* __restrict__ ranges,
    const uint32_t* __restrict__ ids, const float4* __restrict__ splat, int W, int H, int tiles_x, int n_tiles,
    float bg0, float bg1, float bg2, float* __restrict__ rgb, uint32_t* __restrict__ contrib,
    unsigned long long* __restrict__ work) {
  constexpr bool RECORD = MODE == 1, PROD = MODE == 2;
  constexpr int NT = T == 8 ? 64 : 256;  // threads
  constexpr int NB = T * T / 64;         // 8x8 pixel blocks per tile
  constexpr int BPW = NB / (NT / 64);    // blocks per wave (1, 1, 4)
  constexpr int BATCH = NT;              // one staged splat per thread per batch
  // staged records, one array so that a fragment's three reads share one
  // address: [k][0] = u, v relative to the first pixel centre of the tile's
  // 32-pixel block, F row 1; [k][1] = F row 2, log2(opacity), r; [k][2] = g, b
  __shared__ float4 s_rec[BATCH][3];
  __shared__ uint32_t s_ov[T == 8 ? 1 : BATCH];  // bit b: the footprint box touches 8x8 block b
  __shared__ uint32_t s_p[RECORD ? BATCH : 1];
  const bool split = nch > 1;
  if (split && (int64_t)ic.split_off[it.x] + nch > ic.cap_split) return;  // over capacity: the frame is flagged
  const int key = (int)ic.order[it.x];
  const int cam = key / n_tiles, tile = key % n_tiles;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  uint32_t start = ranges[2 * (int64_t)key], end = ranges[2 * (int64_t)key + 1];
  if (split) {
    const uint32_t clen = (end - start + nch - 1) / nch;
    start = min(end, start + it.y * clen);
    end = min(end, start + clen);
  }
  const int64_t sbase = split ? ((int64_t)ic.split_off[it.x] + it.y) * (T * T) : 0;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  auto pix_x = [&](int j) { return tx * T + ((wave * BPW + j) % (T / 8)) * 8 + (lane & 7); };
  auto pix_y = [&](int j) { return ty * T + ((wave * BPW + j) / (T / 8)) * 8 + (lane >> 3); };
  float px[BPW], py[BPW], Tr[BPW], cr[BPW], cg[BPW], cb[BPW];
  bool before[BPW];
  uint32_t stop[BPW];  // statistics: list position at which the pixel stopped (end if it never did)
#pragma unroll
  for (int j = 0; j < BPW; ++j) {
    stop[j] = end;
    const int blk = wave * BPW + j;
    const int x = pix_x(j), y = pix_y(j);
    // pixel offsets within the 32-pixel block holding the tile (the staged
    // centres are relative to it, the same for every tile size)
    px[j] = (x < W && y < H) ? (float)(x & 31) : kFar;
    py[j] = (float)(y & 31);
    Tr[j] = 1.f;
    cr[j] = cg[j] = cb[j] = 0.f;
    before[j] = false;
    if (split && !PROD && it.y > 0) {
      // transmittance entering this chunk: product of the earlier chunks' products
      const int64_t pix = blk * 64 + lane;
      const int64_t b0 = (int64_t)ic.split_off[it.x] * (T * T) + pix;
      float tin = 1.f;
      for (uint32_t q = 0; q < it.y; ++q) tin *= ic.prod[b0 + (int64_t)q * (T * T)];
      Tr[j] = tin;
      before[j] = tin < kTMin;
      px[j] = before[j] ? kFar : px[j];
    }
  }
  // the next batch's record of this thread, fetched while the current one is composited
  float4 qa = make_float4(0.f, 0.f, 0.f, 0.f), qb = qa, qc = qa;
  float2 qd = make_float2(0.f, 0.f);  // pair id, extents
  if (start + t < end) {
    const float4* r = splat + 4 * (int64_t)ids[start + t];
    qa = r[0];
    qb = r[1];
    qc = r[2];
    qd = *reinterpret_cast<const float2*>(r + 3);
  }
  uint32_t b0k = start;
  // composite staged splat k into pixel block j.  Branch-free: a fragment that
  // is skipped (outside the 1/255 level set, alpha < 1/255, pixel stopped)
  // contributes weight 0; one whose blend would take T below 1e-4 stops the
  // pixel instead (Sec. 4.1).  The product pass multiplies (1 - alpha) of the
  // passing fragments, stopping once below 1e-4 (later chunks only test that).
  auto step = [&](int j, int k) {
    const float4 g = s_rec[k][0];
    const float4 h = s_rec[k][1];
    const float dx = px[j] - g.x, dy = py[j] - g.y;
    // alpha = min(0.99, o 2^pw) with pw = -log2(e) d^T conic d / 2 = -|F d|^2,
    // as 2^(pw + log2 o)
    const float t1 = fmaf(g.z, dx, g.w * dy);
    const float t2 = fmaf(h.x, dx, h.y * dy);
    const float q = fmaf(-t1, t1, fmaf(-t2, t2, h.z));
    const float al = fminf(kAlphaMax, __builtin_amdgcn_exp2f(q));
    const bool ok = al >= kAlphaMin;
    const float w0 = al * Tr[j];
    const float Tn = Tr[j] - w0;  // T (1 - alpha)
    if (PROD) {
      Tr[j] = ok ? Tn : Tr[j];
      px[j] = Tr[j] < kTMin ? kFar : px[j];
      return;
    }
    const float4 c = s_rec[k][2];
    // Tn >= 0, so the FP32 order is the order of the bit patterns
    const bool low = __float_as_uint(Tn) < __float_as_uint(kTMin);
    const bool halt = ok && low;
    const bool take = ok != halt;  // ok and not low
    const float w = take ? w0 : 0.f;
    cr[j] = fmaf(w, h.w, cr[j]);
    cg[j] = fmaf(w, c.x, cg[j]);
    cb[j] = fmaf(w, c.y, cb[j]);
    Tr[j] = take ? Tn : Tr[j];
    if (STATS) stop[j] = halt ? b0k + (uint32_t)k : stop[j];
    px[j] = halt ? kFar : px[j];
    // contribution: alpha T of a blended fragment; the stopping fragment was
    // reached but not blended and records the smallest positive float
    if (RECORD && ok) atomicMax(contrib + s_p[k], take ? __float_as_uint(w) : 1u);
  };
  auto live = [&](int j) { return px[j] < kFarTest; };
  for (uint32_t b0 = start; b0 < end; b0 += BATCH) {
    bool any = false;
#pragma unroll
    for (int j = 0; j < BPW; ++j) any |= live(j);
    if (__syncthreads_count(any) == 0) break;  // also: the previous batch is consumed
    const int cnt = (int)min((uint32_t)BATCH, end - b0);
    b0k = b0;
    uint64_t pm = 0;  // 8x8 tiles: bit p = pixel p of the tile lies in this thread's footprint box
    if (t < cnt) {
      // the centre relative to the first pixel centre of the tile's 32-pixel
      // block, from its hi + lo parts (qc.z, qc.w): for a splat over the
      // tile, u - origin is (nearly) exact in FP32, so d = offset - centre
      // keeps the centre's precision, and the same for every tile size
      const int bx = (tx * T) & ~31, by = (ty * T) & ~31;
      const float ur = (qa.x - ((float)bx + 0.5f)) + qc.z;
      const float vr = (qa.y - ((float)by + 0.5f)) + qc.w;
      s_rec[t][0] = make_float4(ur, vr, qa.z, qa.w);
      s_rec[t][1] = qb;
      s_rec[t][2] = qc;
      if (T == 8) {
        // pixels of the tile whose centre lies in the footprint box (the
        // alpha >= 1/255 bound of the tile rectangle, with the same widening);
        // qd.y = the half extents, rounded up to FP16.  Pixel p = 8 row + column.
        const __half2 exy = __builtin_bit_cast(__half2, qd.y);
        const float ex = __low2float(exy), ey = __high2float(exy);
        const float wx = 1e-4f * ex + 1e-3f, wy = 1e-4f * ey + 1e-3f;
        const float ox = (float)(tx * T - bx), oy = (float)(ty * T - by);
        const float c0 = fmaxf(0.f, ceilf(ur - ox - ex - wx)), c1 = fminf(7.f, floorf(ur - ox + ex + wx));
        const float r0 = fmaxf(0.f, ceilf(vr - oy - ey - wy)), r1 = fminf(7.f, floorf(vr - oy + ey + wy));
        if (c0 <= c1 && r0 <= r1) {
          const uint32_t cols = (2u << (int)c1) - (1u << (int)c0);
          const uint64_t rows = (~0ull >> (56 - 8 * (int)r1)) & (~0ull << (8 * (int)r0));
          pm = ((uint64_t)cols * 0x0101010101010101ull) & rows;
        }
      } else {
        // 8x8 blocks of the tile touched by the footprint box (same widening
        // as the tile rectangle); qd.y = the half extents, rounded up to FP16
        const __half2 exy = __builtin_bit_cast(__half2, qd.y);
        const float ex = __low2float(exy), ey = __high2float(exy);
        const float wx = 1e-4f * ex + 1e-3f, wy = 1e-4f * ey + 1e-3f;
        const float ox = (float)(tx * T - bx), oy = (float)(ty * T - by);
        const float x0 = fmaxf(-1.f, (ur - ox - ex - wx) * 0.125f);
        const float x1 = fminf((float)T, (ur - ox + ex + wx) * 0.125f);
        const float y0 = fmaxf(-1.f, (vr - oy - ey - wy) * 0.125f);
        const float y1 = fminf((float)T, (vr - oy + ey + wy) * 0.125f);
        const int bx0 = max(0, (int)floorf(x0)), bx1 = min(T / 8 - 1, (int)floorf(x1));
        const int by0 = max(0, (int)floorf(y0)), by1 = min(T / 8 - 1, (int)floorf(y1));
        uint32_t m = 0;
        for (int by = by0; by <= by1; ++by)
          for (int bx = bx0; bx <= bx1; ++bx) m |= 1u << (by * (T / 8) + bx);
        s_ov[t] = m;
      }
      if (RECORD) s_p[t] = __float_as_uint(qd.x);
    }
    __syncthreads();
    if (b0 + BATCH + t < end) {  // overlaps the compositing below
      const float4* r = splat + 4 * (int64_t)ids[b0 + BATCH + t];
      qa = r[0];
      qb = r[1];
      qc = r[2];
      qd = *reinterpret_cast<const float2*>(r + 3);
    }
#pragma unroll
    for (int j = 0; j < BPW; ++j) {
      if (__ballot(live(j)) == 0) continue;
      if (T == 8) {
        // the batch's splats in list order, skipping those whose footprint
        // box holds no live pixel of the tile: their alpha is below 1/255 at
        // every live pixel, so compositing them would change nothing (lane k
        // staged splat k; the set is refreshed every 8 splats)
        uint64_t lm = __ballot(live(j));
        uint64_t set = __ballot((pm & lm) != 0);
        int n = 0;
        while (set) {
          const int k = __builtin_ctzll(set);
          set &= set - 1;
          step(j, k);
          if (++n == 8) {
            n = 0;
            lm = __ballot(live(j));
            set &= __ballot((pm & lm) != 0);
          }
        }
      } else {
        // splats whose box touches this wave's block, as 64-bit ballot sets
        const int blk = wave * BPW + j;
        uint64_t set[BATCH / 64];
#pragma unroll
        for (int c = 0; c < BATCH / 64; ++c) {
          const int k = c * 64 + lane;
          set[c] = __ballot(k < cnt && ((s_ov[k] >> blk) & 1u));
        }
#pragma unroll
        for (int c = 0; c < BATCH / 64; ++c) {
          uint64_t m = set[c];
          while (m) {
            const int k = c * 64 + __builtin_ctzll(m);
            m &= m - 1;
            step(j, k);
          }
          if (__ballot(live(j)) == 0) break;
        }
      }
    }
  }
  if (PROD) {
#pragma unroll
    for (int j = 0; j < BPW; ++j) ic.prod[sbase + (wave * BPW + j) * 64 + lane] = Tr[j];
    return;
  }
  if (STATS && work) {
    // entries of the tile list each pixel examined: up to and including its stop
    uint32_t wk = 0;
#pragma unroll
    for (int j = 0; j < BPW; ++j) {
      const int x = pix_x(j), y = pix_y(j);
      if (x < W && y < H && !before[j]) wk += (stop[j] < end ? stop[j] + 1 : end) - start;
    }
    for (int o = 32; o > 0; o >>= 1) wk += __shfl_xor(wk, o);
    if (lane == 0) atomicAdd(work, (unsigned long long)wk);
  }
#pragma unroll
  for (int j = 0; j < BPW; ++j) {
    const int x = pix_x(j), y = pix_y(j);
    if (split) {
      // chunk record: colour and a flag: 0 if the pixel stopped in an earlier
      // chunk, -T if it stopped in this one, else the transmittance leaving it
      // (pixels outside the image are never read back)
      const bool stopped_here = !before[j] && !live(j);
      const float flag = before[j] ? 0.f : (stopped_here ? -Tr[j] : Tr[j]);
      ic.part[sbase + (wave * BPW + j) * 64 + lane] = make_float4(cr[j], cg[j], cb[j], flag);
      if (FIRST_PROD) ic.prod[sbase + (wave * BPW + j) * 64 + lane] = stopped_here ? 0.f : Tr[j];
      continue;
    }
    if (x < W && y < H) {
      float* o = rgb + (((int64_t)cam * H + y) * W + x) * 3;
      o[0] = fmaf(Tr[j], bg0, cr[j]);
      o[1] = fmaf(Tr[j], bg1, cg[j]);
      o[2] = fmaf(Tr[j], bg2, cb[j]);
    }
  }
}

// Compositing in two launches.  PHASE 0: the first chunk of every split list,
// composited from T = 1 (storing its product, 0 where the pixel stopped), and
// the product pass over the middle chunks; PHASE 1: lists that are not split,
// and the later chunks of split ones, each starting from the product of the
// chunks before it.
template <int T, int MODE, bool STATS, int PHASE>
__global__ __launch_bounds__(T == 8 ? 64 : 256) void k_blend(
    ItemCtx ic, const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ ids,
    const float4* __restrict__ splat, int W, int H, int tiles_x, int n_tiles, float bg0, float bg1, float bg2,
    float* __restrict__ rgb, uint32_t* __restrict__ contrib, unsigned long long* __restrict__ work) {
  const int64_t item = blockIdx.x;
  if (item >= min((int64_t)*ic.n_items, ic.cap_items)) return;
  const uint2 it = ic.items[item];
  const uint32_t nch = ic.nch[it.x];
  const bool split = nch > 1;
  if (PHASE == 0) {
    if (!split || it.y + 1 == nch) return;  // the last chunk's product is never needed
    if (it.y == 0)
      blend_item<T, MODE, STATS, true>(ic, it, nch, ranges, ids, splat, W, H, tiles_x, n_tiles, bg0, bg1, bg2, rgb,
                                       contrib, work);
    else
      blend_item<T, 2, false, false>(ic, it, nch, ranges, ids, splat, W, H, tiles_x, n_tiles, bg0, bg1, bg2, rgb,
                                     contrib, nullptr);
    return;
  }
  if (split && it.y == 0) return;  // composited in phase 0
  blend_item<T, MODE, STATS, false>(ic, it, nch, ranges, ids, splat, W, H, tiles_x, n_tiles, bg0, bg1, bg2, rgb,
                                    contrib, work);
}

// pixels of split tiles: chunk colours summed in list order, the final
// transmittance from the chunk where the pixel stopped (or the last one)
template <int T>
__global__ __launch_bounds__(256) void k_blend_combine(ItemCtx ic, int W, int H, int tiles_x, int n_tiles, float bg0,
                                                       float bg1, float bg2, float* __restrict__ rgb) {
  // work-groups loop over the launch positions; a split one is combined when
  // all of its chunks were composited (items within the capacity)
  const int64_t live_items = min((int64_t)*ic.n_items, ic.cap_items);
  for (int64_t p = blockIdx.x; p < ic.nkeys; p += gridDim.x) {
    const uint32_t nch = ic.nch[p];
    if (nch <= 1) continue;
    if ((int64_t)ic.item_off[p] + nch > live_items) continue;
    if ((int64_t)ic.split_off[p] + nch > ic.cap_split) continue;
    const int key = (int)ic.order[p];
    const int cam = key / n_tiles, tile = key % n_tiles;
    const int tx = tile % tiles_x, ty = tile / tiles_x;
    const int64_t base = (int64_t)ic.split_off[p] * (T * T);
    for (int pix = threadIdx.x; pix < T * T; pix += 256) {
      const int blk = pix / 64, lane = pix % 64;
      const int x = tx * T + (blk % (T / 8)) * 8 + (lane & 7), y = ty * T + (blk / (T / 8)) * 8 + (lane >> 3);
      if (!(x < W && y < H)) continue;
      float r = 0.f, g = 0.f, b = 0.f, tf = 1.f;
      for (uint32_t q = 0; q < nch; ++q) {
        const float4 v = ic.part[base + (int64_t)q * (T * T) + pix];
        if (v.w == 0.f) break;  // stopped before this chunk: tf is the last chunk's exit value
        r += v.x;
        g += v.y;
        b += v.z;
        if (v.w < 0.f) {
          tf = -v.w;
          break;
        }
        tf = v.w;
      }
      float* o = rgb + (((int64_t)cam * H + y) * W + x) * 3;
      o[0] = fmaf(tf, bg0, r);
      o[1] = fmaf(tf, bg1, g);
      o[2] = fmaf(tf, bg2, b);
    }
  }
}

template <int T>
static void launch_blend_t(bool record, const ItemCtx& ic, bool any_split, hipStream_t st, const uint32_t* ranges,
                           const uint32_t* ids, const float4* splat, int W, int H, int tiles_x, int n_tiles, float b0,
                           float b1, float b2, float* rgb, float* contrib, unsigned long long* work) {
  constexpr int NT = T == 8 ? 64 : 256;
  const dim3 grid((unsigned)ic.cap_items);
  uint32_t* cu = reinterpret_cast<uint32_t*>(contrib);
#define NVGS_BL(M, S, P)                                                                                         \
  hipLaunchKernelGGL((k_blend<T, M, S, P>), grid, dim3(NT), 0, st, ic, ranges, ids, splat, W, H, tiles_x, n_tiles, \
                     b0, b1, b2, rgb, cu, work)
#define NVGS_BL_MS(P)                                          \
  do {                                                         \
    if (record) {                                              \
      if (work) NVGS_BL(1, true, P); else NVGS_BL(1, false, P); \
    } else {                                                   \
      if (work) NVGS_BL(0, true, P); else NVGS_BL(0, false, P); \
    }                                                          \
  } while (0)
  if (any_split) NVGS_BL_MS(0);
  NVGS_BL_MS(1);
#undef NVGS_BL_MS
#undef NVGS_BL
  if (any_split)
    hipLaunchKernelGGL((k_blend_combine<T>), dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(ic.nkeys, 2048))), dim3(256), 0, st, ic, W,
                       H, tiles_x, n_tiles, b0, b1, b2, rgb);
}

// chunks per launch position, their offsets and the totals (items, split slots)
hipError_t launch_split_count(const uint32_t* ranges, const uint32_t* order, int64_t nkeys, int split_len,
                              const uint32_t* n_dev, int64_t cap, int64_t split_div, uint32_t* nch, uint32_t* nsp,
                              uint32_t* item_off, uint32_t* split_off, uint32_t* n_items, uint32_t* n_split,
                              uint32_t* chunk_len, uint32_t* partials, hipStream_t st) {
  if (nkeys == 0) return hipSuccess;
  if (split_len == kSplitAuto && split_div < 1) return hipErrorInvalidValue;
  const unsigned grid = (unsigned)std::min<int64_t>((nkeys + 255) / 256, 65536);
  hipLaunchKernelGGL(k_split_count, dim3(grid), dim3(256), 0, st, ranges, order, nkeys, split_len, n_dev, cap,
                     split_div, nch, nsp, chunk_len);
  hipError_t e = launch_scan_u32_dev(nch, item_off, nkeys, nullptr, n_items, partials, st, nullptr);
  if (e != hipSuccess) return e;
  return launch_scan_u32_dev(nsp, split_off, nkeys, nullptr, n_split, partials, st, nullptr);
}

hipError_t launch_split_expand(const uint32_t* nch, const uint32_t* item_off, int64_t nkeys, uint2* items,
                               int64_t cap_items, const uint32_t* n_split, int64_t cap_split, uint32_t* overflow,
                               hipStream_t st) {
  if (nkeys == 0) return hipSuccess;
  const unsigned grid = (unsigned)std::min<int64_t>((nkeys + 255) / 256, 65536);
  hipLaunchKernelGGL(k_split_expand, dim3(grid), dim3(256), 0, st, nch, item_off, nkeys, cap_items, items, n_split,
                     cap_split, overflow);
  return hipGetLastError();
}

hipError_t launch_blend(const BlendItems& bi, const uint32_t* ranges, const uint32_t* ids, const float4* splat, int W,
                        int H, int tile, int tiles_x, int tiles_y, float bg0, float bg1, float bg2, float* rgb,
                        float* contrib, unsigned long long* work, hipStream_t st) {
  const int n_tiles = tiles_x * tiles_y;
  if (bi.cap_items == 0) return hipSuccess;
  const ItemCtx ic{bi.items, bi.n_items, bi.cap_items, bi.cap_split, bi.order,   bi.nch,
                   bi.split_off, bi.prod,   bi.part,      bi.item_off,  bi.nkeys};
  const bool record = contrib != nullptr;
  const bool any_split = bi.split_len != 0;
  if (tile == 8)
    launch_blend_t<8>(record, ic, any_split, st, ranges, ids, splat, W, H, tiles_x, n_tiles, bg0, bg1, bg2, rgb,
                      contrib, work);
  else if (tile == 16)
    launch_blend_t<16>(record, ic, any_split, st, ranges, ids, splat, W, H, tiles_x, n_tiles, bg0, bg1, bg2, rgb,
                       contrib, work);
  else if (tile == 32)
    launch_blend_t<32>(record, ic, any_split, st, ranges, ids, splat, W, H, tiles_x, n_tiles, bg0, bg1, bg2, rgb,
                       contrib, work);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace nvgs
