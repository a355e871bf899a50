// NVGS oracle: a plain, slow, FP64 CPU implementation of the per-frame path of
// "NVGS: Neural Visibility for Occlusion Culling in 3D Gaussian Splatting".
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include,
// link or call this file; only the tests, the smoke check and the CPU
// baseline leg of the benchmark use it.  It shares no code with the HIP path.
//
// Every step is written in the order the method states it, with no blocking
// or fusion, so that each function can be read against the paper:
//   scene transform + frustum test on the Gaussian mean          (Sec. 3.3)
//   MLP input: camera in the asset frame, FoV/scale correction
//          (Sec. 3.3, Eq. 2), frequency encoding (Sec. 3.2 counting)
//   visibility MLP, keep iff logit >= 0 (sigmoid >= 0.5)
//   EWA projection of the 3D covariance, SH colour               (Sec. 3.3:
//          the original 3DGS tiled rasterization)
//   footprint: exact AABB of the alpha = 1/255 level set
//   (tile, depth, id) ordering and front-to-back compositing with the
//          1/255 skip and the 1e-4 transmittance stop          (Sec. 4.1)
//   contribution alpha*T and visibility labels                 (Sec. 3.1)
//   BCE-with-logits loss, backward, Adam                       (Sec. 4.1)
//
// Built with g++ -O2 (no fast-math, no FMA contraction) and OpenMP over
// independent outputs only, so results do not depend on the thread count.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kAlphaMin = 1.0 / 255.0;   // skip fragments below this alpha
constexpr double kAlphaMax = 0.99;          // alpha clamp
constexpr double kTMin = 1e-4;              // transmittance stop threshold
constexpr double kGuard = 1.3;              // frustum / Jacobian side guard
constexpr double kDilate = 0.3;             // screen-space low-pass added to Sigma2D

// Instance record: R[9] (asset -> world, row-major), s, t[3]
struct Inst {
  double R[9], s, t[3];
};
// Camera record: pos[3], R[9] (world -> camera rows right, down, forward),
// fovy, width, height, near
struct Cam {
  double pos[3], R[9], fovy, W, H, near;
  double focal() const { return 0.5 * H / std::tan(0.5 * fovy); }
  double tanx() const { return 0.5 * W / focal(); }
  double tany() const { return std::tan(0.5 * fovy); }
};

Inst load_inst(const double* p) {
  Inst r;
  for (int k = 0; k < 9; ++k) r.R[k] = p[k];
  r.s = p[9];
  for (int k = 0; k < 3; ++k) r.t[k] = p[10 + k];
  return r;
}
Cam load_cam(const double* p) {
  Cam c;
  for (int k = 0; k < 3; ++k) c.pos[k] = p[k];
  for (int k = 0; k < 9; ++k) c.R[k] = p[3 + k];
  c.fovy = p[12];
  c.W = p[13];
  c.H = p[14];
  c.near = p[15];
  return c;
}

// y = M x for a row-major 3x3 M
void mat3_vec(const double* M, const double* x, double* y) {
  for (int r = 0; r < 3; ++r) y[r] = M[3 * r] * x[0] + M[3 * r + 1] * x[1] + M[3 * r + 2] * x[2];
}
// y = M^T x
void mat3t_vec(const double* M, const double* x, double* y) {
  for (int r = 0; r < 3; ++r) y[r] = M[r] * x[0] + M[3 + r] * x[1] + M[6 + r] * x[2];
}
// C = A B (3x3, row-major)
void mat3_mul(const double* A, const double* B, double* C) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int k = 0; k < 3; ++k) s += A[3 * i + k] * B[3 * k + j];
      C[3 * i + j] = s;
    }
}

// World position of Gaussian mean mu under instance (R, s, t).
void world_mean(const Inst& in, const double* mu, double* w) {
  double r[3];
  mat3_vec(in.R, mu, r);
  for (int k = 0; k < 3; ++k) w[k] = in.s * r[k] + in.t[k];
}
// Camera-space position p = R_c (w - c).
void cam_space(const Cam& c, const double* w, double* p) {
  double d[3] = {w[0] - c.pos[0], w[1] - c.pos[1], w[2] - c.pos[2]};
  mat3_vec(c.R, d, p);
}

// Frustum test on the mean.  Returns in/out and a relative margin (the
// smallest relative slack of the three inequalities) used by the tests to
// recognise FP32-vs-FP64 threshold cases.
bool in_frustum(const Cam& c, const double* p, double* margin) {
  double tx = kGuard * c.tanx(), ty = kGuard * c.tany();
  double mz = (p[2] - c.near) / std::max(std::fabs(p[2]), c.near);
  double mx = (tx * p[2] - std::fabs(p[0])) / (std::fabs(p[0]) + tx * std::fabs(p[2]) + 1e-300);
  double my = (ty * p[2] - std::fabs(p[1])) / (std::fabs(p[1]) + ty * std::fabs(p[2]) + 1e-300);
  bool in = p[2] > c.near && std::fabs(p[0]) <= tx * p[2] && std::fabs(p[1]) <= ty * p[2];
  if (margin) *margin = std::min(std::fabs(mz), std::min(std::fabs(mx), std::fabs(my)));
  return in;
}

// Camera position in the asset frame.  The global->local transform undoes
// the instance rotation, translation and scale; the factor f_t / f_r of
// Eq. 2, with focal lengths in pixels (so it accounts for both field of view
// and resolution), is applied to the position so that its length is the
// corrected distance.  If a far bound d_max is set, the local distance is
// clamped to it (the distance input is normalised to a fixed range).
void local_camera(const Inst& in, const Cam& c, double train_focal, double d_max, double* cl) {
  double d[3] = {c.pos[0] - in.t[0], c.pos[1] - in.t[1], c.pos[2] - in.t[2]};
  double r[3];
  mat3t_vec(in.R, d, r);
  double f = train_focal / c.focal();
  for (int k = 0; k < 3; ++k) cl[k] = r[k] / in.s * f;
  if (d_max > 0) {
    double len = std::sqrt(cl[0] * cl[0] + cl[1] * cl[1] + cl[2] * cl[2]);
    if (len > d_max)
      for (int k = 0; k < 3; ++k) cl[k] *= d_max / len;
  }
}

// Frequency encoding.  For each scalar x_j and band k = 0..bands-1 emit
// sin(2^k pi x_j) then cos(2^k pi x_j); no identity term (Sec. 3.2 counts
// 5 bands x 6 inputs as 60 values, i.e. two values per band).
void encode(const double* x, int nscalar, int bands, double* out) {
  int o = 0;
  for (int j = 0; j < nscalar; ++j)
    for (int k = 0; k < bands; ++k) {
      double a = std::ldexp(kPi * x[j], k);
      out[o++] = std::sin(a);
      out[o++] = std::cos(a);
    }
}

// The visibility MLP.  P is the packed parameter vector
// (W1 [W x in], b1, W2 [W x W], b2, W3 [W x W], b3, wo [W], bo).  Writes the
// pre-activations of the hidden layers to pre (3*W, nullable) and returns
// the logit together with the scale sum |wo_j h3_j| + |bo| (for tolerances).
double mlp_eval(const double* P, int W, int in_dim, const double* x, double* pre, double* scale) {
  std::vector<double> h(x, x + in_dim), nh(W);
  const double* p = P;
  int fan = in_dim;
  for (int l = 0; l < 3; ++l) {
    const double* Wl = p;
    const double* bl = p + (size_t)W * fan;
    for (int r = 0; r < W; ++r) {
      double s = bl[r];
      for (int k = 0; k < fan; ++k) s += Wl[(size_t)r * fan + k] * h[k];
      if (pre) pre[l * W + r] = s;
      nh[r] = s > 0 ? s : 0.0;
    }
    p = bl + W;
    h.assign(nh.begin(), nh.end());
    fan = W;
  }
  double z = p[W];
  double sc = std::fabs(p[W]);
  for (int k = 0; k < W; ++k) {
    z += p[k] * h[k];
    sc += std::fabs(p[k] * h[k]);
  }
  if (scale) *scale = sc;
  return z;
}

// Real spherical harmonics, l <= 3, order (l, m = -l..l), without the
// Condon-Shortley phase.  Constants follow from
// Y_lm = sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) P_l^|m|(cos th) {sqrt2 cos, sqrt2 sin}.
void sh_basis(const double* d, int degree, double* Y) {
  double x = d[0], y = d[1], z = d[2];
  Y[0] = 0.5 * std::sqrt(1.0 / kPi);
  if (degree < 1) return;
  double c1 = std::sqrt(3.0 / (4.0 * kPi));
  Y[1] = c1 * y;
  Y[2] = c1 * z;
  Y[3] = c1 * x;
  if (degree < 2) return;
  Y[4] = 0.5 * std::sqrt(15.0 / kPi) * x * y;
  Y[5] = 0.5 * std::sqrt(15.0 / kPi) * y * z;
  Y[6] = 0.25 * std::sqrt(5.0 / kPi) * (3.0 * z * z - 1.0);
  Y[7] = 0.5 * std::sqrt(15.0 / kPi) * x * z;
  Y[8] = 0.25 * std::sqrt(15.0 / kPi) * (x * x - y * y);
  if (degree < 3) return;
  Y[9] = 0.25 * std::sqrt(35.0 / (2.0 * kPi)) * y * (3.0 * x * x - y * y);
  Y[10] = 0.5 * std::sqrt(105.0 / kPi) * x * y * z;
  Y[11] = 0.25 * std::sqrt(21.0 / (2.0 * kPi)) * y * (5.0 * z * z - 1.0);
  Y[12] = 0.25 * std::sqrt(7.0 / kPi) * z * (5.0 * z * z - 3.0);
  Y[13] = 0.25 * std::sqrt(21.0 / (2.0 * kPi)) * x * (5.0 * z * z - 1.0);
  Y[14] = 0.25 * std::sqrt(105.0 / kPi) * z * (x * x - y * y);
  Y[15] = 0.25 * std::sqrt(35.0 / (2.0 * kPi)) * x * (x * x - 3.0 * y * y);
}

// rotation matrix of a (not necessarily normalised) quaternion (w, x, y, z)
void quat_to_rot(const double* q0, double* R) {
  double n = std::sqrt(q0[0] * q0[0] + q0[1] * q0[1] + q0[2] * q0[2] + q0[3] * q0[3]);
  double w = 1, x = 0, y = 0, z = 0;
  if (n > 0) { w = q0[0] / n; x = q0[1] / n; y = q0[2] / n; z = q0[3] / n; }
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

// Splat record written by the projection (doubles):
//  0 u, 1 v, 2 a, 3 b, 4 c (Sigma2D), 5..7 conic (A, B, C), 8 depth,
//  9 opacity, 10..12 rgb, 13 ex, 14 ey (footprint half extents), 15 kappa^2
constexpr int kRec = 16;

}  // namespace

extern "C" {

// ---------------------------------------------------------------------------
// Encoding alone (for pins): x [nscalar] -> out [nscalar * bands * 2]
void orc_encode(const double* x, int nscalar, int bands, double* out) { encode(x, nscalar, bands, out); }
void orc_encode_batch(const double* X, int64_t B, int nscalar, int bands, double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < B; ++b) encode(X + b * nscalar, nscalar, bands, out + b * nscalar * bands * 2);
}

// MLP alone (for pins): X [B][in_dim] -> z [B]; pre [B][3W] nullable
void orc_mlp_forward(const double* P, int W, int in_dim, const double* X, int64_t B, double* z,
                     double* pre, double* scale) {
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < B; ++b) {
    double sc;
    z[b] = mlp_eval(P, W, in_dim, X + b * in_dim, pre ? pre + b * 3 * W : nullptr, &sc);
    if (scale) scale[b] = sc;
  }
}

// SH basis alone (for pins): d [3] unit -> Y [(deg+1)^2]
void orc_sh_basis(const double* d, int degree, double* Y) { sh_basis(d, degree, Y); }

// Local camera position for one instance / camera.
void orc_local_camera(const double* inst, const double* cam, double train_focal, double d_max, double* out) {
  local_camera(load_inst(inst), load_cam(cam), train_focal, d_max, out);
}

// ---------------------------------------------------------------------------
// Cull + MLP query for one (camera, instance): state [n] (0 frustum-culled, 1 MLP-culled,
// 2 kept), logit [n] (NaN where the MLP was not queried), margins [n] nullable
// (relative decision margin of the deciding test).
void orc_query(int64_t n, const float* mean, const double* inst_p, const double* cam_p,
               const double* P, int W, int bands, double mean_scale, double cam_scale,
               double train_focal, double d_min, double d_max, int use_mlp,
               uint8_t* state, double* logit, double* margin) {
  Inst in = load_inst(inst_p);
  Cam c = load_cam(cam_p);
  double cl[3];
  local_camera(in, c, train_focal, d_max, cl);
  double cl_len = std::sqrt(cl[0] * cl[0] + cl[1] * cl[1] + cl[2] * cl[2]);
  bool gate_open = cl_len >= d_min;  // below d_min every in-frustum Gaussian is kept
  int in_dim = 6 * bands * 2;
#pragma omp parallel for schedule(static)
  for (int64_t g = 0; g < n; ++g) {
    double mu[3] = {mean[g], mean[n + g], mean[2 * n + g]};
    double w[3], p[3], fm;
    world_mean(in, mu, w);
    cam_space(c, w, p);
    bool inside = in_frustum(c, p, &fm);
    logit[g] = std::numeric_limits<double>::quiet_NaN();
    if (margin) margin[g] = fm;
    if (!inside) { state[g] = 0; continue; }
    if (!use_mlp || !gate_open) { state[g] = 2; continue; }
    double x[6] = {mean_scale * mu[0], mean_scale * mu[1], mean_scale * mu[2],
                   cam_scale * cl[0], cam_scale * cl[1], cam_scale * cl[2]};
    std::vector<double> e(in_dim);
    encode(x, 6, bands, e.data());
    double sc;
    double z = mlp_eval(P, W, in_dim, e.data(), nullptr, &sc);
    logit[g] = z;
    state[g] = z >= 0.0 ? 2 : 1;
    if (margin) margin[g] = std::min(fm, std::fabs(z) / std::max(sc, 1e-300));
  }
}

// ---------------------------------------------------------------------------
// Projection + footprint for m kept Gaussians g[m] of one asset under one (instance, camera).
// Asset arrays are the float32 SoA inputs (stride n).  rec [m][16] doubles,
// prect [m][4] inclusive pixel rectangle (x0, x1, y0, y1); x0 > x1 = empty.
void orc_project(int64_t m, const int64_t* gidx, int64_t n, const float* mean, const float* scale,
                 const float* quat, const float* opacity, const float* sh, int sh_degree,
                 const double* inst_p, const double* cam_p, double* rec, int32_t* prect) {
  Inst in = load_inst(inst_p);
  Cam c = load_cam(cam_p);
  double f = c.focal();
  double tx = kGuard * c.tanx(), ty = kGuard * c.tany();
  double RcRi[9];
  mat3_mul(c.R, in.R, RcRi);
  int K = (sh_degree + 1) * (sh_degree + 1);
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < m; ++j) {
    int64_t g = gidx[j];
    double mu[3] = {mean[g], mean[n + g], mean[2 * n + g]};
    double w[3], p[3];
    world_mean(in, mu, w);
    cam_space(c, w, p);
    // Sigma_l = R(q) diag(s^2) R(q)^T
    double q[4] = {quat[g], quat[n + g], quat[2 * n + g], quat[3 * n + g]};
    double Rq[9];
    quat_to_rot(q, Rq);
    double s2[3] = {(double)scale[g] * scale[g], (double)scale[n + g] * scale[n + g],
                    (double)scale[2 * n + g] * scale[2 * n + g]};
    double Sl[9];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double s = 0;
        for (int k = 0; k < 3; ++k) s += Rq[3 * a + k] * s2[k] * Rq[3 * b + k];
        Sl[3 * a + b] = s;
      }
    // Sigma_c = s_i^2 (Rc Ri) Sigma_l (Rc Ri)^T
    double T1[9], Sc[9];
    mat3_mul(RcRi, Sl, T1);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double s = 0;
        for (int k = 0; k < 3; ++k) s += T1[3 * a + k] * RcRi[3 * b + k];
        Sc[3 * a + b] = in.s * in.s * s;
      }
    // perspective Jacobian with the guard-clamped tangent position
    double z = p[2];
    double txz = std::min(tx, std::max(-tx, p[0] / z)) * z;
    double tyz = std::min(ty, std::max(-ty, p[1] / z)) * z;
    double J[6] = {f / z, 0.0, -f * txz / (z * z), 0.0, f / z, -f * tyz / (z * z)};
    double JS[6];
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 3; ++b) {
        double s = 0;
        for (int k = 0; k < 3; ++k) s += J[3 * a + k] * Sc[3 * k + b];
        JS[3 * a + b] = s;
      }
    double S2[4];
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        double s = 0;
        for (int k = 0; k < 3; ++k) s += JS[3 * a + k] * J[3 * b + k];
        S2[2 * a + b] = s;
      }
    double A = S2[0] + kDilate, B = 0.5 * (S2[1] + S2[2]), C = S2[3] + kDilate;
    double det = A * C - B * B;
    double* r = rec + j * kRec;
    r[0] = f * p[0] / z + 0.5 * c.W;
    r[1] = f * p[1] / z + 0.5 * c.H;
    r[2] = A; r[3] = B; r[4] = C;
    r[5] = C / det; r[6] = -B / det; r[7] = A / det;
    r[8] = z;
    double o = opacity[g];
    r[9] = o;
    // colour from SH along the asset-frame view direction
    double dw[3] = {w[0] - c.pos[0], w[1] - c.pos[1], w[2] - c.pos[2]};
    double dl[3];
    mat3t_vec(in.R, dw, dl);
    double dn = std::sqrt(dl[0] * dl[0] + dl[1] * dl[1] + dl[2] * dl[2]);
    for (int k = 0; k < 3; ++k) dl[k] /= dn;
    double Y[16];
    sh_basis(dl, sh_degree, Y);
    for (int ch = 0; ch < 3; ++ch) {
      double s = 0.5;
      for (int k = 0; k < K; ++k) s += Y[k] * sh[(size_t)(3 * k + ch) * n + g];
      r[10 + ch] = s > 0 ? s : 0.0;
    }
    // footprint: exact AABB of { d : d^T Sigma2D^-1 d <= kappa^2 }, kappa^2 = 2 ln(255 o),
    // widened by 1e-4 e + 1e-3 px
    int32_t* pr = prect + 4 * j;
    double k2 = 2.0 * std::log(255.0 * o);
    r[15] = k2;
    if (k2 < 0) {
      r[13] = r[14] = 0;
      pr[0] = 1; pr[1] = 0; pr[2] = 1; pr[3] = 0;
      continue;
    }
    double ex = std::sqrt(k2 * A), ey = std::sqrt(k2 * C);
    r[13] = ex; r[14] = ey;
    double wx = 1e-4 * ex + 1e-3, wy = 1e-4 * ey + 1e-3;
    double x0 = std::ceil(r[0] - ex - 0.5 - wx), x1 = std::floor(r[0] + ex - 0.5 + wx);
    double y0 = std::ceil(r[1] - ey - 0.5 - wy), y1 = std::floor(r[1] + ey - 0.5 + wy);
    x0 = std::max(x0, 0.0); y0 = std::max(y0, 0.0);
    x1 = std::min(x1, c.W - 1); y1 = std::min(y1, c.H - 1);
    if (x0 > x1 || y0 > y1) { pr[0] = 1; pr[1] = 0; pr[2] = 1; pr[3] = 0; continue; }
    pr[0] = (int32_t)x0; pr[1] = (int32_t)x1; pr[2] = (int32_t)y0; pr[3] = (int32_t)y1;
  }
}

// ---------------------------------------------------------------------------
// Binning + compositing for one camera: splats rec [m][16] (already in S order, id = index),
// prect [m][4] pixel rectangles, tile size T.  Builds the (tile, depth, id)
// ordered lists and composites each pixel front to back.
//   image [H][W][3], tfinal [H][W], contrib [m] (max alpha*T over blended
//   fragments; accumulated with max so several cameras may share it),
//   reached [m] (set to 1 if tested with alpha >= 1/255 before the stop),
//   margin [H][W][2] nullable: [0] smallest relative margin of any alpha /
//   stop decision taken at the pixel, [1] smallest relative depth gap between
//   consecutive fragments with alpha >= 1/255, up to and including the first
//   such fragment after the stop (how close the pixel's blend order is to a
//   tie).
//   order_out nullable: the sorted (tile, id) list, ntile_entries returned.
//   smargin [m][2] nullable: per splat, the smallest pixel margins ([0] alpha /
//   stop, [1] depth order, as in `margin`) of every decision taken at a pixel
//   up to and including that splat's own test there, and, at a pixel that
//   stopped, of all decisions up to the stop for every splat listed after it
//   (min-accumulated like contrib): how close the splat's contribution and
//   "reached" state are to changing with a decision elsewhere.
int64_t orc_render(int64_t m, const double* rec, const int32_t* prect, const double* cam_p, int T,
                   const double* bg, double* image, double* tfinal, double* contrib, uint8_t* reached,
                   double* margin, int64_t* order_out, int64_t order_cap, double* smargin) {
  Cam c = load_cam(cam_p);
  int W = (int)c.W, H = (int)c.H;
  int tw = (W + T - 1) / T, th = (H + T - 1) / T;
  struct Entry { int64_t tile; double depth; int64_t id; };
  std::vector<Entry> ent;
  for (int64_t j = 0; j < m; ++j) {
    const int32_t* pr = prect + 4 * j;
    if (pr[0] > pr[1] || pr[2] > pr[3]) continue;
    for (int ty = pr[2] / T; ty <= pr[3] / T; ++ty)
      for (int tx = pr[0] / T; tx <= pr[1] / T; ++tx)
        ent.push_back({(int64_t)ty * tw + tx, rec[j * kRec + 8], j});
  }
  std::stable_sort(ent.begin(), ent.end(), [](const Entry& a, const Entry& b) {
    if (a.tile != b.tile) return a.tile < b.tile;
    if (a.depth != b.depth) return a.depth < b.depth;
    return a.id < b.id;
  });
  if (order_out)
    for (size_t k = 0; k < ent.size() && (int64_t)k < order_cap; ++k) {
      order_out[2 * k] = ent[k].tile;
      order_out[2 * k + 1] = ent[k].id;
    }
  std::vector<int64_t> start(tw * th + 1, (int64_t)ent.size());
  for (int64_t k = (int64_t)ent.size() - 1; k >= 0; --k) start[ent[k].tile] = k;
  for (int t = tw * th - 1; t >= 0; --t) start[t] = std::min(start[t], start[t + 1]);
  // per-pixel compositing; contrib/reached updates are collected per thread
  int nthreads = 1;
#ifdef _OPENMP
  nthreads = omp_get_max_threads();
#endif
  std::vector<std::vector<double>> cmax(nthreads);
  std::vector<std::vector<uint8_t>> rch(nthreads);
  std::vector<std::vector<double>> smg(nthreads);
#pragma omp parallel
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    cmax[tid].assign(contrib ? m : 0, 0.0);
    rch[tid].assign(reached ? m : 0, 0);
    smg[tid].assign(smargin ? 2 * m : 0, std::numeric_limits<double>::infinity());
    auto note = [&](int64_t j, double a_m, double d_m) {
      if (!smargin) return;
      smg[tid][2 * j] = std::min(smg[tid][2 * j], a_m);
      smg[tid][2 * j + 1] = std::min(smg[tid][2 * j + 1], d_m);
    };
#pragma omp for schedule(dynamic, 16)
    for (int64_t pix = 0; pix < (int64_t)W * H; ++pix) {
      int px = (int)(pix % W), py = (int)(pix / W);
      int64_t tile = (int64_t)(py / T) * tw + px / T;
      double cx = px + 0.5, cy = py + 0.5;
      double Tr = 1.0, col[3] = {0, 0, 0};
      double mg = std::numeric_limits<double>::infinity();
      double mgd = std::numeric_limits<double>::infinity();
      double prev_depth = -1.0;
      for (int64_t k = start[tile]; k < start[tile + 1]; ++k) {
        int64_t j = ent[k].id;
        const double* r = rec + j * kRec;
        double dx = cx - r[0], dy = cy - r[1];
        double q = r[5] * dx * dx + 2.0 * r[6] * dx * dy + r[7] * dy * dy;
        double power = -0.5 * q;
        if (power > 0) continue;
        double a = std::min(kAlphaMax, r[9] * std::exp(power));
        mg = std::min(mg, std::fabs(a - kAlphaMin) / kAlphaMin);
        if (a < kAlphaMin) {
          note(j, mg, mgd);
          continue;
        }
        if (prev_depth >= 0) mgd = std::min(mgd, (r[8] - prev_depth) / r[8]);
        prev_depth = r[8];
        double Tn = Tr * (1.0 - a);
        mg = std::min(mg, std::fabs(Tn - kTMin) / kTMin);
        note(j, mg, mgd);
        if (reached) rch[tid][j] = 1;
        if (Tn < kTMin) {
          // the next fragment with alpha >= 1/255 comes after the stop only
          // by its depth: a renderer whose depths tie them may blend it
          // before this one, so its depth gap is a decision margin too
          for (int64_t k2 = k + 1; k2 < start[tile + 1]; ++k2) {
            const double* r2 = rec + ent[k2].id * kRec;
            const double ex = cx - r2[0], ey = cy - r2[1];
            const double q2 = r2[5] * ex * ex + 2.0 * r2[6] * ex * ey + r2[7] * ey * ey;
            if (std::min(kAlphaMax, r2[9] * std::exp(-0.5 * q2)) < kAlphaMin) continue;
            mgd = std::min(mgd, (r2[8] - r[8]) / r2[8]);
            break;
          }
          note(j, mg, mgd);
          for (int64_t k2 = k + 1; smargin && k2 < start[tile + 1]; ++k2) note(ent[k2].id, mg, mgd);
          break;
        }
        for (int ch = 0; ch < 3; ++ch) col[ch] += a * Tr * r[10 + ch];
        if (contrib) cmax[tid][j] = std::max(cmax[tid][j], a * Tr);
        Tr = Tn;
      }
      for (int ch = 0; ch < 3; ++ch) image[3 * pix + ch] = col[ch] + Tr * bg[ch];
      if (tfinal) tfinal[pix] = Tr;
      if (margin) { margin[2 * pix] = mg; margin[2 * pix + 1] = mgd; }
    }
  }
  for (int t = 0; t < nthreads; ++t) {
    if (contrib && !cmax[t].empty())
      for (int64_t j = 0; j < m; ++j) contrib[j] = std::max(contrib[j], cmax[t][j]);
    if (reached && !rch[t].empty())
      for (int64_t j = 0; j < m; ++j) reached[j] |= rch[t][j];
    if (smargin && !smg[t].empty())
      for (int64_t j = 0; j < 2 * m; ++j) smargin[j] = std::min(smargin[j], smg[t][j]);
  }
  return (int64_t)ent.size();
}

// Tile-free reference: every pixel visits every splat in (depth, id) order,
// with no footprint rectangle at all.  Used to pin the tiled renderer.
void orc_render_brute(int64_t m, const double* rec, const double* cam_p, const double* bg,
                      double* image, double* tfinal) {
  Cam c = load_cam(cam_p);
  int W = (int)c.W, H = (int)c.H;
  std::vector<int64_t> ord(m);
  for (int64_t j = 0; j < m; ++j) ord[j] = j;
  std::stable_sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) {
    double da = rec[a * kRec + 8], db = rec[b * kRec + 8];
    if (da != db) return da < db;
    return a < b;
  });
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t pix = 0; pix < (int64_t)W * H; ++pix) {
    double cx = (double)(pix % W) + 0.5, cy = (double)(pix / W) + 0.5;
    double Tr = 1.0, col[3] = {0, 0, 0};
    for (int64_t k = 0; k < m; ++k) {
      const double* r = rec + ord[k] * kRec;
      double dx = cx - r[0], dy = cy - r[1];
      double q = r[5] * dx * dx + 2.0 * r[6] * dx * dy + r[7] * dy * dy;
      double power = -0.5 * q;
      if (power > 0) continue;
      double a = std::min(kAlphaMax, r[9] * std::exp(power));
      if (a < kAlphaMin) continue;
      double Tn = Tr * (1.0 - a);
      if (Tn < kTMin) break;
      for (int ch = 0; ch < 3; ++ch) col[ch] += a * Tr * r[10 + ch];
      Tr = Tn;
    }
    for (int ch = 0; ch < 3; ++ch) image[3 * pix + ch] = col[ch] + Tr * bg[ch];
    if (tfinal) tfinal[pix] = Tr;
  }
}

// ---------------------------------------------------------------------------
// Mean BCE-with-logits over a batch, its gradient w.r.t. all packed
// parameters (dP, same layout as P), and optionally dX.  Optional per-sample
// weights w [B] (nullable = 1).  Returns the loss.
double orc_bce_backward(const double* P, int W, int in_dim, const double* X, const double* y,
                        const double* wts, int64_t B, double* dP, double* dX) {
  size_t np = (size_t)in_dim * W + W + 2 * ((size_t)W * W + W) + W + 1;
  std::fill(dP, dP + np, 0.0);
  double loss = 0.0;
  // serial over the batch: the gradient is a sum and its order stays fixed
  std::vector<double> h0(in_dim), pre(3 * W), h(3 * W), d(W), dn(W);
  const double* Wl[3];
  double* dWl[3];
  double* dbl[3];
  {
    size_t off = 0;
    int fan = in_dim;
    for (int l = 0; l < 3; ++l) {
      Wl[l] = P + off; dWl[l] = dP + off;
      off += (size_t)W * fan;
      dbl[l] = dP + off;
      off += W;
      fan = W;
    }
  }
  const double* wo = P + np - W - 1;
  double* dwo = dP + np - W - 1;
  for (int64_t b = 0; b < B; ++b) {
    const double* x = X + b * in_dim;
    double z = mlp_eval(P, W, in_dim, x, pre.data(), nullptr);
    for (int k = 0; k < 3 * W; ++k) h[k] = pre[k] > 0 ? pre[k] : 0.0;
    double wb = wts ? wts[b] : 1.0;
    double yb = y[b];
    loss += wb * (std::max(z, 0.0) - z * yb + std::log1p(std::exp(-std::fabs(z))));
    double sig = 1.0 / (1.0 + std::exp(-z));
    double dz = wb * (sig - yb) / (double)B;
    // output layer
    for (int k = 0; k < W; ++k) {
      dwo[k] += dz * h[2 * W + k];
      d[k] = dz * wo[k] * (pre[2 * W + k] > 0 ? 1.0 : 0.0);
    }
    dwo[W] += dz;
    // hidden layers 3, 2, 1
    for (int l = 2; l >= 0; --l) {
      int fan = l == 0 ? in_dim : W;
      const double* hin = l == 0 ? x : h.data() + (l - 1) * W;
      for (int r = 0; r < W; ++r) {
        dbl[l][r] += d[r];
        for (int k = 0; k < fan; ++k) dWl[l][(size_t)r * fan + k] += d[r] * hin[k];
      }
      if (l > 0) {
        for (int k = 0; k < W; ++k) {
          double s = 0;
          for (int r = 0; r < W; ++r) s += d[r] * Wl[l][(size_t)r * W + k];
          dn[k] = s * (pre[(l - 1) * W + k] > 0 ? 1.0 : 0.0);
        }
        d.swap(dn);
      } else if (dX) {
        for (int k = 0; k < in_dim; ++k) {
          double s = 0;
          for (int r = 0; r < W; ++r) s += d[r] * Wl[0][(size_t)r * in_dim + k];
          dX[b * in_dim + k] = s;
        }
      }
    }
  }
  return loss / (double)B;
}

// Adam (beta1, beta2, eps; bias-corrected), one step t >= 1, in place.
void orc_adam_step(int64_t n, double* p, const double* g, double* m, double* v, int64_t t, double lr,
                   double b1, double b2, double eps) {
  double c1 = 1.0 - std::pow(b1, (double)t), c2 = 1.0 - std::pow(b2, (double)t);
  for (int64_t k = 0; k < n; ++k) {
    m[k] = b1 * m[k] + (1.0 - b1) * g[k];
    v[k] = b2 * v[k] + (1.0 - b2) * g[k] * g[k];
    double mh = m[k] / c1, vh = v[k] / c2;
    p[k] -= lr * mh / (std::sqrt(vh) + eps);
  }
}

// ---------------------------------------------------------------------------
// Reduced-precision forms of the visibility MLP: operands rounded to BF16 or
// to OCP FP8 E4M3 where the GEMM chain consumes them, everything else in
// FP64 (FP32 where the value is stored as FP32).  prec: 1 = BF16, 2 = FP8.
//   BF16: round-to-nearest-even to 8 significant bits of the float32 value.
//   E4M3: 4 exponent bits (bias 7), 3 mantissa bits, largest finite 448,
//         subnormal spacing 2^-9, round-to-nearest-even.
// FP8 per-layer scales are powers of two: weights by 448 / max|W| of each
// GEMM, inputs by 448 over an interval bound of the activations
// (|gamma| <= 1; |h1| <= max_r sum_k |W1[r,k]| + |b1[r]|;
//  |h2| <= max_r sum_k |W2[r,k]| |h1|max + |b2[r]|).
static double to_f32(double x) { return (double)(float)x; }

static double to_bf16(double x) {
  float f = (float)x;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  uint32_t lsb = (u >> 16) & 1u;
  u = (u + 0x7FFFu + lsb) & 0xFFFF0000u;
  std::memcpy(&f, &u, 4);
  return (double)f;
}

static double to_e4m3(double x) {
  double a = std::fabs(x);
  if (a == 0.0) return 0.0;
  int e = (int)std::floor(std::log2(a));
  if (e < -6) e = -6;                       // subnormal range: fixed spacing 2^-9
  double q = std::ldexp(1.0, e - 3);         // spacing of representable values
  double m = a / q;
  double r = std::nearbyint(m);              // ties to even (default rounding mode)
  double v = std::min(r * q, 448.0);
  return x < 0 ? -v : v;
}

static double pow2_floor(double x) { return std::ldexp(1.0, (int)std::floor(std::log2(x))); }

}  // extern "C" (reopened below)
extern "C" {

// scales[9]: invU, inv2, inv3, saH1, saH2, saG, sw1, sw2, sw3
void orc_fp8_scales(const double* P, int W, double* scales) {
  const double* W1 = P;
  const double* b1 = W1 + (size_t)W * 72;
  const double* W2 = b1 + W;
  const double* b2 = W2 + (size_t)W * W;
  const double* W3 = b2 + W;
  double m1 = 0, m2 = 0, m3 = 0, B1 = 0, B2 = 0;
  for (int r = 0; r < W; ++r)
    for (int k = 0; k < 36; ++k) m1 = std::max(m1, std::fabs(W1[(size_t)r * 72 + k]));
  for (size_t i = 0; i < (size_t)W * W; ++i) {
    m2 = std::max(m2, std::fabs(W2[i]));
    m3 = std::max(m3, std::fabs(W3[i]));
  }
  for (int r = 0; r < W; ++r) {
    double s = std::fabs(b1[r]);
    for (int k = 0; k < 72; ++k) s += std::fabs(W1[(size_t)r * 72 + k]);
    B1 = std::max(B1, s);
  }
  for (int r = 0; r < W; ++r) {
    double s = 0;
    for (int k = 0; k < W; ++k) s += std::fabs(W2[(size_t)r * W + k]);
    B2 = std::max(B2, s * B1 + std::fabs(b2[r]));
  }
  double sw1 = pow2_floor(448.0 / m1), sw2 = pow2_floor(448.0 / m2), sw3 = pow2_floor(448.0 / m3);
  double sag = pow2_floor(448.0), sa1 = pow2_floor(448.0 / B1), sa2 = pow2_floor(448.0 / B2);
  double out[9] = {1.0 / (sw1 * sag), 1.0 / (sw2 * sa1), 1.0 / (sw3 * sa2), sa1, sa2, sag, sw1, sw2, sw3};
  for (int k = 0; k < 9; ++k) scales[k] = out[k];
}

// X [B][72] encoded inputs (Gaussian half first), z [B]
void orc_mlp_forward_q(const double* P, int W, const double* X, int64_t B, int prec, double* z) {
  double sc[9] = {1, 1, 1, 1, 1, 1, 1, 1, 1};
  if (prec == 2) orc_fp8_scales(P, W, sc);
  auto q = [&](double v) { return prec == 1 ? to_bf16(v) : to_e4m3(v); };
  const double* W1 = P;
  const double* b1 = W1 + (size_t)W * 72;
  const double* W2 = b1 + W;
  const double* b2 = W2 + (size_t)W * W;
  const double* W3 = b2 + W;
  const double* b3 = W3 + (size_t)W * W;
  const double* wo = b3 + W;
  std::vector<double> W1q((size_t)W * 36), W2q((size_t)W * W), W3q((size_t)W * W);
  for (int r = 0; r < W; ++r)
    for (int k = 0; k < 36; ++k) W1q[(size_t)r * 36 + k] = q(W1[(size_t)r * 72 + k] * sc[6]);
  for (size_t i = 0; i < (size_t)W * W; ++i) {
    W2q[i] = q(W2[i] * sc[7]);
    W3q[i] = q(W3[i] * sc[8]);
  }
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < B; ++b) {
    const double* x = X + b * 72;
    std::vector<double> g(36), h1(W), h2(W);
    for (int k = 0; k < 36; ++k) g[k] = q(to_f32(x[k]) * sc[5]);
    for (int r = 0; r < W; ++r) {
      double u = 0, c = b1[r];
      for (int k = 0; k < 36; ++k) u += W1q[(size_t)r * 36 + k] * g[k];
      for (int k = 36; k < 72; ++k) c += W1[(size_t)r * 72 + k] * x[k];
      double h = to_f32(to_f32(u) * sc[0] + to_f32(c));
      h1[r] = q(to_f32(std::max(h, 0.0)) * sc[3]);
    }
    for (int r = 0; r < W; ++r) {
      double a = 0;
      for (int k = 0; k < W; ++k) a += W2q[(size_t)r * W + k] * h1[k];
      h2[r] = q(to_f32(std::max(to_f32(a) * sc[1] + b2[r], 0.0)) * sc[4]);
    }
    double zz = wo[W];
    for (int r = 0; r < W; ++r) {
      double a = 0;
      for (int k = 0; k < W; ++k) a += W3q[(size_t)r * W + k] * h2[k];
      zz += wo[r] * std::max(to_f32(a) * sc[2] + b3[r], 0.0);
    }
    z[b] = zz;
  }
}

// OpenMP threads of the parallel loops (for timing the oracle on 1 core and on
// all cores); results do not depend on it.
void orc_set_threads(int n) {
#ifdef _OPENMP
  omp_set_num_threads(n > 0 ? n : omp_get_num_procs());
#else
  (void)n;
#endif
}
int orc_max_threads() {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// The two roundings on their own (for the pins of the reduced-precision checker).
double orc_to_bf16(double x) { return to_bf16(x); }
double orc_to_e4m3(double x) { return to_e4m3(x); }

// Learning rate of step t (0-based) of a T-step run under the schedule of
// Sec. 4.1: the rate rises along a cosine from 0 to lr over the first 20 % of
// the iterations (Tw = max(1, round(0.2 T)) steps; step t < Tw uses the
// warm-up curve evaluated at the end of the step, (t + 1) / Tw, so the last
// warm-up step runs at lr), then decays exponentially from lr at step Tw to
// lr_final at the last step T - 1 (a fixed ratio per step).
double orc_lr_schedule(double lr, double lr_final, int64_t T, int64_t t) {
  const int64_t Tw = std::max<int64_t>(1, (int64_t)std::llround(0.2 * (double)T));
  if (t < Tw) {
    const double phase = (double)(t + 1) / (double)Tw;  // in (0, 1]
    return lr * 0.5 * (1.0 - std::cos(kPi * phase));
  }
  if (T - Tw <= 1) return lr_final;  // a single decay step ends at lr_final
  const double frac = (double)(t - Tw) / (double)(T - 1 - Tw);  // 0 at Tw, 1 at T - 1
  return lr * std::pow(lr_final / lr, frac);
}

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) evaluated at counter i:
// the i-th output of the generator seeded with `seed`.
uint64_t orc_splitmix64(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// The paper's compact MLP form (Sec. 3.2, 3.3, 4.1).  A secondary MLP maps a
// Gaussian's opacity, scales and rotation to a 6-D embedding, computed once
// per asset; the visibility MLP takes 16 inputs: the normalised mean, the
// unit direction from the camera to the Gaussian, the camera distance mapped
// to [-1, 1] by min-max over the asset's distance range, the camera forward
// vector (all in the asset frame) and the embedding.  Both have two hidden
// layers of 32 ReLU units; outputs 1 (logit) and 6 (linear).
// Parameters (one packed vector): visibility W1[32][16] b1[32] W2[32][32]
// b2[32] wo[32] bo, then embedding E1[32][8] e1[32] E2[32][32] e2[32]
// E3[6][32] e3[6].
// ---------------------------------------------------------------------------
constexpr int kCH = 32, kCIn = 16, kCEIn = 8, kCEOut = 6;
constexpr int kCVis = kCH * kCIn + kCH + kCH * kCH + kCH + kCH + 1;                // 1633
constexpr int kCEmb = kCH * kCEIn + kCH + kCH * kCH + kCH + kCEOut * kCH + kCEOut;  // 1542

// y = W x + b for a row-major W [rows][cols]
static void dense(const double* W, const double* b, int rows, int cols, const double* x, double* y) {
  for (int r = 0; r < rows; ++r) {
    double s = b[r];
    for (int k = 0; k < cols; ++k) s += W[(size_t)r * cols + k] * x[k];
    y[r] = s;
  }
}

// embedding inputs: opacity, log scales, unit quaternion with w >= 0 (q and -q
// are the same rotation)
static void cembed_input(double o, const double* s, const double* q, double* xe) {
  xe[0] = o;
  for (int k = 0; k < 3; ++k) xe[1 + k] = std::log(s[k]);
  double n = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  double sg = q[0] < 0 ? -1.0 : 1.0;
  for (int k = 0; k < 4; ++k) xe[4 + k] = sg * q[k] / n;
}

// embedding MLP; pre1/pre2 (nullable) receive the hidden pre-activations
static void cembed(const double* PE, const double* xe, double* e, double* pre1, double* pre2) {
  const double* E1 = PE;
  const double* e1 = E1 + kCH * kCEIn;
  const double* E2 = e1 + kCH;
  const double* e2 = E2 + kCH * kCH;
  const double* E3 = e2 + kCH;
  const double* e3 = E3 + kCEOut * kCH;
  double a[kCH], h[kCH], a2[kCH], h2[kCH];
  dense(E1, e1, kCH, kCEIn, xe, a);
  for (int r = 0; r < kCH; ++r) h[r] = a[r] > 0 ? a[r] : 0.0;
  dense(E2, e2, kCH, kCH, h, a2);
  for (int r = 0; r < kCH; ++r) h2[r] = a2[r] > 0 ? a2[r] : 0.0;
  dense(E3, e3, kCEOut, kCH, h2, e);
  if (pre1) std::copy(a, a + kCH, pre1);
  if (pre2) std::copy(a2, a2 + kCH, pre2);
}

// visibility MLP: logit; scale (nullable) = sum |wo h2| + |bo| (the size of
// the terms the logit is a sum of)
static double cvis(const double* PV, const double* x, double* pre1, double* pre2, double* scale) {
  const double* W1 = PV;
  const double* b1 = W1 + kCH * kCIn;
  const double* W2 = b1 + kCH;
  const double* b2 = W2 + kCH * kCH;
  const double* wo = b2 + kCH;
  double a[kCH], h[kCH], a2[kCH];
  dense(W1, b1, kCH, kCIn, x, a);
  for (int r = 0; r < kCH; ++r) h[r] = a[r] > 0 ? a[r] : 0.0;
  dense(W2, b2, kCH, kCH, h, a2);
  double z = wo[kCH], sc = std::fabs(wo[kCH]);
  for (int r = 0; r < kCH; ++r) {
    double h2 = a2[r] > 0 ? a2[r] : 0.0;
    z += wo[r] * h2;
    sc += std::fabs(wo[r] * h2);
  }
  if (pre1) std::copy(a, a + kCH, pre1);
  if (pre2) std::copy(a2, a2 + kCH, pre2);
  if (scale) *scale = sc;
  return z;
}

// The first ten visibility inputs of Gaussian mean mu (asset frame) under an
// instance and camera: sigma_mu mu, the unit direction from the camera to the
// Gaussian, the distance corrected by f_t / f_r (Eq. 2, pixel focal lengths;
// the instance scale is undone by working in the asset frame) and mapped to
// [-1, 1] over [d_min, d_max] (clamped), and the camera forward vector.
static void cinputs10(const Inst& in, const Cam& c, double train_focal, double d_min, double d_max,
                      double mean_scale, const double* mu, double* x) {
  double d[3] = {c.pos[0] - in.t[0], c.pos[1] - in.t[1], c.pos[2] - in.t[2]};
  double r[3], cl[3];
  mat3t_vec(in.R, d, r);
  for (int k = 0; k < 3; ++k) cl[k] = r[k] / in.s;
  double v[3] = {mu[0] - cl[0], mu[1] - cl[1], mu[2] - cl[2]};
  double len = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  double dt = len * train_focal / c.focal();
  double dn = 2.0 * (dt - d_min) / (d_max - d_min) - 1.0;
  dn = std::min(1.0, std::max(-1.0, dn));
  double fw[3];
  mat3t_vec(in.R, c.R + 6, fw);  // forward row of R_c, into the asset frame
  for (int k = 0; k < 3; ++k) {
    x[k] = mean_scale * mu[k];
    x[3 + k] = v[k] / len;
    x[7 + k] = fw[k];
  }
  x[6] = dn;
}

extern "C" {

int orc_compact_sizes(int which) { return which == 0 ? kCVis : kCEmb; }

// embeddings E [n][6] of every Gaussian of an asset (P: full parameter vector)
void orc_cembed(int64_t n, const float* scale, const float* quat, const float* opacity, const double* P,
                double* E, double* XE) {
#pragma omp parallel for schedule(static)
  for (int64_t g = 0; g < n; ++g) {
    double s[3] = {scale[g], scale[n + g], scale[2 * n + g]};
    double q[4] = {quat[g], quat[n + g], quat[2 * n + g], quat[3 * n + g]};
    double xe[kCEIn];
    cembed_input(opacity[g], s, q, xe);
    cembed(P + kCVis, xe, E + g * kCEOut, nullptr, nullptr);
    if (XE) std::copy(xe, xe + kCEIn, XE + g * kCEIn);
  }
}

// visibility inputs X [m][16] of Gaussians gidx under an instance and camera
void orc_cinputs(int64_t m, const int64_t* gidx, int64_t n, const float* mean, const double* E,
                 const double* inst_p, const double* cam_p, double train_focal, double d_min, double d_max,
                 double mean_scale, double* X) {
  Inst in = load_inst(inst_p);
  Cam c = load_cam(cam_p);
  for (int64_t j = 0; j < m; ++j) {
    const int64_t g = gidx[j];
    double mu[3] = {mean[g], mean[n + g], mean[2 * n + g]};
    double* x = X + j * kCIn;
    cinputs10(in, c, train_focal, d_min, d_max, mean_scale, mu, x);
    for (int k = 0; k < kCEOut; ++k) x[10 + k] = E[g * kCEOut + k];
  }
}

void orc_cmlp_forward(const double* P, const double* X, int64_t B, double* z, double* scale) {
  for (int64_t b = 0; b < B; ++b) z[b] = cvis(P, X + b * kCIn, nullptr, nullptr, scale ? scale + b : nullptr);
}

// The joint compact model on raw inputs: the embedding of each sample from
// its eight embedding inputs XE [B][8], then the visibility MLP on the ten
// other inputs XV [B][10] and that embedding.  z [B]; scale [B] (nullable)
// as in cvis.
void orc_cjoint_forward(const double* P, const double* XV, const double* XE, int64_t B, double* z, double* scale) {
  for (int64_t b = 0; b < B; ++b) {
    double x[kCIn];
    std::copy(XV + b * 10, XV + b * 10 + 10, x);
    cembed(P + kCVis, XE + b * kCEIn, x + 10, nullptr, nullptr);
    z[b] = cvis(P, x, nullptr, nullptr, scale ? scale + b : nullptr);
  }
}

// Logits of the compact visibility MLP with its second-layer operands (the
// weights and the first hidden layer's activations) rounded to BF16; the
// first layer and the output in FP64 otherwise.  X [B][16].
void orc_cmlp_forward_bf16(const double* P, const double* X, int64_t B, double* z) {
  const double* W1 = P;
  const double* b1 = W1 + kCH * kCIn;
  const double* W2 = b1 + kCH;
  const double* b2 = W2 + kCH * kCH;
  const double* wo = b2 + kCH;
  for (int64_t b = 0; b < B; ++b) {
    double a[kCH], h[kCH];
    dense(W1, b1, kCH, kCIn, X + b * kCIn, a);
    for (int r = 0; r < kCH; ++r) h[r] = to_bf16(to_f32(a[r] > 0 ? a[r] : 0.0));
    double zz = wo[kCH];
    for (int r = 0; r < kCH; ++r) {
      double s = b2[r];
      for (int k = 0; k < kCH; ++k) s += to_bf16(W2[r * kCH + k]) * h[k];
      zz += wo[r] * (s > 0 ? s : 0.0);
    }
    z[b] = zz;
  }
}

// Cull + compact-MLP query for every Gaussian of one (instance, camera): as
// orc_query; the gate compares the corrected distance of the camera from the
// asset centre with d_min.
void orc_cquery(int64_t n, const float* mean, const double* E, const double* inst_p, const double* cam_p,
                const double* P, double mean_scale, double train_focal, double d_min, double d_max, int use_mlp,
                uint8_t* state, double* logit, double* margin) {
  Inst in = load_inst(inst_p);
  Cam c = load_cam(cam_p);
  double cl[3];
  local_camera(in, c, train_focal, 0.0, cl);
  double cl_len = std::sqrt(cl[0] * cl[0] + cl[1] * cl[1] + cl[2] * cl[2]);
  bool gate_open = cl_len >= d_min;
#pragma omp parallel for schedule(static)
  for (int64_t g = 0; g < n; ++g) {
    double mu[3] = {mean[g], mean[n + g], mean[2 * n + g]};
    double w[3], p[3], fm;
    world_mean(in, mu, w);
    cam_space(c, w, p);
    bool inside = in_frustum(c, p, &fm);
    logit[g] = std::numeric_limits<double>::quiet_NaN();
    if (margin) margin[g] = fm;
    if (!inside) { state[g] = 0; continue; }
    if (!use_mlp || !gate_open) { state[g] = 2; continue; }
    double x[kCIn];
    cinputs10(in, c, train_focal, d_min, d_max, mean_scale, mu, x);
    for (int k = 0; k < kCEOut; ++k) x[10 + k] = E[g * kCEOut + k];
    double sc;
    double z = cvis(P, x, nullptr, nullptr, &sc);
    logit[g] = z;
    state[g] = z >= 0.0 ? 2 : 1;
    if (margin) margin[g] = std::min(fm, std::fabs(z) / std::max(sc, 1e-300));
  }
}

// Weighted BCE-with-logits over a batch of the joint model (the embedding of
// each sample computed from its inputs XE [B][8], the other ten visibility
// inputs XV [B][10]), and the gradient dP [kCVis + kCEmb] of the mean loss.
double orc_cbce_backward(const double* P, const double* XV, const double* XE, const double* y, const double* wts,
                         int64_t B, double* dP) {
  std::fill(dP, dP + kCVis + kCEmb, 0.0);
  const double* W1 = P;
  const double* W2 = W1 + kCH * kCIn + kCH;
  const double* wo = W2 + kCH * kCH + kCH;
  const double* PE = P + kCVis;
  const double* E2 = PE + kCH * kCEIn + kCH;
  const double* E3 = E2 + kCH * kCH + kCH;
  double* dW1 = dP;
  double* db1 = dW1 + kCH * kCIn;
  double* dW2 = db1 + kCH;
  double* db2 = dW2 + kCH * kCH;
  double* dwo = db2 + kCH;
  double* dE1 = dP + kCVis;
  double* de1 = dE1 + kCH * kCEIn;
  double* dE2 = de1 + kCH;
  double* de2 = dE2 + kCH * kCH;
  double* dE3 = de2 + kCH;
  double* de3 = dE3 + kCEOut * kCH;
  double loss = 0.0;
  // serial over the batch: the gradient is a sum in a fixed order
  for (int64_t b = 0; b < B; ++b) {
    double x[kCIn], pe1[kCH], pe2[kCH], p1[kCH], p2[kCH];
    const double* xe = XE + b * kCEIn;
    for (int k = 0; k < 10; ++k) x[k] = XV[b * 10 + k];
    cembed(PE, xe, x + 10, pe1, pe2);
    double z = cvis(P, x, p1, p2, nullptr);
    double wb = wts ? wts[b] : 1.0, yb = y[b];
    loss += wb * (std::max(z, 0.0) - z * yb + std::log1p(std::exp(-std::fabs(z))));
    double dz = wb * (1.0 / (1.0 + std::exp(-z)) - yb) / (double)B;
    // visibility output and hidden layers
    double d2[kCH], d1[kCH], dx[kCIn];
    for (int r = 0; r < kCH; ++r) {
      double h2 = p2[r] > 0 ? p2[r] : 0.0;
      dwo[r] += dz * h2;
      d2[r] = dz * wo[r] * (p2[r] > 0 ? 1.0 : 0.0);
    }
    dwo[kCH] += dz;
    for (int r = 0; r < kCH; ++r) {
      db2[r] += d2[r];
      for (int k = 0; k < kCH; ++k) dW2[r * kCH + k] += d2[r] * (p1[k] > 0 ? p1[k] : 0.0);
    }
    for (int k = 0; k < kCH; ++k) {
      double s = 0;
      for (int r = 0; r < kCH; ++r) s += d2[r] * W2[r * kCH + k];
      d1[k] = s * (p1[k] > 0 ? 1.0 : 0.0);
    }
    for (int r = 0; r < kCH; ++r) {
      db1[r] += d1[r];
      for (int k = 0; k < kCIn; ++k) dW1[r * kCIn + k] += d1[r] * x[k];
    }
    for (int k = 0; k < kCIn; ++k) {
      double s = 0;
      for (int r = 0; r < kCH; ++r) s += d1[r] * W1[r * kCIn + k];
      dx[k] = s;
    }
    // embedding: output (linear), then its two hidden layers
    double g2[kCH], g1[kCH];
    for (int r = 0; r < kCEOut; ++r) {
      const double de = dx[10 + r];
      de3[r] += de;
      for (int k = 0; k < kCH; ++k) dE3[r * kCH + k] += de * (pe2[k] > 0 ? pe2[k] : 0.0);
    }
    for (int k = 0; k < kCH; ++k) {
      double s = 0;
      for (int r = 0; r < kCEOut; ++r) s += dx[10 + r] * E3[r * kCH + k];
      g2[k] = s * (pe2[k] > 0 ? 1.0 : 0.0);
    }
    for (int r = 0; r < kCH; ++r) {
      de2[r] += g2[r];
      for (int k = 0; k < kCH; ++k) dE2[r * kCH + k] += g2[r] * (pe1[k] > 0 ? pe1[k] : 0.0);
    }
    for (int k = 0; k < kCH; ++k) {
      double s = 0;
      for (int r = 0; r < kCH; ++r) s += g2[r] * E2[r * kCH + k];
      g1[k] = s * (pe1[k] > 0 ? 1.0 : 0.0);
    }
    for (int r = 0; r < kCH; ++r) {
      de1[r] += g1[r];
      for (int k = 0; k < kCEIn; ++k) dE1[r * kCEIn + k] += g1[r] * xe[k];
    }
  }
  return loss / (double)B;
}

}  // extern "C"
