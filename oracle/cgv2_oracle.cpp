// cgv2_oracle.cpp -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow FP64 CPU reference of the differentiable 2D-Gaussian (surfel)
// tile rasterizer used by CityGaussianV2 (Sec. 3.1, Eq. 1; Sec. 3.2, Eq. 2).
// Only the tests, the smoke check and the benchmark's CPU-baseline leg may
// load it.  It shares no code, header or constant table with the HIP library:
// every formula here is written from its mathematical definition.
//
// What each function follows:
//   orc_project      surfel parameters -> per-view screen transform M = K [R s_u t_u | R s_v t_v | R mu + t],
//                    SH colour, camera-facing normal, opacity, exact conic bounding box
//                    (2DGS surfel model, Sec. 3.1; low-pass filter, Sec. 3.2)
//   orc_tile_reach   which tiles of a surfel's rect its cutoff region can reach (the list rule)
//   orc_bin          per-tile lists ordered by (fp32 depth bits, id) using std::sort
//   orc_render       front-to-back alpha blending of Eq. 1 per pixel, over the tile lists
//   orc_render_brute the same blend over *all* surviving surfels (no tiling): pins the lists
//   orc_render_bwd   reverse-mode of orc_render over stored fragments (chain rule, no T division)
//   orc_project_bwd  chain from d(M, colour, normal, opacity) to the parameters
//   orc_contribution per-surfel contribution of one view (Sec. 3.3, Eq. 3) over the blended pixels;
//                    orc_contribution_brute the same over every surviving surfel (pins the tiled pass)
//   orc_ssim_loss    (1-l) L1 + l (1 - SSIM) with an 11x11 Gaussian window (Sec. 3.1) and its gradient,
//                    once in total and once for the SSIM term alone (the DGD source of Eq. 2)
//   orc_sh_eval      real spherical harmonics from the associated-Legendre definition
//   orc_eval_pairs / orc_blend_trace  the per-pair evaluation and one pixel's fragments with the bounds of the
//                    FP32 error model behind the decision margins (so that tests can check the model)
//
// Readings where the paper is silent are the numbered R* items of the design notes:
// pixel centres at (i+0.5, j+0.5); sigma of the screen low-pass filter sqrt(2)/2 px;
// alpha = min(0.99, o G), skip alpha < 1/255, stop when T(1-alpha) < 1e-4; median depth =
// depth of the last fragment whose incoming T > 0.5; lossless opacity-aware cutoff
// k^2 = 2 ln(255 o); SH colour = max(0, 0.5 + sum f Y).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

const double kPi = 3.14159265358979323846;
const int kTile = 16;
const double kAlphaMin = 1.0 / 255.0;
const double kAlphaMax = 0.99;
const double kTmin = 1e-4;
const double kSigmaF2 = 0.5;  // filter variance in px^2 -> rho2d = |x - c|^2 / sigma^2 = 2 |x - c|^2

// project flags
const int F_VISIBLE = 1, F_NEAR = 2, F_OPACITY = 4, F_BEHIND = 8, F_NONFINITE = 16, F_LOWPASS = 32;

struct Cam {
  int W, H;
  double fx, fy, cx, cy, R[9], t[3], znear, bg[3];
};

Cam load_cam(const double* c) {
  Cam k;
  k.W = (int)c[0];
  k.H = (int)c[1];
  k.fx = c[2]; k.fy = c[3]; k.cx = c[4]; k.cy = c[5];
  for (int i = 0; i < 9; ++i) k.R[i] = c[6 + i];
  for (int i = 0; i < 3; ++i) k.t[i] = c[15 + i];
  k.znear = c[18];
  for (int i = 0; i < 3; ++i) k.bg[i] = c[19 + i];
  return k;
}

// ---------------------------------------------------------------------------------------------
// Real spherical harmonics, from the definition
//   Y_l^m = sqrt(2) K_l^m P_l^m(cos t) cos(m p)   (m > 0)
//   Y_l^-m = sqrt(2) K_l^m P_l^m(cos t) sin(m p)  (m > 0)
//   Y_l^0 = K_l^0 P_l(cos t)
// with the Condon-Shortley phase inside P_l^m.  On the unit sphere
// P_l^m(z) (cos, sin)(m p) = (-1)^m P_l^(m)(z) (Re, Im)((x + i y)^m), so each Y is a polynomial
// in (x, y, z) whose gradient is exact.  Coefficient index = l^2 + l + m.
// ---------------------------------------------------------------------------------------------
struct Poly { std::vector<double> c; };  // ascending powers of z

std::vector<Poly> legendre(int lmax) {
  std::vector<Poly> P(lmax + 1);
  P[0].c = {1.0};
  if (lmax >= 1) P[1].c = {0.0, 1.0};
  for (int l = 1; l < lmax; ++l) {  // (l+1) P_{l+1} = (2l+1) z P_l - l P_{l-1}
    std::vector<double> r(l + 2, 0.0);
    for (size_t k = 0; k < P[l].c.size(); ++k) r[k + 1] += (2 * l + 1) * P[l].c[k];
    for (size_t k = 0; k < P[l - 1].c.size(); ++k) r[k] -= l * P[l - 1].c[k];
    for (auto& v : r) v /= (l + 1);
    P[l + 1].c = r;
  }
  return P;
}

Poly deriv(const Poly& p, int times) {
  Poly r = p;
  for (int t = 0; t < times; ++t) {
    if (r.c.size() <= 1) { r.c = {0.0}; break; }
    std::vector<double> d(r.c.size() - 1);
    for (size_t k = 1; k < r.c.size(); ++k) d[k - 1] = k * r.c[k];
    r.c = d;
  }
  return r;
}

void peval(const Poly& p, double z, double* v, double* dv) {
  double s = 0, ds = 0;
  for (int k = (int)p.c.size() - 1; k >= 0; --k) {
    ds = ds * z + s;
    s = s * z + p.c[k];
  }
  *v = s;
  *dv = ds;
}

double fact(int n) { double r = 1; for (int i = 2; i <= n; ++i) r *= i; return r; }

// Y[k] and dY[k][3] (gradient in R^3 of the polynomial extension) for k < (deg+1)^2
void sh_eval(int deg, const double d[3], double* Y, double (*dY)[3]) {
  static std::vector<Poly> P = legendre(3);
  const double x = d[0], y = d[1], z = d[2];
  for (int l = 0; l <= deg; ++l) {
    for (int m = 0; m <= l; ++m) {
      Poly Pm = deriv(P[l], m);
      double pv, pd;
      peval(Pm, z, &pv, &pd);
      double K = std::sqrt((2 * l + 1) / (4 * kPi) * fact(l - m) / fact(l + m));
      double sgn = (m % 2) ? -1.0 : 1.0;
      // (x + i y)^m and its derivative m (x + i y)^(m-1)
      double re = 1, im = 0, dre = 0, dim = 0;
      for (int k = 0; k < m; ++k) {
        dre = re; dim = im;  // holds (x+iy)^(m-1) after the loop
        double nr = re * x - im * y, ni = re * y + im * x;
        re = nr; im = ni;
      }
      if (m > 0) { dre *= m; dim *= m; }
      if (m == 0) {
        int k = l * l + l;
        Y[k] = K * pv;
        if (dY) { dY[k][0] = 0; dY[k][1] = 0; dY[k][2] = K * pd; }
      } else {
        double c = std::sqrt(2.0) * K * sgn;
        int kp = l * l + l + m, kn = l * l + l - m;
        Y[kp] = c * pv * re;
        Y[kn] = c * pv * im;
        if (dY) {
          // d/dx (x+iy)^m = m (x+iy)^(m-1); d/dy = i m (x+iy)^(m-1)
          dY[kp][0] = c * pv * dre;
          dY[kp][1] = c * pv * (-dim);
          dY[kp][2] = c * pd * re;
          dY[kn][0] = c * pv * dim;
          dY[kn][1] = c * pv * dre;
          dY[kn][2] = c * pd * im;
        }
      }
    }
  }
}

// rotation from a unit quaternion (w, x, y, z); columns are t_u, t_v, n
void quat_to_rot(const double q[4], double R[9]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z); R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z); R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y); R[7] = 2 * (y * z + w * x); R[8] = 1 - 2 * (x * x + y * y);
}

// dR_ij / dq_k for the formula above, d[9][4]
void quat_to_rot_jac(const double q[4], double d[9][4]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  double J[9][4] = {
      {0, 0, -4 * y, -4 * z},          {-2 * z, 2 * y, 2 * x, -2 * w}, {2 * y, 2 * z, 2 * w, 2 * x},
      {2 * z, 2 * y, 2 * x, 2 * w},    {0, -4 * x, 0, -4 * z},         {-2 * x, -2 * w, 2 * z, 2 * y},
      {-2 * y, 2 * z, -2 * w, 2 * x},  {2 * x, 2 * w, 2 * z, 2 * y},   {0, -4 * x, -4 * y, 0}};
  std::memcpy(d, J, sizeof(J));
}

inline double sigmoid(double v) { return 1.0 / (1.0 + std::exp(-v)); }

struct Params {
  int64_t n;
  int deg;
  const double *mean, *log_scale, *quat, *logit, *sh;
};

// geometric quantities of one surfel in one view
struct Geo {
  double su, sv, o, qn[4], Rw[9], tu[3], tv[3], nw[3];
  double pc[3];    // camera-space centre R mu + t
  double M[9];     // row-major 3x3
  double nc[3];    // camera normal after flip
  double flip;     // +1 or -1
  double dir[3], dist;  // view direction (mu - C)/|mu - C|
};

void geometry(const Params& P, const Cam& cam, int64_t i, Geo& g) {
  const int64_t n = P.n;
  g.su = std::exp(P.log_scale[i]);
  g.sv = std::exp(P.log_scale[n + i]);
  g.o = sigmoid(P.logit[i]);
  double q[4] = {P.quat[i], P.quat[n + i], P.quat[2 * n + i], P.quat[3 * n + i]};
  double qq = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int k = 0; k < 4; ++k) g.qn[k] = q[k] / qq;
  quat_to_rot(g.qn, g.Rw);
  for (int r = 0; r < 3; ++r) { g.tu[r] = g.Rw[3 * r]; g.tv[r] = g.Rw[3 * r + 1]; g.nw[r] = g.Rw[3 * r + 2]; }
  const double mu[3] = {P.mean[i], P.mean[n + i], P.mean[2 * n + i]};
  double cu[3], cv[3];
  for (int r = 0; r < 3; ++r) {
    g.pc[r] = cam.t[r];
    cu[r] = cv[r] = 0;
    g.nc[r] = 0;
    for (int c = 0; c < 3; ++c) {
      g.pc[r] += cam.R[3 * r + c] * mu[c];
      cu[r] += cam.R[3 * r + c] * g.su * g.tu[c];
      cv[r] += cam.R[3 * r + c] * g.sv * g.tv[c];
      g.nc[r] += cam.R[3 * r + c] * g.nw[c];
    }
  }
  // M = K [cu | cv | pc]
  const double* cols[3] = {cu, cv, g.pc};
  for (int c = 0; c < 3; ++c) {
    g.M[0 + c] = cam.fx * cols[c][0] + cam.cx * cols[c][2];
    g.M[3 + c] = cam.fy * cols[c][1] + cam.cy * cols[c][2];
    g.M[6 + c] = cols[c][2];
  }
  double dp = g.nc[0] * g.pc[0] + g.nc[1] * g.pc[1] + g.nc[2] * g.pc[2];
  g.flip = dp > 0 ? -1.0 : 1.0;
  for (int r = 0; r < 3; ++r) g.nc[r] *= g.flip;
  // camera centre C = -R^T t
  double C[3];
  for (int c = 0; c < 3; ++c) C[c] = -(cam.R[c] * cam.t[0] + cam.R[3 + c] * cam.t[1] + cam.R[6 + c] * cam.t[2]);
  double v[3] = {mu[0] - C[0], mu[1] - C[1], mu[2] - C[2]};
  g.dist = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  for (int r = 0; r < 3; ++r) g.dir[r] = v[r] / g.dist;
}

// Fragility margins only (never results): an FP32 evaluation of the intersection is modelled as
// exact arithmetic on data carrying a relative error of kU32 -- every coefficient of the affine map
// (x', y') -> p written in the frame centred on the projected centre, and the offsets x', y' themselves
// (rounded relative to a tile origin at most 16 px away) -- propagated to first order through
// u = p0/p2, v = p1/p2 and rho, times a safety factor.  (Emulating the FP32 evaluation of 1.6e5
// (pixel, surfel) pairs of a 10 M-surfel aerial view gave actual / bound <= 1.32 before the factor.)
// T carries the relative errors of its alpha factors and two roundings per step.
const double kU32 = 5.9604644775390625e-8;  // 2^-24
const double kErrSafety = 3.0;

// ray-splat evaluation at pixel sample (x, y) for a screen transform M (row-major)
struct Eval {
  double a[3], b[3], p[3], rho3, rho2, rho, G, araw, alpha, zf, u, v, cxp, cyp;
  double drho3, drho2, dalpha_rel;  // error bounds of rho3, rho2 and relative bound of alpha (FP32 model)
  bool is3d, clamped;
};

inline void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

void evaluate(const double* M, double o, double x, double y, Eval& e) {
  const double* m1 = M;
  const double* m2 = M + 3;
  const double* m3 = M + 6;
  for (int k = 0; k < 3; ++k) { e.a[k] = x * m3[k] - m1[k]; e.b[k] = y * m3[k] - m2[k]; }
  e.p[0] = e.a[1] * e.b[2] - e.a[2] * e.b[1];
  e.p[1] = e.a[2] * e.b[0] - e.a[0] * e.b[2];
  e.p[2] = e.a[0] * e.b[1] - e.a[1] * e.b[0];
  if (std::fabs(e.p[2]) > 0) {
    e.u = e.p[0] / e.p[2];
    e.v = e.p[1] / e.p[2];
    e.rho3 = e.u * e.u + e.v * e.v;
  } else {
    e.u = e.v = 0;
    e.rho3 = INFINITY;
  }
  e.cxp = M[2] / M[8];
  e.cyp = M[5] / M[8];
  const double dx = x - e.cxp, dy = y - e.cyp;
  e.rho2 = (dx * dx + dy * dy) / kSigmaF2;
  e.is3d = e.rho3 <= e.rho2;
  e.rho = e.is3d ? e.rho3 : e.rho2;
  e.G = std::exp(-0.5 * e.rho);
  e.araw = o * e.G;
  e.clamped = e.araw > kAlphaMax;
  e.alpha = e.clamped ? kAlphaMax : e.araw;
  e.zf = e.is3d ? (m3[0] * e.u + m3[1] * e.v + m3[2]) : M[8];

  // error model (see kU32): with a = dx m3 + a0, b = dy m3 + b0 (a0 = cx m3 - m1, b0 = cy m3 - m2),
  // p = dx (m3 x b0) + dy (a0 x m3) + a0 x b0
  const double eps = kErrSafety * kU32;
  double a0[3], b0[3], px[3], py[3], p0[3];
  for (int k = 0; k < 3; ++k) { a0[k] = e.cxp * m3[k] - m1[k]; b0[k] = e.cyp * m3[k] - m2[k]; }
  cross3(m3, b0, px);
  cross3(a0, m3, py);
  cross3(a0, b0, p0);
  const double ax = std::fabs(dx), ay = std::fabs(dy);
  double dp[3];
  for (int k = 0; k < 3; ++k)
    dp[k] = eps * (std::fabs(p0[k]) + (2 * ax + kTile) * std::fabs(px[k]) + (2 * ay + kTile) * std::fabs(py[k]));
  if (std::isfinite(e.rho3)) {
    const double ap2 = std::fabs(e.p[2]);
    const double du = (dp[0] + std::fabs(e.u) * dp[2]) / ap2, dv = (dp[1] + std::fabs(e.v) * dp[2]) / ap2;
    e.drho3 = 2 * (std::fabs(e.u) * du + std::fabs(e.v) * dv) + eps * e.rho3;
  } else {
    e.drho3 = INFINITY;
  }
  e.drho2 = eps * (e.rho2 + 2 * (ax * (ax + kTile) + ay * (ay + kTile)) / kSigmaF2);
  // alpha = o exp(-rho/2): relative error rho's half plus the rounding of log2(o) and exp2
  e.dalpha_rel = 0.5 * (e.is3d ? e.drho3 : e.drho2) + eps * (2 + std::fabs(std::log2(o)));
}

uint32_t f32bits(double z) {
  float f = (float)z;
  uint32_t b;
  std::memcpy(&b, &f, 4);
  return b;
}

// relative distance of a positive quantity to a threshold, in log space (|ln(v / thr)|, which is the
// relative difference near the threshold and compares directly with a relative error bound)
inline double relmargin(double v, double thr) { return v > 0 ? std::fabs(std::log(v / thr)) : INFINITY; }

struct PixOut {
  double C[3], D, Dmed, N[3], A, T;
  int64_t last, med, n_eval, n_con;
  double margin;
  uint64_t sig;
};

// One pixel's front-to-back blend over an ordered list of surfel indices.  'order[e]' gives
// the surfel of list entry e; entries [start, end).
// on_frag(n, alpha, T, dalpha, dT) is called for every contributing fragment with the transmittance in
// front of it and the relative error bounds of alpha and T under the FP32 error model.
struct NoFrag {
  void operator()(int64_t, double, double, double, double) const {}
};

template <class IdOf, class OnFrag = NoFrag>
void blend_pixel(IdOf id_of, int64_t start, int64_t end, const double* M, const double* rgb,
                 const double* nrm, const double* opac, const Cam& cam, double x, double y, PixOut& o,
                 OnFrag on_frag = OnFrag()) {
  double T = 1, C[3] = {0, 0, 0}, D = 0, N[3] = {0, 0, 0}, Dmed = 0;
  int64_t med = -1, last = start, n_eval = 0, n_con = 0;
  double margin = INFINITY;
  double dT = 0;  // relative error bound of T under the FP32 error model
  uint64_t sig = 1469598103934665603ull;
  auto mix = [&](uint64_t v) { sig = (sig ^ v) * 1099511628211ull; };
  Eval e;
  // each margin is a relative distance to a decision threshold, net of the FP32 error bound of the
  // quantity decided on
  for (int64_t k = start; k < end; ++k) {
    const int64_t n = id_of(k);
    ++n_eval;
    evaluate(M + 9 * n, opac[n], x, y, e);
    margin = std::min(margin, relmargin(e.alpha, kAlphaMin) - e.dalpha_rel);
    if (e.alpha < kAlphaMin) continue;
    const double Tn = T * (1 - e.alpha);
    const double dTn =
        dT + (e.clamped ? 0.0 : e.alpha / (1 - e.alpha) * e.dalpha_rel) + 2 * kErrSafety * kU32;
    margin = std::min(margin, relmargin(Tn, kTmin) - dTn);
    if (Tn < kTmin) { mix(0xffffffffull); break; }
    ++n_con;
    margin = std::min(margin, relmargin(e.araw, kAlphaMax) - e.dalpha_rel);
    if (std::isfinite(e.rho3))
      margin = std::min(margin, (std::fabs(e.rho3 - e.rho2) - e.drho3 - e.drho2) / std::max(e.rho3, e.rho2));
    margin = std::min(margin, relmargin(T, 0.5) - dT);
    dT = dTn;
    mix((uint64_t)n * 4 + (e.is3d ? 1 : 0) + (e.clamped ? 2 : 0));
    on_frag(n, e.alpha, T, e.clamped ? 0.0 : e.dalpha_rel, dT);
    const double w = e.alpha * T;
    for (int c = 0; c < 3; ++c) { C[c] += w * rgb[3 * n + c]; N[c] += w * nrm[3 * n + c]; }
    D += w * e.zf;
    if (T > 0.5) { Dmed = e.zf; med = k; }
    T = Tn;
    last = k + 1;
  }
  mix((uint64_t)(med + 7));
  for (int c = 0; c < 3; ++c) o.C[c] = C[c] + T * cam.bg[c];
  o.D = D; o.Dmed = Dmed;
  for (int c = 0; c < 3; ++c) o.N[c] = N[c];
  o.A = 1 - T; o.T = T; o.last = last; o.med = med; o.n_eval = n_eval; o.n_con = n_con;
  o.margin = margin; o.sig = sig;
}

void store_pix(const PixOut& po, int64_t p, int64_t HW, double* out_rgb, double* out_depth, double* out_dmed,
               double* out_normal, double* out_alpha, double* out_T, int64_t* out_last, int64_t* out_med,
               double* out_margin, uint64_t* out_sig) {
  for (int c = 0; c < 3; ++c) { out_rgb[c * HW + p] = po.C[c]; out_normal[c * HW + p] = po.N[c]; }
  out_depth[p] = po.D; out_dmed[p] = po.Dmed; out_alpha[p] = po.A; out_T[p] = po.T;
  out_last[p] = po.last; out_med[p] = po.med;
  if (out_margin) out_margin[p] = po.margin;
  if (out_sig) out_sig[p] = po.sig;
}

template <class Range>
void contribution_pass(Range range, const double* M, const double* rgb, const double* nrm, const double* opac,
                       const Cam& cam, double gamma, double fragile_thr, double* out_sum, int64_t* out_cnt,
                       int32_t* out_fragile, double* out_err) {
#pragma omp parallel for schedule(dynamic)
  for (int j = 0; j < cam.H; ++j) {
    for (int i = 0; i < cam.W; ++i) {
      int64_t start, end;
      auto id_of = range(i, j, start, end);
      PixOut po;
      blend_pixel(id_of, start, end, M, rgb, nrm, opac, cam, i + 0.5, j + 0.5, po,
                  [&](int64_t n, double alpha, double T, double da, double dT) {
                    const double c = std::pow(alpha, gamma) * std::pow(T, 1 - gamma);
#pragma omp atomic
                    out_sum[n] += c;
#pragma omp atomic
                    out_cnt[n] += 1;
                    if (out_err) {
                      // first-order error of c = alpha^g T^(1-g) from those of alpha and T, plus the FP32
                      // evaluation of exp2(g log2 alpha + (1 - g) log2 T) (argument error ~ 16 ulp)
                      const double e = c * (gamma * da + (1 - gamma) * dT + 16 * kU32);
#pragma omp atomic
                      out_err[n] += e;
                    }
                  });
      if (po.margin < fragile_thr)
        for (int64_t k = start; k < start + po.n_eval; ++k) {
#pragma omp atomic
          out_fragile[id_of(k)] += 1;
        }
    }
  }
}

// Tile reach helpers (see orc_tile_reach).
void cross(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// x in [xl, xh], y in [yl, yh], centre-relative
bool tile_reached(const double* M, double K, double xl, double xh, double yl, double yh) {
  // screen-filter branch: rho2d = 2 |x - c|^2
  const double dx = xl > 0 ? xl : (xh < 0 ? xh : 0.0), dy = yl > 0 ? yl : (yh < 0 ? yh : 0.0);
  if (2 * (dx * dx + dy * dy) <= K) return true;
  double c1[3], c2[3], c3[3];
  cross(M + 3, M + 6, c1);
  cross(M + 6, M, c2);
  cross(M, M + 3, c3);
  const double cx = M[2] / M[8], cy = M[5] / M[8];
  double pc[3];
  for (int k = 0; k < 3; ++k) pc[k] = cx * c1[k] + cy * c2[k] + c3[k];
  // q(x, y) = Q00 x^2 + 2 Q01 x y + Q11 y^2 + 2 B0 x + 2 B1 y + D
  auto dot = [&](const double* u, const double* v) { return u[0] * v[0] + u[1] * v[1] - K * u[2] * v[2]; };
  const double Q00 = dot(c1, c1), Q01 = dot(c1, c2), Q11 = dot(c2, c2);
  const double B0 = dot(c1, pc), B1 = dot(c2, pc), D = dot(pc, pc);
  const double det = Q00 * Q11 - Q01 * Q01;
  if (!(Q00 > 0 && Q11 > 0 && det > 0)) return true;
  const double xs = -(Q11 * B0 - Q01 * B1) / det, ys = -(Q00 * B1 - Q01 * B0) / det;
  if (xs >= xl && xs <= xh && ys >= yl && ys <= yh) return true;
  auto q = [&](double x, double y) { return Q00 * x * x + 2 * Q01 * x * y + Q11 * y * y + 2 * B0 * x + 2 * B1 * y + D; };
  auto clamp = [](double v, double lo, double hi) { return std::min(std::max(v, lo), hi); };
  double best = INFINITY;
  for (double X : {xl, xh}) best = std::min(best, q(X, clamp(-(Q01 * X + B1) / Q11, yl, yh)));
  for (double Y : {yl, yh}) best = std::min(best, q(clamp(-(Q01 * Y + B0) / Q00, xl, xh), Y));
  return best <= 0;
}

bool tile_reach_at(const double* M, double k2, int tx, int ty, double Kscale, double pad) {
  const double K = (k2 * (1 + 2e-3) + 2e-3) * Kscale;
  const double cx = M[2] / M[8], cy = M[5] / M[8];
  const double xl = kTile * tx + 0.5 - pad - cx, xh = kTile * tx + kTile - 0.5 + pad - cx;
  const double yl = kTile * ty + 0.5 - pad - cy, yh = kTile * ty + kTile - 0.5 + pad - cy;
  return tile_reached(M, K, xl, xh, yl, yh);
}

}  // namespace

extern "C" {

// ------------------------------------------------------------------------------------------
// Projection of every surfel into one view.  Outputs (row-major per surfel):
//   M[n][9], rgb[n][3] (clamped), rgb_raw[n][3] (0.5 + sum f Y, before the clamp), normal[n][3],
//   opac[n], k2[n], bbox[n][4] (x_lo, x_hi, y_lo, y_hi), pix_rect[n][4] (i0, i1, j0, j1 inclusive),
//   tile_rect[n][4] (tx0, ty0, tx1, ty1; end exclusive), radius[n], flags[n]
// ------------------------------------------------------------------------------------------
int orc_project(int64_t n, int deg, const double* mean, const double* log_scale, const double* quat,
                const double* logit, const double* sh, const double* camv, double* M, double* rgb,
                double* rgb_raw, double* normal, double* opac, double* k2o, double* bbox, int32_t* pix_rect,
                int32_t* tile_rect, double* radius, int32_t* flags) {
  if (n < 0 || deg < 0 || deg > 3) return -1;
  const Params P{n, deg, mean, log_scale, quat, logit, sh};
  const Cam cam = load_cam(camv);
  const int K = (deg + 1) * (deg + 1);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    Geo g;
    geometry(P, cam, i, g);
    int fl = 0;
    for (int k = 0; k < 9; ++k) M[9 * i + k] = g.M[k];
    for (int c = 0; c < 3; ++c) normal[3 * i + c] = g.nc[c];
    opac[i] = g.o;
    double Y[16];
    sh_eval(deg, g.dir, Y, nullptr);
    for (int c = 0; c < 3; ++c) {
      double s = 0.5;
      for (int k = 0; k < K; ++k) s += sh[(int64_t)(k * 3 + c) * n + i] * Y[k];
      rgb_raw[3 * i + c] = s;
      rgb[3 * i + c] = std::max(0.0, s);
    }
    bool finite = true;
    for (int k = 0; k < 9; ++k) finite = finite && std::isfinite(g.M[k]);
    finite = finite && std::isfinite(g.o);
    double k2 = 2 * std::log(255.0 * g.o);
    k2o[i] = k2;
    pix_rect[4 * i] = 0; pix_rect[4 * i + 1] = -1; pix_rect[4 * i + 2] = 0; pix_rect[4 * i + 3] = -1;
    for (int k = 0; k < 4; ++k) { tile_rect[4 * i + k] = 0; bbox[4 * i + k] = 0; }
    radius[i] = 0;
    if (!finite) fl |= F_NONFINITE;
    else if (!(g.M[8] > cam.znear)) fl |= F_NEAR;
    else if (!(k2 > 0)) fl |= F_OPACITY;
    if (fl) { flags[i] = fl; continue; }
    const double* Mm = g.M;
    auto Q = [&](int a, int b) {
      return Mm[3 * a] * Mm[3 * b] + Mm[3 * a + 1] * Mm[3 * b + 1] - Mm[3 * a + 2] * Mm[3 * b + 2] / k2;
    };
    const double Q33 = Q(2, 2);
    if (!(Q33 < 0)) { flags[i] = F_BEHIND; continue; }
    const double xb = Q(0, 2) / Q33, yb = Q(1, 2) / Q33;
    const double ex = std::sqrt(std::max(0.0, xb * xb - Q(0, 0) / Q33));
    const double ey = std::sqrt(std::max(0.0, yb * yb - Q(1, 1) / Q33));
    const double ccx = Mm[2] / Mm[8], ccy = Mm[5] / Mm[8];
    const double rf = std::sqrt(k2 * kSigmaF2);  // rho2d <= k2  <=>  |x - c| <= k sigma_f
    const double xlo = std::min(xb - ex, ccx - rf), xhi = std::max(xb + ex, ccx + rf);
    const double ylo = std::min(yb - ey, ccy - rf), yhi = std::max(yb + ey, ccy + rf);
    bbox[4 * i] = xlo; bbox[4 * i + 1] = xhi; bbox[4 * i + 2] = ylo; bbox[4 * i + 3] = yhi;
    radius[i] = std::max(std::max(ex, ey), rf);
    // low-pass dominance at the pixel sample nearest the centre
    {
      Eval e;
      evaluate(Mm, g.o, std::floor(ccx) + 0.5, std::floor(ccy) + 0.5, e);
      if (e.rho2 < e.rho3) fl |= F_LOWPASS;
    }
    const double i0 = std::max(0.0, std::ceil(xlo - 0.5)), i1 = std::min(cam.W - 1.0, std::floor(xhi - 0.5));
    const double j0 = std::max(0.0, std::ceil(ylo - 0.5)), j1 = std::min(cam.H - 1.0, std::floor(yhi - 0.5));
    if (i0 <= i1 && j0 <= j1) {
      fl |= F_VISIBLE;
      pix_rect[4 * i] = (int)i0; pix_rect[4 * i + 1] = (int)i1;
      pix_rect[4 * i + 2] = (int)j0; pix_rect[4 * i + 3] = (int)j1;
      tile_rect[4 * i] = (int)i0 / kTile; tile_rect[4 * i + 1] = (int)j0 / kTile;
      tile_rect[4 * i + 2] = (int)i1 / kTile + 1; tile_rect[4 * i + 3] = (int)j1 / kTile + 1;
    }
    flags[i] = fl;
  }
  return 0;
}

// ------------------------------------------------------------------------------------------
// Tile reach (which tiles of a surfel's rect can hold a blended pixel; reading of the binning).
// A tile lists the surfel when some point of its pixel-sample box [16 tx + 0.5, 16 tx + 15.5] x
// [16 ty + 0.5, 16 ty + 15.5], padded by 1/64 px, has rho = min(rho3d, rho2d) <= K with the cutoff
// enlarged to K = k2 (1 + 2e-3) + 2e-3.  (A pixel can only take the surfel where rho <= k2; the
// enlargement keeps every such pixel whatever the rounding of an FP32 evaluation.)
//   rho2d <= K  <=>  |x - c|^2 <= K / 2: the distance from the projected centre c to the box;
//   rho3d <= K  <=>  q(x) = p0^2 + p1^2 - K p2^2 <= 0, with p = a x b of evaluate() linear in x:
//                    p = x (m2 x m3) + y (m3 x m1) + m1 x m2.  When the quadratic part of q is positive
//                    definite the set is an ellipse and q is convex: it meets the box iff its minimiser
//                    lies in the box or q <= 0 at the minimum along one of the four edges.  Otherwise
//                    (the cutoff ellipse on the surfel's plane reaches the camera plane) every tile of
//                    the rect is kept.
// keep[j] / fragile[j] for the rect tiles of the visible surfels in order (surfel, then tile rows);
// fragile marks decisions that change between K (1 -+ 1e-5) with the pad -+ 1e-3 px.
// ------------------------------------------------------------------------------------------

int64_t orc_tile_reach(int64_t n, const double* M, const double* k2, const int32_t* tile_rect, uint8_t* keep,
                       uint8_t* fragile) {
  std::vector<int64_t> start((size_t)n + 1, 0);
  for (int64_t i = 0; i < n; ++i) {
    const int32_t* r = tile_rect + 4 * i;
    start[i + 1] = start[i] + (int64_t)std::max(0, r[2] - r[0]) * std::max(0, r[3] - r[1]);
  }
  if (!keep) return start[n];
  const double pad = 1.0 / 64.0;
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t i = 0; i < n; ++i) {
    const int32_t* r = tile_rect + 4 * i;
    int64_t j = start[i];
    for (int y = r[1]; y < r[3]; ++y)
      for (int x = r[0]; x < r[2]; ++x, ++j) {
        keep[j] = tile_reach_at(M + 9 * i, k2[i], x, y, 1.0, pad);
        if (fragile)
          fragile[j] = tile_reach_at(M + 9 * i, k2[i], x, y, 1 + 1e-5, pad + 1e-3) !=
                       tile_reach_at(M + 9 * i, k2[i], x, y, 1 - 1e-5, pad - 1e-3);
      }
  }
  return start[n];
}

// ------------------------------------------------------------------------------------------
// Binning: for each tile, the surfels whose tile rect covers it (and, when keep is given, whose
// rect-tile entry of orc_tile_reach is set), ordered by (float32 bits of the centre depth, id).
// offsets[tiles + 1]; ids[K].  Returns K (ids untouched if cap < K).
// ------------------------------------------------------------------------------------------
int64_t orc_bin(int64_t n, int W, int H, const int32_t* tile_rect, const float* depth32, const uint8_t* keep,
                int64_t* offsets, int32_t* ids, int64_t cap) {
  const int tx = (W + kTile - 1) / kTile, ty = (H + kTile - 1) / kTile;
  std::vector<std::vector<std::pair<uint64_t, int32_t>>> lists((size_t)tx * ty);
  int64_t j = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int32_t* r = tile_rect + 4 * i;
    uint32_t bits;
    std::memcpy(&bits, depth32 + i, 4);
    for (int y = r[1]; y < r[3]; ++y)
      for (int x = r[0]; x < r[2]; ++x, ++j)
        if (!keep || keep[j]) lists[(size_t)y * tx + x].push_back({((uint64_t)bits << 32) | (uint32_t)i, (int32_t)i});
  }
  int64_t K = 0;
  offsets[0] = 0;
  for (size_t t = 0; t < lists.size(); ++t) {
    K += (int64_t)lists[t].size();
    offsets[t + 1] = K;
  }
  if (cap < K) return K;
#pragma omp parallel for schedule(dynamic)
  for (int64_t t = 0; t < (int64_t)lists.size(); ++t) {
    auto& L = lists[t];
    std::sort(L.begin(), L.end());
    for (size_t k = 0; k < L.size(); ++k) ids[offsets[t] + k] = L[k].second;
  }
  return K;
}

// ------------------------------------------------------------------------------------------
// Tiled forward render.  Images are planar [c][H][W].  last/med are list indices (med = -1: none).
// counters[0] = evaluated (pixel, entry) pairs, counters[1] = contributing pairs.
// margin[p] = smallest relative margin of any discrete decision at p; sig[p] = decision hash.
// ------------------------------------------------------------------------------------------
int orc_render(int64_t n, const double* M, const double* rgb, const double* nrm, const double* opac,
               const double* camv, const int64_t* offsets, const int32_t* ids, double* out_rgb,
               double* out_depth, double* out_dmed, double* out_normal, double* out_alpha, double* out_T,
               int64_t* out_last, int64_t* out_med, int64_t* counters, double* out_margin, uint64_t* out_sig) {
  (void)n;
  const Cam cam = load_cam(camv);
  const int tx = (cam.W + kTile - 1) / kTile;
  const int64_t HW = (int64_t)cam.W * cam.H;
  int64_t ne = 0, nc = 0;
#pragma omp parallel for schedule(dynamic) reduction(+ : ne, nc)
  for (int j = 0; j < cam.H; ++j) {
    for (int i = 0; i < cam.W; ++i) {
      const int64_t t = (int64_t)(j / kTile) * tx + i / kTile;
      PixOut po;
      blend_pixel([&](int64_t k) { return (int64_t)ids[k]; }, offsets[t], offsets[t + 1], M, rgb, nrm, opac, cam,
                  i + 0.5, j + 0.5, po);
      const int64_t p = (int64_t)j * cam.W + i;
      store_pix(po, p, HW, out_rgb, out_depth, out_dmed, out_normal, out_alpha, out_T, out_last, out_med,
                out_margin, out_sig);
      ne += po.n_eval;
      nc += po.n_con;
    }
  }
  if (counters) { counters[0] = ne; counters[1] = nc; }
  return 0;
}

// Tiled render restricted to a set of tiles (for sampled parity and CPU timing at large sizes).
// Outputs are per listed tile, each 256 pixels in row-major tile order (pixels outside the image
// are left untouched).
int orc_render_tiles(const double* M, const double* rgb, const double* nrm, const double* opac,
                     const double* camv, const int64_t* offsets, const int32_t* ids, int64_t ntiles,
                     const int32_t* tiles, double* out /*[ntiles][256][13]*/, int64_t* counters) {
  const Cam cam = load_cam(camv);
  const int tx = (cam.W + kTile - 1) / kTile;
  int64_t ne = 0, nc = 0;
#pragma omp parallel for schedule(dynamic) reduction(+ : ne, nc)
  for (int64_t s = 0; s < ntiles; ++s) {
    const int t = tiles[s];
    const int ox = (t % tx) * kTile, oy = (t / tx) * kTile;
    for (int ly = 0; ly < kTile; ++ly)
      for (int lx = 0; lx < kTile; ++lx) {
        const int i = ox + lx, j = oy + ly;
        if (i >= cam.W || j >= cam.H) continue;
        PixOut po;
        blend_pixel([&](int64_t k) { return (int64_t)ids[k]; }, offsets[t], offsets[t + 1], M, rgb, nrm, opac,
                    cam, i + 0.5, j + 0.5, po);
        double* o = out + ((s * 256) + ly * kTile + lx) * 13;
        o[0] = po.C[0]; o[1] = po.C[1]; o[2] = po.C[2]; o[3] = po.D; o[4] = po.Dmed;
        o[5] = po.N[0]; o[6] = po.N[1]; o[7] = po.N[2]; o[8] = po.A; o[9] = po.T;
        o[10] = po.margin;
        o[11] = (double)(po.med >= 0 ? ids[po.med] : -1);
        o[12] = (double)(po.last > offsets[t] ? ids[po.last - 1] : -1);
        ne += po.n_eval;
        nc += po.n_con;
      }
  }
  if (counters) { counters[0] = ne; counters[1] = nc; }
  return 0;
}

// ------------------------------------------------------------------------------------------
// Brute force: every pixel blends every surfel that survives the culls (flags without cull bits),
// ordered by (float32 bits of depth, id), with no bounding boxes or tiles.
// ------------------------------------------------------------------------------------------
int orc_render_brute(int64_t n, const double* M, const double* rgb, const double* nrm, const double* opac,
                     const int32_t* flags, const double* camv, double* out_rgb, double* out_depth,
                     double* out_dmed, double* out_normal, double* out_alpha, double* out_T, int64_t* out_med_id) {
  const Cam cam = load_cam(camv);
  const int64_t HW = (int64_t)cam.W * cam.H;
  std::vector<std::pair<uint64_t, int64_t>> order;
  for (int64_t i = 0; i < n; ++i) {
    if (flags[i] & (F_NEAR | F_OPACITY | F_BEHIND | F_NONFINITE)) continue;
    order.push_back({((uint64_t)f32bits(M[9 * i + 8]) << 32) | (uint32_t)i, i});
  }
  std::sort(order.begin(), order.end());
#pragma omp parallel for schedule(dynamic)
  for (int j = 0; j < cam.H; ++j)
    for (int i = 0; i < cam.W; ++i) {
      PixOut po;
      blend_pixel([&](int64_t k) { return order[k].second; }, 0, (int64_t)order.size(), M, rgb, nrm, opac, cam,
                  i + 0.5, j + 0.5, po);
      const int64_t p = (int64_t)j * cam.W + i;
      for (int c = 0; c < 3; ++c) { out_rgb[c * HW + p] = po.C[c]; out_normal[c * HW + p] = po.N[c]; }
      out_depth[p] = po.D; out_dmed[p] = po.Dmed; out_alpha[p] = po.A; out_T[p] = po.T;
      out_med_id[p] = po.med >= 0 ? order[po.med].second : -1;
    }
  return 0;
}

// ------------------------------------------------------------------------------------------
// Contribution of every surfel in one view (Sec. 3.3, Eq. 3): over the pixels P_k at which the surfel
// is blended as a fragment, the sum of alpha^gamma T^(1 - gamma) with T the transmittance in front of
// it, and |P_k|; C_{n,k} = sum / |P_k| (0 when P_k is empty).  fragile[n] counts the pixels at which
// the surfel is evaluated and whose smallest decision margin is below fragile_thr (there an FP32
// evaluation may decide differently, moving the surfel's count by at most 1 and its sum by at most one
// term).  out_err (optional) receives a first-order bound of the error an FP32 evaluation makes in the
// sum, from the FP32 error model of alpha and T.  Accumulates into out_sum / out_cnt / out_fragile /
// out_err (caller zeroes).
// ------------------------------------------------------------------------------------------
int orc_contribution(int64_t n, const double* M, const double* rgb, const double* nrm, const double* opac,
                     const double* camv, const int64_t* offsets, const int32_t* ids, double gamma, double fragile_thr,
                     double* out_sum, int64_t* out_cnt, int32_t* out_fragile, double* out_err) {
  (void)n;
  const Cam cam = load_cam(camv);
  const int tx = (cam.W + kTile - 1) / kTile;
  contribution_pass(
      [&](int i, int j, int64_t& start, int64_t& end) {
        const int64_t t = (int64_t)(j / kTile) * tx + i / kTile;
        start = offsets[t];
        end = offsets[t + 1];
        return [ids](int64_t k) { return (int64_t)ids[k]; };
      },
      M, rgb, nrm, opac, cam, gamma, fragile_thr, out_sum, out_cnt, out_fragile, out_err);
  return 0;
}

// The same over every surviving surfel per pixel (no tiles): pins the tiled pass.
int orc_contribution_brute(int64_t n, const double* M, const double* rgb, const double* nrm, const double* opac,
                           const int32_t* flags, const double* camv, double gamma, double* out_sum,
                           int64_t* out_cnt) {
  const Cam cam = load_cam(camv);
  std::vector<std::pair<uint64_t, int64_t>> order;
  for (int64_t i = 0; i < n; ++i) {
    if (flags[i] & (F_NEAR | F_OPACITY | F_BEHIND | F_NONFINITE)) continue;
    order.push_back({((uint64_t)f32bits(M[9 * i + 8]) << 32) | (uint32_t)i, i});
  }
  std::sort(order.begin(), order.end());
  std::vector<int32_t> fragile((size_t)std::max<int64_t>(n, 1), 0);
  const std::vector<std::pair<uint64_t, int64_t>>* ord = &order;
  contribution_pass(
      [&](int, int, int64_t& start, int64_t& end) {
        start = 0;
        end = (int64_t)ord->size();
        return [ord](int64_t k) { return (*ord)[k].second; };
      },
      M, rgb, nrm, opac, cam, gamma, -1.0, out_sum, out_cnt, fragile.data(), nullptr);
  return 0;
}

// ------------------------------------------------------------------------------------------
// Backward of orc_render.  Upstream images (any may be NULL = zero): d_rgb[3][H][W], d_depth,
// d_dmed, d_normal[3][H][W], d_alpha.  Accumulates (+=) into dM[n][9], d_rgb_s[n][3],
// d_nrm_s[n][3], d_opac[n].  Fragments are stored per pixel; T_i is the product of the
// preceding (1 - alpha), never recovered by division.  counters[0] += (pixel, entry) pairs
// between each pixel's list start and its 'last'.  tile_mask (nullable): only pixels of tiles with
// a non-zero entry are processed (used to time the oracle on a sample of tiles).
// ------------------------------------------------------------------------------------------
int orc_render_bwd(int64_t n, const double* M, const double* rgb, const double* nrm, const double* opac,
                   const double* camv, const int64_t* offsets, const int32_t* ids, const double* d_rgb,
                   const double* d_depth, const double* d_dmed, const double* d_normal, const double* d_alpha,
                   double* dM, double* d_rgb_s, double* d_nrm_s, double* d_opac, int64_t* counters,
                   const uint8_t* tile_mask) {
  const Cam cam = load_cam(camv);
  const int tx = (cam.W + kTile - 1) / kTile;
  const int64_t HW = (int64_t)cam.W * cam.H;
  // per-thread accumulation buffers, reduced at the end in thread order
  std::vector<std::vector<double>> acc;
  int64_t pairs = 0;
#pragma omp parallel reduction(+ : pairs)
  {
#pragma omp single
    {
      int T = 1;
#ifdef _OPENMP
      T = omp_get_num_threads();
#endif
      acc.assign(T, std::vector<double>());
    }
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    std::vector<double>& A = acc[tid];
    A.assign((size_t)n * 16, 0.0);  // 9 M + 3 rgb + 3 nrm + 1 opac
    struct Frag { int64_t n, k; Eval e; double T; };
    std::vector<Frag> fr;
#pragma omp for schedule(dynamic)
    for (int j = 0; j < cam.H; ++j) {
      for (int i = 0; i < cam.W; ++i) {
        const int64_t p = (int64_t)j * cam.W + i;
        const int64_t t = (int64_t)(j / kTile) * tx + i / kTile;
        if (tile_mask && !tile_mask[t]) continue;
        const double x = i + 0.5, y = j + 0.5;
        // forward, storing contributing fragments
        fr.clear();
        double T = 1;
        int64_t med = -1, last = offsets[t];
        for (int64_t k = offsets[t]; k < offsets[t + 1]; ++k) {
          Frag f;
          f.n = ids[k];
          f.k = k;
          evaluate(M + 9 * f.n, opac[f.n], x, y, f.e);
          if (f.e.alpha < kAlphaMin) continue;
          const double Tn = T * (1 - f.e.alpha);
          if (Tn < kTmin) break;
          f.T = T;
          if (T > 0.5) med = k;
          fr.push_back(f);
          T = Tn;
          last = k + 1;
        }
        pairs += last - offsets[t];
        const double Tf = T;
        double gC[3], gN[3];
        for (int c = 0; c < 3; ++c) {
          gC[c] = d_rgb ? d_rgb[c * HW + p] : 0;
          gN[c] = d_normal ? d_normal[c * HW + p] : 0;
        }
        const double gD = d_depth ? d_depth[p] : 0, gDm = d_dmed ? d_dmed[p] : 0, gA = d_alpha ? d_alpha[p] : 0;
        // after-sums S_i = sum_{j > i} w_j x_j (+ T_final * bg for colour)
        double SC[3] = {Tf * cam.bg[0], Tf * cam.bg[1], Tf * cam.bg[2]}, SD = 0, SN[3] = {0, 0, 0};
        for (int64_t q = (int64_t)fr.size() - 1; q >= 0; --q) {
          const Frag& f = fr[q];
          const Eval& e = f.e;
          const int64_t s = f.n;
          const double w = e.alpha * f.T;
          const double* c_s = rgb + 3 * s;
          const double* n_s = nrm + 3 * s;
          // d out / d alpha_i
          double dL_dalpha = 0;
          for (int c = 0; c < 3; ++c) {
            dL_dalpha += gC[c] * (f.T * c_s[c] - SC[c] / (1 - e.alpha));
            dL_dalpha += gN[c] * (f.T * n_s[c] - SN[c] / (1 - e.alpha));
          }
          dL_dalpha += gD * (f.T * e.zf - SD / (1 - e.alpha));
          dL_dalpha += gA * Tf / (1 - e.alpha);
          double* As = A.data() + (size_t)s * 16;
          for (int c = 0; c < 3; ++c) { As[9 + c] += gC[c] * w; As[12 + c] += gN[c] * w; }
          double dL_dzf = gD * w + (f.k == med ? gDm : 0.0);
          // update after-sums to include fragment i (for the next, earlier fragment)
          for (int c = 0; c < 3; ++c) { SC[c] += w * c_s[c]; SN[c] += w * n_s[c]; }
          SD += w * e.zf;
          double dL_drho = 0;
          if (!e.clamped) {
            As[15] += dL_dalpha * e.G;
            dL_drho = dL_dalpha * opac[s] * e.G * (-0.5);
          }
          const double* m3 = M + 9 * s + 6;
          double* dm1 = As;
          double* dm2 = As + 3;
          double* dm3 = As + 6;
          if (e.is3d) {
            const double p1 = e.p[0], p2 = e.p[1], p3 = e.p[2];
            double g[3];
            g[0] = dL_drho * 2 * p1 / (p3 * p3) + dL_dzf * m3[0] / p3;
            g[1] = dL_drho * 2 * p2 / (p3 * p3) + dL_dzf * m3[1] / p3;
            g[2] = dL_drho * (-2) * (p1 * p1 + p2 * p2) / (p3 * p3 * p3) - dL_dzf * (m3[0] * p1 + m3[1] * p2) / (p3 * p3);
            // p = a x b: dL/da = b x g, dL/db = g x a
            const double* a = e.a;
            const double* b = e.b;
            double ga[3] = {b[1] * g[2] - b[2] * g[1], b[2] * g[0] - b[0] * g[2], b[0] * g[1] - b[1] * g[0]};
            double gb[3] = {g[1] * a[2] - g[2] * a[1], g[2] * a[0] - g[0] * a[2], g[0] * a[1] - g[1] * a[0]};
            for (int k = 0; k < 3; ++k) {
              dm1[k] -= ga[k];
              dm2[k] -= gb[k];
              dm3[k] += x * ga[k] + y * gb[k];
            }
            dm3[0] += dL_dzf * e.u;
            dm3[1] += dL_dzf * e.v;
            dm3[2] += dL_dzf;
          } else {
            // rho2 = (|x - c|^2) / sigma^2, c = (M13, M23) / M33; depth = M33
            const double M13 = M[9 * s + 2], M23 = M[9 * s + 5], M33 = M[9 * s + 8];
            const double dcx = dL_drho * (-2) * (x - e.cxp) / kSigmaF2;
            const double dcy = dL_drho * (-2) * (y - e.cyp) / kSigmaF2;
            dm1[2] += dcx / M33;
            dm2[2] += dcy / M33;
            dm3[2] += -dcx * M13 / (M33 * M33) - dcy * M23 / (M33 * M33) + dL_dzf;
          }
        }
      }
    }
  }
  for (auto& A : acc)
    for (int64_t s = 0; s < n; ++s) {
      const double* a = A.data() + (size_t)s * 16;
      for (int k = 0; k < 9; ++k) dM[9 * s + k] += a[k];
      for (int c = 0; c < 3; ++c) { d_rgb_s[3 * s + c] += a[9 + c]; d_nrm_s[3 * s + c] += a[12 + c]; }
      d_opac[s] += a[15];
    }
  if (counters) counters[0] += pairs;
  return 0;
}

// ------------------------------------------------------------------------------------------
// Chain rule from per-view d(M, colour, normal, opacity) to the parameters; accumulates (+=).
// ------------------------------------------------------------------------------------------
int orc_project_bwd(int64_t n, int deg, const double* mean, const double* log_scale, const double* quat,
                    const double* logit, const double* sh, const double* camv, const double* dM,
                    const double* d_rgb_s, const double* d_nrm_s, const double* d_opac, double* d_mean,
                    double* d_log_scale, double* d_quat, double* d_logit, double* d_sh) {
  const Params P{n, deg, mean, log_scale, quat, logit, sh};
  const Cam cam = load_cam(camv);
  const int K = (deg + 1) * (deg + 1);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    Geo g;
    geometry(P, cam, i, g);
    const double* G = dM + 9 * i;
    // column c of M = K_int * col_c  =>  d col_c = K_int^T dM[:, c]
    double dcol[3][3];
    for (int c = 0; c < 3; ++c) {
      dcol[c][0] = cam.fx * G[c];
      dcol[c][1] = cam.fy * G[3 + c];
      dcol[c][2] = cam.cx * G[c] + cam.cy * G[3 + c] + G[6 + c];
    }
    // world-space: d(world vector) = R_c^T d(camera vector)
    double vw[3][3];
    for (int c = 0; c < 3; ++c)
      for (int r = 0; r < 3; ++r)
        vw[c][r] = cam.R[r] * dcol[c][0] + cam.R[3 + r] * dcol[c][1] + cam.R[6 + r] * dcol[c][2];
    double d_su = 0, d_sv = 0, dtu[3], dtv[3], dnw[3];
    for (int r = 0; r < 3; ++r) {
      d_su += vw[0][r] * g.tu[r];
      d_sv += vw[1][r] * g.tv[r];
      dtu[r] = g.su * vw[0][r];
      dtv[r] = g.sv * vw[1][r];
    }
    const double* dn = d_nrm_s + 3 * i;
    for (int r = 0; r < 3; ++r)
      dnw[r] = g.flip * (cam.R[r] * dn[0] + cam.R[3 + r] * dn[1] + cam.R[6 + r] * dn[2]);
    double dmu[3] = {vw[2][0], vw[2][1], vw[2][2]};
    // rotation columns -> normalized quaternion -> raw quaternion
    double dR[9];
    for (int r = 0; r < 3; ++r) { dR[3 * r] = dtu[r]; dR[3 * r + 1] = dtv[r]; dR[3 * r + 2] = dnw[r]; }
    double J[9][4];
    quat_to_rot_jac(g.qn, J);
    double dqn[4] = {0, 0, 0, 0};
    for (int e = 0; e < 9; ++e)
      for (int k = 0; k < 4; ++k) dqn[k] += dR[e] * J[e][k];
    double q[4] = {quat[i], quat[n + i], quat[2 * n + i], quat[3 * n + i]};
    double qq = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    double dot = 0;
    for (int k = 0; k < 4; ++k) dot += g.qn[k] * dqn[k];
    for (int k = 0; k < 4; ++k) d_quat[k * n + i] += (dqn[k] - g.qn[k] * dot) / qq;
    d_log_scale[i] += d_su * g.su;
    d_log_scale[n + i] += d_sv * g.sv;
    d_logit[i] += d_opac[i] * g.o * (1 - g.o);
    // colour through SH (clamped channels pass nothing)
    double Y[16], dY[16][3];
    sh_eval(deg, g.dir, Y, dY);
    double ddir[3] = {0, 0, 0};
    for (int c = 0; c < 3; ++c) {
      double raw = 0.5;
      for (int k = 0; k < K; ++k) raw += sh[(int64_t)(k * 3 + c) * n + i] * Y[k];
      if (raw < 0) continue;
      const double gc = d_rgb_s[3 * i + c];
      for (int k = 0; k < K; ++k) {
        d_sh[(int64_t)(k * 3 + c) * n + i] += gc * Y[k];
        const double f = sh[(int64_t)(k * 3 + c) * n + i];
        for (int r = 0; r < 3; ++r) ddir[r] += gc * f * dY[k][r];
      }
    }
    // dir = v / |v|: d v = (I - dir dir^T) d dir / |v|
    double dd = ddir[0] * g.dir[0] + ddir[1] * g.dir[1] + ddir[2] * g.dir[2];
    for (int r = 0; r < 3; ++r) dmu[r] += (ddir[r] - g.dir[r] * dd) / g.dist;
    for (int r = 0; r < 3; ++r) d_mean[r * n + i] += dmu[r];
  }
  return 0;
}

// ------------------------------------------------------------------------------------------
// The per-pair evaluation and its FP32 error model, exposed so that a test can hold the model against
// an emulated FP32 evaluation (the model decides which pixels count as fragile).  For m (surfel,
// sample) pairs: M[m][9], opac[m], xy[m][2] -> out[m][8] = rho3, rho2, alpha (clamped), drho3, drho2,
// dalpha_rel (relative), the 3D branch flag, the clamp flag.
// ------------------------------------------------------------------------------------------
int orc_eval_pairs(int64_t m, const double* M, const double* opac, const double* xy, double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    Eval e;
    evaluate(M + 9 * i, opac[i], xy[2 * i], xy[2 * i + 1], e);
    double* o = out + 8 * i;
    o[0] = e.rho3; o[1] = e.rho2; o[2] = e.alpha; o[3] = e.drho3; o[4] = e.drho2; o[5] = e.dalpha_rel;
    o[6] = e.is3d ? 1.0 : 0.0; o[7] = e.clamped ? 1.0 : 0.0;
  }
  return 0;
}

// ------------------------------------------------------------------------------------------
// The contributing fragments of one pixel sample (x, y) over the list ids[0 .. count), in blend order:
// frag[k][5] = surfel id, alpha, transmittance in front, relative bound of alpha, relative bound of the
// transmittance behind it (T (1 - alpha)) under the FP32 error model.  Returns the number of fragments
// (at most cap are written) and the pixel's smallest decision margin in *margin.
// ------------------------------------------------------------------------------------------
int64_t orc_blend_trace(const double* M, const double* rgb, const double* nrm, const double* opac,
                        const double* camv, const int32_t* ids, int64_t count, double x, double y, double* frag,
                        int64_t cap, double* margin) {
  const Cam cam = load_cam(camv);
  PixOut po;
  int64_t k = 0;
  blend_pixel([&](int64_t e) { return (int64_t)ids[e]; }, 0, count, M, rgb, nrm, opac, cam, x, y, po,
              [&](int64_t n, double alpha, double T, double da, double dT) {
                if (k < cap) {
                  double* f = frag + 5 * k;
                  f[0] = (double)n; f[1] = alpha; f[2] = T; f[3] = da; f[4] = dT;
                }
                ++k;
              });
  *margin = po.margin;
  return k;
}

// ------------------------------------------------------------------------------------------
// Threads of the OpenMP loops (the CPU baseline times the oracle at one thread and at all cores);
// returns the number in effect.
// ------------------------------------------------------------------------------------------
int orc_set_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
  return omp_get_max_threads();
#else
  (void)t;
  return 1;
#endif
}

// ------------------------------------------------------------------------------------------
// SH basis values for test pins: Y[m][(deg+1)^2] at m unit directions dirs[m][3].
// ------------------------------------------------------------------------------------------
int orc_sh_eval(int deg, int64_t m, const double* dirs, double* Y, double* dY) {
  const int K = (deg + 1) * (deg + 1);
  for (int64_t i = 0; i < m; ++i) {
    double y[16], dy[16][3];
    sh_eval(deg, dirs + 3 * i, y, dy);
    for (int k = 0; k < K; ++k) {
      Y[i * K + k] = y[k];
      if (dY)
        for (int r = 0; r < 3; ++r) dY[(i * K + k) * 3 + r] = dy[k][r];
    }
  }
  return 0;
}

// ------------------------------------------------------------------------------------------
// L = (1 - lam) mean|x - y| + lam (1 - SSIM(x, y)) over [3][H][W].  SSIM (Wang et al. 2004):
// 11x11 Gaussian window, sigma 1.5, zero padding ('same'), C1 = 0.01^2, C2 = 0.03^2, mean over
// pixels and channels.  Outputs parts[3] = {L, mean L1, SSIM}; dL/dx (total) and d(lam(1-SSIM))/dx;
// ssim_map (nullable) receives the per-pixel SSIM values.
// ------------------------------------------------------------------------------------------
int orc_ssim_loss(int H, int W, const double* x, const double* y, double lam, double* parts, double* dx_total,
                  double* dx_ssim, double* ssim_map) {
  const int R = 5;
  double g[11], gs = 0;
  for (int a = -R; a <= R; ++a) { g[a + R] = std::exp(-(a * a) / (2 * 1.5 * 1.5)); gs += g[a + R]; }
  for (auto& v : g) v /= gs;
  const double C1 = 0.01 * 0.01, C2 = 0.03 * 0.03;
  const int64_t HW = (int64_t)H * W;
  const double Ninv = 1.0 / (3.0 * HW);
  std::vector<double> dmu(3 * HW), dxx(3 * HW), dxy(3 * HW);
  double ssim_sum = 0, l1_sum = 0;
#pragma omp parallel for schedule(static) reduction(+ : ssim_sum, l1_sum)
  for (int64_t cp = 0; cp < 3 * HW; ++cp) {
    const int64_t c = cp / HW, p = cp % HW;
    const int j = (int)(p / W), i = (int)(p % W);
    const double* X = x + c * HW;
    const double* Yv = y + c * HW;
    double mx = 0, my = 0, exx = 0, eyy = 0, exy = 0;
    for (int b = -R; b <= R; ++b)
      for (int a = -R; a <= R; ++a) {
        const int jj = j + b, ii = i + a;
        if (jj < 0 || jj >= H || ii < 0 || ii >= W) continue;
        const double w = g[a + R] * g[b + R];
        const double xv = X[(int64_t)jj * W + ii], yv = Yv[(int64_t)jj * W + ii];
        mx += w * xv; my += w * yv; exx += w * xv * xv; eyy += w * yv * yv; exy += w * xv * yv;
      }
    const double sx = exx - mx * mx, sy = eyy - my * my, sxy = exy - mx * my;
    const double A1 = 2 * mx * my + C1, A2 = 2 * sxy + C2;
    const double B1 = mx * mx + my * my + C1, B2 = sx + sy + C2;
    const double m = A1 * A2 / (B1 * B2);
    if (ssim_map) ssim_map[cp] = m;
    ssim_sum += m;
    // partial derivatives of m w.r.t. (mu_x, E[x^2], E[xy]) with mu_y, E[y^2] fixed
    dmu[cp] = (2 * my * A2 + A1 * 2 * (-my)) / (B1 * B2) - m * (2 * mx / B1 + (-2 * mx) / B2);
    dxx[cp] = -m / B2;
    dxy[cp] = 2 * A1 / (B1 * B2);
    l1_sum += std::fabs(X[p] - Yv[p]);
  }
  const double ssim = ssim_sum * Ninv;
  parts[0] = (1 - lam) * l1_sum * Ninv + lam * (1 - ssim);
  parts[1] = l1_sum * Ninv;
  parts[2] = ssim;
#pragma omp parallel for schedule(static)
  for (int64_t cq = 0; cq < 3 * HW; ++cq) {
    const int64_t c = cq / HW, q = cq % HW;
    const int j = (int)(q / W), i = (int)(q % W);
    double s_mu = 0, s_xx = 0, s_xy = 0;
    for (int b = -R; b <= R; ++b)
      for (int a = -R; a <= R; ++a) {
        const int jj = j - b, ii = i - a;  // output pixel p = q - (a, b) sees q through tap (a, b)
        if (jj < 0 || jj >= H || ii < 0 || ii >= W) continue;
        const double w = g[a + R] * g[b + R];
        const int64_t pp = c * HW + (int64_t)jj * W + ii;
        s_mu += w * dmu[pp]; s_xx += w * dxx[pp]; s_xy += w * dxy[pp];
      }
    const double xv = x[cq], yv = y[cq];
    const double dssim = Ninv * (s_mu + 2 * xv * s_xx + yv * s_xy);
    const double d = xv - yv;
    const double sgn = d > 0 ? 1.0 : (d < 0 ? -1.0 : 0.0);
    dx_ssim[cq] = -lam * dssim;
    dx_total[cq] = (1 - lam) * sgn * Ninv - lam * dssim;
  }
  return 0;
}

}  // extern "C"
