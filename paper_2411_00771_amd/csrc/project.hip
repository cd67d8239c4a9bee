// Per-surfel projection (2DGS surfel model of CityGaussianV2 Sec. 3.1, low-pass filter of
// Sec. 3.2) and its reverse (chain from per-view record gradients to the parameters).
//
// One thread per (surfel, view).  Parameters are read as coalesced planar SoA; the geometry
// (screen transform, centre, inverse homography, conic bound) is computed in FP64, which on
// MI355X runs at the non-packed FP32 rate and keeps the projected centre exact to ~1e-9 px at
// 1600-px widths; the kernel is HBM-bound either way.  SH colour is FP32.
#include "cgv2r_device.h"
#include "cgv2r_kernels.h"

#include <algorithm>

namespace cgv2 {

// Real spherical harmonics (Condon-Shortley phase, index l*l + l + m) as polynomials in the unit
// direction; constants are the normalisations sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) times the
// polynomial factors of the derivatives of P_l.
struct SH {
  static constexpr float c0 = 0.28209479177387814f;   // 1/(2 sqrt(pi))
  static constexpr float c1 = 0.48860251190291992f;   // sqrt(3/(4 pi))
  static constexpr float c2a = 1.0925484305920792f;   // sqrt(15/(4 pi))
  static constexpr float c2b = 0.31539156525252005f;  // sqrt(5/(16 pi))
  static constexpr float c2c = 0.54627421529603959f;  // sqrt(15/(16 pi))
  static constexpr float c3a = 0.59004358992664352f;  // sqrt(35/(32 pi))
  static constexpr float c3b = 2.8906114426405538f;   // sqrt(105/(4 pi))
  static constexpr float c3c = 0.45704579946446572f;  // sqrt(21/(32 pi))
  static constexpr float c3d = 0.37317633259011540f;  // sqrt(7/(16 pi))
  static constexpr float c3e = 1.4453057213202769f;   // sqrt(105/(16 pi))
};

// Y[k] and, if dY != nullptr, the gradient of each polynomial w.r.t. (x, y, z).
template <int deg>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float* Y, float (*dY)[3]) {
  Y[0] = SH::c0;
  if (dY) { dY[0][0] = dY[0][1] = dY[0][2] = 0.f; }
  if (deg < 1) return;
  Y[1] = -SH::c1 * y; Y[2] = SH::c1 * z; Y[3] = -SH::c1 * x;
  if (dY) {
    dY[1][0] = 0.f; dY[1][1] = -SH::c1; dY[1][2] = 0.f;
    dY[2][0] = 0.f; dY[2][1] = 0.f; dY[2][2] = SH::c1;
    dY[3][0] = -SH::c1; dY[3][1] = 0.f; dY[3][2] = 0.f;
  }
  if (deg < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[4] = SH::c2a * x * y;
  Y[5] = -SH::c2a * y * z;
  Y[6] = SH::c2b * (3.f * zz - 1.f);
  Y[7] = -SH::c2a * x * z;
  Y[8] = SH::c2c * (xx - yy);
  if (dY) {
    dY[4][0] = SH::c2a * y; dY[4][1] = SH::c2a * x; dY[4][2] = 0.f;
    dY[5][0] = 0.f; dY[5][1] = -SH::c2a * z; dY[5][2] = -SH::c2a * y;
    dY[6][0] = 0.f; dY[6][1] = 0.f; dY[6][2] = SH::c2b * 6.f * z;
    dY[7][0] = -SH::c2a * z; dY[7][1] = 0.f; dY[7][2] = -SH::c2a * x;
    dY[8][0] = 2.f * SH::c2c * x; dY[8][1] = -2.f * SH::c2c * y; dY[8][2] = 0.f;
  }
  if (deg < 3) return;
  Y[9] = -SH::c3a * y * (3.f * xx - yy);
  Y[10] = SH::c3b * x * y * z;
  Y[11] = -SH::c3c * y * (5.f * zz - 1.f);
  Y[12] = SH::c3d * z * (5.f * zz - 3.f);
  Y[13] = -SH::c3c * x * (5.f * zz - 1.f);
  Y[14] = SH::c3e * z * (xx - yy);
  Y[15] = -SH::c3a * x * (xx - 3.f * yy);
  if (dY) {
    dY[9][0] = -SH::c3a * 6.f * x * y; dY[9][1] = -SH::c3a * (3.f * xx - 3.f * yy); dY[9][2] = 0.f;
    dY[10][0] = SH::c3b * y * z; dY[10][1] = SH::c3b * x * z; dY[10][2] = SH::c3b * x * y;
    dY[11][0] = 0.f; dY[11][1] = -SH::c3c * (5.f * zz - 1.f); dY[11][2] = -SH::c3c * 10.f * y * z;
    dY[12][0] = 0.f; dY[12][1] = 0.f; dY[12][2] = SH::c3d * (15.f * zz - 3.f);
    dY[13][0] = -SH::c3c * (5.f * zz - 1.f); dY[13][1] = 0.f; dY[13][2] = -SH::c3c * 10.f * x * z;
    dY[14][0] = 2.f * SH::c3e * x * z; dY[14][1] = -2.f * SH::c3e * y * z; dY[14][2] = SH::c3e * (xx - yy);
    dY[15][0] = -SH::c3a * (3.f * xx - 3.f * yy); dY[15][1] = SH::c3a * 6.f * x * y; dY[15][2] = 0.f;
  }
}

// sum_k g[k] grad Y_k(x, y, z): the direction gradient of a weighted SH sum without the per-basis
// gradient table.
template <int deg>
__device__ __forceinline__ void sh_grad_dot(const float* g, float x, float y, float z, float* out) {
  float gx = 0.f, gy = 0.f, gz = 0.f;
  if (deg >= 1) {
    gy -= SH::c1 * g[1];
    gz += SH::c1 * g[2];
    gx -= SH::c1 * g[3];
  }
  if (deg >= 2) {
    gx += SH::c2a * y * g[4];
    gy += SH::c2a * x * g[4];
    gy -= SH::c2a * z * g[5];
    gz -= SH::c2a * y * g[5];
    gz += SH::c2b * 6.f * z * g[6];
    gx -= SH::c2a * z * g[7];
    gz -= SH::c2a * x * g[7];
    gx += 2.f * SH::c2c * x * g[8];
    gy -= 2.f * SH::c2c * y * g[8];
  }
  if (deg >= 3) {
    const float xx = x * x, yy = y * y, zz = z * z;
    gx -= SH::c3a * 6.f * x * y * g[9];
    gy -= SH::c3a * (3.f * xx - 3.f * yy) * g[9];
    gx += SH::c3b * y * z * g[10];
    gy += SH::c3b * x * z * g[10];
    gz += SH::c3b * x * y * g[10];
    gy -= SH::c3c * (5.f * zz - 1.f) * g[11];
    gz -= SH::c3c * 10.f * y * z * g[11];
    gz += SH::c3d * (15.f * zz - 3.f) * g[12];
    gx -= SH::c3c * (5.f * zz - 1.f) * g[13];
    gz -= SH::c3c * 10.f * x * z * g[13];
    gx += 2.f * SH::c3e * x * z * g[14];
    gy -= 2.f * SH::c3e * y * z * g[14];
    gz += SH::c3e * (xx - yy) * g[14];
    gx -= SH::c3a * (3.f * xx - 3.f * yy) * g[15];
    gy += SH::c3a * 6.f * x * y * g[15];
  }
  out[0] = gx; out[1] = gy; out[2] = gz;
}

// A surfel's SH block sh[i][K][3] (3K contiguous floats, 16-B aligned when 3K % 4 == 0).
template <int N>
__device__ __forceinline__ void load_row(const float* p, float (&v)[N]) {
  if constexpr (N % 4 == 0) {
    const float4* q = (const float4*)p;
#pragma unroll
    for (int j = 0; j < N / 4; ++j) {
      const float4 t = q[j];
      v[4 * j] = t.x; v[4 * j + 1] = t.y; v[4 * j + 2] = t.z; v[4 * j + 3] = t.w;
    }
  } else {
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] = p[j];
  }
}

template <int N>
__device__ __forceinline__ void store_row(float* p, const float (&v)[N]) {
  if constexpr (N % 4 == 0) {
    float4* q = (float4*)p;
#pragma unroll
    for (int j = 0; j < N / 4; ++j) q[j] = make_float4(v[4 * j], v[4 * j + 1], v[4 * j + 2], v[4 * j + 3]);
  } else {
#pragma unroll
    for (int j = 0; j < N; ++j) p[j] = v[j];
  }
}

struct Geom {
  double su, sv, o, qn[4], qlen, Rw[9];
  double pc[3];   // camera-space centre
  double M[9];    // screen transform, row-major
  double flip;    // normal orientation (+1 / -1)
  float nc[3];    // camera-space normal after the flip
  float dir[3];   // unit view direction (mu - C) / |mu - C|
  float dist;
};

__device__ __forceinline__ void rot_from_quat(const double q[4], double R[9]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z); R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z); R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y); R[7] = 2 * (y * z + w * x); R[8] = 1 - 2 * (x * x + y * y);
}

// Parameter sources of the forward projection.  Both hand the same float32 values to the same
// arithmetic, so a compact set projects bit for bit like its decoded float32 copy.
struct FullSource {
  const cgv2_surfels& s;
  __device__ int64_t n() const { return s.n; }
  __device__ float mean(int k, int64_t i) const { return s.mean[k * s.n + i]; }
  __device__ float log_scale(int k, int64_t i) const { return s.log_scale[k * s.n + i]; }
  __device__ float quat(int k, int64_t i) const { return s.quat[k * s.n + i]; }
  __device__ float opacity_logit(int64_t i) const { return s.opacity_logit[i]; }
  __device__ bool valid(int64_t) const { return true; }
  template <int N>
  __device__ void sh(int64_t i, float (&f)[N]) const { load_row<N>(s.sh + i * N, f); }
};

__device__ __forceinline__ float half_bits(uint16_t b) { return (float)__builtin_bit_cast(_Float16, b); }

// Serving storage (Sec. 3.3 and the appendix's vector-tree quantization): float16 shape, rotation and
// opacity; float16 SH for the surfels [0, n_full), a codebook row for the rest.
struct CompactSource {
  const cgv2_surfels_compact& s;
  __device__ int64_t n() const { return s.n; }
  __device__ float mean(int k, int64_t i) const { return s.mean[k * s.n + i]; }
  __device__ float log_scale(int k, int64_t i) const { return half_bits(s.log_scale[k * s.n + i]); }
  __device__ float quat(int k, int64_t i) const { return half_bits(s.quat[k * s.n + i]); }
  __device__ float opacity_logit(int64_t i) const { return half_bits(s.opacity_logit[i]); }
  __device__ bool valid(int64_t i) const { return i < s.n_full || s.code[i - s.n_full] < (uint32_t)s.codebook_size; }
  template <int N>
  __device__ void sh(int64_t i, float (&f)[N]) const {
    const uint16_t* p = i < s.n_full ? s.sh + i * N : s.codebook + (int64_t)s.code[i - s.n_full] * N;
#pragma unroll
    for (int j = 0; j < N; ++j) f[j] = half_bits(p[j]);
  }
};

template <class Src>
__device__ __forceinline__ void load_geom(const Src& s, const DevCam& c, int64_t i, Geom& g) {
  g.su = (double)expf(s.log_scale(0, i));
  g.sv = (double)expf(s.log_scale(1, i));
  g.o = 1.0 / (1.0 + (double)expf(-s.opacity_logit(i)));
  const double q[4] = {s.quat(0, i), s.quat(1, i), s.quat(2, i), s.quat(3, i)};
  g.qlen = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  const double iq = 1.0 / g.qlen;
  for (int k = 0; k < 4; ++k) g.qn[k] = q[k] * iq;
  rot_from_quat(g.qn, g.Rw);
  const double mu[3] = {s.mean(0, i), s.mean(1, i), s.mean(2, i)};
  double cu[3], cv[3], ncd[3];
  for (int r = 0; r < 3; ++r) {
    const double R0 = c.R[3 * r], R1 = c.R[3 * r + 1], R2 = c.R[3 * r + 2];
    g.pc[r] = (double)c.t[r] + R0 * mu[0] + R1 * mu[1] + R2 * mu[2];
    cu[r] = g.su * (R0 * g.Rw[0] + R1 * g.Rw[3] + R2 * g.Rw[6]);
    cv[r] = g.sv * (R0 * g.Rw[1] + R1 * g.Rw[4] + R2 * g.Rw[7]);
    ncd[r] = R0 * g.Rw[2] + R1 * g.Rw[5] + R2 * g.Rw[8];
  }
  const double* cols[3] = {cu, cv, g.pc};
  for (int k = 0; k < 3; ++k) {
    g.M[k] = (double)c.fx * cols[k][0] + (double)c.cx * cols[k][2];
    g.M[3 + k] = (double)c.fy * cols[k][1] + (double)c.cy * cols[k][2];
    g.M[6 + k] = cols[k][2];
  }
  g.flip = (ncd[0] * g.pc[0] + ncd[1] * g.pc[1] + ncd[2] * g.pc[2]) > 0 ? -1.0 : 1.0;
  for (int r = 0; r < 3; ++r) g.nc[r] = (float)(g.flip * ncd[r]);
  // camera centre C = -R^T t
  double v[3];
  for (int k = 0; k < 3; ++k) {
    const double Ck = -((double)c.R[k] * c.t[0] + (double)c.R[3 + k] * c.t[1] + (double)c.R[6 + k] * c.t[2]);
    v[k] = mu[k] - Ck;
  }
  const double d = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  g.dist = (float)d;
  for (int k = 0; k < 3; ++k) g.dir[k] = (float)(v[k] / d);
}

// Centre, inverse-homography coefficients (unscaled) in the centre-shifted pixel frame.
struct Homog {
  double cx, cy, al1, al2, be1, be2, A[4], W[3], scale;
};

__device__ __forceinline__ void homography(const double* M, Homog& h) {
  h.cx = M[2] / M[8];
  h.cy = M[5] / M[8];
  h.al1 = M[0] - h.cx * M[6];
  h.al2 = M[1] - h.cx * M[7];
  h.be1 = M[3] - h.cy * M[6];
  h.be2 = M[4] - h.cy * M[7];
  const double g1 = M[6], g2 = M[7], g3 = M[8];
  h.A[0] = g3 * h.be2;
  h.A[1] = -g3 * h.al2;
  h.A[2] = -g3 * h.be1;
  h.A[3] = g3 * h.al1;
  h.W[0] = h.al1 * h.be2 - h.al2 * h.be1;
  h.W[1] = h.be1 * g2 - h.be2 * g1;
  h.W[2] = g1 * h.al2 - g2 * h.al1;
  double m = 0;
  for (int k = 0; k < 4; ++k) m = fmax(m, fabs(h.A[k]));
  for (int k = 0; k < 3; ++k) m = fmax(m, fabs(h.W[k]));
  h.scale = m > 0 ? 1.0 / m : 1.0;
}

// Projects surfel i into view v; returns whether it is binned (visible).
template <int DEG, class Src>
__device__ __forceinline__ bool project_one(const Src& s, const DevCam& c, int v, int64_t i,
                                            const cgv2_proj& out) {
  const int64_t n = s.n();
  const int64_t vi = (int64_t)v * n + i;
  uint16_t* rect = out.rect + 4 * vi;
  Geom g;
  load_geom(s, c, i, g);
  unsigned fl = 0;
  bool finite = isfinite(g.o) && isfinite(g.su) && isfinite(g.sv) && isfinite(g.qlen) && g.qlen > 0 && s.valid(i);
  for (int k = 0; k < 9; ++k) finite = finite && isfinite(g.M[k]);
  const double k2 = 2.0 * log(255.0 * g.o);
  if (!finite) fl = CGV2_F_NONFINITE;
  else if (!(g.M[8] > (double)c.znear)) fl = CGV2_F_NEAR;
  else if (!(k2 > 0)) fl = CGV2_F_OPACITY;
  double Q33 = 0;
  if (!fl) {
    Q33 = g.M[6] * g.M[6] + g.M[7] * g.M[7] - g.M[8] * g.M[8] / k2;
    if (!(Q33 < 0)) fl = CGV2_F_BEHIND;
  }
  if (fl) {
    out.flags[vi] = (uint8_t)fl;
    out.radius[vi] = 0.f;
    *(uint2*)rect = make_uint2(0u, 0u);
    return false;
  }
  const double* M = g.M;
  const double ik2 = 1.0 / k2;
  const double Q13 = M[0] * M[6] + M[1] * M[7] - M[2] * M[8] * ik2;
  const double Q23 = M[3] * M[6] + M[4] * M[7] - M[5] * M[8] * ik2;
  const double Q11 = M[0] * M[0] + M[1] * M[1] - M[2] * M[2] * ik2;
  const double Q22 = M[3] * M[3] + M[4] * M[4] - M[5] * M[5] * ik2;
  const double xb = Q13 / Q33, yb = Q23 / Q33;
  const double ex = sqrt(fmax(0.0, xb * xb - Q11 / Q33));
  const double ey = sqrt(fmax(0.0, yb * yb - Q22 / Q33));
  Homog h;
  homography(M, h);
  const double rf = sqrt(0.5 * k2);
  // a 1e-4 px pad keeps every pixel the exact bound includes, whatever the rounding
  const double pad = 1e-4;
  const double xlo = fmin(xb - ex, h.cx - rf) - pad, xhi = fmax(xb + ex, h.cx + rf) + pad;
  const double ylo = fmin(yb - ey, h.cy - rf) - pad, yhi = fmax(yb + ey, h.cy + rf) + pad;
  // low-pass dominance at the sample nearest the centre
  {
    const double xr = floor(h.cx) + 0.5 - h.cx, yr = floor(h.cy) + 0.5 - h.cy;
    const double P1 = h.A[0] * xr + h.A[1] * yr, P2 = h.A[2] * xr + h.A[3] * yr;
    const double w = h.W[0] + h.W[1] * xr + h.W[2] * yr;
    const double rho2 = 2.0 * (xr * xr + yr * yr);
    // rho2 < rho3 = (P1^2 + P2^2) / w^2
    if (rho2 * w * w < P1 * P1 + P2 * P2) fl |= CGV2_F_LOWPASS;
  }
  const double i0 = fmax(0.0, ceil(xlo - 0.5)), i1 = fmin((double)(c.W - 1), floor(xhi - 0.5));
  const double j0 = fmax(0.0, ceil(ylo - 0.5)), j1 = fmin((double)(c.H - 1), floor(yhi - 0.5));
  out.radius[vi] = (float)fmax(fmax(ex, ey), rf);
  if (!(i0 <= i1 && j0 <= j1)) {
    out.flags[vi] = (uint8_t)fl;
    *(uint2*)rect = make_uint2(0u, 0u);
    return false;
  }
  fl |= CGV2_F_VISIBLE;
  out.flags[vi] = (uint8_t)fl;
  const uint32_t tx0 = (uint32_t)i0 / kTile, tx1 = (uint32_t)i1 / kTile + 1;
  const uint32_t ty0 = (uint32_t)j0 / kTile, ty1 = (uint32_t)j1 / kTile + 1;
  *(uint2*)rect = make_uint2(tx0 | (ty0 << 16), tx1 | (ty1 << 16));

  // SH colour
  constexpr int K = (DEG + 1) * (DEG + 1);
  float Y[K];
  sh_basis<DEG>(g.dir[0], g.dir[1], g.dir[2], Y, nullptr);
  float f[3 * K];
  s.template sh<3 * K>(i, f);
  float col[3];
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    float acc = 0.5f;
#pragma unroll
    for (int k = 0; k < K; ++k) acc = fmaf(f[k * 3 + ch], Y[k], acc);
    col[ch] = fmaxf(acc, 0.f);
  }
  // record
  const double cxh = rint(fmin(fmax(h.cx, -16777216.0), 16777216.0));
  const double cyh = rint(fmin(fmax(h.cy, -16777216.0), 16777216.0));
  float4* rp = (float4*)(out.rec + (size_t)vi * kRec);
  const double sc = h.scale;
  rp[0] = make_float4((float)cxh, (float)cyh, (float)(h.cx - cxh), (float)(h.cy - cyh));
  rp[1] = make_float4((float)(h.A[0] * sc), (float)(h.A[1] * sc), (float)(h.A[2] * sc), (float)(h.A[3] * sc));
  rp[2] = make_float4((float)(h.W[0] * sc), (float)(h.W[1] * sc), (float)(h.W[2] * sc), (float)M[8]);
  rp[3] = make_float4((float)g.o, col[0], col[1], col[2]);
  rp[4] = make_float4(g.nc[0], g.nc[1], g.nc[2], (float)k2);
  const uint32_t pxr = (uint32_t)i0 | ((uint32_t)i1 << 16), pyr = (uint32_t)j0 | ((uint32_t)j1 << 16);
  rp[5] = make_float4(__uint_as_float(pxr), __uint_as_float(pyr), 0.f, 0.f);
  return true;
}

template <int DEG>
__global__ __launch_bounds__(256) void k_project(cgv2_surfels s, CamPack cams, cgv2_proj out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int v = cams.v0 + (int)blockIdx.y;
  if (i < s.n) project_one<DEG>(FullSource{s}, cams.c[blockIdx.y], v, i, out);
}

template <int DEG>
__global__ __launch_bounds__(256) void k_project_compact(cgv2_surfels_compact s, CamPack cams, cgv2_proj out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int v = cams.v0 + (int)blockIdx.y;
  if (i < s.n) project_one<DEG>(CompactSource{s}, cams.c[blockIdx.y], v, i, out);
}

// ------------------------------------------------------------------------------------------
// Reverse: record gradients of every view -> parameter gradients (+=), view-space gradients.
// ------------------------------------------------------------------------------------------
// One view (cams.c[0], view index cams.v0), one thread per entry of its visible list
// (list[vstart[0] .. vstart[1])); each surfel appears once per list, so the parameter gradients are
// added without atomics.  Every load of a surfel (parameters, record gradients, the gradient values
// being added to) is issued before its first store: the stores may alias the loaded arrays, so an
// interleaved read-modify-write would cost one full memory round trip per element.
template <int DEG>
__global__ __launch_bounds__(64) void k_project_bwd(cgv2_surfels s, CamPack cams,
                                                      const uint32_t* __restrict__ list,
                                                      const uint32_t* __restrict__ vstart,
                                                      RecGrads rg, cgv2_grads gr) {
  const int64_t n = s.n;
  const uint32_t e0 = vstart[0], e1 = vstart[1];
  constexpr int K = (DEG + 1) * (DEG + 1);
  const int v = cams.v0;
  const DevCam& c = cams.c[0];
  for (uint32_t e = e0 + blockIdx.x * blockDim.x + threadIdx.x; e < e1; e += gridDim.x * blockDim.x) {
    const int64_t i = list[e];
    // ---- loads
    float d[kGradFields];
    {
      const float4* r = (const float4*)(rg.row + ((int64_t)v * n + i) * kGradRow);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float4 q = r[k];
        d[4 * k] = q.x;
        d[4 * k + 1] = q.y;
        d[4 * k + 2] = q.z;
        d[4 * k + 3] = q.w;
      }
      const float4 q = *(const float4*)(rg.nrm + ((int64_t)v * n + i) * kGradNrm);
      d[G_NX] = q.x;
      d[G_NY] = q.y;
      d[G_NZ] = q.z;
    }
    float f[3 * K], gsh[3 * K];  // index k * 3 + channel
    load_row<3 * K>(s.sh + i * 3 * K, f);
    load_row<3 * K>(gr.d_sh + i * 3 * K, gsh);
    float gmu[3], gq[4], gls[2], glo;
#pragma unroll
    for (int k = 0; k < 3; ++k) gmu[k] = gr.d_mean[k * n + i];
#pragma unroll
    for (int k = 0; k < 4; ++k) gq[k] = gr.d_quat[k * n + i];
    gls[0] = gr.d_log_scale[i];
    gls[1] = gr.d_log_scale[n + i];
    glo = gr.d_opacity_logit[i];
    Geom g;
    load_geom(FullSource{s}, c, i, g);

    // ---- record -> (alpha, beta, gamma) -> M; the common scale of the coefficients leaves every
    // output unchanged, so it is held constant
    double dmu[3] = {0, 0, 0}, dq[4] = {0, 0, 0, 0};
    Homog h;
    homography(g.M, h);
    const double* M = g.M;
    const double sc = h.scale;
    const double dA11 = d[G_A11] * sc, dA12 = d[G_A12] * sc, dA21 = d[G_A21] * sc, dA22 = d[G_A22] * sc;
    const double dW0 = d[G_W0] * sc, dW1 = d[G_W1] * sc, dW2 = d[G_W2] * sc;
    const double g1 = M[6], g2 = M[7], g3 = M[8];
    const double dal1 = dA22 * g3 + dW0 * h.be2 - dW2 * g2;
    const double dal2 = -dA12 * g3 - dW0 * h.be1 + dW2 * g1;
    const double dbe1 = -dA21 * g3 - dW0 * h.al2 + dW1 * g2;
    const double dbe2 = dA11 * g3 + dW0 * h.al1 - dW1 * g1;
    const double dg1 = -dW1 * h.be2 + dW2 * h.al2;
    const double dg2 = dW1 * h.be1 - dW2 * h.al1;
    const double dg3 = dA11 * h.be2 - dA12 * h.al2 - dA21 * h.be1 + dA22 * h.al1 + d[G_ZC];
    double dM[9];
    dM[0] = dal1; dM[1] = dal2; dM[3] = dbe1; dM[4] = dbe2;
    dM[6] = dg1 - dal1 * h.cx - dbe1 * h.cy;
    dM[7] = dg2 - dal2 * h.cx - dbe2 * h.cy;
    const double dcx = (double)d[G_CX] - dal1 * M[6] - dal2 * M[7];
    const double dcy = (double)d[G_CY] - dbe1 * M[6] - dbe2 * M[7];
    dM[2] = dcx / M[8];
    dM[5] = dcy / M[8];
    dM[8] = dg3 - (dcx * h.cx + dcy * h.cy) / M[8];
    // M columns = K_int [cu | cv | pc]
    double vw[3][3];
    for (int k = 0; k < 3; ++k) {
      const double a = (double)c.fx * dM[k], b = (double)c.fy * dM[3 + k];
      const double e2 = (double)c.cx * dM[k] + (double)c.cy * dM[3 + k] + dM[6 + k];
      for (int r2 = 0; r2 < 3; ++r2) vw[k][r2] = (double)c.R[r2] * a + (double)c.R[3 + r2] * b + (double)c.R[6 + r2] * e2;
    }
    double dsu = 0, dsv = 0, dR[9];
    for (int r2 = 0; r2 < 3; ++r2) {
      dsu += vw[0][r2] * g.Rw[3 * r2];
      dsv += vw[1][r2] * g.Rw[3 * r2 + 1];
      dR[3 * r2] = g.su * vw[0][r2];
      dR[3 * r2 + 1] = g.sv * vw[1][r2];
      dmu[r2] += vw[2][r2];
    }
    const double dn[3] = {d[G_NX], d[G_NY], d[G_NZ]};
    for (int r2 = 0; r2 < 3; ++r2)
      dR[3 * r2 + 2] = g.flip * ((double)c.R[r2] * dn[0] + (double)c.R[3 + r2] * dn[1] + (double)c.R[6 + r2] * dn[2]);
    // rotation -> normalised quaternion
    {
      const double w = g.qn[0], x = g.qn[1], y = g.qn[2], z = g.qn[3];
      double dqn[4];
      dqn[0] = -2 * z * dR[1] + 2 * y * dR[2] + 2 * z * dR[3] - 2 * x * dR[5] - 2 * y * dR[6] + 2 * x * dR[7];
      dqn[1] = 2 * y * dR[1] + 2 * z * dR[2] + 2 * y * dR[3] - 4 * x * dR[4] - 2 * w * dR[5] + 2 * z * dR[6] +
               2 * w * dR[7] - 4 * x * dR[8];
      dqn[2] = -4 * y * dR[0] + 2 * x * dR[1] + 2 * w * dR[2] + 2 * x * dR[3] + 2 * z * dR[5] - 2 * w * dR[6] +
               2 * z * dR[7] - 4 * y * dR[8];
      dqn[3] = -4 * z * dR[0] - 2 * w * dR[1] + 2 * x * dR[2] + 2 * w * dR[3] - 4 * z * dR[4] + 2 * y * dR[5] +
               2 * x * dR[6] + 2 * y * dR[7];
      const double dot = g.qn[0] * dqn[0] + g.qn[1] * dqn[1] + g.qn[2] * dqn[2] + g.qn[3] * dqn[3];
      for (int k = 0; k < 4; ++k) dq[k] += (dqn[k] - g.qn[k] * dot) / g.qlen;
    }
    const double dls0 = dsu * g.su, dls1 = dsv * g.sv;
    const double dlogit = (double)d[G_OP] * g.o * (1 - g.o);
    // colour through SH: the coefficient gradients are added per view, the direction gradient is
    // contracted on the fly; a channel clamped at zero passes nothing
    float Y[K], gY[K];
    sh_basis<DEG>(g.dir[0], g.dir[1], g.dir[2], Y, nullptr);
#pragma unroll
    for (int k = 0; k < K; ++k) gY[k] = 0.f;
    const float dcol[3] = {d[G_R], d[G_G], d[G_B]};
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      float raw = 0.5f;
#pragma unroll
      for (int k = 0; k < K; ++k) raw = fmaf(f[k * 3 + ch], Y[k], raw);
      const float dc = raw < 0.f ? 0.f : dcol[ch];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        gY[k] = fmaf(dc, f[k * 3 + ch], gY[k]);
        gsh[k * 3 + ch] = fmaf(dc, Y[k], gsh[k * 3 + ch]);
      }
    }
    float ddir[3];
    sh_grad_dot<DEG>(gY, g.dir[0], g.dir[1], g.dir[2], ddir);
    const float dd = ddir[0] * g.dir[0] + ddir[1] * g.dir[1] + ddir[2] * g.dir[2];
    for (int k = 0; k < 3; ++k) dmu[k] += (double)((ddir[k] - g.dir[k] * dd) / g.dist);

    // ---- stores
    if (gr.g_view_total) {
      float* gvt = gr.g_view_total + (int64_t)v * 2 * n;
      gvt[i] = d[G_CX] * (0.5f * (float)c.W);
      gvt[n + i] = d[G_CY] * (0.5f * (float)c.H);
    }
    if (gr.g_view_ssim) {
      float* gvs = gr.g_view_ssim + (int64_t)v * 2 * n;
      gvs[i] = d[G_SCX] * (0.5f * (float)c.W);
      gvs[n + i] = d[G_SCY] * (0.5f * (float)c.H);
    }
    // channels clamped at zero store their unchanged values back
    store_row<3 * K>(gr.d_sh + i * 3 * K, gsh);
#pragma unroll
    for (int k = 0; k < 3; ++k) gr.d_mean[k * n + i] = gmu[k] + (float)dmu[k];
#pragma unroll
    for (int k = 0; k < 4; ++k) gr.d_quat[k * n + i] = gq[k] + (float)dq[k];
    gr.d_log_scale[i] = gls[0] + (float)dls0;
    gr.d_log_scale[n + i] = gls[1] + (float)dls1;
    gr.d_opacity_logit[i] = glo + (float)dlogit;
  }
}

}  // namespace cgv2

hipError_t cgv2_launch_project_compact(const cgv2_surfels_compact& s, const cgv2::CamPack& cams, const cgv2_proj& p,
                                      hipStream_t st) {
  if (s.n == 0) return hipSuccess;
  dim3 grid((unsigned)((s.n + 255) / 256), (unsigned)cams.count);
  switch (s.sh_degree) {
    case 0: hipLaunchKernelGGL(cgv2::k_project_compact<0>, grid, dim3(256), 0, st, s, cams, p); break;
    case 1: hipLaunchKernelGGL(cgv2::k_project_compact<1>, grid, dim3(256), 0, st, s, cams, p); break;
    case 2: hipLaunchKernelGGL(cgv2::k_project_compact<2>, grid, dim3(256), 0, st, s, cams, p); break;
    default: hipLaunchKernelGGL(cgv2::k_project_compact<3>, grid, dim3(256), 0, st, s, cams, p); break;
  }
  return hipGetLastError();
}

hipError_t cgv2_launch_project(const cgv2_surfels& s, const cgv2::CamPack& cams, const cgv2_proj& p, hipStream_t st) {
  if (s.n == 0) return hipSuccess;
  dim3 grid((unsigned)((s.n + 255) / 256), (unsigned)cams.count);
  switch (s.sh_degree) {
    case 0: hipLaunchKernelGGL(cgv2::k_project<0>, grid, dim3(256), 0, st, s, cams, p); break;
    case 1: hipLaunchKernelGGL(cgv2::k_project<1>, grid, dim3(256), 0, st, s, cams, p); break;
    case 2: hipLaunchKernelGGL(cgv2::k_project<2>, grid, dim3(256), 0, st, s, cams, p); break;
    default: hipLaunchKernelGGL(cgv2::k_project<3>, grid, dim3(256), 0, st, s, cams, p); break;
  }
  return hipGetLastError();
}

namespace cgv2 {

// Zeroing of the parameter gradients: one grid walks the five arrays with 16-byte stores (the floats
// before an array's first 16-byte boundary and after its last one singly), about eight per thread.
struct ZeroList {
  float* p[5];
  int64_t count[5];
};

__global__ __launch_bounds__(256) void k_zero_grads(ZeroList z) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, nt = (int64_t)gridDim.x * blockDim.x;
#pragma unroll 1
  for (int a = 0; a < 5; ++a) {
    float* p = z.p[a];
    const int64_t c = z.count[a];
    const int64_t head = std::min<int64_t>(c, (int64_t)(((16u - ((uintptr_t)p & 15u)) & 15u) / 4u));
    if (tid < head) p[tid] = 0.f;
    float4* q = (float4*)(p + head);
    const int64_t n4 = (c - head) / 4;
    for (int64_t i = tid; i < n4; i += nt) q[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    const int64_t t0 = head + 4 * n4;
    if (tid < c - t0) p[t0 + tid] = 0.f;
  }
}

}  // namespace cgv2

hipError_t cgv2_launch_zero_grads(const cgv2_grads& g, int64_t n, int sh_degree, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int64_t K = (int64_t)(sh_degree + 1) * (sh_degree + 1);
  cgv2::ZeroList z;
  float* p[5] = {g.d_mean, g.d_log_scale, g.d_quat, g.d_opacity_logit, g.d_sh};
  const int64_t c[5] = {3 * n, 2 * n, 4 * n, n, 3 * K * n};
  for (int a = 0; a < 5; ++a) {
    z.p[a] = p[a];
    z.count[a] = c[a];
  }
  const int64_t total = (3 * K + 10) * n;
  const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((total / 4 + 2047) / 2048, 4096));
  hipLaunchKernelGGL(cgv2::k_zero_grads, dim3(blocks), dim3(256), 0, st, z);
  return hipGetLastError();
}

hipError_t cgv2_launch_project_bwd(const cgv2_surfels& s, const cgv2::CamPack& cams, const cgv2_proj& p,
                                   const cgv2::RecGrads& rg, const cgv2_grads& g, hipStream_t st) {
  if (s.n == 0) return hipSuccess;
  const int64_t n = s.n;
  // one wave per workgroup: the visible surfels (a few percent of n) then spread over every CU instead
  // of filling the first few with four-wave workgroups
  const unsigned blocks = (unsigned)std::min<int64_t>((n + 63) / 64, 16384);
  // g_view rows are overwritten: zero for surfels outside each view's list
  const int64_t rows = (int64_t)cams.count * 2 * n;
  const unsigned fill_blocks = (unsigned)std::min<int64_t>((rows + 255) / 256, 65535);
  if (g.g_view_total || g.g_view_ssim)
    hipLaunchKernelGGL(cgv2::k_zero2<float>, dim3(fill_blocks), dim3(256), 0, st,
                       g.g_view_total ? g.g_view_total + (int64_t)cams.v0 * 2 * n : nullptr,
                       g.g_view_ssim ? g.g_view_ssim + (int64_t)cams.v0 * 2 * n : nullptr, rows);
  for (int lv = 0; lv < cams.count; ++lv) {
    const int v = cams.v0 + lv;
    cgv2::CamPack one;
    one.c[0] = cams.c[lv];
    one.v0 = v;
    one.count = 1;
    const uint32_t* list = p.visible;
    const uint32_t* cnt = p.visible_start + v;
    switch (s.sh_degree) {
      case 0: hipLaunchKernelGGL(cgv2::k_project_bwd<0>, dim3(blocks), dim3(64), 0, st, s, one, list, cnt, rg, g); break;
      case 1: hipLaunchKernelGGL(cgv2::k_project_bwd<1>, dim3(blocks), dim3(64), 0, st, s, one, list, cnt, rg, g); break;
      case 2: hipLaunchKernelGGL(cgv2::k_project_bwd<2>, dim3(blocks), dim3(64), 0, st, s, one, list, cnt, rg, g); break;
      default: hipLaunchKernelGGL(cgv2::k_project_bwd<3>, dim3(blocks), dim3(64), 0, st, s, one, list, cnt, rg, g); break;
    }
  }
  return hipGetLastError();
}
