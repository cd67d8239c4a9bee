// Visibility-frequency crop volume of the CityGaussianV2 evaluation protocol (Sec. 4): every
// ground-truth point is a small isotropic Gaussian; over all views, count the views in which its visible
// mask is set; keep the points seen often enough, take their height range and their ground-plane
// coordinates (for the alpha shape, which runs on the host).
//
// A point's footprint is the image of the sphere of radius rho around it, hulled with a disc of rf
// pixels around its projected centre; it is visible when its centre depth exceeds znear and a pixel
// sample (i + 0.5, j + 0.5) lies in the footprint's box (a sphere reaching the camera plane, depth <=
// rho, is visible).  Every decision is taken in FP64.
//
//   k_vis_table  per view: the camera in FP64 (a row) and, as columns across the views, eight
//                world-space planes: four that bound where a footprint can reach the image, four that bound
//                where every projected centre is inside it
//   k_vis_count  per workgroup of kVisSuper consecutive points: the box of its points is classified
//                against 256 views at a time, one view per thread, then each of its sub-boxes against the
//                views left undecided.  A view that cannot see any point of
//                the box is skipped; a view in which every centre projects inside the sample range
//                counts for all points at once (rf >= 0.5 guarantees the nearest sample is covered); only
//                the remaining views, whose image edge crosses the box, test the points one by one (with
//                rf >= 0.5, the sphere's extent is computed only for centres outside the extended image).
//                Points in spatially coherent order make the boxes small; any order gives the same counts.
//   k_crop_*     threshold, FP64 ground transform, height range, order-preserving compaction
#include "cgv2r_device.h"
#include "cgv2r_kernels.h"

#include <algorithm>
#include <cmath>

namespace cgv2 {

constexpr int kVisThreads = 256;
constexpr int kVisPts = 2;
constexpr int kVisChunk = kVisThreads * kVisPts;  // points per sub-box
constexpr int kVisSub = 8;                         // sub-boxes per workgroup
constexpr int kVisSuper = kVisChunk * kVisSub;
// Per-view table in the workspace: an FP64 camera row per view (read with scalar loads by the per-point
// test) and, for the workgroup classification, one column per plane coefficient across the views (one
// view per lane: coalesced loads).
constexpr int kRow = 36;                 // doubles per camera row: camera (20), four exact edge planes
constexpr int kCols = 37;                // classification columns: depth row (4), znear, 8 planes x 4
constexpr double kEdgeMarginPx = 1e-2;   // the plane tests keep this far from every decision edge
constexpr double kDepthMargin = 1e-7;

enum : int { T_R = 0, T_T = 9, T_FX = 12, T_FY, T_CX, T_CY, T_ZN, T_W, T_H, T_E = 20 };
enum : int { C_Z = 0, C_ZN = 4, C_PL = 5 };  // column index of the depth row, znear, plane q at C_PL + 4 q
enum : int { V_OUT = 0, V_IN = 1, V_EDGE = 2 };

struct VisTable {
  double* row;  // [V][kRow]
  double* col;  // [kCols][V]
  int V;
};

__global__ void k_vis_table(CamPack cams, double rho, double rf, VisTable tab) {
  const int k = threadIdx.x;
  if (k >= cams.count) return;
  const DevCam& c = cams.c[k];
  const int v = cams.v0 + k;
  double* T = tab.row + (int64_t)v * kRow;
  auto col = [&](int q) -> double& { return tab.col[(int64_t)q * tab.V + v]; };
  double R[9], t[3];
  for (int i = 0; i < 9; ++i) R[i] = T[T_R + i] = (double)c.R[i];
  for (int i = 0; i < 3; ++i) t[i] = T[T_T + i] = (double)c.t[i];
  const double fx = c.fx, fy = c.fy, cx = c.cx, cy = c.cy, W = c.W, H = c.H, zn = c.znear;
  T[T_FX] = fx, T[T_FY] = fy, T[T_CX] = cx, T[T_CY] = cy, T[T_ZN] = zn, T[T_W] = W, T[T_H] = H;
  T[19] = 0.0;
  for (int i = 0; i < 3; ++i) col(C_Z + i) = R[6 + i];
  col(C_Z + 3) = t[2];
  col(C_ZN) = zn;
  // u >= k  <=>  fx Xc + (cx - k) Zc >= 0 (Zc > 0); world plane w . p + off with w = fx R0 + (cx - k) R2
  auto plane = [&](int q, int row, double f, double cc, double kk, double sign) {
    for (int i = 0; i < 3; ++i) col(C_PL + 4 * q + i) = sign * (f * R[3 * row + i] + (cc - kk) * R[6 + i]);
    col(C_PL + 4 * q + 3) = sign * (f * t[row] + (cc - kk) * t[2]);
  };
  // exact edge planes of the centre's disc (row): uc + rf >= 0.5, uc - rf <= W - 0.5, likewise v
  auto edge_plane = [&](int q, int row, double f, double cc, double kk, double sign) {
    double* P = T + T_E + 4 * q;
    for (int i = 0; i < 3; ++i) P[i] = sign * (f * R[3 * row + i] + (cc - kk) * R[6 + i]);
    P[3] = sign * (f * t[row] + (cc - kk) * t[2]);
  };
  edge_plane(0, 0, fx, cx, 0.5 - rf, 1.0);
  edge_plane(1, 0, fx, cx, W - 0.5 + rf, -1.0);
  edge_plane(2, 1, fy, cy, 0.5 - rf, 1.0);
  edge_plane(3, 1, fy, cy, H - 0.5 + rf, -1.0);
  // reach planes: beyond them no footprint touches a sample
  plane(0, 0, fx, cx, 0.5 - rf - kEdgeMarginPx, 1.0);
  plane(1, 0, fx, cx, W - 0.5 + rf + kEdgeMarginPx, -1.0);
  plane(2, 1, fy, cy, 0.5 - rf - kEdgeMarginPx, 1.0);
  plane(3, 1, fy, cy, H - 0.5 + rf + kEdgeMarginPx, -1.0);
  // interior planes: inside all four every projected centre lies within the sample range
  plane(4, 0, fx, cx, 0.5 + kEdgeMarginPx, 1.0);
  plane(5, 0, fx, cx, W - 0.5 - kEdgeMarginPx, -1.0);
  plane(6, 1, fy, cy, 0.5 + kEdgeMarginPx, 1.0);
  plane(7, 1, fy, cy, H - 0.5 - kEdgeMarginPx, -1.0);
}

// Class of view v for the points inside the box c +- h (world, FP64).
__device__ __forceinline__ int classify(const double* __restrict__ col, int V, int v, const double c[3],
                                        const double h[3], double rho, bool interior) {
  auto at = [&](int q) { return col[(int64_t)q * V + v]; };
  const double z0 = at(C_Z), z1 = at(C_Z + 1), z2 = at(C_Z + 2);
  const double zc = z0 * c[0] + z1 * c[1] + z2 * c[2] + at(C_Z + 3);
  const double zr = fabs(z0) * h[0] + fabs(z1) * h[1] + fabs(z2) * h[2];
  const double zn = at(C_ZN);
  if (zc + zr < zn - kDepthMargin) return V_OUT;  // every centre at or before znear
  if (zc - zr > rho + kDepthMargin) {
    // no sphere reaches the camera plane: the box grown by rho bounds every sphere
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double p0 = at(C_PL + 4 * q), p1 = at(C_PL + 4 * q + 1), p2 = at(C_PL + 4 * q + 2);
      const double s = p0 * c[0] + p1 * c[1] + p2 * c[2] + at(C_PL + 4 * q + 3) + fabs(p0) * (h[0] + rho) +
                       fabs(p1) * (h[1] + rho) + fabs(p2) * (h[2] + rho);
      if (s < 0.0) return V_OUT;
    }
  }
  if (interior && zc - zr > zn + kDepthMargin) {
    bool in = true;
#pragma unroll
    for (int q = 4; q < 8; ++q) {
      const double p0 = at(C_PL + 4 * q), p1 = at(C_PL + 4 * q + 1), p2 = at(C_PL + 4 * q + 2);
      const double s = p0 * c[0] + p1 * c[1] + p2 * c[2] + at(C_PL + 4 * q + 3) - fabs(p0) * h[0] -
                       fabs(p1) * h[1] - fabs(p2) * h[2];
      in = in && s > 0.0;
    }
    if (in) return V_IN;
  }
  return V_EDGE;
}

// The visible mask of one point in one view, as defined (FP64): any filter reach.
__device__ __forceinline__ bool vis_exact(const double* T, double x, double y, double z, double rho,
                                          double rf) {
  const double X = T[0] * x + T[1] * y + T[2] * z + T[9];
  const double Y = T[3] * x + T[4] * y + T[5] * z + T[10];
  const double Z = T[6] * x + T[7] * y + T[8] * z + T[11];
  if (!(Z > T[T_ZN])) return false;
  if (Z <= rho) return true;
  const double fx = T[T_FX], fy = T[T_FY], cx = T[T_CX], cy = T[T_CY];
  const double iden = 1.0 / (Z * Z - rho * rho), iz = 1.0 / Z;
  const double sx = sqrt(X * X + Z * Z - rho * rho), sy = sqrt(Y * Y + Z * Z - rho * rho);
  const double u0 = fx * ((X * Z - rho * sx) * iden) + cx, u1 = fx * ((X * Z + rho * sx) * iden) + cx;
  const double v0 = fy * ((Y * Z - rho * sy) * iden) + cy, v1 = fy * ((Y * Z + rho * sy) * iden) + cy;
  const double uc = fx * (X * iz) + cx, vc = fy * (Y * iz) + cy;
  const double ulo = fmin(u0, uc - rf), uhi = fmax(u1, uc + rf);
  const double vlo = fmin(v0, vc - rf), vhi = fmax(v1, vc + rf);
  const double i0 = fmax(0.0, ceil(ulo - 0.5)), i1 = fmin(T[T_W] - 1.0, floor(uhi - 0.5));
  const double j0 = fmax(0.0, ceil(vlo - 0.5)), j1 = fmin(T[T_H] - 1.0, floor(vhi - 0.5));
  return i0 <= i1 && j0 <= j1;
}

// The same mask when rf >= 0.5.  Then the footprint's extent along an axis is at least one pixel, so it
// holds a sample exactly when it overlaps [0.5, W - 0.5]: on x, max(u1, uc + rf) >= 0.5 and
// min(u0, uc - rf) <= W - 0.5.  With Z > 0, uc + rf >= 0.5 is the sign of a world-space plane through
// the camera (likewise the other three), so the common case costs four plane evaluations; since
// u0 <= uc <= u1, the sphere's bounds are computed only on a side whose plane test fails.
__device__ __forceinline__ bool vis_exact_wide(const double* T, double x, double y, double z,
                                               double rho) {
  const double Z = T[6] * x + T[7] * y + T[8] * z + T[11];
  if (!(Z > T[T_ZN])) return false;
  if (Z <= rho) return true;
  double e[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double* P = T + T_E + 4 * q;
    e[q] = P[0] * x + P[1] * y + P[2] * z + P[3];
  }
  if (e[0] >= 0.0 && e[1] >= 0.0 && e[2] >= 0.0 && e[3] >= 0.0) return true;
  const double iden = 1.0 / (Z * Z - rho * rho);
  if (e[0] < 0.0 || e[1] < 0.0) {
    const double X = T[0] * x + T[1] * y + T[2] * z + T[9];
    const double sx = sqrt(X * X + Z * Z - rho * rho);
    const bool ok = e[0] < 0.0 ? T[T_FX] * ((X * Z + rho * sx) * iden) + T[T_CX] >= 0.5
                               : T[T_FX] * ((X * Z - rho * sx) * iden) + T[T_CX] <= T[T_W] - 0.5;
    if (!ok) return false;
  }
  if (e[2] < 0.0 || e[3] < 0.0) {
    const double Y = T[3] * x + T[4] * y + T[5] * z + T[10];
    const double sy = sqrt(Y * Y + Z * Z - rho * rho);
    return e[2] < 0.0 ? T[T_FY] * ((Y * Z + rho * sy) * iden) + T[T_CY] >= 0.5
                      : T[T_FY] * ((Y * Z - rho * sy) * iden) + T[T_CY] <= T[T_H] - 0.5;
  }
  return true;
}

// Box of the kVisPts points per thread at pts[base + k kVisThreads] (k < kVisPts, below m) over the
// workgroup: c +- h in FP64.  Ends with a barrier; red is reused only after the caller's next barrier.
__device__ __forceinline__ void block_box(const float (&p)[kVisPts][3], const bool (&ok)[kVisPts],
                                          float (&red)[6][kVisThreads / 64], double c[3], double h[3]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
#pragma unroll
  for (int k = 0; k < kVisPts; ++k) {
    if (!ok[k]) continue;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      lo[d] = fminf(lo[d], p[k][d]);
      hi[d] = fmaxf(hi[d], p[k][d]);
    }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) {
      lo[d] = fminf(lo[d], __shfl_xor(lo[d], s, 64));
      hi[d] = fmaxf(hi[d], __shfl_xor(hi[d], s, 64));
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      red[d][w] = lo[d];
      red[3 + d][w] = hi[d];
    }
  }
  __syncthreads();
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    float a = red[d][0], b = red[3 + d][0];
#pragma unroll
    for (int q = 1; q < kVisThreads / 64; ++q) {
      a = fminf(a, red[d][q]);
      b = fmaxf(b, red[3 + d][q]);
    }
    c[d] = 0.5 * ((double)a + (double)b);
    h[d] = 0.5 * ((double)b - (double)a);
  }
}

// Classifies the views list[0 .. n) (or 0 .. n when list is null) against the box c +- h: adds the
// inside views to *n_in and appends the edge views to out (*n_out).  Every thread must call it.
__device__ __forceinline__ void classify_views(const VisTable& tab, int v_begin, const uint32_t* list, int n,
                                               const double c[3], const double h[3], double rho, bool wide,
                                               uint32_t* n_in, uint32_t* out, uint32_t* n_out) {
  const int lane = threadIdx.x & 63;
  for (int q0 = 0; q0 < n; q0 += kVisThreads) {
    const int q = q0 + (int)threadIdx.x;
    uint32_t v = 0;
    int cls = V_OUT;
    if (q < n) {
      v = list ? list[q] : (uint32_t)q;
      cls = classify(tab.col, tab.V, v_begin + (int)v, c, h, rho, wide);
    }
    const unsigned long long in_mask = __ballot(cls == V_IN);
    const unsigned long long ed_mask = __ballot(cls == V_EDGE);
    uint32_t at = 0;
    if (lane == 0) {
      if (in_mask) atomicAdd(n_in, (uint32_t)__popcll(in_mask));
      if (ed_mask) at = atomicAdd(n_out, (uint32_t)__popcll(ed_mask));
    }
    at = __shfl(at, 0, 64);
    if (cls == V_EDGE) out[at + __popcll(ed_mask & ((1ull << lane) - 1ull))] = v;
  }
}

// One workgroup per kVisSuper consecutive points, in kVisSub sub-boxes of kVisChunk: the views are
// classified once against the whole box; only its edge views are classified again per sub-box, and only a
// sub-box's edge views test its points one by one.
__global__ __launch_bounds__(kVisThreads) void k_vis_count(const float* __restrict__ pts, int64_t m, VisTable tab,
                                                           int v_begin, int V, double rho, double rf,
                                                           uint32_t* __restrict__ count) {
  __shared__ float red[6][kVisThreads / 64];
  __shared__ uint32_t edge_all[kVisMaxViews], edge_sub[kVisMaxViews];
  __shared__ uint32_t n_all, in_all, n_sub, in_sub;
  const bool wide = rf >= 0.5;
  const int64_t base = (int64_t)blockIdx.x * kVisSuper + threadIdx.x;

  // whole box: every point of the workgroup, in kVisSub passes of kVisPts per thread
  {
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int k = 0; k < kVisSub * kVisPts; ++k) {
      const int64_t i = base + (int64_t)k * kVisThreads;
      if (i >= m) break;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const float x = pts[d * m + i];
        lo[d] = fminf(lo[d], x);
        hi[d] = fmaxf(hi[d], x);
      }
    }
    float p1[kVisPts][3];
    bool ok1[kVisPts];
#pragma unroll
    for (int k = 0; k < kVisPts; ++k) {
      ok1[k] = k < 2 && lo[0] <= hi[0];
#pragma unroll
      for (int d = 0; d < 3; ++d) p1[k][d] = k == 0 ? lo[d] : hi[d];
    }
    if (threadIdx.x == 0) n_all = in_all = 0;
    double c[3], h[3];
    block_box(p1, ok1, red, c, h);
    classify_views(tab, v_begin, nullptr, V, c, h, rho, wide, &in_all, edge_all, &n_all);
    __syncthreads();
  }
  const uint32_t na = n_all, ia = in_all;

  for (int sb = 0; sb < kVisSub; ++sb) {
    const int64_t sbase = base + (int64_t)sb * kVisChunk;
    if (sbase - threadIdx.x >= m) break;  // uniform: the sub-box starts past the end
    float p[kVisPts][3];
    bool ok[kVisPts];
#pragma unroll
    for (int k = 0; k < kVisPts; ++k) {
      const int64_t i = sbase + (int64_t)k * kVisThreads;
      ok[k] = i < m;
#pragma unroll
      for (int d = 0; d < 3; ++d) p[k][d] = ok[k] ? pts[d * m + i] : 0.f;
    }
    if (threadIdx.x == 0) n_sub = in_sub = 0;
    double c[3], h[3];
    block_box(p, ok, red, c, h);
    classify_views(tab, v_begin, edge_all, (int)na, c, h, rho, wide, &in_sub, edge_sub, &n_sub);
    __syncthreads();
    const uint32_t ne = n_sub;
    uint32_t cnt[kVisPts];
#pragma unroll
    for (int k = 0; k < kVisPts; ++k) cnt[k] = ia + in_sub;
    for (uint32_t e = 0; e < ne; ++e) {
      // the view index is uniform: its camera row is read with scalar loads
      const double* T = tab.row + (int64_t)(v_begin + (int)__builtin_amdgcn_readfirstlane(edge_sub[e])) * kRow;
      if (wide) {
#pragma unroll
        for (int k = 0; k < kVisPts; ++k)
          cnt[k] += vis_exact_wide(T, (double)p[k][0], (double)p[k][1], (double)p[k][2], rho) ? 1u : 0u;
      } else {
#pragma unroll
        for (int k = 0; k < kVisPts; ++k)
          cnt[k] += vis_exact(T, (double)p[k][0], (double)p[k][1], (double)p[k][2], rho, rf) ? 1u : 0u;
      }
    }
#pragma unroll
    for (int k = 0; k < kVisPts; ++k)
      if (ok[k]) count[sbase + (int64_t)k * kVisThreads] += cnt[k];
    __syncthreads();  // edge_sub, the counters and red are rewritten by the next sub-box
  }
}

// ---- crop: threshold, ground transform, height range, compaction ---------------------------------

constexpr int kCropBlock = 256;
constexpr int kCropItems = 8;
constexpr int kCropChunk = kCropBlock * kCropItems;

struct Ground {
  double T[12];
};

__device__ __forceinline__ void ground_of(const Ground& g, const float* pts, int64_t m, int64_t i, double& gx,
                                          double& gy, double& gh) {
  const double x = pts[i], y = pts[m + i], z = pts[2 * m + i];
  gx = g.T[0] * x + g.T[1] * y + g.T[2] * z + g.T[3];
  gy = g.T[4] * x + g.T[5] * y + g.T[6] * z + g.T[7];
  gh = g.T[8] * x + g.T[9] * y + g.T[10] * z + g.T[11];
}

// per workgroup: kept count, height min and max of its kept points
__global__ __launch_bounds__(kCropBlock) void k_crop_count(const float* __restrict__ pts, int64_t m,
                                                           const uint32_t* __restrict__ count, uint32_t tau, Ground g,
                                                           uint8_t* __restrict__ keep, uint32_t* __restrict__ kpart,
                                                           double* __restrict__ hpart) {
  __shared__ uint32_t lds[kCropBlock / 64];
  __shared__ double hred[2][kCropBlock / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t base = (int64_t)blockIdx.x * kCropChunk + threadIdx.x;
  uint32_t k_local = 0;
  double hmin = INFINITY, hmax = -INFINITY;
#pragma unroll
  for (int k = 0; k < kCropItems; ++k) {
    const int64_t i = base + (int64_t)k * kCropBlock;
    if (i >= m) break;
    const bool kp = count[i] >= tau;
    keep[i] = kp ? 1 : 0;
    if (kp) {
      double gx, gy, gh;
      ground_of(g, pts, m, i, gx, gy, gh);
      hmin = fmin(hmin, gh);
      hmax = fmax(hmax, gh);
      ++k_local;
    }
  }
  uint32_t tot;
  block_exscan<kCropBlock>(k_local, lds, tot);
#pragma unroll
  for (int s = 32; s > 0; s >>= 1) {
    hmin = fmin(hmin, __shfl_xor(hmin, s, 64));
    hmax = fmax(hmax, __shfl_xor(hmax, s, 64));
  }
  if (lane == 0) {
    hred[0][w] = hmin;
    hred[1][w] = hmax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = hred[0][0], b = hred[1][0];
    for (int q = 1; q < kCropBlock / 64; ++q) {
      a = fmin(a, hred[0][q]);
      b = fmax(b, hred[1][q]);
    }
    kpart[blockIdx.x] = tot;
    hpart[2 * blockIdx.x] = a;
    hpart[2 * blockIdx.x + 1] = b;
  }
}

// one workgroup: exclusive offsets of the kept points per workgroup, the kept total, the height range
__global__ __launch_bounds__(kCropBlock) void k_crop_scan(uint32_t* __restrict__ kpart, const double* __restrict__ hpart,
                                                          int nb, int64_t* __restrict__ kept,
                                                          double* __restrict__ hrange) {
  __shared__ unsigned long long lds[kCropBlock / 64];
  __shared__ double hred[2][kCropBlock / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  unsigned long long carry = 0;
  double hmin = INFINITY, hmax = -INFINITY;
  for (int b0 = 0; b0 < nb; b0 += kCropBlock) {
    const int b = b0 + (int)threadIdx.x;
    const unsigned long long v = b < nb ? kpart[b] : 0ull;
    if (b < nb) {
      hmin = fmin(hmin, hpart[2 * b]);
      hmax = fmax(hmax, hpart[2 * b + 1]);
    }
    unsigned long long tot;
    const unsigned long long ex = block_exscan<kCropBlock>(v, lds, tot) + carry;
    if (b < nb) kpart[b] = (uint32_t)ex;
    carry += tot;
  }
#pragma unroll
  for (int s = 32; s > 0; s >>= 1) {
    hmin = fmin(hmin, __shfl_xor(hmin, s, 64));
    hmax = fmax(hmax, __shfl_xor(hmax, s, 64));
  }
  if (lane == 0) {
    hred[0][w] = hmin;
    hred[1][w] = hmax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = hred[0][0], b = hred[1][0];
    for (int q = 1; q < kCropBlock / 64; ++q) {
      a = fmin(a, hred[0][q]);
      b = fmax(b, hred[1][q]);
    }
    *kept = (int64_t)carry;
    hrange[0] = carry ? a : NAN;
    hrange[1] = carry ? b : NAN;
  }
}

// per workgroup: ground coordinates of its kept points at their slots (id order)
__global__ __launch_bounds__(kCropBlock) void k_crop_write(const float* __restrict__ pts, int64_t m,
                                                           const uint8_t* __restrict__ keep, Ground g,
                                                           const uint32_t* __restrict__ koff,
                                                           double* __restrict__ ground) {
  __shared__ uint32_t lds[kCropBlock / 64];
  const int64_t chunk = (int64_t)blockIdx.x * kCropChunk;
  const int64_t base = chunk + (int64_t)threadIdx.x * kCropItems;
  uint32_t kp[kCropItems];
  uint32_t k_local = 0;
#pragma unroll
  for (int k = 0; k < kCropItems; ++k) {
    kp[k] = base + k < m ? keep[base + k] : 0u;
    k_local += kp[k];
  }
  uint32_t tot;
  uint32_t at = koff[blockIdx.x] + block_exscan<kCropBlock>(k_local, lds, tot);
#pragma unroll
  for (int k = 0; k < kCropItems; ++k) {
    if (!kp[k]) continue;
    double gx, gy, gh;
    ground_of(g, pts, m, base + k, gx, gy, gh);
    ground[at] = gx;
    ground[m + at] = gy;
    ++at;
  }
}

}  // namespace cgv2

size_t cgv2_vis_ws_layout(int V) {
  return (((size_t)V * (cgv2::kRow + cgv2::kCols) * sizeof(double)) + 255) & ~(size_t)255;
}

static cgv2::VisTable vis_table(void* ws, int V) {
  cgv2::VisTable t;
  t.row = (double*)ws;
  t.col = t.row + (size_t)V * cgv2::kRow;
  t.V = V;
  return t;
}

hipError_t cgv2_launch_vis_table(const cgv2::CamPack& cams, int V, double rho, double rf, void* ws, hipStream_t st) {
  hipLaunchKernelGGL(cgv2::k_vis_table, dim3(1), dim3(64), 0, st, cams, rho, rf, vis_table(ws, V));
  return hipGetLastError();
}

hipError_t cgv2_launch_vis_count(const float* pts, int64_t m, int V, double rho, double rf, uint32_t* count,
                                 void* ws, hipStream_t st) {
  if (m == 0) return hipGetLastError();
  const unsigned nb = (unsigned)((m + cgv2::kVisSuper - 1) / cgv2::kVisSuper);
  for (int v0 = 0; v0 < V; v0 += kVisMaxViews) {
    const int vc = std::min(V - v0, kVisMaxViews);
    hipLaunchKernelGGL(cgv2::k_vis_count, dim3(nb), dim3(cgv2::kVisThreads), 0, st, pts, m, vis_table(ws, V), v0, vc,
                       rho, rf, count);
  }
  return hipGetLastError();
}

size_t cgv2_crop_ws_layout(int64_t m, size_t* off) {
  const int64_t nb = std::max<int64_t>((m + cgv2::kCropChunk - 1) / cgv2::kCropChunk, 1);
  // off: [0] kept count / offset per workgroup (u32), [1] height min / max per workgroup (f64 x 2)
  off[0] = 0;
  off[1] = ((size_t)4 * (size_t)nb + 255) & ~(size_t)255;
  return off[1] + (((size_t)16 * (size_t)nb + 255) & ~(size_t)255);
}

hipError_t cgv2_launch_crop(const float* pts, int64_t m, const uint32_t* count, uint32_t tau, const double* T,
                            uint8_t* keep, double* ground, double* hrange, int64_t* kept, void* ws, hipStream_t st) {
  size_t off[kCropOffs];
  cgv2_crop_ws_layout(m, off);
  const int nb = (int)std::max<int64_t>((m + cgv2::kCropChunk - 1) / cgv2::kCropChunk, 1);
  uint32_t* kpart = (uint32_t*)((char*)ws + off[0]);
  double* hpart = (double*)((char*)ws + off[1]);
  cgv2::Ground g;
  for (int i = 0; i < 12; ++i) g.T[i] = T[i];
  if (m > 0) {
    hipLaunchKernelGGL(cgv2::k_crop_count, dim3((unsigned)nb), dim3(cgv2::kCropBlock), 0, st, pts, m, count, tau, g,
                       keep, kpart, hpart);
  } else {
    hipLaunchKernelGGL((cgv2::k_fill<uint32_t>), dim3(1), dim3(64), 0, st, kpart, (int64_t)1, 0u);
    hipLaunchKernelGGL((cgv2::k_fill<double>), dim3(1), dim3(64), 0, st, hpart, (int64_t)2, 0.0);
  }
  hipLaunchKernelGGL(cgv2::k_crop_scan, dim3(1), dim3(cgv2::kCropBlock), 0, st, kpart, hpart, nb, kept, hrange);
  if (m > 0)
    hipLaunchKernelGGL(cgv2::k_crop_write, dim3((unsigned)nb), dim3(cgv2::kCropBlock), 0, st, pts, m, keep, g, kpart,
                       ground);
  return hipGetLastError();
}
