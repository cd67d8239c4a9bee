// Device-side helpers shared by the gfx950 kernels of the surfel rasterizer.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/cgv2r.h"

namespace cgv2 {

constexpr int kTile = CGV2_TILE;
constexpr int kRec = CGV2_REC_FLOATS;
constexpr int kGradFields = 19;  // per-surfel, per-view record gradients accumulated by render_bwd

// record field offsets
enum : int {
  R_CXH = 0, R_CYH, R_CXL, R_CYL, R_A11, R_A12, R_A21, R_A22, R_W0, R_W1, R_W2,
  R_ZC, R_OP, R_R, R_G, R_B, R_NX, R_NY, R_NZ, R_K2, R_PXR, R_PYR
};

// record-gradient fields accumulated by the reverse pass; the first 16 are the slots of its wave
// reduce-scatter
enum : int {
  G_CX = 0, G_CY, G_A11, G_A12, G_A21, G_A22, G_W0, G_W1, G_W2, G_OP, G_R, G_G, G_B, G_SCX, G_SCY, G_ZC,
  G_NX, G_NY, G_NZ
};

// Record gradients in the backward workspace.  Fields G_CX..G_ZC of (view v, surfel i) form one 64-B
// row row[(v n + i) 16 + f], so the 16 atomics a wave issues for a (surfel, tile) fall in one cache
// line; the normal fields follow all views' rows as 16-B rows nrm[(v n + i) 4 + c] (c < 3).
constexpr int kGradRow = 16;
constexpr int kGradNrm = 4;
struct RecGrads {
  float* row;
  float* nrm;
};

constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTmin = 1e-4f;
constexpr float kNegHalfLog2e = -0.72134752044448170368f;  // -0.5 / ln 2

struct DevCam {
  int W, H;
  float fx, fy, cx, cy, R[9], t[3], znear, bg[3];
};

// Cameras travel as kernel arguments (the library allocates nothing): up to kMaxViews per launch,
// views [v0, v0 + count) of the call.
constexpr int kMaxViews = 32;
struct CamPack {
  DevCam c[kMaxViews];
  int v0, count;
};

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// DPP move (gfx9 encodings); lanes of rows outside kRowMask receive 0.
template <int kCtrl, int kRowMask = 0xf>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kCtrl, kRowMask, 0xf, false));
}

// Sum over the 64 lanes of a wave with DPP row operations only (no LDS traffic); the total is
// valid in lane 63.
__device__ __forceinline__ float wave_sum_lane63(float v) {
  v += dpp<0xB1>(v);        // quad_perm [1,0,3,2]
  v += dpp<0x4E>(v);        // quad_perm [2,3,0,1]
  v += dpp<0x141>(v);       // row_half_mirror: 4-lane groups -> 8
  v += dpp<0x140>(v);       // row_mirror: 8 -> 16 (every lane holds its row's sum)
  v += dpp<0x142, 0xa>(v);  // row_bcast:15 -> rows 1 and 3 add rows 0 and 2
  v += dpp<0x143, 0xc>(v);  // row_bcast:31 -> rows 2 and 3 add rows 0+1
  return v;
}

// Reduce-scatter of 16 per-lane values over a wave: on return every lane holds the wave total of
// value index reduce16_index(lane).  Exchanges: xor 32 and xor 16 with the gfx950 row-swap
// instructions (x' + y' after a swap is already the pairwise sum of the kept half), xor 1 and xor 2
// with DPP quad permutations, then an all-reduce over lane bits 2-3 with two row rotations.
// About 35 VALU operations for 16 values, against 96 for 16 separate reductions.
__device__ __forceinline__ int reduce16_index(int lane) {
  return ((lane >> 1) & 1) | ((lane & 1) << 1) | (((lane >> 4) & 1) << 2) | (((lane >> 5) & 1) << 3);
}

__device__ __forceinline__ float reduce16_scatter(float (&v)[16]) {
  const int lane = (int)(threadIdx.x & 63u);
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[j]), __float_as_uint(v[j + 8]), false, false);
    v[j] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[j]), __float_as_uint(v[j + 4]), false, false);
    v[j] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  const bool b0 = lane & 1, b1 = lane & 2;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const float send = b0 ? v[j] : v[j + 2];
    const float keep = b0 ? v[j + 2] : v[j];
    v[j] = keep + dpp<0xB1>(send);
  }
  float t;
  {
    const float send = b1 ? v[0] : v[1];
    const float keep = b1 ? v[1] : v[0];
    t = keep + dpp<0x4E>(send);
  }
  t += dpp<0x124>(t);  // row_ror:4
  t += dpp<0x128>(t);  // row_ror:8
  return t;
}

// Where a surfel can reach alpha >= 1/255 (Sec. 3.1 cutoff).  rho is the smaller of the ray-splat
// distance |A x|^2 / w(x)^2 and the screen-filter distance |x|^2, both halved (x relative to the
// projected centre; A = the record's a_ij / sqrt 2, w(x) = w0 + w1 x + w2 y as the renderer stages
// them, so this is the function its evaluation rounds), and the cutoff is rho <= ln(255 o) = k2 / 2.
// {|A x|^2 <= c w(x)^2} is the conic g(x) = x'Gx + 2 b'x + d <= 0; when G is positive definite it is an
// ellipse, met by a box iff its centre lies in the box or g <= 0 somewhere on one of the four edges
// (g is convex, so each edge's minimum is at the clamped stationary point).  FP64, with the cutoff
// enlarged to c = 0.5 k2 (1 + 2e-3) + 1e-3 and every box padded by kReachPad: far beyond the FP32
// error of the evaluation and of the reciprocals used here, so a box is reported unreachable only
// where no pixel sample in it can take the surfel.  A conic that is not an ellipse reaches every box.
constexpr float kInvSqrt2 = 0.70710678118654752440f;
constexpr double kReachPad = 1.0 / 64.0;

struct Reach {
  double G00, G01, G11, b0, b1, d, c, i00, i11, xs, ys;
  bool ellipse;
};

__device__ __forceinline__ void reach_setup(float a11, float a12, float a21, float a22, float w0f, float w1f, float w2f,
                                            float k2, Reach& q) {
  q.c = 0.5 * (double)k2 * (1.0 + 2e-3) + 1e-3;
  const double A11 = a11, A12 = a12, A21 = a21, A22 = a22, w0 = w0f, w1 = w1f, w2 = w2f, c = q.c;
  q.G00 = A11 * A11 + A21 * A21 - c * w1 * w1;
  q.G01 = A11 * A12 + A21 * A22 - c * w1 * w2;
  q.G11 = A12 * A12 + A22 * A22 - c * w2 * w2;
  const double det = q.G00 * q.G11 - q.G01 * q.G01;
  q.ellipse = q.G00 > 0.0 && q.G11 > 0.0 && det > 0.0 && det < 1e300;
  q.b0 = -c * w0 * w1;
  q.b1 = -c * w0 * w2;
  q.d = -c * w0 * w0;
  // single-precision reciprocals are enough: they only place the points at which g is evaluated
  const float r00 = __builtin_amdgcn_rcpf((float)q.G00), r11 = __builtin_amdgcn_rcpf((float)q.G11);
  const float rdet = __builtin_amdgcn_rcpf((float)det);
  // (a reciprocal that overflows or underflows in single precision leaves the conic unused)
  const bool fin = isfinite(r00) && isfinite(r11) && isfinite(rdet) && r00 > 0.f && r11 > 0.f && rdet > 0.f;
  q.ellipse = q.ellipse && fin;
  q.i00 = q.ellipse ? (double)r00 : 0.0;
  q.i11 = q.ellipse ? (double)r11 : 0.0;
  const double idet = q.ellipse ? (double)rdet : 0.0;
  q.xs = -(q.G11 * q.b0 - q.G01 * q.b1) * idet;
  q.ys = -(q.G00 * q.b1 - q.G01 * q.b0) * idet;
}

// Does the box [xl, xh] x [yl, yh] (centre-relative, already padded) hold a point with rho <= c?
__device__ __forceinline__ bool reach_box(const Reach& q, double xl, double xh, double yl, double yh) {
  // screen-filter disc |x|^2 <= c
  const double dx = xl > 0.0 ? xl : (xh < 0.0 ? xh : 0.0), dy = yl > 0.0 ? yl : (yh < 0.0 ? yh : 0.0);
  if (dx * dx + dy * dy <= q.c) return true;
  if (!q.ellipse || (q.xs >= xl && q.xs <= xh && q.ys >= yl && q.ys <= yh)) return true;
  auto g = [&](double x, double y) {
    return fma(q.G00 * x, x, fma(2.0 * q.G01 * x, y, fma(q.G11 * y, y, fma(2.0 * q.b0, x, fma(2.0 * q.b1, y, q.d)))));
  };
  const double yA = fmin(fmax(-(q.G01 * xl + q.b1) * q.i11, yl), yh);
  const double yB = fmin(fmax(-(q.G01 * xh + q.b1) * q.i11, yl), yh);
  const double xA = fmin(fmax(-(q.G01 * yl + q.b0) * q.i00, xl), xh);
  const double xB = fmin(fmax(-(q.G01 * yh + q.b0) * q.i00, xl), xh);
  return fmin(fmin(g(xl, yA), g(xh, yB)), fmin(g(xA, yl), g(xB, yh))) <= 0.0;
}

// Box of the pixel samples [x0 + 0.5, x0 + span - 0.5] x [y0 + ...] of a tile-relative cell, relative to
// the tile-relative centre (cxt, cyt), padded.
__device__ __forceinline__ bool reach_cell(const Reach& q, float cxt, float cyt, int x0, int y0, int span) {
  const double xl = (double)x0 + 0.5 - (double)cxt - kReachPad, xh = xl + (double)(span - 1) + 2.0 * kReachPad;
  const double yl = (double)y0 + 0.5 - (double)cyt - kReachPad, yh = yl + (double)(span - 1) + 2.0 * kReachPad;
  return reach_box(q, xl, xh, yl, yh);
}

template <typename T>
__global__ __launch_bounds__(256) void k_fill(T* p, int64_t count, T v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Zeroes count elements of a and of b (either may be null) in one launch.
template <typename T>
__global__ __launch_bounds__(256) void k_zero2(T* a, T* b, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
    if (a) a[i] = T(0);
    if (b) b[i] = T(0);
  }
}

// Exclusive scan over a workgroup of kThreads threads (a multiple of 64); lds holds kThreads / 64
// values; 'total' receives the workgroup sum.  Every thread of the workgroup must call it.
template <int kThreads, typename T>
__device__ __forceinline__ T block_exscan(T v, T* lds, T& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  T x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const T y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) lds[w] = x;
  __syncthreads();
  T off = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kThreads / 64; ++k) {
    if (k < w) off += lds[k];
    tot += lds[k];
  }
  __syncthreads();
  total = tot;
  return off + x - v;
}

// Block -> tile mapping.  Hardware dispatches workgroup b to XCD b % 8.  Here XCD x receives the
// runs of kXcdChunk consecutive tiles with run index = x (mod 8): neighbouring tiles of a run share
// that XCD's L2, while the runs of every XCD are spread over the whole image.  (Giving each XCD one
// contiguous band instead leaves the XCD with the densest band -- the far field of an oblique view --
// with up to twice the mean work.)  Blocks past the last full round of 8 runs map to themselves.
constexpr uint32_t kXcdChunk = 4;
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t nb) {
  const uint32_t span = 8u * kXcdChunk;
  const uint32_t full = nb - nb % span;
  if (b >= full) return b;
  const uint32_t x = b % 8u, k = b / 8u;  // XCD and the block's rank on it
  return (x + 8u * (k / kXcdChunk)) * kXcdChunk + k % kXcdChunk;
}

}  // namespace cgv2
