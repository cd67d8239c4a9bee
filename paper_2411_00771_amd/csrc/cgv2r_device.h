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
  R_ZC, R_OP, R_R, R_G, R_B, R_NX, R_NY, R_NZ, R_K2
};

// record-gradient field offsets ([V][kGradFields][n] in the backward workspace)
enum : int {
  G_CX = 0, G_CY, G_A11, G_A12, G_A21, G_A22, G_W0, G_W1, G_W2, G_ZC, G_OP,
  G_R, G_G, G_B, G_NX, G_NY, G_NZ, G_SCX, G_SCY
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

// Per-pixel evaluation of one surfel, shared by the forward and the backward kernels so that
// both take bit-identical decisions.  (xr, yr) = pixel sample minus the projected centre.
struct PairEval {
  float P1, P2, w, nn, ww, rho, G, araw, alpha;
  bool is3d;
};

__device__ __forceinline__ void eval_pair(float xr, float yr, float a11, float a12, float a21, float a22, float w0,
                                          float w1, float w2, float op, PairEval& e) {
  e.P1 = fmaf(a11, xr, a12 * yr);
  e.P2 = fmaf(a21, xr, a22 * yr);
  e.w = fmaf(w1, xr, fmaf(w2, yr, w0));
  e.nn = fmaf(e.P1, e.P1, e.P2 * e.P2);
  e.ww = e.w * e.w;
  const float rho2 = 2.0f * fmaf(xr, xr, yr * yr);
  // rho_3d = nn / ww <= rho_2d, evaluated without a division; ww == 0 means the ray is parallel
  // to the plane (rho_3d infinite)
  e.is3d = (e.ww > 0.0f) && (e.nn <= rho2 * e.ww);
  e.rho = e.is3d ? e.nn * __builtin_amdgcn_rcpf(e.ww) : rho2;
  e.G = exp2f(e.rho * kNegHalfLog2e);
  e.araw = op * e.G;
  e.alpha = fminf(kAlphaMax, e.araw);
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Sum over the 64 lanes of a wave; the result is valid in every lane.
__device__ __forceinline__ float wave_sum(float v) {
  v += __shfl_xor(v, 1);
  v += __shfl_xor(v, 2);
  v += __shfl_xor(v, 4);
  v += __shfl_xor(v, 8);
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}

// Block -> tile mapping that keeps neighbouring tiles on one XCD: hardware dispatches
// workgroup b to XCD b % 8, so XCD x receives the contiguous run [x*q, (x+1)*q).
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t nb) {
  const uint32_t q = nb / 8u, r = nb % 8u;
  const uint32_t x = b % 8u, k = b / 8u;
  // the first r XCDs take q + 1 blocks each
  const uint32_t base = x < r ? x * (q + 1u) : r * (q + 1u) + (x - r) * q;
  return base + k;
}

}  // namespace cgv2
