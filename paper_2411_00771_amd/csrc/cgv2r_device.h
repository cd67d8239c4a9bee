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

template <typename T>
__global__ __launch_bounds__(256) void k_fill(T* p, int64_t count, T v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
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
