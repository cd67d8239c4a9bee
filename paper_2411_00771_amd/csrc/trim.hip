// Contribution-based trimming of CityGaussianV2 Sec. 3.3 (Eq. 3, Eq. 4 and the percentile bound).
//
// The per-view sums are accumulated by the contribution mode of the forward traversal (render.hip);
// here:
//   k_zero_pairs      clears the (sum, count) pairs of the surfels in each view's visible list
//   k_contrib_final   C_{n,k} = sum / count (0 for surfels without a blended pixel), the running sum
//                     over the call's views (fixed order), |P_k|
//   k_sel_*           exact k-th smallest of a non-negative float array: four 8-bit radix passes over
//                     the float bits (per-workgroup histograms, one workgroup picks the digit)
//   k_trim_apply      mask = c <= bound, per-workgroup counts, reduced by one workgroup
#include "cgv2r_device.h"
#include "cgv2r_kernels.h"

#include <algorithm>

namespace cgv2 {

constexpr int kSelBlock = 256;
constexpr int kSelMaxBlocks = 1024;

__global__ __launch_bounds__(256) void k_zero_pairs(const uint32_t* __restrict__ visible,
                                                   const uint32_t* __restrict__ vstart, int64_t n, float2* cws,
                                                   int v0) {
  const int v = v0 + (int)blockIdx.y;
  const uint32_t e0 = vstart[v], e1 = vstart[v + 1];
  for (uint32_t e = e0 + blockIdx.x * blockDim.x + threadIdx.x; e < e1; e += gridDim.x * blockDim.x)
    cws[(int64_t)v * n + visible[e]] = make_float2(0.f, 0.f);
}

__global__ __launch_bounds__(256) void k_contrib_final(const uint8_t* __restrict__ flags,
                                                      const float2* __restrict__ cws, int64_t n, int V,
                                                      float* __restrict__ c_view, float* __restrict__ c_sum,
                                                      uint32_t* __restrict__ pixels) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    float acc = 0.f;
    for (int v = 0; v < V; ++v) {
      const int64_t vi = (int64_t)v * n + i;
      float C = 0.f, cnt = 0.f;
      if (flags[vi] & CGV2_F_VISIBLE) {
        const float2 q = cws[vi];
        cnt = q.y;
        C = cnt > 0.f ? q.x / cnt : 0.f;
      }
      if (c_view) c_view[vi] = C;
      if (pixels) pixels[vi] = (uint32_t)cnt;
      acc += C;
    }
    if (c_sum) c_sum[i] += acc;
  }
}

// selection state: [0] prefix of the bits found so far, [1] mask of those bits, [2] rank still sought
__global__ void k_sel_init(uint32_t* __restrict__ state, uint32_t k) {
  if (threadIdx.x == 0) {
    state[0] = 0;
    state[1] = 0;
    state[2] = k;
  }
}

__global__ __launch_bounds__(kSelBlock) void k_sel_hist(const float* __restrict__ c, int64_t n,
                                                       const uint32_t* __restrict__ state, int shift,
                                                       uint32_t* __restrict__ part) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t prefix = state[0], mask = state[1];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t key = __float_as_uint(c[i]);
    if ((key & mask) == prefix) atomicAdd(&h[(key >> shift) & 255u], 1u);
  }
  __syncthreads();
  part[(int64_t)blockIdx.x * 256 + threadIdx.x] = h[threadIdx.x];
}

// One workgroup of kPickThreads: the per-workgroup histograms are summed by kPickThreads / 256 groups
// of threads with kPickUnroll independent loads in flight each (the sum is latency-bound); a scan over
// the 256 bins then finds the digit whose count range holds the rank sought.
constexpr int kPickThreads = 1024;
constexpr int kPickUnroll = 8;

__global__ __launch_bounds__(kPickThreads) void k_sel_pick(const uint32_t* __restrict__ part, int nblocks, int shift,
                                                          uint32_t* __restrict__ state) {
  constexpr int kGroups = kPickThreads / 256;
  __shared__ uint32_t tot[kGroups][256];
  __shared__ uint32_t wsum[4];
  const uint32_t k = state[2];  // read by every thread before any write below
  const int bin = threadIdx.x & 255, grp = threadIdx.x >> 8;
  uint32_t acc[kPickUnroll] = {};
  int b = grp;
  for (; b + (kPickUnroll - 1) * kGroups < nblocks; b += kPickUnroll * kGroups) {
#pragma unroll
    for (int u = 0; u < kPickUnroll; ++u) acc[u] += part[(int64_t)(b + u * kGroups) * 256 + bin];
  }
  for (; b < nblocks; b += kGroups) acc[0] += part[(int64_t)b * 256 + bin];
  uint32_t t = 0;
#pragma unroll
  for (int u = 0; u < kPickUnroll; ++u) t += acc[u];
  tot[grp][bin] = t;
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t c = 0, x = 0;
  if (threadIdx.x < 256) {
#pragma unroll
    for (int g = 0; g < kGroups; ++g) c += tot[g][threadIdx.x];
    x = c;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(x, d, 64);
      if (lane >= d) x += y;
    }
    if (lane == 63) wsum[w] = x;
  }
  __syncthreads();
  if (threadIdx.x < 256) {
    uint32_t off = 0;
    for (int q = 0; q < w; ++q) off += wsum[q];
    const uint32_t incl = off + x, below = incl - c;
    // digit d: below(d) <= k < below(d) + count(d); the last digit also takes a rank past the total
    if (below <= k && (k < incl || threadIdx.x == 255)) {
      state[0] |= (uint32_t)threadIdx.x << shift;
      state[1] |= 255u << shift;
      state[2] = k - below;
    }
  }
}

__global__ __launch_bounds__(kSelBlock) void k_trim_apply(const float* __restrict__ c, int64_t n,
                                                         const uint32_t* __restrict__ state,
                                                         uint8_t* __restrict__ mask, uint32_t* __restrict__ part) {
  __shared__ uint32_t red[kSelBlock];
  const float bound = __uint_as_float(state[0]);
  uint32_t cnt = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const bool rm = c[i] <= bound;
    mask[i] = rm ? 1 : 0;
    cnt += rm ? 1u : 0u;
  }
  red[threadIdx.x] = cnt;
  __syncthreads();
  for (int off = kSelBlock / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kSelBlock) void k_trim_count(const uint32_t* __restrict__ part, int nblocks,
                                                         const uint32_t* __restrict__ state, float* __restrict__ bound,
                                                         uint32_t* __restrict__ removed) {
  __shared__ uint32_t red[kSelBlock];
  uint32_t t = 0;
  for (int b = threadIdx.x; b < nblocks; b += kSelBlock) t += part[b];
  red[threadIdx.x] = t;
  __syncthreads();
  for (int off = kSelBlock / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (removed) *removed = red[0];
    if (bound) *bound = __uint_as_float(state[0]);
  }
}

}  // namespace cgv2

size_t cgv2_contribution_ws_layout(int64_t n, int V) {
  return ((size_t)8 * (size_t)n * (size_t)V + 255) & ~(size_t)255;
}

hipError_t cgv2_launch_contribution_final(const cgv2_proj& p, const cgv2::CamPack& cams, int64_t n, int V_total,
                                          void* ws, bool zero, float* c_view, float* c_sum, uint32_t* pixels,
                                          hipStream_t st) {
  float2* cws = (float2*)ws;
  if (zero) {
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(cgv2::k_zero_pairs, dim3(blocks, (unsigned)cams.count), dim3(256), 0, st, p.visible,
                       p.visible_start, n, cws, cams.v0);
  } else {
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(cgv2::k_contrib_final, dim3(blocks), dim3(256), 0, st, p.flags, cws, n, V_total, c_view, c_sum,
                       pixels);
  }
  return hipGetLastError();
}

size_t cgv2_trim_ws_layout(int64_t n, size_t* off) {
  const int64_t nb = std::min<int64_t>(std::max<int64_t>((n + cgv2::kSelBlock * 8 - 1) / (cgv2::kSelBlock * 8), 1),
                                       cgv2::kSelMaxBlocks);
  // off: [0] selection state (u32 x 4), [1] per-workgroup histograms (u32, nb x 256), [2] counts (u32, nb)
  off[0] = 0;
  off[1] = 256;
  off[2] = off[1] + ((4 * 256 * (size_t)nb + 255) & ~(size_t)255);
  return off[2] + ((4 * (size_t)nb + 255) & ~(size_t)255);
}

hipError_t cgv2_launch_trim(const float* c, int64_t n, uint32_t k, float* bound, uint8_t* mask, uint32_t* removed,
                            void* ws, hipStream_t st) {
  size_t off[kTrimOffs];
  cgv2_trim_ws_layout(n, off);
  const int nb = (int)std::min<int64_t>(std::max<int64_t>((n + cgv2::kSelBlock * 8 - 1) / (cgv2::kSelBlock * 8), 1),
                                        cgv2::kSelMaxBlocks);
  uint32_t* state = (uint32_t*)((char*)ws + off[0]);
  uint32_t* part = (uint32_t*)((char*)ws + off[1]);
  uint32_t* cnt = (uint32_t*)((char*)ws + off[2]);
  hipLaunchKernelGGL(cgv2::k_sel_init, dim3(1), dim3(64), 0, st, state, k);
  for (int shift = 24; shift >= 0; shift -= 8) {
    hipLaunchKernelGGL(cgv2::k_sel_hist, dim3((unsigned)nb), dim3(cgv2::kSelBlock), 0, st, c, n, state, shift, part);
    hipLaunchKernelGGL(cgv2::k_sel_pick, dim3(1), dim3(cgv2::kPickThreads), 0, st, part, nb, shift, state);
  }
  hipLaunchKernelGGL(cgv2::k_trim_apply, dim3((unsigned)nb), dim3(cgv2::kSelBlock), 0, st, c, n, state, mask, cnt);
  hipLaunchKernelGGL(cgv2::k_trim_count, dim3(1), dim3(cgv2::kSelBlock), 0, st, cnt, nb, state, bound, removed);
  return hipGetLastError();
}
