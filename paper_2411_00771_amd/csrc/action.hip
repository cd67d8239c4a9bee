// Densification action: the candidates of CityGaussianV2 Sec. 3.2 (DGD high gradient, not elongated)
// are cloned or split, and the surfels trimmed by Sec. 3.3 (or below the minimum opacity) are removed,
// by the clone / split rule of the 3DGS / 2DGS training the method builds on.
//
// plan (per source surfel, order-preserving):
//   k_act_count  per workgroup of kAChunk surfels: each surfel's action and the workgroup's four
//                action counts
//   k_act_scan   one workgroup: exclusive offsets of the survivors and of the new surfels per
//                workgroup; the totals and the output count
//   k_act_dst    per workgroup: each surfel's survivor slot and first new slot, in id order
// apply (per output slot: every write is coalesced, reads follow the sources in order):
//   k_src_fill   inverse map slot -> (source id, kind: survivor, copy, child 0, child 1)
//   k_apply      geometry of each slot (a split child is placed in FP64 and rounded once), then the
//                slots' SH blocks copied by the whole workgroup
//   k_gather     the same re-layout for any other per-surfel float field
#include "cgv2r_device.h"
#include "cgv2r_kernels.h"

#include <algorithm>

namespace cgv2 {

constexpr int kABlock = 256;
constexpr int kAItems = 8;
constexpr int kAChunk = kABlock * kAItems;
constexpr uint32_t kNone = 0xffffffffu;

enum : uint32_t { A_KEEP = 0, A_CLONE = 1, A_SPLIT = 2, A_REMOVE = 3 };
enum : uint32_t { S_SURVIVOR = 0, S_COPY = 1, S_CHILD0 = 2, S_CHILD1 = 3 };

// The action of surfel i, decided in FP64 on the float32 parameters.
__device__ __forceinline__ uint32_t action_of(const uint8_t* __restrict__ mask, const uint8_t* __restrict__ remove,
                                              const float* __restrict__ ls, const float* __restrict__ logit,
                                              int64_t n, int64_t i, double dense_scale, double min_opacity) {
  const double o = 1.0 / (1.0 + exp(-(double)logit[i]));
  if ((remove && remove[i]) || o < min_opacity) return A_REMOVE;
  if (!(mask[i] & 4u)) return A_KEEP;
  const double smax = fmax(exp((double)ls[i]), exp((double)ls[n + i]));
  return smax <= dense_scale ? A_CLONE : A_SPLIT;
}

// Items k * kABlock + thread of the workgroup's chunk: every load and the action store are coalesced
// (the counts need no order).
__global__ __launch_bounds__(kABlock) void k_act_count(const uint8_t* __restrict__ mask,
                                                       const uint8_t* __restrict__ remove,
                                                       const float* __restrict__ ls,
                                                       const float* __restrict__ logit, int64_t n,
                                                       double dense_scale, double min_opacity,
                                                       uint8_t* __restrict__ actions, uint32_t* __restrict__ part) {
  __shared__ unsigned long long lds[kABlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kAChunk + threadIdx.x;
  // four counts of at most kAChunk each, 16 bits apiece
  unsigned long long c = 0;
#pragma unroll
  for (int k = 0; k < kAItems; ++k) {
    const int64_t i = base + (int64_t)k * kABlock;
    if (i < n) {
      const uint32_t a = action_of(mask, remove, ls, logit, n, i, dense_scale, min_opacity);
      actions[i] = (uint8_t)a;
      c += 1ull << (16 * a);
    }
  }
  unsigned long long tot;
  block_exscan<kABlock>(c, lds, tot);
  if (threadIdx.x < 4) part[(int64_t)blockIdx.x * 4 + threadIdx.x] = (uint32_t)((tot >> (16 * threadIdx.x)) & 0xffffu);
}

// counts: [0] keep, [1] clone, [2] split, [3] removed, [4] output surfels = keep + 2 clone + 2 split
__global__ __launch_bounds__(kABlock) void k_act_scan(const uint32_t* __restrict__ part, int nb,
                                                      uint2* __restrict__ offs, int64_t* __restrict__ counts) {
  __shared__ unsigned long long lds[kABlock / 64];
  __shared__ unsigned long long red[4][kABlock / 64];
  unsigned long long carry = 0;
  unsigned long long acc[4] = {0, 0, 0, 0};
  for (int b0 = 0; b0 < nb; b0 += kABlock) {
    const int b = b0 + (int)threadIdx.x;
    uint32_t q[4] = {0, 0, 0, 0};
    if (b < nb) {
#pragma unroll
      for (int k = 0; k < 4; ++k) q[k] = part[(int64_t)b * 4 + k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] += q[k];
    // survivors in the low half, new surfels in the high half (each total < 2^32 for n < 2^30)
    const unsigned long long v = (unsigned long long)(q[A_KEEP] + q[A_CLONE]) |
                                 ((unsigned long long)(q[A_CLONE] + 2u * q[A_SPLIT]) << 32);
    unsigned long long tot;
    const unsigned long long ex = block_exscan<kABlock>(v, lds, tot) + carry;
    if (b < nb) offs[b] = make_uint2((uint32_t)ex, (uint32_t)(ex >> 32));
    carry += tot;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    unsigned long long x = acc[k];
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) x += __shfl_xor(x, d, 64);
    if (lane == 0) red[k][w] = x;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    unsigned long long t = 0;
#pragma unroll
    for (int k = 0; k < kABlock / 64; ++k) t += red[threadIdx.x][k];
    counts[threadIdx.x] = (int64_t)t;
  }
  if (threadIdx.x == 0) counts[4] = (int64_t)(carry & 0xffffffffull) + (int64_t)(carry >> 32);
}

// Each thread scans kAItems consecutive surfels; the slots go through LDS so that the stores of
// dst[0] and dst[1] are coalesced.
__global__ __launch_bounds__(kABlock) void k_act_dst(const uint8_t* __restrict__ actions, int64_t n,
                                                     const uint2* __restrict__ offs,
                                                     const int64_t* __restrict__ counts,
                                                     uint32_t* __restrict__ dst) {
  __shared__ uint32_t lds[kABlock / 64];
  __shared__ uint32_t s_d0[kAChunk], s_d1[kAChunk];
  const int64_t chunk = (int64_t)blockIdx.x * kAChunk;
  const int64_t base = chunk + (int64_t)threadIdx.x * kAItems;
  uint32_t a[kAItems];
  if (base + kAItems <= n) {
    const uint2 w = *(const uint2*)(actions + base);
#pragma unroll
    for (int k = 0; k < kAItems; ++k) a[k] = ((k < 4 ? w.x : w.y) >> (8 * (k & 3))) & 255u;
  } else {
#pragma unroll
    for (int k = 0; k < kAItems; ++k) a[k] = base + k < n ? actions[base + k] : A_REMOVE;
  }
  // survivors (<= 8) in the low half, new surfels (<= 16) in the high half
  uint32_t v = 0;
#pragma unroll
  for (int k = 0; k < kAItems; ++k)
    v += (a[k] <= A_CLONE ? 1u : 0u) + (a[k] == A_CLONE ? 1u << 16 : a[k] == A_SPLIT ? 2u << 16 : 0u);
  uint32_t tot;
  const uint32_t ex = block_exscan<kABlock>(v, lds, tot);
  const uint2 o = offs[blockIdx.x];
  const uint32_t survivors = (uint32_t)(counts[A_KEEP] + counts[A_CLONE]);
  uint32_t rs = o.x + (ex & 0xffffu);
  uint32_t rn = survivors + o.y + (ex >> 16);
#pragma unroll
  for (int k = 0; k < kAItems; ++k) {
    uint32_t d0 = kNone, d1 = kNone;
    if (a[k] <= A_CLONE) d0 = rs++;
    if (a[k] == A_CLONE || a[k] == A_SPLIT) {
      d1 = rn;
      rn += a[k] == A_CLONE ? 1u : 2u;
    }
    s_d0[threadIdx.x * kAItems + k] = d0;
    s_d1[threadIdx.x * kAItems + k] = d1;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kAItems; ++k) {
    const int e = k * kABlock + (int)threadIdx.x;
    const int64_t i = chunk + e;
    if (i < n) {
      dst[i] = s_d0[e];
      dst[n + i] = s_d1[e];
    }
  }
}

__device__ __forceinline__ int64_t live_slots(const int64_t* counts, int64_t cap) {
  return counts[4] < cap ? counts[4] : cap;
}

__global__ __launch_bounds__(kABlock) void k_src_fill(const uint8_t* __restrict__ actions,
                                                      const uint32_t* __restrict__ dst, int64_t n,
                                                      const int64_t* __restrict__ counts, int64_t cap,
                                                      uint32_t* __restrict__ src) {
  const int64_t lim = live_slots(counts, cap);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t a = actions[i];
    const uint32_t d0 = dst[i], d1 = dst[n + i];
    const uint32_t id = (uint32_t)i << 2;
    if (a <= A_CLONE && d0 < lim) src[d0] = id | S_SURVIVOR;
    if (a == A_CLONE && d1 < lim) src[d1] = id | S_COPY;
    if (a == A_SPLIT) {
      if (d1 < lim) src[d1] = id | S_CHILD0;
      if ((int64_t)d1 + 1 < lim) src[d1 + 1] = id | S_CHILD1;
    }
  }
}

// One workgroup per run of kABlock output slots: each thread places its slot's geometry, then the
// workgroup copies the slots' SH blocks together (float4 where a block is a whole number of them), so
// the SH writes of the run form one contiguous, fully coalesced stream.
template <int kF>  // floats per SH block: 3 (deg + 1)^2
__global__ __launch_bounds__(kABlock) void k_apply(cgv2_surfels s, const uint32_t* __restrict__ src,
                                                   const int64_t* __restrict__ counts,
                                                   const float* __restrict__ z, double log_shrink,
                                                   cgv2_surfels_out out) {
  constexpr int kV = (kF % 4 == 0) ? 4 : 1;  // floats per copy unit
  constexpr int kU = kF / kV;                // copy units per SH block
  __shared__ uint32_t s_src[kABlock];
  const int64_t n = s.n, cap = out.n;
  const int64_t lim = live_slots(counts, cap);
  for (int64_t j0 = (int64_t)blockIdx.x * kABlock; j0 < lim; j0 += (int64_t)gridDim.x * kABlock) {
    const int64_t j = j0 + threadIdx.x;
    uint32_t e = kNone;
    if (j < lim) {
      e = src[j];
      const int64_t i = e >> 2;
      const uint32_t kind = e & 3u;
      if (i < n) {
        float q[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          q[c] = s.quat[c * n + i];
          out.quat[c * cap + j] = q[c];
        }
        out.opacity_logit[j] = s.opacity_logit[i];
        const float l0 = s.log_scale[i], l1 = s.log_scale[n + i];
        if (kind < S_CHILD0) {
#pragma unroll
          for (int c = 0; c < 3; ++c) out.mean[c * cap + j] = s.mean[c * n + i];
          out.log_scale[j] = l0;
          out.log_scale[cap + j] = l1;
        } else {
          // child: mu + s_u z0 t_u + s_v z1 t_v, with t_u, t_v the first two columns of the rotation
          const double w = q[0], x = q[1], y = q[2], zq = q[3];
          const double r = 1.0 / sqrt(w * w + x * x + y * y + zq * zq);
          const double qw = w * r, qx = x * r, qy = y * r, qz = zq * r;
          const double tu[3] = {1.0 - 2.0 * (qy * qy + qz * qz), 2.0 * (qx * qy + qw * qz),
                                2.0 * (qx * qz - qw * qy)};
          const double tv[3] = {2.0 * (qx * qy - qw * qz), 1.0 - 2.0 * (qx * qx + qz * qz),
                                2.0 * (qy * qz + qw * qx)};
          const float* zz = z + i * 4 + (kind - S_CHILD0) * 2;
          const double du = exp((double)l0) * (double)zz[0], dv = exp((double)l1) * (double)zz[1];
#pragma unroll
          for (int c = 0; c < 3; ++c)
            out.mean[c * cap + j] = (float)((double)s.mean[c * n + i] + du * tu[c] + dv * tv[c]);
          out.log_scale[j] = (float)((double)l0 - log_shrink);
          out.log_scale[cap + j] = (float)((double)l1 - log_shrink);
        }
      }
    }
    s_src[threadIdx.x] = e;
    __syncthreads();
    const int cnt = (int)((lim - j0) < kABlock ? (lim - j0) : kABlock);
    for (int t = threadIdx.x; t < cnt * kU; t += kABlock) {
      const int slot = t / kU, k = t - slot * kU;
      const int64_t i = s_src[slot] >> 2;
      if (i >= n) continue;
      if constexpr (kV == 4) {
        const float4 v = ((const float4*)s.sh)[i * kU + k];
        ((float4*)out.sh)[(j0 + slot) * kU + k] = v;
      } else {
        out.sh[(j0 + slot) * kF + k] = s.sh[i * kF + k];
      }
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kABlock) void k_gather(const float* __restrict__ f, int64_t n, int C, int blocked,
                                                    const uint32_t* __restrict__ src,
                                                    const int64_t* __restrict__ counts, int64_t cap, int zero_new,
                                                    float* __restrict__ out) {
  const int64_t lim = live_slots(counts, cap);
  const int64_t total = lim * C;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    int64_t j, c;
    if (blocked) {
      j = t / C;
      c = t - j * C;
    } else {
      c = t / lim;
      j = t - c * lim;
    }
    const uint32_t e = src[j];
    const int64_t i = e >> 2;
    if (i >= n) continue;
    const float v = (zero_new && (e & 3u) != S_SURVIVOR) ? 0.f : f[blocked ? i * C + c : c * n + i];
    out[blocked ? j * C + c : c * cap + j] = v;
  }
}

inline unsigned grid_for(int64_t items, int64_t cap_blocks = 8192) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((items + kABlock - 1) / kABlock, cap_blocks));
}

}  // namespace cgv2

size_t cgv2_action_ws_layout(int64_t n, size_t* off) {
  const int64_t nb = std::max<int64_t>((n + cgv2::kAChunk - 1) / cgv2::kAChunk, 1);
  // off: [0] per-workgroup action counts (u32 x 4), [1] per-workgroup offsets (uint2)
  off[0] = 0;
  off[1] = ((size_t)16 * (size_t)nb + 255) & ~(size_t)255;
  return off[1] + (((size_t)8 * (size_t)nb + 255) & ~(size_t)255);
}

hipError_t cgv2_launch_densify_plan(const cgv2_surfels& s, const uint8_t* mask, const uint8_t* remove,
                                    const cgv2_action_params& prm, uint8_t* actions, uint32_t* dst, int64_t* counts,
                                    void* ws, hipStream_t st) {
  const int64_t n = s.n;
  const int nb = (int)std::max<int64_t>((n + cgv2::kAChunk - 1) / cgv2::kAChunk, 1);
  size_t off[kActionOffs];
  cgv2_action_ws_layout(n, off);
  uint32_t* part = (uint32_t*)((char*)ws + off[0]);
  uint2* offs = (uint2*)((char*)ws + off[1]);
  if (n > 0)
    hipLaunchKernelGGL(cgv2::k_act_count, dim3((unsigned)nb), dim3(cgv2::kABlock), 0, st, mask, remove, s.log_scale,
                       s.opacity_logit, n, (double)prm.dense_scale, (double)prm.min_opacity, actions, part);
  else
    hipLaunchKernelGGL((cgv2::k_fill<uint32_t>), dim3(1), dim3(64), 0, st, part, (int64_t)4, 0u);
  hipLaunchKernelGGL(cgv2::k_act_scan, dim3(1), dim3(cgv2::kABlock), 0, st, part, nb, offs, counts);
  if (n > 0)
    hipLaunchKernelGGL(cgv2::k_act_dst, dim3((unsigned)nb), dim3(cgv2::kABlock), 0, st, actions, n, offs, counts,
                       dst);
  return hipGetLastError();
}

hipError_t cgv2_launch_densify_apply(const cgv2_surfels& s, const uint8_t* actions, const uint32_t* dst,
                                     const int64_t* counts, const float* z, const cgv2_action_params& prm,
                                     const cgv2_surfels_out& out, uint32_t* src, hipStream_t st) {
  const int64_t n = s.n, cap = out.n;
  if (n == 0 || cap == 0) return hipGetLastError();
  hipLaunchKernelGGL(cgv2::k_src_fill, dim3(cgv2::grid_for(n)), dim3(cgv2::kABlock), 0, st, actions, dst, n, counts,
                     cap, src);
  const unsigned g = cgv2::grid_for(cap, 16384);
  const double ls = log((double)prm.split_shrink);
  switch (s.sh_degree) {
    case 0: hipLaunchKernelGGL((cgv2::k_apply<3>), dim3(g), dim3(cgv2::kABlock), 0, st, s, src, counts, z, ls, out); break;
    case 1: hipLaunchKernelGGL((cgv2::k_apply<12>), dim3(g), dim3(cgv2::kABlock), 0, st, s, src, counts, z, ls, out); break;
    case 2: hipLaunchKernelGGL((cgv2::k_apply<27>), dim3(g), dim3(cgv2::kABlock), 0, st, s, src, counts, z, ls, out); break;
    default: hipLaunchKernelGGL((cgv2::k_apply<48>), dim3(g), dim3(cgv2::kABlock), 0, st, s, src, counts, z, ls, out); break;
  }
  return hipGetLastError();
}

hipError_t cgv2_launch_densify_gather(const float* f, int64_t n, int C, int blocked, const uint32_t* src,
                                      const int64_t* counts, int zero_new, float* out, int64_t cap, hipStream_t st) {
  if (n == 0 || cap == 0) return hipGetLastError();
  hipLaunchKernelGGL(cgv2::k_gather, dim3(cgv2::grid_for(cap * C, 16384)), dim3(cgv2::kABlock), 0, st, f, n, C,
                     blocked, src, counts, cap, zero_new, out);
  return hipGetLastError();
}
