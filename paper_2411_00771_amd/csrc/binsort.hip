// Tile binning and per-tile depth sort.
//
// Instead of a global LSD radix sort over (view | tile | depth) keys, intersections are bucketed
// by tile directly:
//   k_count      one thread per (surfel, view): atomic +1 on every covered tile's counter
//   k_scan_*     exclusive prefix sum of the V * tiles counters -> ranges (two small launches)
//   k_scatter    one thread per (surfel, view): atomic cursor per tile, writes (depth bits << 32 | id)
//   k_sort_small one workgroup per tile: LDS bitonic sort of lists up to kSmall entries
//   k_sort_big   lists up to kBig entries in 128 KB of LDS; longer lists are sorted in kBig chunks
//                and merged in global memory by rank (binary search)
// (depth bits, id) is unique within a tile, so the atomic scatter order does not matter and the
// result is deterministic and bit-exact.  HBM traffic is about 8 B written + 8 B read + 4 B
// written per intersection.
#include "cgv2r_device.h"
#include "cgv2r_kernels.h"

namespace cgv2 {

constexpr int kSmall = 2048;   // entries sorted by k_sort_small (16 KB of LDS)
constexpr int kBig = 16384;    // entries sorted in LDS by k_sort_big (128 KB)
constexpr int kScanBlock = 1024;
constexpr int kScanItems = 4;  // counters per thread per scan block

__device__ __forceinline__ void tile_rect(const uint16_t* r4, uint32_t& tx0, uint32_t& ty0, uint32_t& tx1,
                                          uint32_t& ty1) {
  const uint2 r = *(const uint2*)r4;
  tx0 = r.x & 0xffffu; ty0 = r.x >> 16; tx1 = r.y & 0xffffu; ty1 = r.y >> 16;
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* p, int64_t count, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

__global__ __launch_bounds__(256) void k_count(const uint16_t* __restrict__ rect, int64_t n, int tiles_x,
                                               int tiles_per_view, uint32_t* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y;
  if (i >= n) return;
  uint32_t tx0, ty0, tx1, ty1;
  tile_rect(rect + 4 * ((int64_t)v * n + i), tx0, ty0, tx1, ty1);
  uint32_t* c = cnt + (int64_t)v * tiles_per_view;
  for (uint32_t ty = ty0; ty < ty1; ++ty)
    for (uint32_t tx = tx0; tx < tx1; ++tx) atomicAdd(c + ty * tiles_x + tx, 1u);
}

// block-wide exclusive scan of kScanBlock * kScanItems counters; returns the block total
__device__ __forceinline__ uint64_t block_scan(uint64_t (&vals)[kScanItems], uint64_t* lds) {
  uint64_t s = 0;
  for (int k = 0; k < kScanItems; ++k) { const uint64_t t = vals[k]; vals[k] = s; s += t; }
  // Hillis-Steele over thread sums
  const int t = threadIdx.x;
  lds[t] = s;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    const uint64_t add = t >= off ? lds[t - off] : 0;
    __syncthreads();
    lds[t] += add;
    __syncthreads();
  }
  const uint64_t incl = lds[t];
  const uint64_t total = lds[kScanBlock - 1];
  const uint64_t excl = incl - s;
  for (int k = 0; k < kScanItems; ++k) vals[k] += excl;
  __syncthreads();
  return total;
}

// pass 1: per-block sums
__global__ __launch_bounds__(kScanBlock) void k_scan_sums(const uint32_t* __restrict__ cnt, int64_t m,
                                                          uint64_t* __restrict__ sums) {
  __shared__ uint64_t lds[kScanBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock * kScanItems;
  uint64_t s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t idx = base + (int64_t)k * kScanBlock + threadIdx.x;
    if (idx < m) s += cnt[idx];
  }
  lds[threadIdx.x] = s;
  __syncthreads();
  for (int off = kScanBlock / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) lds[threadIdx.x] += lds[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = lds[0];
}

// pass 2: each block adds the sums of the blocks before it, scans its counters, writes ranges and
// cursors; the last block writes the total, the overflow status and clears the big-list counter.
__global__ __launch_bounds__(kScanBlock) void k_scan_apply(const uint32_t* __restrict__ cnt, int64_t m,
                                                           const uint64_t* __restrict__ sums, int nblocks,
                                                           uint32_t* __restrict__ ranges,
                                                           uint32_t* __restrict__ cursor, int64_t capacity,
                                                           int32_t* __restrict__ status, int64_t* __restrict__ needed,
                                                           uint32_t* __restrict__ big_count) {
  __shared__ uint64_t lds[kScanBlock];
  uint64_t carry = 0;
  for (int b = 0; b < (int)blockIdx.x; ++b) carry += sums[b];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock * kScanItems + (int64_t)threadIdx.x * kScanItems;
  uint64_t vals[kScanItems];
  for (int k = 0; k < kScanItems; ++k) vals[k] = base + k < m ? cnt[base + k] : 0;
  const uint64_t total = block_scan(vals, lds);
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < m) {
      const uint32_t v = (uint32_t)(vals[k] + carry);
      ranges[base + k] = v;
      cursor[base + k] = v;
    }
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
    const uint64_t K = carry + total;
    ranges[m] = (uint32_t)(K > 0xffffffffull ? 0xffffffffull : K);
    *needed = (int64_t)K;
    if ((int64_t)K > capacity) *status = 1;
    *big_count = 0;
  }
  (void)nblocks;
}

__global__ __launch_bounds__(256) void k_scatter(const uint16_t* __restrict__ rect, const float* __restrict__ rec,
                                                 int64_t n, int tiles_x, int tiles_per_view,
                                                 uint32_t* __restrict__ cursor, uint64_t* __restrict__ keys,
                                                 const int32_t* __restrict__ status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y;
  if (i >= n || *status != 0) return;
  const int64_t vi = (int64_t)v * n + i;
  uint32_t tx0, ty0, tx1, ty1;
  tile_rect(rect + 4 * vi, tx0, ty0, tx1, ty1);
  if (tx1 <= tx0) return;
  const uint64_t key = ((uint64_t)__float_as_uint(rec[vi * kRec + R_ZC]) << 32) | (uint32_t)i;
  uint32_t* cur = cursor + (int64_t)v * tiles_per_view;
  for (uint32_t ty = ty0; ty < ty1; ++ty)
    for (uint32_t tx = tx0; tx < tx1; ++tx) {
      const uint32_t pos = atomicAdd(cur + ty * tiles_x + tx, 1u);
      keys[pos] = key;
    }
}

// In-LDS bitonic sort of 'len' keys padded to the next power of two 'p' with UINT64_MAX.
template <int NT>
__device__ __forceinline__ void lds_bitonic(uint64_t* s, int p) {
  for (int k = 2; k <= p; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < (p >> 1); t += NT) {
        // index of the lower element of pair t at distance j
        const int i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
        const int l = i | j;
        const bool up = (i & k) == 0;
        const uint64_t a = s[i], b = s[l];
        if ((a > b) == up) { s[i] = b; s[l] = a; }
      }
      __syncthreads();
    }
  }
}

__device__ __forceinline__ int next_pow2(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

__global__ __launch_bounds__(256) void k_sort_small(const uint32_t* __restrict__ ranges, int num_tiles,
                                                    const uint64_t* __restrict__ keys, uint32_t* __restrict__ ids,
                                                    uint32_t* __restrict__ big_list, uint32_t* __restrict__ big_count,
                                                    const int32_t* __restrict__ status) {
  __shared__ uint64_t s[kSmall];
  const int t = blockIdx.x;
  if (t >= num_tiles || *status != 0) return;
  const uint32_t a = ranges[t], b = ranges[t + 1];
  const int len = (int)(b - a);
  if (len == 0) return;
  if (len > kSmall) {
    if (threadIdx.x == 0) big_list[atomicAdd(big_count, 1u)] = (uint32_t)t;
    return;
  }
  if (len == 1) {
    if (threadIdx.x == 0) ids[a] = (uint32_t)keys[a];
    return;
  }
  const int p = next_pow2(len);
  for (int k = threadIdx.x; k < p; k += 256) s[k] = k < len ? keys[a + k] : ~0ull;
  __syncthreads();
  lds_bitonic<256>(s, p);
  for (int k = threadIdx.x; k < len; k += 256) ids[a + k] = (uint32_t)s[k];
}

// rank of key x in sorted run r[0..len): number of elements < x
__device__ __forceinline__ uint32_t lower_rank(const uint64_t* r, uint32_t len, uint64_t x) {
  uint32_t lo = 0, hi = len;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (r[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(1024) void k_sort_big(const uint32_t* __restrict__ ranges,
                                                   uint64_t* __restrict__ keys, uint64_t* __restrict__ scratch,
                                                   uint32_t* __restrict__ ids, const uint32_t* __restrict__ big_list,
                                                   const uint32_t* __restrict__ big_count,
                                                   const int32_t* __restrict__ status) {
  __shared__ uint64_t s[kBig];
  if (*status != 0) return;
  const uint32_t nbig = *big_count;
  for (uint32_t q = blockIdx.x; q < nbig; q += gridDim.x) {
    const uint32_t t = big_list[q];
    const uint32_t a = ranges[t], b = ranges[t + 1];
    const uint32_t len = b - a;
    // 1) sort chunks of kBig in LDS
    for (uint32_t c0 = 0; c0 < len; c0 += kBig) {
      const int cl = (int)min((uint32_t)kBig, len - c0);
      const int p = next_pow2(cl);
      for (int k = threadIdx.x; k < p; k += 1024) s[k] = k < cl ? keys[a + c0 + k] : ~0ull;
      __syncthreads();
      lds_bitonic<1024>(s, p);
      if (len <= (uint32_t)kBig) {
        for (int k = threadIdx.x; k < cl; k += 1024) ids[a + k] = (uint32_t)s[k];
      } else {
        for (int k = threadIdx.x; k < cl; k += 1024) keys[a + c0 + k] = s[k];
      }
      __syncthreads();
    }
    if (len <= (uint32_t)kBig) continue;
    // 2) merge sorted runs of width w pairwise, ping-ponging between keys and scratch
    uint64_t* src = keys + a;
    uint64_t* dst = scratch + a;
    for (uint32_t w = kBig; w < len; w <<= 1) {
      for (uint32_t k = threadIdx.x; k < len; k += 1024) {
        const uint32_t run = k / w;
        const uint32_t r0 = (run & ~1u) * w;  // start of the left run of this pair
        const uint32_t llen = min(w, len - r0);
        const uint32_t rlen = r0 + w < len ? min(w, len - r0 - w) : 0;
        const uint64_t x = src[k];
        uint32_t pos;
        if ((run & 1u) == 0) pos = (k - r0) + lower_rank(src + r0 + w, rlen, x);
        else pos = (k - r0 - w) + lower_rank(src + r0, llen, x);
        dst[r0 + pos] = x;
      }
      __syncthreads();
      __threadfence_block();
      uint64_t* tmp = src; src = dst; dst = tmp;
    }
    for (uint32_t k = threadIdx.x; k < len; k += 1024) ids[a + k] = (uint32_t)src[k];
    __syncthreads();
  }
}

}  // namespace cgv2

size_t cgv2_binsort_ws_layout(int64_t capacity, int V, int tiles, size_t* off) {
  // off: [0] cnt (u32, m), [1] cursor (u32, m), [2] sums (u64), [3] big_list (u32, m), [4] big_count,
  //      [5] keys (u64, capacity), [6] scratch (u64, capacity)
  const int64_t m = (int64_t)V * tiles;
  const int64_t nsb = (m + cgv2::kScanBlock * cgv2::kScanItems - 1) / (cgv2::kScanBlock * cgv2::kScanItems);
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o += (bytes + 255) & ~(size_t)255; return r; };
  off[0] = take(4 * (size_t)m);
  off[1] = take(4 * (size_t)m);
  off[2] = take(8 * (size_t)(nsb + 1));
  off[3] = take(4 * (size_t)m);
  off[4] = take(4);
  off[5] = take(8 * (size_t)capacity);
  off[6] = take(8 * (size_t)capacity);
  return o;
}

hipError_t cgv2_launch_bin_sort(const cgv2_proj& p, int64_t n, int V, int tiles_x, int tiles_y, const cgv2_bins& b,
                                void* ws, hipStream_t st) {
  using namespace cgv2;
  const int tiles = tiles_x * tiles_y;
  const int64_t m = (int64_t)V * tiles;
  size_t off[7];
  cgv2_binsort_ws_layout(b.capacity, V, tiles, off);
  char* w = (char*)ws;
  uint32_t* cnt = (uint32_t*)(w + off[0]);
  uint32_t* cursor = (uint32_t*)(w + off[1]);
  uint64_t* sums = (uint64_t*)(w + off[2]);
  uint32_t* big_list = (uint32_t*)(w + off[3]);
  uint32_t* big_count = (uint32_t*)(w + off[4]);
  uint64_t* keys = (uint64_t*)(w + off[5]);
  uint64_t* scratch = (uint64_t*)(w + off[6]);
  const int nsb = (int)((m + kScanBlock * kScanItems - 1) / (kScanBlock * kScanItems));
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, cnt, m, 0u);
  if (n > 0) {
    hipLaunchKernelGGL(k_count, dim3((unsigned)((n + 255) / 256), (unsigned)V), dim3(256), 0, st, p.rect, n, tiles_x,
                       tiles, cnt);
  }
  hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nsb), dim3(kScanBlock), 0, st, cnt, m, sums);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nsb), dim3(kScanBlock), 0, st, cnt, m, sums, nsb, b.ranges, cursor,
                     b.capacity, b.status, b.needed, big_count);
  if (n > 0) {
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)((n + 255) / 256), (unsigned)V), dim3(256), 0, st, p.rect, p.rec, n,
                       tiles_x, tiles, cursor, keys, b.status);
  }
  hipLaunchKernelGGL(k_sort_small, dim3((unsigned)m), dim3(256), 0, st, b.ranges, (int)m, keys, b.ids, big_list,
                     big_count, b.status);
  hipLaunchKernelGGL(k_sort_big, dim3(256), dim3(1024), 0, st, b.ranges, keys, scratch, b.ids, big_list, big_count,
                     b.status);
  return hipGetLastError();
}
