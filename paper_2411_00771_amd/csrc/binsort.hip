// Tile binning and per-tile depth sort.
//
// Instead of a global LSD radix sort over (view | tile | depth) keys, intersections are bucketed
// by tile directly:
//   surfel scan   exclusive prefix sum of every (surfel, view)'s tile count (from its rect)
//   k_stage       one thread per (surfel, view): writes (tile, depth bits << 32 | id) of each
//                 covered tile into its own slice and counts the tile (fire-and-forget atomics)
//   tile scan     exclusive prefix sum of the V * tiles counters -> ranges and cursors
//   k_place       one thread per intersection: a returning atomic on the tile cursor places the key
//   k_sort_small  one workgroup per tile: LDS bitonic sort of lists up to kSmall entries
//   k_sort_big    lists up to kBig entries in 128 KB of LDS; longer lists are sorted in kBig chunks
//                 and merged in global memory by rank (binary search)
// (depth bits, id) is unique within a tile, so the atomic placement order does not matter and the
// result is deterministic and bit-exact.  HBM traffic is about 12 B staged + 12 B read + 8 B placed
// + 8 B read + 4 B written per intersection.
#include "cgv2r_device.h"
#include "cgv2r_kernels.h"

#include <algorithm>

namespace cgv2 {

constexpr int kSmall = 2048;   // entries sorted by k_sort_small (16 KB of LDS)
constexpr int kBig = 16384;    // entries sorted in LDS by k_sort_big (128 KB)
constexpr int kScanBlock = 1024;
constexpr int kScanItems = 8;  // elements per thread per scan block
constexpr int kScanChunk = kScanBlock * kScanItems;

__device__ __forceinline__ void tile_rect(const uint16_t* r4, uint32_t& tx0, uint32_t& ty0, uint32_t& tx1,
                                          uint32_t& ty1) {
  const uint2 r = *(const uint2*)r4;
  tx0 = r.x & 0xffffu; ty0 = r.x >> 16; tx1 = r.y & 0xffffu; ty1 = r.y >> 16;
}

__device__ __forceinline__ uint32_t rect_count(const uint16_t* r4) {
  uint32_t tx0, ty0, tx1, ty1;
  tile_rect(r4, tx0, ty0, tx1, ty1);
  return (tx1 - tx0) * (ty1 - ty0);
}

// scan inputs: a u32 array, the tile counts of the rects, or the rects' non-empty bits
struct ScanIn {
  const uint32_t* u32;
  const uint16_t* rect;
  int nonzero;
  __device__ __forceinline__ uint32_t operator()(int64_t i) const {
    if (u32) return u32[i];
    const uint32_t c = rect_count(rect + 4 * i);
    return nonzero ? (c != 0u) : c;
  }
};


// block-wide exclusive scan of kScanChunk values held kScanItems per thread; returns the total
__device__ __forceinline__ uint64_t block_scan(uint64_t (&vals)[kScanItems], uint64_t* lds) {
  uint64_t s = 0;
  for (int k = 0; k < kScanItems; ++k) { const uint64_t t = vals[k]; vals[k] = s; s += t; }
  const int t = threadIdx.x;
  lds[t] = s;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    const uint64_t add = t >= off ? lds[t - off] : 0;
    __syncthreads();
    lds[t] += add;
    __syncthreads();
  }
  const uint64_t total = lds[kScanBlock - 1];
  const uint64_t excl = lds[t] - s;
  for (int k = 0; k < kScanItems; ++k) vals[k] += excl;
  __syncthreads();
  return total;
}

// pass 1: per-chunk sums
__global__ __launch_bounds__(kScanBlock) void k_scan_sums(ScanIn in, int64_t m, uint64_t* __restrict__ sums) {
  __shared__ uint64_t lds[kScanBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  uint64_t s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t idx = base + (int64_t)k * kScanBlock + threadIdx.x;
    if (idx < m) s += in(idx);
  }
  lds[threadIdx.x] = s;
  __syncthreads();
  for (int off = kScanBlock / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) lds[threadIdx.x] += lds[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = lds[0];
}

// pass 2: one workgroup scans the chunk sums in place (any count, kScanChunk at a time)
__global__ __launch_bounds__(kScanBlock) void k_scan_top(uint64_t* __restrict__ sums, int64_t nb,
                                                         uint64_t* __restrict__ total) {
  __shared__ uint64_t lds[kScanBlock];
  uint64_t carry = 0;
  for (int64_t base = 0; base < nb; base += kScanChunk) {
    const int64_t b0 = base + (int64_t)threadIdx.x * kScanItems;
    uint64_t vals[kScanItems];
    for (int k = 0; k < kScanItems; ++k) vals[k] = b0 + k < nb ? sums[b0 + k] : 0;
    const uint64_t tot = block_scan(vals, lds);
    for (int k = 0; k < kScanItems; ++k)
      if (b0 + k < nb) sums[b0 + k] = vals[k] + carry;
    carry += tot;
  }
  if (threadIdx.x == 0) *total = carry;
}

// pass 3: scan each chunk with its offset; out[m] = total (clamped to u32).  When 'cursor' is set
// it receives a copy.  When 'capacity' >= 0 the total is checked against it.
__global__ __launch_bounds__(kScanBlock) void k_scan_apply(ScanIn in, int64_t m, const uint64_t* __restrict__ sums,
                                                           const uint64_t* __restrict__ total,
                                                           uint32_t* __restrict__ out, uint32_t* __restrict__ cursor,
                                                           int64_t capacity, int32_t* __restrict__ status,
                                                           int64_t* __restrict__ needed) {
  __shared__ uint64_t lds[kScanBlock];
  const uint64_t carry = sums[blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
  uint64_t vals[kScanItems];
  for (int k = 0; k < kScanItems; ++k) vals[k] = base + k < m ? in(base + k) : 0;
  block_scan(vals, lds);
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < m) {
      const uint64_t v = vals[k] + carry;
      const uint32_t v32 = (uint32_t)(v > 0xffffffffull ? 0xffffffffull : v);
      out[base + k] = v32;
      if (cursor) cursor[base + k] = v32;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const uint64_t K = *total;
    out[m] = (uint32_t)(K > 0xffffffffull ? 0xffffffffull : K);
    if (capacity >= 0) {
      *needed = (int64_t)K;
      if ((int64_t)K > capacity) *status = 1;
    }
  }
}

// compaction: visible[pos] = surfel id of every (view, surfel) with a non-empty rect, in (view, id)
// order; vstart[v] = first entry of view v, vstart[V] = total
__global__ __launch_bounds__(kScanBlock) void k_visible_apply(ScanIn in, int64_t m, int64_t n,
                                                              const uint64_t* __restrict__ sums,
                                                              const uint64_t* __restrict__ total,
                                                              uint32_t* __restrict__ visible,
                                                              uint32_t* __restrict__ vstart, int V) {
  __shared__ uint64_t lds[kScanBlock];
  const uint64_t carry = sums[blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
  uint64_t vals[kScanItems];
  uint32_t flag[kScanItems];
  for (int k = 0; k < kScanItems; ++k) {
    flag[k] = base + k < m ? in(base + k) : 0u;
    vals[k] = flag[k];
  }
  block_scan(vals, lds);
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t e = base + k;
    if (e >= m) continue;
    const uint32_t pos = (uint32_t)(vals[k] + carry);
    const int64_t i = e % n;
    if (flag[k]) visible[pos] = (uint32_t)i;
    if (i == 0) vstart[e / n] = pos;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) vstart[V] = (uint32_t)*total;
}

// Groups of 8 lanes take one visible surfel of view blockIdx.y each and spread its tiles over the
// group, so a surfel that covers hundreds of tiles does not hold up a wave.
constexpr int kGroup = 8;
__global__ __launch_bounds__(256) void k_stage(const uint16_t* __restrict__ rect, const float* __restrict__ rec,
                                               int64_t n, int tiles_x, int tiles_per_view,
                                               const uint32_t* __restrict__ visible,
                                               const uint32_t* __restrict__ vstart,
                                               const uint32_t* __restrict__ soff, uint32_t* __restrict__ cnt,
                                               uint32_t* __restrict__ st_tile, uint64_t* __restrict__ st_key,
                                               const int32_t* __restrict__ status) {
  const int v = blockIdx.y;
  if (*status != 0) return;
  const uint32_t nv = vstart[v + 1] - vstart[v];
  const uint32_t* list = visible + vstart[v];
  const uint32_t g = threadIdx.x % kGroup;
  const uint32_t tbase = (uint32_t)v * (uint32_t)tiles_per_view;
  for (uint32_t e = (blockIdx.x * blockDim.x + threadIdx.x) / kGroup; e < nv;
       e += gridDim.x * blockDim.x / kGroup) {
    const uint32_t i = list[e];
    const int64_t vi = (int64_t)v * n + i;
    uint32_t tx0, ty0, tx1, ty1;
    tile_rect(rect + 4 * vi, tx0, ty0, tx1, ty1);
    const uint32_t w = tx1 - tx0, total = w * (ty1 - ty0);
    const uint64_t key = ((uint64_t)__float_as_uint(rec[vi * kRec + R_ZC]) << 32) | i;
    const uint32_t o = soff[vi];
    for (uint32_t k = g; k < total; k += kGroup) {
      const uint32_t t = tbase + (ty0 + k / w) * tiles_x + tx0 + k % w;
      st_tile[o + k] = t;
      st_key[o + k] = key;
      atomicAdd(cnt + t, 1u);
    }
  }
}

__global__ __launch_bounds__(256) void k_place(const uint32_t* __restrict__ soff_total,
                                               const uint32_t* __restrict__ st_tile,
                                               const uint64_t* __restrict__ st_key, uint32_t* __restrict__ cursor,
                                               uint64_t* __restrict__ keys, const int32_t* __restrict__ status) {
  if (*status != 0) return;
  const uint32_t K = *soff_total;
  for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < K; e += gridDim.x * blockDim.x) {
    const uint32_t pos = atomicAdd(cursor + st_tile[e], 1u);
    keys[pos] = st_key[e];
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

static int64_t scan_blocks(int64_t m) { return (m + cgv2::kScanChunk - 1) / cgv2::kScanChunk; }

size_t cgv2_binsort_ws_layout(int64_t capacity, int V, int tiles, int64_t n, size_t* off) {
  // off: [0] cnt (u32, m), [1] cursor (u32, m), [2] scan sums (u64), [3] big_list (u32, m),
  //      [4] big_count + scan totals, [5] keys (u64, capacity), [6] staged keys / merge scratch
  //      (u64, capacity), [7] staged tiles (u32, capacity), [8] surfel offsets (u32, V n + 1)
  const int64_t m = (int64_t)V * tiles;
  const int64_t vn = (int64_t)V * n;
  const int64_t nsb = scan_blocks(m > vn ? m : vn);
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o += (bytes + 255) & ~(size_t)255; return r; };
  off[0] = take(4 * (size_t)m);
  off[1] = take(4 * (size_t)m);
  off[2] = take(8 * (size_t)(nsb + 1));
  off[3] = take(4 * (size_t)m);
  off[4] = take(64);
  off[5] = take(8 * (size_t)capacity);
  off[6] = take(8 * (size_t)capacity);
  off[7] = take(4 * (size_t)capacity);
  off[8] = take(4 * (size_t)(vn + 1));
  return o;
}

hipError_t cgv2_launch_bin_sort(const cgv2_proj& p, int64_t n, int V, int tiles_x, int tiles_y, const cgv2_bins& b,
                                void* ws, hipStream_t st) {
  using namespace cgv2;
  const int tiles = tiles_x * tiles_y;
  const int64_t m = (int64_t)V * tiles;
  const int64_t vn = (int64_t)V * n;
  size_t off[9];
  cgv2_binsort_ws_layout(b.capacity, V, tiles, n, off);
  char* w = (char*)ws;
  uint32_t* cnt = (uint32_t*)(w + off[0]);
  uint32_t* cursor = (uint32_t*)(w + off[1]);
  uint64_t* sums = (uint64_t*)(w + off[2]);
  uint32_t* big_list = (uint32_t*)(w + off[3]);
  uint32_t* big_count = (uint32_t*)(w + off[4]);
  uint64_t* totals = (uint64_t*)(w + off[4] + 8);  // [0] surfel scan, [1] tile scan, [2] visible scan
  uint64_t* keys = (uint64_t*)(w + off[5]);
  uint64_t* stk = (uint64_t*)(w + off[6]);
  uint32_t* stt = (uint32_t*)(w + off[7]);
  uint32_t* soff = (uint32_t*)(w + off[8]);
  hipLaunchKernelGGL(k_fill<uint32_t>, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, cnt, m, 0u);
  hipLaunchKernelGGL(k_fill<uint32_t>, dim3(1), dim3(256), 0, st, big_count, (int64_t)1, 0u);
  // surfel offsets, total and overflow check
  ScanIn sin{nullptr, p.rect, 0};
  const int64_t nbs = scan_blocks(vn > 0 ? vn : 1);
  hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nbs), dim3(kScanBlock), 0, st, sin, vn, sums);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanBlock), 0, st, sums, nbs, totals);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nbs), dim3(kScanBlock), 0, st, sin, vn, sums, totals, soff,
                     (uint32_t*)nullptr, b.capacity, b.status, b.needed);
  // visible lists (consumed by the staging here and by the reverse pass)
  if (n > 0) {
    ScanIn vin{nullptr, p.rect, 1};
    hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nbs), dim3(kScanBlock), 0, st, vin, vn, sums);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanBlock), 0, st, sums, nbs, totals + 2);
    hipLaunchKernelGGL(k_visible_apply, dim3((unsigned)nbs), dim3(kScanBlock), 0, st, vin, vn, n, sums, totals + 2,
                       p.visible, p.visible_start, V);
    const unsigned blocks = (unsigned)std::min<int64_t>((n * kGroup + 255) / 256, 2048);
    hipLaunchKernelGGL(k_stage, dim3(blocks, (unsigned)V), dim3(256), 0, st, p.rect, p.rec, n, tiles_x, tiles,
                       p.visible, p.visible_start, soff, cnt, stt, stk, b.status);
  } else {
    hipLaunchKernelGGL(k_fill<uint32_t>, dim3(1), dim3(256), 0, st, p.visible_start, (int64_t)V + 1, 0u);
  }
  // tile ranges and cursors
  ScanIn tin{cnt, nullptr, 0};
  const int64_t nbt = scan_blocks(m);
  hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nbt), dim3(kScanBlock), 0, st, tin, m, sums);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanBlock), 0, st, sums, nbt, totals + 1);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nbt), dim3(kScanBlock), 0, st, tin, m, sums, totals + 1, b.ranges,
                     cursor, (int64_t)-1, b.status, b.needed);
  hipLaunchKernelGGL(k_place, dim3(2048), dim3(256), 0, st, soff + vn, stt, stk, cursor, keys, b.status);
  hipLaunchKernelGGL(k_sort_small, dim3((unsigned)m), dim3(256), 0, st, b.ranges, (int)m, keys, b.ids, big_list,
                     big_count, b.status);
  hipLaunchKernelGGL(k_sort_big, dim3(256), dim3(1024), 0, st, b.ranges, keys, stk, b.ids, big_list, big_count,
                     b.status);
  return hipGetLastError();
}
