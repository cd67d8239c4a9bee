// Tile binning and per-tile depth sort.
//
// Instead of a global LSD radix sort over (view | tile | depth) keys, intersections are bucketed
// by tile directly:
//   surfel scan   one fused pass of three kernels (two up to kSurfLocal chunks) over every (view,
//                 surfel): the exclusive prefix sum of its tile count (from its rect) and the compaction
//                 of the visible ones into per-view lists, plus the capacity check
//   k_stage       groups of lanes per visible surfel: for each tile of its rect that the surfel's
//                 alpha >= 1/255 region reaches (reach_cell over the tile's pixel samples), a returning
//                 atomic on the tile's counter gives the entry's rank within the tile; (tile, rank,
//                 depth bits << 32 | id) goes to the surfel's own slice, a sentinel tile to the slots of
//                 the rect tiles it cannot reach
//   k_tile_scan   one workgroup: exclusive prefix sum of the V * tiles counters -> ranges; up to
//                 kScanChunk tiles of at most kMaxViews views, k_tile_scan_order also computes the
//                 launch order in the same workgroup (the multi-workgroup order kernels otherwise)
//   k_place       one thread per staged slot: keys[ranges[tile] + rank] = key (no atomics)
//   k_sort_wave   one wave per tile: bitonic sort of lists up to kWaveSort entries in registers
//   k_sort_big    longer lists, up to kBig entries in 128 KB of LDS; longer still are sorted in kBig
//                 chunks and merged in global memory by rank (binary search)
// (depth bits, id) is unique within a tile, so the order in which the atomics hand out ranks does not
// matter: the result is deterministic and bit-exact.  HBM traffic is about 16 B staged + 16 B read +
// 8 B placed + 8 B read + 4 B written per intersection.
#include "cgv2r_device.h"
#include "cgv2r_kernels.h"

#include <algorithm>

namespace cgv2 {

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

__device__ __forceinline__ uint64_t shfl_up64(uint64_t x, unsigned d) {
  const uint32_t lo = __shfl_up((uint32_t)x, d, 64), hi = __shfl_up((uint32_t)(x >> 32), d, 64);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_xor64(uint64_t x, int m) {
  const uint32_t lo = __shfl_xor((uint32_t)x, m, 64), hi = __shfl_xor((uint32_t)(x >> 32), m, 64);
  return ((uint64_t)hi << 32) | lo;
}

// inclusive prefix sum over the 64 lanes of a wave
__device__ __forceinline__ uint64_t wave_scan(uint64_t x) {
  const unsigned lane = threadIdx.x & 63u;
#pragma unroll
  for (unsigned d = 1; d < 64; d <<= 1) {
    const uint64_t y = shfl_up64(x, d);
    if (lane >= d) x += y;
  }
  return x;
}

// inclusive prefix sum over the 64 lanes of a wave (32-bit) with DPP row shifts and row broadcasts
// only: each row of 16 lanes scans itself, then rows 1 and 3 add the total of the row before, then
// rows 2 and 3 that of rows 0-1 (lanes a shift or broadcast does not reach receive 0)
template <int kCtrl, int kRowMask = 0xf>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kCtrl, kRowMask, 0xf, false);
}

__device__ __forceinline__ uint32_t wave_scan_u32(uint32_t x) {
  x += dpp_u32<0x111>(x);       // row_shr:1
  x += dpp_u32<0x112>(x);       // row_shr:2
  x += dpp_u32<0x114>(x);       // row_shr:4
  x += dpp_u32<0x118>(x);       // row_shr:8
  x += dpp_u32<0x142, 0xa>(x);  // row_bcast:15
  x += dpp_u32<0x143, 0xc>(x);  // row_bcast:31
  return x;
}

// the value of lane 63 (a wave total after wave_scan_u32)
__device__ __forceinline__ uint32_t lane63(uint32_t x) { return (uint32_t)__builtin_amdgcn_readlane((int)x, 63); }

constexpr int kScanWaves = kScanBlock / 64;

// block-wide exclusive scan of kScanChunk values held kScanItems per thread (consecutive items per
// thread); returns the total.  Lane scans in registers, one LDS round for the 16 wave totals; lds
// holds at least 2 * kScanWaves entries.
__device__ __forceinline__ uint64_t block_scan(uint64_t (&vals)[kScanItems], uint64_t* lds) {
  uint64_t s = 0;
  for (int k = 0; k < kScanItems; ++k) { const uint64_t t = vals[k]; vals[k] = s; s += t; }
  const unsigned lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  const uint64_t inc = wave_scan(s);
  if (lane == 63u) lds[w] = inc;
  __syncthreads();
  if (w == 0) {
    const uint64_t x = wave_scan(lane < (unsigned)kScanWaves ? lds[lane] : 0);
    if (lane < (unsigned)kScanWaves) lds[kScanWaves + lane] = x;
  }
  __syncthreads();
  const uint64_t excl = (w > 0 ? lds[kScanWaves + w - 1] : 0) + inc - s;
  const uint64_t total = lds[2 * kScanWaves - 1];
  for (int k = 0; k < kScanItems; ++k) vals[k] += excl;
  __syncthreads();
  return total;
}

// block-wide sum, valid in thread 0; lds holds at least kScanWaves entries (a second call right after
// needs another lds array: thread 0 may still be reading this one)
__device__ __forceinline__ uint64_t block_sum(uint64_t x, uint64_t* lds) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) x += shfl_xor64(x, m);
  if ((threadIdx.x & 63u) == 0) lds[threadIdx.x >> 6] = x;
  __syncthreads();
  uint64_t t = 0;
  if (threadIdx.x == 0)
    for (int q = 0; q < kScanWaves; ++q) t += lds[q];
  return t;
}

// pass 2 of the surfel scan: workgroup 0 scans the chunk sums of the counts in place, workgroup 1
// those of the visible flags (any count, kScanChunk at a time); totals[blockIdx.x] = grand total
__global__ __launch_bounds__(kScanBlock) void k_scan_top(uint64_t* __restrict__ sums0, uint64_t* __restrict__ sums1,
                                                         int64_t nb, uint64_t* __restrict__ totals) {
  __shared__ uint64_t lds[2 * kScanWaves];
  uint64_t* sums = blockIdx.x == 0 ? sums0 : sums1;
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
  if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

// The surfel scan runs over chunks of kSurfChunk (view, surfel) entries, one 256-thread workgroup each;
// a wave owns kSurfRows consecutive rows of 64 entries (coalesced loads), scans them with shuffles and
// ballots, and only the wave totals go through LDS.
constexpr int kSurfBlock = 256;
constexpr int kSurfWaves = kSurfBlock / 64;
constexpr int kSurfRows = 8;
constexpr int kSurfChunk = kSurfBlock * kSurfRows;
constexpr int kSurfLocal = 4 * kSurfBlock;  // up to this many chunks, each apply workgroup adds up those before it

// pass 1 of the surfel scan: per-chunk sums of the tile counts and of the visible flags; the workgroups
// also zero the nz tile counters (and the counts after them), which the staging uses two launches later
__global__ __launch_bounds__(kSurfBlock) void k_surfel_sums(const uint16_t* __restrict__ rect, int64_t m,
                                                            uint64_t* __restrict__ sums_cnt,
                                                            uint64_t* __restrict__ sums_vis,
                                                            uint32_t* __restrict__ zero, int64_t nz) {
  __shared__ uint64_t red[2][kSurfWaves];
  for (int64_t z = (int64_t)blockIdx.x * kSurfBlock + threadIdx.x; z < nz; z += (int64_t)gridDim.x * kSurfBlock)
    zero[z] = 0u;
  const int64_t base = (int64_t)blockIdx.x * kSurfChunk;
  uint64_t c = 0, f = 0;
  for (int k = 0; k < kSurfRows; ++k) {
    const int64_t idx = base + (int64_t)k * kSurfBlock + threadIdx.x;
    if (idx < m) {
      const uint32_t t = rect_count(rect + 4 * idx);
      c += t;
      f += t != 0u;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    c += shfl_xor64(c, o);
    f += shfl_xor64(f, o);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][w] = c;
    red[1][w] = f;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t sc = 0, sf = 0;
    for (int q = 0; q < kSurfWaves; ++q) {
      sc += red[0][q];
      sf += red[1][q];
    }
    sums_cnt[blockIdx.x] = sc;
    sums_vis[blockIdx.x] = sf;
  }
}

// pass 3 of the surfel scan: soff[e] = first staged slot of (view, surfel) e, soff[m] = total;
// visible[pos] = surfel id of every (view, surfel) with a non-empty rect in (view, id) order,
// vstart[v] = first entry of view v, vstart[V] = total; the total is checked against the capacity.
// local_nsb > 0 (at most kSurfLocal chunks): the sums are pass 1's raw chunk sums and each workgroup
// adds up those before it (pass 2 is skipped); 0: the sums are pass 2's scanned ones, totals its totals.
__global__ __launch_bounds__(kSurfBlock) void k_surfel_apply(
    const uint16_t* __restrict__ rect, int64_t m, int64_t n, const uint64_t* __restrict__ sums_cnt,
    const uint64_t* __restrict__ sums_vis, const uint64_t* __restrict__ totals, int local_nsb,
    uint32_t* __restrict__ soff, uint32_t* __restrict__ visible, uint32_t* __restrict__ vstart, int V,
    int64_t capacity, int32_t* __restrict__ status, int64_t* __restrict__ needed) {
  __shared__ uint64_t red[4][kSurfWaves];
  __shared__ uint32_t wt[2][kSurfWaves];
  __shared__ uint64_t carry[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (local_nsb > 0) {
    uint64_t r[4] = {0, 0, 0, 0};  // counts and flags before this chunk, then their totals
    for (int j = threadIdx.x; j < local_nsb; j += kSurfBlock) {
      const uint64_t sc = sums_cnt[j], sv = sums_vis[j];
      if (j < (int)blockIdx.x) {
        r[0] += sc;
        r[1] += sv;
      }
      r[2] += sc;
      r[3] += sv;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) r[k] += shfl_xor64(r[k], o);
      if (lane == 0) red[k][w] = r[k];
    }
    __syncthreads();
    if (threadIdx.x < 4) {
      uint64_t t = 0;
      for (int q = 0; q < kSurfWaves; ++q) t += red[threadIdx.x][q];
      carry[threadIdx.x] = t;
    }
  } else if (threadIdx.x == 0) {
    carry[0] = sums_cnt[blockIdx.x];
    carry[1] = sums_vis[blockIdx.x];
    carry[2] = totals[0];
    carry[3] = totals[1];
  }
  // wave scans of the counts and of the visible flags over the wave's rows (32-bit: a chunk's counts
  // stay far below 2^32)
  const int64_t wbase = (int64_t)blockIdx.x * kSurfChunk + (int64_t)w * (64 * kSurfRows);
  const unsigned long long lt = (1ull << lane) - 1ull;
  uint32_t c[kSurfRows], ex[kSurfRows], fx[kSurfRows];
  uint32_t cc = 0, fc = 0;
#pragma unroll
  for (int r = 0; r < kSurfRows; ++r) {
    const int64_t idx = wbase + 64 * r + lane;
    c[r] = idx < m ? rect_count(rect + 4 * idx) : 0u;
  }
#pragma unroll
  for (int r = 0; r < kSurfRows; ++r) {
    const uint32_t inc = wave_scan_u32(c[r]);
    ex[r] = cc + inc - c[r];
    cc += lane63(inc);
    const unsigned long long fb = __ballot(c[r] != 0u);
    fx[r] = fc + (uint32_t)__popcll(fb & lt);
    fc += (uint32_t)__popcll(fb);
  }
  if (lane == 0) {
    wt[0][w] = cc;
    wt[1][w] = fc;
  }
  __syncthreads();
  uint64_t oc = carry[0], ov = carry[1];
  for (int q = 0; q < w; ++q) {
    oc += wt[0][q];
    ov += wt[1][q];
  }
#pragma unroll
  for (int r = 0; r < kSurfRows; ++r) {
    const int64_t e = wbase + 64 * r + lane;
    if (e >= m) continue;
    const uint64_t cs = oc + ex[r];
    soff[e] = (uint32_t)(cs > 0xffffffffull ? 0xffffffffull : cs);
    const uint32_t pos = (uint32_t)(ov + fx[r]);
    const int64_t i = e % n;
    if (c[r] != 0u) visible[pos] = (uint32_t)i;
    if (i == 0) vstart[e / n] = pos;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const uint64_t K = carry[2];
    soff[m] = (uint32_t)(K > 0xffffffffull ? 0xffffffffull : K);
    vstart[V] = (uint32_t)carry[3];
    *needed = (int64_t)K;
    if ((int64_t)K > capacity) *status = 1;
  }
}

// Groups of 32 lanes take one visible surfel of view blockIdx.y each and spread its rect tiles over the
// group.  A group stages at most the first kFirstTiles tiles of a surfel itself; the rest of a larger rect
// (a surfel near the camera, or a long thin one) goes to a queue of kChunkTiles-tile chunks that
// k_stage_big spreads over all groups, so no group walks one rect for long while the others idle.
// (Measured: 8 or 16 lanes per surfel are slower on the training views, 64 saves 7 us there but costs
// 20 % of the served latency on the 5 M-surfel 4K views; batches of 64 surfels with their tiles
// flattened over the lanes are slower; up to 8192 workgroups per view instead of 2048 saves 3 us.)
constexpr int kGroup = 32;
constexpr uint32_t kNoTile = 0xffffffffu;  // staged slot of a rect tile the surfel cannot reach
constexpr uint32_t kChunkTiles = 4 * kGroup;
#ifndef CGV2_FIRST_CHUNKS
#define CGV2_FIRST_CHUNKS 2
#endif
constexpr uint32_t kFirstTiles = CGV2_FIRST_CHUNKS * kChunkTiles;

// One visible surfel of view v as the staging sees it.
struct StageSurfel {
  uint32_t tx0, ty0, w, total, o;
  float4 r0;
  uint64_t key;
  Reach q;
};

__device__ __forceinline__ void stage_surfel(const uint16_t* rect, const float* rec, const uint32_t* soff, int64_t n,
                                             int v, uint32_t i, StageSurfel& u) {
  const int64_t vi = (int64_t)v * n + i;
  uint32_t tx1, ty1;
  tile_rect(rect + 4 * vi, u.tx0, u.ty0, tx1, ty1);
  u.w = tx1 - u.tx0;
  u.total = u.w * (ty1 - u.ty0);
  const float4* rp = (const float4*)(rec + vi * kRec);
  const float4 r1 = rp[1], r2 = rp[2], r4 = rp[4];
  u.r0 = rp[0];
  u.key = ((uint64_t)__float_as_uint(r2.w) << 32) | i;
  reach_setup(r1.x * kInvSqrt2, r1.y * kInvSqrt2, r1.z * kInvSqrt2, r1.w * kInvSqrt2, r2.x, r2.y, r2.z, r4.w, u.q);
  u.o = soff[vi];
}

// Rect tiles [kb, ke) of surfel u, tile k on lane kb + g + 32 j of the group: for each tile the surfel's
// alpha >= 1/255 region reaches, a returning atomic on the tile's counter gives the entry's rank; (tile,
// rank) and the key go to the surfel's slot o + k, a sentinel tile to the slots of the tiles it cannot
// reach.  Four independent returning atomics are in flight per lane before their results are used.
__device__ __forceinline__ void stage_range(const StageSurfel& u, uint32_t tbase, int tiles_x, uint32_t kb, uint32_t ke,
                                            uint32_t g, uint32_t* __restrict__ cnt, uint2* __restrict__ st_pos,
                                            uint64_t* __restrict__ st_key) {
  for (uint32_t k0 = kb + g; k0 < ke; k0 += 4 * kGroup) {
    uint32_t t[4], r[4];
    bool keep[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t k = k0 + (uint32_t)j * kGroup;
      const uint32_t tx = u.tx0 + k % u.w, ty = u.ty0 + k / u.w;
      t[j] = tbase + ty * tiles_x + tx;
      // the tile-relative centre exactly as the renderer stages it
      const float fox = (float)(tx * kTile), foy = (float)(ty * kTile);
      keep[j] = k < ke && reach_cell(u.q, (u.r0.x - fox) + u.r0.z, (u.r0.y - foy) + u.r0.w, 0, 0, kTile);
      r[j] = keep[j] ? atomicAdd(cnt + t[j], 1u) : 0u;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t k = k0 + (uint32_t)j * kGroup;
      if (k < ke) {
        st_pos[u.o + k] = make_uint2(keep[j] ? t[j] : kNoTile, r[j]);
        if (keep[j]) st_key[u.o + k] = u.key;
      }
    }
  }
}

// chunk queue entry: (index into 'visible', view << 16 | chunk); chunk c covers rect tiles
// [kFirstTiles + c kChunkTiles, ... + kChunkTiles).  A surfel with T > kFirstTiles tiles queues
// ceil((T - kFirstTiles) / kChunkTiles) < T / kChunkTiles chunks, so capacity / kChunkTiles + 1 entries
// hold every queue whose rect slots fit the capacity (the staging does not run otherwise).
__global__ __launch_bounds__(256) void k_stage(const uint16_t* __restrict__ rect, const float* __restrict__ rec,
                                               int64_t n, int tiles_x, int tiles_per_view,
                                               const uint32_t* __restrict__ visible,
                                               const uint32_t* __restrict__ vstart,
                                               const uint32_t* __restrict__ soff, uint32_t* __restrict__ cnt,
                                               uint2* __restrict__ st_pos, uint64_t* __restrict__ st_key,
                                               uint2* __restrict__ chunks, uint32_t* __restrict__ n_chunks,
                                               uint32_t max_chunks, const int32_t* __restrict__ status) {
  const int v = blockIdx.y;
  if (*status != 0) return;
  const uint32_t nv = vstart[v + 1] - vstart[v];
  const uint32_t* list = visible + vstart[v];
  const uint32_t g = threadIdx.x % kGroup;
  const uint32_t tbase = (uint32_t)v * (uint32_t)tiles_per_view;
  for (uint32_t e = (blockIdx.x * blockDim.x + threadIdx.x) / kGroup; e < nv;
       e += gridDim.x * blockDim.x / kGroup) {
    StageSurfel u;
    stage_surfel(rect, rec, soff, n, v, list[e], u);
    stage_range(u, tbase, tiles_x, 0u, min(u.total, kFirstTiles), g, cnt, st_pos, st_key);
    if (u.total > kFirstTiles) {
      const uint32_t nc = (u.total - kFirstTiles + kChunkTiles - 1) / kChunkTiles;
      uint32_t base = 0;
      if (g == 0) base = atomicAdd(n_chunks, nc);
      base = __shfl(base, (int)(threadIdx.x & 63u & ~(uint32_t)(kGroup - 1)), 64);
      for (uint32_t c = g; c < nc; c += kGroup)
        if (base + c < max_chunks) chunks[base + c] = make_uint2(vstart[v] + e, ((uint32_t)v << 16) | c);
    }
  }
}

// The queued chunks of the large rects, one chunk per group.
__global__ __launch_bounds__(256) void k_stage_big(const uint16_t* __restrict__ rect, const float* __restrict__ rec,
                                                   int64_t n, int tiles_x, int tiles_per_view,
                                                   const uint32_t* __restrict__ visible,
                                                   const uint32_t* __restrict__ soff, uint32_t* __restrict__ cnt,
                                                   uint2* __restrict__ st_pos, uint64_t* __restrict__ st_key,
                                                   const uint2* __restrict__ chunks,
                                                   const uint32_t* __restrict__ n_chunks, uint32_t max_chunks,
                                                   const int32_t* __restrict__ status) {
  if (*status != 0) return;
  const uint32_t nc = min(*n_chunks, max_chunks);
  const uint32_t g = threadIdx.x % kGroup;
  for (uint32_t it = (blockIdx.x * blockDim.x + threadIdx.x) / kGroup; it < nc;
       it += gridDim.x * blockDim.x / kGroup) {
    const uint2 c = chunks[it];
    const int v = (int)(c.y >> 16);
    StageSurfel u;
    stage_surfel(rect, rec, soff, n, v, visible[c.x], u);
    const uint32_t kb = kFirstTiles + (c.y & 0xffffu) * kChunkTiles;
    stage_range(u, (uint32_t)v * (uint32_t)tiles_per_view, tiles_x, kb, min(u.total, kb + kChunkTiles), g, cnt,
                st_pos, st_key);
  }
}

__global__ __launch_bounds__(kScanBlock) void k_tile_scan(const uint32_t* __restrict__ cnt, int64_t m,
                                                          uint32_t* __restrict__ ranges) {
  __shared__ uint64_t lds[2 * kScanWaves];
  uint64_t carry = 0;
  for (int64_t base = 0; base < m; base += kScanChunk) {
    const int64_t b0 = base + (int64_t)threadIdx.x * kScanItems;
    uint64_t vals[kScanItems];
    for (int k = 0; k < kScanItems; ++k) vals[k] = b0 + k < m ? cnt[b0 + k] : 0;
    const uint64_t tot = block_scan(vals, lds);
    for (int k = 0; k < kScanItems; ++k)
      if (b0 + k < m) ranges[b0 + k] = (uint32_t)(vals[k] + carry);
    carry += tot;
  }
  if (threadIdx.x == 0) ranges[m] = (uint32_t)carry;
}

// Multi-workgroup form of the tile scan for many tiles: chunk sums, then (after k_scan_top) each chunk
// scanned with its carry.
__global__ __launch_bounds__(kScanBlock) void k_u32_sums(const uint32_t* __restrict__ a, int64_t m,
                                                         uint64_t* __restrict__ sums) {
  __shared__ uint64_t lds[2 * kScanWaves];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  uint64_t c = 0;
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t idx = base + (int64_t)k * kScanBlock + threadIdx.x;
    if (idx < m) c += a[idx];
  }
  const uint64_t t = block_sum(c, lds);
  if (threadIdx.x == 0) sums[blockIdx.x] = t;
}

__global__ __launch_bounds__(kScanBlock) void k_u32_apply(const uint32_t* __restrict__ a, int64_t m,
                                                          const uint64_t* __restrict__ sums,
                                                          const uint64_t* __restrict__ total,
                                                          uint32_t* __restrict__ out) {
  __shared__ uint64_t lds[2 * kScanWaves];
  const uint64_t carry = sums[blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
  uint64_t vals[kScanItems];
  for (int k = 0; k < kScanItems; ++k) vals[k] = base + k < m ? a[base + k] : 0;
  block_scan(vals, lds);
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < m) out[base + k] = (uint32_t)(vals[k] + carry);
  if (blockIdx.x == 0 && threadIdx.x == 0) out[m] = (uint32_t)*total;
}

__global__ __launch_bounds__(256) void k_place(const uint32_t* __restrict__ soff_total,
                                               const uint2* __restrict__ st_pos, const uint64_t* __restrict__ st_key,
                                               const uint32_t* __restrict__ ranges, uint64_t* __restrict__ keys,
                                               const int32_t* __restrict__ status) {
  if (*status != 0) return;
  const uint32_t K = *soff_total;
  for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < K; e += gridDim.x * blockDim.x) {
    const uint2 tp = st_pos[e];
    if (tp.x != kNoTile) keys[ranges[tp.x] + tp.y] = st_key[e];
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

// ---- per-tile sort of up to kWaveSort keys in one wave's registers ----------------------------------
// A bitonic network over 64 E keys, E per lane in blocked order (key x = E lane + e).  Steps whose partner
// distance j is below E pair two registers of a lane; the others pair register e of lanes l and l ^ j / E,
// exchanged with DPP (distances 1, 2, 4, 8) or the gfx950 row-swap instructions (16, 32), so the sort
// touches neither LDS nor a barrier.  A compare-exchange keeps the minimum where the lane holds the
// lower index of an ascending pair or the upper one of a descending pair.
constexpr int kWaveSort = 1024;  // longest list sorted in registers (E = 16)

// value of lane l ^ D for D = 1, 2, 4, 8 (DPP within rows of 16)
template <int D>
__device__ __forceinline__ uint32_t lane_xor(uint32_t x) {
  const int i = (int)x;
  if constexpr (D == 1) return (uint32_t)__builtin_amdgcn_update_dpp(0, i, 0xB1, 0xf, 0xf, false);   // [1,0,3,2]
  if constexpr (D == 2) return (uint32_t)__builtin_amdgcn_update_dpp(0, i, 0x4E, 0xf, 0xf, false);   // [2,3,0,1]
  if constexpr (D == 4) {  // l ^ 7 (row_half_mirror), then ^ 3 (quad_perm [3,2,1,0])
    const int h = __builtin_amdgcn_update_dpp(0, i, 0x141, 0xf, 0xf, false);
    return (uint32_t)__builtin_amdgcn_update_dpp(0, h, 0x1B, 0xf, 0xf, false);
  }
  if constexpr (D == 8) return (uint32_t)__builtin_amdgcn_update_dpp(0, i, 0x128, 0xf, 0xf, false);  // row_ror:8
}

// register e of lanes l and l ^ D: keep the smaller key where keep_min, else the larger
template <int D>
__device__ __forceinline__ void cx_lanes(uint64_t& v, bool keep_min) {
  const uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  uint64_t a, b;  // the two keys of the pair (which one is this lane's does not matter)
  if constexpr (D <= 8) {
    a = v;
    b = ((uint64_t)lane_xor<D>(hi) << 32) | lane_xor<D>(lo);
  } else {
    // a row swap of a register with itself leaves this lane's key in one result and its partner's in
    // the other
    const auto rl = D == 16 ? __builtin_amdgcn_permlane16_swap(lo, lo, false, false)
                            : __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto rh = D == 16 ? __builtin_amdgcn_permlane16_swap(hi, hi, false, false)
                            : __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    a = ((uint64_t)rh[0] << 32) | rl[0];
    b = ((uint64_t)rh[1] << 32) | rl[1];
  }
  v = ((a < b) == keep_min) ? a : b;
}

// registers x (lower index) and y of one lane, ascending or descending
__device__ __forceinline__ void cx_regs(uint64_t& x, uint64_t& y, bool asc) {
  const bool c = (x < y) == asc;
  const uint64_t p = c ? x : y, q = c ? y : x;
  x = p;
  y = q;
}

template <int E, int K, int J>
__device__ __forceinline__ void bitonic_step(uint64_t (&v)[E], unsigned lane) {
  if constexpr (J >= E) {
    // K >= 2 J >= 2 E: the direction follows bit K / E of the lane (all ascending in the last merge)
    const bool asc = K >= 64 * E || (lane & (unsigned)(K / E)) == 0u;
    const bool keep_min = ((lane & (unsigned)(J / E)) == 0u) == asc;
#pragma unroll
    for (int e = 0; e < E; ++e) cx_lanes<J / E>(v[e], keep_min);
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (e & J) continue;
      const bool asc = K < E ? (e & K) == 0 : (K >= 64 * E || (lane & (unsigned)(K / E)) == 0u);
      cx_regs(v[e], v[e | J], asc);
    }
  }
  if constexpr (J > 1) bitonic_step<E, K, J / 2>(v, lane);
}

template <int E, int K = 2>
__device__ __forceinline__ void wave_bitonic(uint64_t (&v)[E], unsigned lane) {
  bitonic_step<E, K, K / 2>(v, lane);
  if constexpr (K < 64 * E) wave_bitonic<E, 2 * K>(v, lane);
}

// keys[a, a + len) sorted by one wave (len <= 64 E), ids written in order; the tail is padded with the
// largest key
template <int E>
__device__ __forceinline__ void sort_list_wave(const uint64_t* __restrict__ keys, uint32_t* __restrict__ ids,
                                               uint32_t a, int len, unsigned lane) {
  uint64_t v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int x = E * (int)lane + e;
    v[e] = x < len ? keys[a + x] : ~0ull;
  }
  wave_bitonic<E>(v, lane);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int x = E * (int)lane + e;
    if (x < len) ids[a + x] = (uint32_t)v[e];
  }
}

// One wave per tile: lists up to kWaveSort entries are sorted in registers with the smallest E that
// holds them; longer ones go to big_list for k_sort_big.
__global__ __launch_bounds__(256) void k_sort_wave(const uint32_t* __restrict__ ranges, int num_tiles,
                                                   const uint64_t* __restrict__ keys, uint32_t* __restrict__ ids,
                                                   uint32_t* __restrict__ big_list, uint32_t* __restrict__ big_count,
                                                   const int32_t* __restrict__ status) {
  const int t = (int)(blockIdx.x * 4u + (threadIdx.x >> 6));
  if (t >= num_tiles || *status != 0) return;
  const unsigned lane = threadIdx.x & 63u;
  const uint32_t a = ranges[t], b = ranges[t + 1];
  const int len = (int)(b - a);
  if (len == 0) return;
  if (len > kWaveSort) {
    if (lane == 0) big_list[atomicAdd(big_count, 1u)] = (uint32_t)t;
    return;
  }
  if (len <= 64) sort_list_wave<1>(keys, ids, a, len, lane);
  else if (len <= 128) sort_list_wave<2>(keys, ids, a, len, lane);
  else if (len <= 256) sort_list_wave<4>(keys, ids, a, len, lane);
  else if (len <= 512) sort_list_wave<8>(keys, ids, a, len, lane);
  else sort_list_wave<16>(keys, ids, a, len, lane);
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

// ---- launch order of the render kernels --------------------------------------------------------
// A render launch holds few tiles per wave slot and tile costs vary by orders of magnitude, so the
// heaviest tiles go first (longest-processing-time order): a stable counting sort of a view chunk's
// tiles by a log-scale bucket of their list length, descending, tiles in index order within a bucket.
constexpr int kOrdBuckets = 64;
static_assert(kOrdBuckets == 64, "the order kernels keep one bucket per lane");
constexpr int kOrdChunk = 1024;  // tiles per workgroup (16 waves)

__device__ __forceinline__ int order_bucket(uint32_t len) {
  if (len == 0) return 0;
  const int e = 31 - __clz(len);  // floor(log2 len)
  const int half = e >= 1 ? (int)((len >> (e - 1)) & 1u) : 0;
  const int b = 2 * e + 1 + half;
  return b < kOrdBuckets ? b : kOrdBuckets - 1;
}

// lanes of this wave whose bucket equals the calling lane's (bk in [0, kOrdBuckets), -1 for none; the
// result is meaningful for bk >= 0): one ballot per bit of the 6-bit bucket
__device__ __forceinline__ unsigned long long same_bucket(int bk) {
  unsigned long long same = __ballot(bk >= 0);
#pragma unroll
  for (int b = 0; b < 6; ++b) {
    const bool bit = bk >= 0 && ((bk >> b) & 1);
    const unsigned long long B = __ballot(bit);
    same &= bit ? B : ~B;
  }
  return same;
}

__global__ __launch_bounds__(kOrdChunk) void k_order_hist(const uint32_t* __restrict__ ranges, int64_t base, int T,
                                                          uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[kOrdBuckets];
  if (threadIdx.x < kOrdBuckets) h[threadIdx.x] = 0;
  __syncthreads();
  const int t = blockIdx.x * kOrdChunk + threadIdx.x;
  if (t < T) atomicAdd(&h[order_bucket(ranges[base + t + 1] - ranges[base + t])], 1u);
  __syncthreads();
  if (threadIdx.x < kOrdBuckets) hist[(int64_t)blockIdx.x * kOrdBuckets + threadIdx.x] = h[threadIdx.x];
}

// one wave: hist[c][k] -> first slot of bucket k's tiles of chunk c, buckets in descending order
__global__ __launch_bounds__(64) void k_order_scan(uint32_t* __restrict__ hist, int nc) {
  const int k = threadIdx.x;  // bucket
  uint32_t tot = 0;
  for (int c = 0; c < nc; ++c) tot += hist[(int64_t)c * kOrdBuckets + k];
  // inclusive suffix sum over the buckets k and above, then exclusive
  uint32_t x = tot;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_down(x, d, 64);
    if (k + d < 64) x += y;
  }
  uint32_t run = x - tot;
  for (int c = 0; c < nc; ++c) {
    const uint32_t v = hist[(int64_t)c * kOrdBuckets + k];
    hist[(int64_t)c * kOrdBuckets + k] = run;
    run += v;
  }
}

__global__ __launch_bounds__(kOrdChunk) void k_order_place(const uint32_t* __restrict__ ranges, int64_t base, int T,
                                                           const uint32_t* __restrict__ hist,
                                                           uint32_t* __restrict__ order) {
  constexpr int kWaves = kOrdChunk / 64;
  __shared__ uint32_t wc[kWaves][kOrdBuckets];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int t = blockIdx.x * kOrdChunk + threadIdx.x;
  const int bk = t < T ? order_bucket(ranges[base + t + 1] - ranges[base + t]) : -1;
  const unsigned long long lt = (1ull << lane) - 1ull;
  const unsigned long long same = same_bucket(bk);
  const uint32_t rank = bk >= 0 ? (uint32_t)__popcll(same & lt) : 0u;
  wc[w][lane] = 0;  // kOrdBuckets == 64: one bucket per lane
  // the first lane of each bucket present writes its count (after the zeroing: one wave, LDS in order)
  if (bk >= 0 && rank == 0) wc[w][bk] = (uint32_t)__popcll(same);
  __syncthreads();
  if (threadIdx.x < kOrdBuckets) {
    uint32_t run = 0;
    for (int q = 0; q < kWaves; ++q) {
      const uint32_t v = wc[q][threadIdx.x];
      wc[q][threadIdx.x] = run;
      run += v;
    }
  }
  __syncthreads();
  if (bk >= 0) order[hist[(int64_t)blockIdx.x * kOrdBuckets + bk] + wc[w][bk] + rank] = (uint32_t)t;
}

// One workgroup for up to kScanChunk tiles of at most kMaxViews views (the common single-view case):
// the tile scan of k_tile_scan and the launch order of k_order_hist / k_order_scan / k_order_place in
// one launch, the same results.  Wave w owns the contiguous tiles [w per, (w + 1) per) and loads their
// counts once, all at the same time (lane l holds tiles w per + 64 k + l); the scan runs over those
// registers (wave scans in k order, one LDS exchange of the 16 wave totals); the order takes LDS counts
// per (wave, bucket), one exchange of the 16 x 64 counts into first slots, and a placing pass with
// stable ranks from the lanes that share a bucket (same_bucket).

__global__ __launch_bounds__(kScanBlock) void k_tile_scan_order(const uint32_t* __restrict__ cnt, int m,
                                                                uint32_t* __restrict__ ranges,
                                                                uint32_t* __restrict__ order) {
  __shared__ uint32_t wtot[kScanWaves];
  __shared__ uint32_t wc[kScanWaves][kOrdBuckets];
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  // kScanWaves * per >= m, per a multiple of 64 and at most 64 kScanItems (m <= kScanChunk)
  const int per = ((m + kScanBlock - 1) / kScanBlock) * 64;
  const int i0 = w * per, i1 = min(m, i0 + per);
  uint32_t c[kScanItems];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int i = i0 + 64 * k + lane;
    c[k] = 64 * k < per && i < i1 ? cnt[i] : 0u;
  }
  // tile scan: exclusive prefix sums within the wave's tiles, then the wave offsets
  uint32_t ex[kScanItems];
  uint32_t carry = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const uint32_t inc = wave_scan_u32(c[k]);
    ex[k] = carry + inc - c[k];
    carry += lane63(inc);
  }
  if (lane == 0) wtot[w] = carry;
  const unsigned long long lt = (1ull << lane) - 1ull;
  wc[w][lane] = 0;  // kOrdBuckets == 64: one bucket per lane
  __syncthreads();
  uint32_t off = 0, total = 0;
  for (int q = 0; q < kScanWaves; ++q) {
    const uint32_t v = wtot[q];
    off += q < w ? v : 0u;
    total += v;
  }
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int i = i0 + 64 * k + lane;
    if (64 * k < per && i < i1) ranges[i] = off + ex[k];
  }
  if (t == 0) ranges[m] = total;
  // counts per (wave, bucket), by LDS atomics that return nothing (no wait between the rows)
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (i0 + 64 * k >= i1) break;
    const int i = i0 + 64 * k + lane;
    if (i < i1) atomicAdd(&wc[w][order_bucket(c[k])], 1u);
  }
  __syncthreads();
  if (t < kOrdBuckets) {
    uint32_t tot = 0;
    for (int q = 0; q < kScanWaves; ++q) tot += wc[q][t];
    // buckets in descending order: bucket t starts after the tiles of the buckets above it
    const uint32_t inc = wave_scan_u32(tot);
    uint32_t run = lane63(inc) - inc;
    for (int q = 0; q < kScanWaves; ++q) {
      const uint32_t v = wc[q][t];
      wc[q][t] = run;
      run += v;
    }
  }
  __syncthreads();
  // wc[w][k]: next slot of bucket k for this wave's tiles
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (i0 + 64 * k >= i1) break;
    const int i = i0 + 64 * k + lane;
    const int bk = i < i1 ? order_bucket(c[k]) : -1;
    const unsigned long long same = same_bucket(bk);
    const uint32_t rank = (uint32_t)__popcll(same & lt);
    const uint32_t first = bk >= 0 ? wc[w][bk] : 0u;
    if (bk >= 0) order[first + rank] = (uint32_t)i;
    // after every lane's read above
    if (bk >= 0 && rank == 0) wc[w][bk] = first + (uint32_t)__popcll(same);
  }
}

}  // namespace cgv2

static int64_t scan_blocks(int64_t m) { return (m + cgv2::kScanChunk - 1) / cgv2::kScanChunk; }
static int64_t surf_blocks(int64_t m) { return (m + cgv2::kSurfChunk - 1) / cgv2::kSurfChunk; }

size_t cgv2_binsort_ws_layout(int64_t capacity, int V, int tiles, int64_t n, size_t* off) {
  // off: [0] tile counters (u32, m) followed by the big-list and chunk-queue counts, [1] chunk sums of the surfel
  //      scan (2 x u64 arrays), [2] big_list (u32, m), [3] scan totals (u64 x 2), [4] keys (u64,
  //      capacity), [5] staged keys / merge scratch (u64, capacity), [6] staged (tile, rank) (u32 x 2,
  //      capacity), [7] surfel offsets (u32, V n + 1), [8] chunk sums of the tile scan (u64)
  const int64_t m = (int64_t)V * tiles;
  const int64_t vn = (int64_t)V * n;
  const int64_t nsb = surf_blocks(vn > 0 ? vn : 1);
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o += (bytes + 255) & ~(size_t)255; return r; };
  off[0] = take(4 * (size_t)(m + 2));
  off[1] = take(16 * (size_t)(nsb + 1));
  off[2] = take(4 * (size_t)m);
  off[3] = take(64);
  off[4] = take(8 * (size_t)capacity);
  off[5] = take(8 * (size_t)capacity);
  off[6] = take(8 * (size_t)capacity);
  off[7] = take(4 * (size_t)(vn + 1));
  off[8] = take(8 * (size_t)(scan_blocks(m) + 1));
  // [9] per-chunk bucket counts of the launch order (one view chunk at a time)
  const int64_t per = (int64_t)std::min(V, cgv2::kMaxViews) * tiles;
  off[9] = take(4 * (size_t)cgv2::kOrdBuckets * (size_t)((per + cgv2::kOrdChunk - 1) / cgv2::kOrdChunk + 1));
  // [10] the chunk queue of the large rects (see k_stage)
  off[10] = take(8 * (size_t)(capacity / cgv2::kChunkTiles + 1));
  return o;
}

hipError_t cgv2_launch_bin_sort(const cgv2_proj& p, int64_t n, int V, int tiles_x, int tiles_y, const cgv2_bins& b,
                                void* ws, hipStream_t st) {
  using namespace cgv2;
  const int tiles = tiles_x * tiles_y;
  const int64_t m = (int64_t)V * tiles;
  const int64_t vn = (int64_t)V * n;
  size_t off[kBinsortOffs];
  cgv2_binsort_ws_layout(b.capacity, V, tiles, n, off);
  char* w = (char*)ws;
  uint32_t* cnt = (uint32_t*)(w + off[0]);
  uint32_t* big_count = cnt + m;
  const int64_t nsb = surf_blocks(vn > 0 ? vn : 1);
  uint64_t* sums_cnt = (uint64_t*)(w + off[1]);
  uint64_t* sums_vis = sums_cnt + nsb + 1;
  uint32_t* big_list = (uint32_t*)(w + off[2]);
  uint64_t* totals = (uint64_t*)(w + off[3]);
  uint64_t* keys = (uint64_t*)(w + off[4]);
  uint64_t* stk = (uint64_t*)(w + off[5]);
  uint2* stp = (uint2*)(w + off[6]);
  uint32_t* soff = (uint32_t*)(w + off[7]);
  uint32_t* n_chunks = cnt + m + 1;
  uint2* chunks = (uint2*)(w + off[10]);
  const uint32_t max_chunks = (uint32_t)std::min<int64_t>(b.capacity / kChunkTiles + 1, 0xffffffffll);
  if (n > 0) {
    // surfel offsets, visible lists (consumed by the staging here and by the reverse pass), total and
    // overflow check; the tile counters and the big-list count are zeroed on the way
    hipLaunchKernelGGL(k_surfel_sums, dim3((unsigned)nsb), dim3(kSurfBlock), 0, st, p.rect, vn, sums_cnt, sums_vis,
                       cnt, m + 2);
    // up to kSurfLocal chunks each apply workgroup adds up the chunk sums before it itself
    const int local_nsb = nsb <= kSurfLocal ? (int)nsb : 0;
    if (!local_nsb) hipLaunchKernelGGL(k_scan_top, dim3(2), dim3(kScanBlock), 0, st, sums_cnt, sums_vis, nsb, totals);
    hipLaunchKernelGGL(k_surfel_apply, dim3((unsigned)nsb), dim3(kSurfBlock), 0, st, p.rect, vn, n, sums_cnt,
                       sums_vis, totals, local_nsb, soff, p.visible, p.visible_start, V, b.capacity, b.status,
                       b.needed);
    const unsigned blocks = (unsigned)std::min<int64_t>((n * kGroup + 255) / 256, 8192);
    hipLaunchKernelGGL(k_stage, dim3(blocks, (unsigned)V), dim3(256), 0, st, p.rect, p.rec, n, tiles_x, tiles,
                       p.visible, p.visible_start, soff, cnt, stp, stk, chunks, n_chunks, max_chunks, b.status);
    hipLaunchKernelGGL(k_stage_big, dim3(1024), dim3(256), 0, st, p.rect, p.rec, n, tiles_x, tiles, p.visible, soff,
                       cnt, stp, stk, chunks, n_chunks, max_chunks, b.status);
  } else {
    // no surfels: empty lists, zero intersections
    hipLaunchKernelGGL(k_fill<uint32_t>, dim3((unsigned)std::min<int64_t>((m + 257) / 256, 65535)), dim3(256), 0, st,
                       cnt, m + 2, 0u);
    hipLaunchKernelGGL(k_fill<uint32_t>, dim3(1), dim3(256), 0, st, p.visible_start, (int64_t)V + 1, 0u);
    hipLaunchKernelGGL(k_fill<uint32_t>, dim3(1), dim3(256), 0, st, soff, (int64_t)1, 0u);
    hipLaunchKernelGGL(k_fill<int64_t>, dim3(1), dim3(256), 0, st, b.needed, (int64_t)1, (int64_t)0);
  }
  const int64_t nbt = scan_blocks(m);
  const bool fused_order = b.order && m <= kScanChunk && V <= kMaxViews;
  if (fused_order) {
    hipLaunchKernelGGL(k_tile_scan_order, dim3(1), dim3(kScanBlock), 0, st, cnt, (int)m, b.ranges, b.order);
  } else if (nbt <= 16) {
    hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(kScanBlock), 0, st, cnt, m, b.ranges);
  } else {
    uint64_t* ts = (uint64_t*)(w + off[8]);
    hipLaunchKernelGGL(k_u32_sums, dim3((unsigned)nbt), dim3(kScanBlock), 0, st, cnt, m, ts);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanBlock), 0, st, ts, ts, nbt, totals + 2);
    hipLaunchKernelGGL(k_u32_apply, dim3((unsigned)nbt), dim3(kScanBlock), 0, st, cnt, m, ts, totals + 2, b.ranges);
  }
  // one staged slot per thread up to 4 M slots (each slot is a chain of dependent loads); the total is
  // only known on the device, so the grid follows the capacity and the surplus threads exit at once
  const unsigned place_blocks = (unsigned)std::min<int64_t>(std::max<int64_t>((b.capacity + 255) / 256, 1), 16384);
  hipLaunchKernelGGL(k_place, dim3(place_blocks), dim3(256), 0, st, soff + vn, stp, stk, b.ranges, keys, b.status);
  hipLaunchKernelGGL(k_sort_wave, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, st, b.ranges, (int)m, keys, b.ids,
                     big_list, big_count, b.status);
  hipLaunchKernelGGL(k_sort_big, dim3(256), dim3(1024), 0, st, b.ranges, keys, stk, b.ids, big_list, big_count,
                     b.status);
  if (b.order && !fused_order) {
    uint32_t* hist = (uint32_t*)(w + off[9]);
    for (int v0 = 0; v0 < V; v0 += kMaxViews) {
      const int T = std::min(V - v0, kMaxViews) * tiles;
      const int nc = (T + kOrdChunk - 1) / kOrdChunk;
      const int64_t base = (int64_t)v0 * tiles;
      hipLaunchKernelGGL(k_order_hist, dim3((unsigned)nc), dim3(kOrdChunk), 0, st, b.ranges, base, T, hist);
      hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(64), 0, st, hist, nc);
      hipLaunchKernelGGL(k_order_place, dim3((unsigned)nc), dim3(kOrdChunk), 0, st, b.ranges, base, T, hist,
                         b.order + base);
    }
  }
  return hipGetLastError();
}
