// Serving storage of CityGaussianV2 (Sec. 3.3: SH degree 2; the appendix's vector-tree quantization):
// the least important surfels' SH vectors are replaced by the nearest row of a k-means codebook, the rest
// of the set is stored in float16.
//
//   k_part_*      stable partition by the quantize mask: kept surfels first, both groups in id order
//   k_vq_init     codeword j = row floor(j m / K) of the quantized vectors
//   k_vq_assign   nearest codeword: |c|^2 - 2 x.c on the matrix cores (FP32 MFMA 16x16x4), the argmin
//                 fused into the epilogue; codewords stream through LDS in chunks, transposed
//   k_vq_accum / k_vq_final   Lloyd update: FP64 sums per codeword, mean, empty codewords kept
//   k_compact_*   the stored arrays in partition order (float16 by round-to-nearest-even)
#include "cgv2r_device.h"
#include "cgv2r_kernels.h"

#include <algorithm>

namespace cgv2 {

typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t to_half_bits(float x) { return __builtin_bit_cast(uint16_t, (_Float16)x); }
__device__ __forceinline__ float from_half_bits(uint16_t b) { return (float)__builtin_bit_cast(_Float16, b); }

// ---- stable partition --------------------------------------------------------------------------

constexpr int kPBlock = 256;
constexpr int kPItems = 8;
constexpr int kPChunk = kPBlock * kPItems;

__global__ __launch_bounds__(kPBlock) void k_part_count(const uint8_t* __restrict__ q, int64_t n,
                                                        uint32_t* __restrict__ part) {
  __shared__ uint32_t lds[kPBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kPChunk + threadIdx.x;
  uint32_t keep = 0;
#pragma unroll
  for (int k = 0; k < kPItems; ++k) {
    const int64_t i = base + (int64_t)k * kPBlock;
    if (i < n && !q[i]) ++keep;
  }
  uint32_t tot;
  block_exscan<kPBlock>(keep, lds, tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kPBlock) void k_part_scan(uint32_t* __restrict__ part, int nb, int64_t* __restrict__ n_full) {
  __shared__ unsigned long long lds[kPBlock / 64];
  unsigned long long carry = 0;
  for (int b0 = 0; b0 < nb; b0 += kPBlock) {
    const int b = b0 + (int)threadIdx.x;
    const unsigned long long v = b < nb ? part[b] : 0ull;
    unsigned long long tot;
    const unsigned long long ex = block_exscan<kPBlock>(v, lds, tot) + carry;
    if (b < nb) part[b] = (uint32_t)ex;
    carry += tot;
  }
  if (threadIdx.x == 0) *n_full = (int64_t)carry;
}

__global__ __launch_bounds__(kPBlock) void k_part_write(const uint8_t* __restrict__ q, int64_t n,
                                                        const uint32_t* __restrict__ koff,
                                                        const int64_t* __restrict__ n_full,
                                                        uint32_t* __restrict__ order) {
  __shared__ uint32_t lds[kPBlock / 64];
  const int64_t chunk = (int64_t)blockIdx.x * kPChunk;
  const int64_t base = chunk + (int64_t)threadIdx.x * kPItems;
  uint32_t qq[kPItems], keep = 0;
#pragma unroll
  for (int k = 0; k < kPItems; ++k) {
    qq[k] = base + k < n ? (q[base + k] ? 1u : 0u) : 1u;
    keep += base + k < n ? 1u - qq[k] : 0u;
  }
  uint32_t tot;
  const uint32_t ex = block_exscan<kPBlock>(keep, lds, tot);
  // kept before this thread's first item, over the whole set; quantized before it = index - kept
  uint32_t kept_before = koff[blockIdx.x] + ex;
  const int64_t nf = *n_full;
#pragma unroll
  for (int k = 0; k < kPItems; ++k) {
    const int64_t i = base + k;
    if (i >= n) break;
    if (!qq[k]) {
      order[kept_before] = (uint32_t)i;
      ++kept_before;
    } else {
      order[nf + (i - kept_before)] = (uint32_t)i;
    }
  }
}

// ---- codebook ------------------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_vq_init(const float* __restrict__ x, int D, const uint32_t* __restrict__ rows,
                                                 int64_t m, int K, float* __restrict__ cb) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)K * D) return;
  const int j = (int)(t / D), d = (int)(t - (int64_t)j * D);
  const int64_t r = ((int64_t)j * m) / K;
  cb[t] = x[(int64_t)rows[r] * D + d];
}

// Nearest codeword for kVqRows query vectors per workgroup (kVqRowsWave per wave: two 16-row MFMA
// tiles), against codewords staged kVqCols at a time in LDS as cwT[dim][col] (conflict-free B reads).
// MFMA 16x16x4 f32 operand layout (wave64): A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k, and
// D[4 (lane / 16) + r][lane % 16] in accumulator element r.
constexpr int kVqThreads = 256;
constexpr int kVqRowsWave = 32;
constexpr int kVqRows = kVqRowsWave * (kVqThreads / 64);
constexpr int kVqCols = 128;

// |c|^2 of every codeword (of its float16 rounding when half_cb), FP32.
__global__ __launch_bounds__(256) void k_vq_norms(const float* __restrict__ cb, int K, int D, int half_cb,
                                                  float* __restrict__ norms) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= K) return;
  float s2 = 0.f;
  for (int d = 0; d < D; ++d) {
    float v = cb[(int64_t)j * D + d];
    if (half_cb) v = (float)(_Float16)v;
    s2 = fmaf(v, v, s2);
  }
  norms[j] = s2;
}

template <int DP>  // dimensions padded to a multiple of 4
__global__ __launch_bounds__(kVqThreads) void k_vq_assign(const float* __restrict__ x, int D,
                                                          const uint32_t* __restrict__ rows, int64_t m,
                                                          const float* __restrict__ cb, const float* __restrict__ norms,
                                                          int K, int half_cb, uint16_t* __restrict__ code) {
  constexpr int kSteps = DP / 4;
  __shared__ float cwT[DP][kVqCols];
  __shared__ float norm[kVqCols];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t row0 = (int64_t)blockIdx.x * kVqRows + (int64_t)w * kVqRowsWave;
  // A operands: query (row0 + 16 t + li), dimension 4 s + lk
  float a[2][kSteps];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int64_t r = row0 + 16 * t + li;
    const float* xr = r < m ? x + (int64_t)rows[r] * D : nullptr;
#pragma unroll
    for (int s = 0; s < kSteps; ++s) {
      const int d = 4 * s + lk;
      a[t][s] = (xr && d < D) ? xr[d] : 0.f;
    }
  }
  float best[2][4];
  int bidx[2][4];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      best[t][r] = INFINITY;
      bidx[t][r] = 0x7fffffff;
    }
  for (int c0 = 0; c0 < K; c0 += kVqCols) {
    __syncthreads();  // the previous chunk is no longer read
    // thread (j, group of 4 dimensions): consecutive threads fill consecutive columns of a row of cwT
    for (int e = threadIdx.x; e < kVqCols * kSteps; e += kVqThreads) {
      const int j = e % kVqCols, d4 = e / kVqCols;
      const bool live = c0 + j < K;
      const float* src = cb + (int64_t)(c0 + j) * D + 4 * d4;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float v = 0.f;
        if (live && 4 * d4 + q < D) {
          v = src[q];
          if (half_cb) v = (float)(_Float16)v;
        }
        cwT[4 * d4 + q][j] = v;
      }
    }
    if (threadIdx.x < kVqCols) norm[threadIdx.x] = c0 + (int)threadIdx.x < K ? norms[c0 + threadIdx.x] : INFINITY;
    __syncthreads();
#pragma unroll
    for (int ct = 0; ct < kVqCols / 16; ++ct) {
      floatx4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < kSteps; ++s) {
        const float b = cwT[4 * s + lk][16 * ct + li];
        acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0][s], b, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1][s], b, acc1, 0, 0, 0);
      }
      const int j = 16 * ct + li;
      const float nj = norm[j];
      const int idx = c0 + j;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float s0 = fmaf(-2.f, acc0[r], nj), s1 = fmaf(-2.f, acc1[r], nj);
        if (s0 < best[0][r]) { best[0][r] = s0; bidx[0][r] = idx; }
        if (s1 < best[1][r]) { best[1][r] = s1; bidx[1][r] = idx; }
      }
    }
  }
  // reduce over the 16 lanes that hold the same rows (lane % 16 = codeword column)
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float b = best[t][r];
      int bi = bidx[t][r];
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) {
        const float ob = __shfl_xor(b, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ob < b || (ob == b && oi < bi)) { b = ob; bi = oi; }
      }
      const int64_t q = row0 + 16 * t + 4 * lk + r;
      if (li == 0 && q < m) code[q] = (uint16_t)bi;
    }
}

__global__ __launch_bounds__(256) void k_vq_accum(const float* __restrict__ x, int D, const uint32_t* __restrict__ rows,
                                                  int64_t m, const uint16_t* __restrict__ code, int K,
                                                  double* __restrict__ sums, uint32_t* __restrict__ counts) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m) return;
  const int c = code[t];
  if (c >= K) return;
  const float* xr = x + (int64_t)rows[t] * D;
  for (int d = 0; d < D; ++d) atomicAdd(&sums[(int64_t)c * D + d], (double)xr[d]);
  atomicAdd(&counts[c], 1u);
}

__global__ __launch_bounds__(256) void k_vq_final(const double* __restrict__ sums,
                                                  const uint32_t* __restrict__ counts, int K, int D,
                                                  float* __restrict__ cb) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)K * D) return;
  const uint32_t c = counts[t / D];
  if (c) cb[t] = (float)(sums[t] / (double)c);
}

// ---- stored arrays ---------------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_compact_geom(cgv2_surfels s, const uint32_t* __restrict__ order,
                                                      cgv2_compact_out out) {
  const int64_t n = s.n;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int64_t i = order[j];
  if (i >= n) return;
#pragma unroll
  for (int c = 0; c < 3; ++c) out.mean[c * n + j] = s.mean[c * n + i];
#pragma unroll
  for (int c = 0; c < 2; ++c) out.log_scale[c * n + j] = to_half_bits(s.log_scale[c * n + i]);
#pragma unroll
  for (int c = 0; c < 4; ++c) out.quat[c * n + j] = to_half_bits(s.quat[c * n + i]);
  out.opacity_logit[j] = to_half_bits(s.opacity_logit[i]);
}

// SH of the kept slots [0, n_full), one value per thread (coalesced writes)
__global__ __launch_bounds__(256) void k_compact_sh(const float* __restrict__ sh, int64_t n, int F,
                                                    const uint32_t* __restrict__ order,
                                                    const int64_t* __restrict__ n_full, uint16_t* __restrict__ out) {
  const int64_t lim = *n_full * F;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < lim; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = t / F;
    const int k = (int)(t - j * F);
    const int64_t i = order[j];
    if (i < n) out[t] = to_half_bits(sh[i * F + k]);
  }
}

__global__ __launch_bounds__(256) void k_to_half(const float* __restrict__ x, int64_t count, uint16_t* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) out[t] = to_half_bits(x[t]);
}

inline unsigned blocks_for(int64_t items, int64_t cap = 1 << 20) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((items + 255) / 256, cap));
}

}  // namespace cgv2

size_t cgv2_part_ws_layout(int64_t n) {
  const int64_t nb = std::max<int64_t>((n + cgv2::kPChunk - 1) / cgv2::kPChunk, 1);
  return ((size_t)4 * (size_t)nb + 255) & ~(size_t)255;
}

hipError_t cgv2_launch_compact_order(const uint8_t* q, int64_t n, uint32_t* order, int64_t* n_full, void* ws,
                                     hipStream_t st) {
  const int nb = (int)std::max<int64_t>((n + cgv2::kPChunk - 1) / cgv2::kPChunk, 1);
  uint32_t* part = (uint32_t*)ws;
  if (n > 0)
    hipLaunchKernelGGL(cgv2::k_part_count, dim3((unsigned)nb), dim3(cgv2::kPBlock), 0, st, q, n, part);
  else
    hipLaunchKernelGGL((cgv2::k_fill<uint32_t>), dim3(1), dim3(64), 0, st, part, (int64_t)1, 0u);
  hipLaunchKernelGGL(cgv2::k_part_scan, dim3(1), dim3(cgv2::kPBlock), 0, st, part, nb, n_full);
  if (n > 0)
    hipLaunchKernelGGL(cgv2::k_part_write, dim3((unsigned)nb), dim3(cgv2::kPBlock), 0, st, q, n, part, n_full, order);
  return hipGetLastError();
}

hipError_t cgv2_launch_vq_init(const float* x, int D, const uint32_t* rows, int64_t m, int K, float* cb,
                               hipStream_t st) {
  hipLaunchKernelGGL(cgv2::k_vq_init, dim3(cgv2::blocks_for((int64_t)K * D)), dim3(256), 0, st, x, D, rows, m, K, cb);
  return hipGetLastError();
}

size_t cgv2_vq_assign_ws_layout(int K) { return (((size_t)K * sizeof(float)) + 255) & ~(size_t)255; }

hipError_t cgv2_launch_vq_assign(const float* x, int D, const uint32_t* rows, int64_t m, const float* cb, int K,
                                 int half_cb, uint16_t* code, void* ws, hipStream_t st) {
  if (m == 0) return hipGetLastError();
  float* norms = (float*)ws;
  hipLaunchKernelGGL(cgv2::k_vq_norms, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, st, cb, K, D, half_cb, norms);
  const unsigned nb = (unsigned)((m + cgv2::kVqRows - 1) / cgv2::kVqRows);
  const int DP = (D + 3) & ~3;
  switch (DP) {
    case 4: hipLaunchKernelGGL((cgv2::k_vq_assign<4>), dim3(nb), dim3(cgv2::kVqThreads), 0, st, x, D, rows, m, cb, norms, K, half_cb, code); break;
    case 12: hipLaunchKernelGGL((cgv2::k_vq_assign<12>), dim3(nb), dim3(cgv2::kVqThreads), 0, st, x, D, rows, m, cb, norms, K, half_cb, code); break;
    case 28: hipLaunchKernelGGL((cgv2::k_vq_assign<28>), dim3(nb), dim3(cgv2::kVqThreads), 0, st, x, D, rows, m, cb, norms, K, half_cb, code); break;
    case 48: hipLaunchKernelGGL((cgv2::k_vq_assign<48>), dim3(nb), dim3(cgv2::kVqThreads), 0, st, x, D, rows, m, cb, norms, K, half_cb, code); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

size_t cgv2_vq_update_ws_layout(int K, int D) {
  return (((size_t)K * D * sizeof(double)) + 255) & ~(size_t)255;
}

hipError_t cgv2_launch_vq_update(const float* x, int D, const uint32_t* rows, int64_t m, const uint16_t* code, int K,
                                 float* cb, uint32_t* counts, void* ws, hipStream_t st) {
  double* sums = (double*)ws;
  hipLaunchKernelGGL((cgv2::k_fill<double>), dim3(cgv2::blocks_for((int64_t)K * D, 4096)), dim3(256), 0, st, sums,
                     (int64_t)K * D, 0.0);
  hipLaunchKernelGGL((cgv2::k_fill<uint32_t>), dim3(cgv2::blocks_for(K, 4096)), dim3(256), 0, st, counts, (int64_t)K, 0u);
  if (m > 0)
    hipLaunchKernelGGL(cgv2::k_vq_accum, dim3(cgv2::blocks_for(m)), dim3(256), 0, st, x, D, rows, m, code, K, sums,
                       counts);
  hipLaunchKernelGGL(cgv2::k_vq_final, dim3(cgv2::blocks_for((int64_t)K * D)), dim3(256), 0, st, sums, counts, K, D, cb);
  return hipGetLastError();
}

hipError_t cgv2_launch_compact_write(const cgv2_surfels& s, const uint32_t* order, const int64_t* n_full,
                                     const float* cb, int K, const cgv2_compact_out& out, hipStream_t st) {
  const int64_t n = s.n;
  const int F = 3 * (s.sh_degree + 1) * (s.sh_degree + 1);
  if (n > 0) {
    hipLaunchKernelGGL(cgv2::k_compact_geom, dim3(cgv2::blocks_for(n)), dim3(256), 0, st, s, order, out);
    hipLaunchKernelGGL(cgv2::k_compact_sh, dim3(cgv2::blocks_for(n * F, 16384)), dim3(256), 0, st, s.sh, n, F, order,
                       n_full, out.sh);
  }
  if (K > 0 && cb)
    hipLaunchKernelGGL(cgv2::k_to_half, dim3(cgv2::blocks_for((int64_t)K * F)), dim3(256), 0, st, cb, (int64_t)K * F,
                       out.codebook);
  return hipGetLastError();
}
