// Densification statistics of CityGaussianV2 Sec. 3.2: the decomposed-gradient densification
// factor of Eq. 2 and the elongation filter.
//
// k_dgd_partial  per view, per block of 512 surfels: sums of |g_total| and |g_ssim| over the
//                visible surfels, tree-reduced in FP64 in a fixed order
// k_dgd_final    one workgroup reduces each view's block partials in a fixed order into
//                scale_v = max(omega a_tot / a_ssim, 1) (deterministic)
// k_densify      updates the per-surfel state and the masks; per-workgroup counter partials
// k_count_final  one workgroup adds the partials to the counters (no same-address atomics)
#include <atomic>

#include "cgv2r_device.h"
#include "cgv2r_kernels.h"

namespace cgv2 {

constexpr int kDBlock = 256;
constexpr int kDItems = 2;  // surfels per thread in k_dgd_partial

__global__ __launch_bounds__(kDBlock) void k_dgd_partial(const uint8_t* __restrict__ flags,
                                                         const float* __restrict__ gt, const float* __restrict__ gs,
                                                         int64_t n, double* __restrict__ partial, int nblocks,
                                                         uint32_t* __restrict__ counters) {
  __shared__ double red[2][kDBlock];
  const int v = blockIdx.y;
  const int64_t base = (int64_t)blockIdx.x * kDBlock * kDItems;
  const float* g1 = gt + (int64_t)v * 2 * n;
  const float* g2 = gs ? gs + (int64_t)v * 2 * n : nullptr;
  double a = 0, b = 0;
  for (int k = 0; k < kDItems; ++k) {
    const int64_t i = base + (int64_t)k * kDBlock + threadIdx.x;
    if (i < n && (flags[(int64_t)v * n + i] & CGV2_F_VISIBLE)) {
      a += sqrt((double)g1[i] * g1[i] + (double)g1[n + i] * g1[n + i]);
      if (g2) b += sqrt((double)g2[i] * g2[i] + (double)g2[n + i] * g2[n + i]);
    }
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  __syncthreads();
  for (int off = kDBlock / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      red[0][threadIdx.x] += red[0][threadIdx.x + off];
      red[1][threadIdx.x] += red[1][threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * ((int64_t)v * nblocks + blockIdx.x)] = red[0][0];
    partial[2 * ((int64_t)v * nblocks + blockIdx.x) + 1] = red[1][0];
  }
  if (blockIdx.x == 0 && v == 0 && threadIdx.x < 8) counters[threadIdx.x] = 0;
}

__global__ __launch_bounds__(kDBlock) void k_dgd_final(const double* __restrict__ partial, int nblocks, int V,
                                                       float omega, float* __restrict__ scale_ws,
                                                       float* __restrict__ scale_out) {
  __shared__ double red[2][kDBlock];
  for (int v = 0; v < V; ++v) {
    double a = 0, b = 0;
    for (int k = threadIdx.x; k < nblocks; k += kDBlock) {
      a += partial[2 * ((int64_t)v * nblocks + k)];
      b += partial[2 * ((int64_t)v * nblocks + k) + 1];
    }
    red[0][threadIdx.x] = a;
    red[1][threadIdx.x] = b;
    __syncthreads();
    for (int off = kDBlock / 2; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) {
        red[0][threadIdx.x] += red[0][threadIdx.x + off];
        red[1][threadIdx.x] += red[1][threadIdx.x + off];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const double at = red[0][0], as = red[1][0];
      const float sc = (float)(as > 0 ? fmax((double)omega * at / as, 1.0) : 1.0);
      scale_ws[v] = sc;
      if (scale_out) scale_out[v] = sc;
    }
    __syncthreads();
  }
}

constexpr int kCounters = 6;

__global__ __launch_bounds__(kDBlock) void k_densify(cgv2_surfels s, const uint8_t* __restrict__ flags,
                                                     const float* __restrict__ radius, const float* __restrict__ gt,
                                                     const float* __restrict__ gs, int V,
                                                     const float* __restrict__ scale_ws, cgv2_densify_params prm,
                                                     cgv2_densify_state st, uint32_t* __restrict__ cpart) {
  __shared__ uint32_t cnt_s[8];
  const int64_t n = s.n;
  if (threadIdx.x < 8) cnt_s[threadIdx.x] = 0;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * kDBlock + threadIdx.x;
  if (i < n) {
    float adgd = st.accum_dgd[i], atot = st.accum_total[i], mr = st.max_radius[i];
    int32_t den = st.denom[i];
    uint32_t nvis = 0, nlp = 0;
    bool lp = false;
    for (int v = 0; v < V; ++v) {
      const int64_t vi = (int64_t)v * n + i;
      const uint8_t f = flags[vi];
      if (!(f & CGV2_F_VISIBLE)) continue;
      const float* g1 = gt + (int64_t)v * 2 * n;
      const float nt = sqrtf(g1[i] * g1[i] + g1[n + i] * g1[n + i]);
      float ns = 0.f;
      if (gs) {
        const float* g2 = gs + (int64_t)v * 2 * n;
        ns = sqrtf(g2[i] * g2[i] + g2[n + i] * g2[n + i]);
      }
      adgd = fmaf(scale_ws[v], ns, adgd);
      atot += nt;
      den += 1;
      mr = fmaxf(mr, radius[vi]);
      ++nvis;
      if (f & CGV2_F_LOWPASS) { ++nlp; lp = true; }
    }
    st.accum_dgd[i] = adgd;
    st.accum_total[i] = atot;
    st.max_radius[i] = mr;
    st.denom[i] = den;
    const float su = expf(s.log_scale[i]), sv = expf(s.log_scale[n + i]);
    const float eta = fminf(su, sv) / fmaxf(su, sv);
    const float avg = den > 0 ? adgd / (float)den : 0.f;
    const bool high = avg >= prm.grad_threshold;
    const bool elong = eta < prm.eta_min;
    const bool cand = high && !elong;
    st.mask[i] = (uint8_t)((high ? 1 : 0) | (elong ? 2 : 0) | (cand ? 4 : 0) | (lp ? 8 : 0));
    if (nvis) atomicAdd(&cnt_s[0], nvis);
    if (high) atomicAdd(&cnt_s[1], 1u);
    if (elong) atomicAdd(&cnt_s[2], 1u);
    if (high && elong) atomicAdd(&cnt_s[3], 1u);
    if (nlp) atomicAdd(&cnt_s[4], nlp);
    if (cand) atomicAdd(&cnt_s[5], 1u);
  }
  __syncthreads();
  if (threadIdx.x < kCounters) cpart[(int64_t)blockIdx.x * kCounters + threadIdx.x] = cnt_s[threadIdx.x];
}

constexpr int kCBlock = 1024;

__global__ __launch_bounds__(kCBlock) void k_count_final(const uint32_t* __restrict__ cpart, int nblocks,
                                                         uint32_t* __restrict__ counters) {
  __shared__ uint32_t red[kCounters][kCBlock / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t a[kCounters] = {0, 0, 0, 0, 0, 0};
#pragma unroll 4
  for (int b = threadIdx.x; b < nblocks; b += kCBlock)
#pragma unroll
    for (int c = 0; c < kCounters; ++c) a[c] += cpart[(int64_t)b * kCounters + c];
#pragma unroll
  for (int c = 0; c < kCounters; ++c) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) a[c] += __shfl_xor(a[c], o, 64);
    if (lane == 0) red[c][w] = a[c];
  }
  __syncthreads();
  if (threadIdx.x < kCounters) {
    uint32_t t = 0;
    for (int q = 0; q < kCBlock / 64; ++q) t += red[threadIdx.x][q];
    counters[threadIdx.x] += t;
  }
}

}  // namespace cgv2

size_t cgv2_densify_ws_layout(int64_t n, int V, size_t* off) {
  // off: [0] scale per view (f32, V), [1] counter partials (u32, 6 per k_densify workgroup); the DGD
  // partial sums (f64) start at 0
  const int64_t nb = (n + cgv2::kDBlock * cgv2::kDItems - 1) / (cgv2::kDBlock * cgv2::kDItems);
  const int64_t nbd = (n + cgv2::kDBlock - 1) / cgv2::kDBlock;
  off[0] = ((size_t)(2 * sizeof(double) * (size_t)(nb > 0 ? nb : 1) * V + 255) & ~(size_t)255);
  off[1] = off[0] + (((size_t)V * sizeof(float) + 255) & ~(size_t)255);
  return off[1] + (((size_t)cgv2::kCounters * sizeof(uint32_t) * (size_t)(nbd > 0 ? nbd : 1) + 255) & ~(size_t)255);
}

hipError_t cgv2_launch_densify(const cgv2_surfels& s, const cgv2_proj& p, const cgv2_grads& g, int V,
                               const cgv2_densify_params& prm, const cgv2_densify_state& st, void* ws,
                               hipStream_t stream) {
  const int64_t n = s.n;
  const int nb = (int)((n + cgv2::kDBlock * cgv2::kDItems - 1) / (cgv2::kDBlock * cgv2::kDItems));
  const int nbp = nb > 0 ? nb : 1;
  size_t off[kDensifyOffs];
  cgv2_densify_ws_layout(n, V, off);
  double* partial = (double*)ws;
  float* scale_ws = (float*)((char*)ws + off[0]);
  uint32_t* cpart = (uint32_t*)((char*)ws + off[1]);
  hipLaunchKernelGGL(cgv2::k_dgd_partial, dim3((unsigned)nbp, (unsigned)V), dim3(cgv2::kDBlock), 0, stream, p.flags,
                     g.g_view_total, g.g_view_ssim, n, partial, nbp, st.counters);
  hipLaunchKernelGGL(cgv2::k_dgd_final, dim3(1), dim3(cgv2::kDBlock), 0, stream, partial, nbp, V, prm.omega, scale_ws,
                     st.scale);
  if (n > 0) {
    const int nbd = (int)((n + cgv2::kDBlock - 1) / cgv2::kDBlock);
    hipLaunchKernelGGL(cgv2::k_densify, dim3((unsigned)nbd), dim3(cgv2::kDBlock), 0, stream, s, p.flags, p.radius,
                       g.g_view_total, g.g_view_ssim, V, scale_ws, prm, st, cpart);
    hipLaunchKernelGGL(cgv2::k_count_final, dim3(1), dim3(cgv2::kCBlock), 0, stream, cpart, nbd, st.counters);
  }
  return hipGetLastError();
}

// ---- fixed device buffer of cgv2_densify_stats_noalloc ------------------------------------------
// One array per GPU, held until the process ends.  Host code never uses the array's name (on the host
// it is a stand-in, not a device address): the first call on each device looks its address up with that
// device current and keeps it.
static __device__ __align__(256) unsigned char scratch[CGV2_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::atomic<void*> g_scratch_ptr[kMaxDevices];
}  // namespace

hipError_t cgv2_densify_scratch(void** ptr) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  void* p = g_scratch_ptr[dev].load(std::memory_order_acquire);
  if (!p) {
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev].store(p, std::memory_order_release);
  }
  *ptr = p;
  return hipSuccess;
}
