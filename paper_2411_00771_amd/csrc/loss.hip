// Photometric loss of CityGaussianV2 Sec. 3.1: L = (1 - lambda) L1 + lambda (1 - SSIM), with the
// SSIM-only part of the gradient kept apart as the source of the decomposed densification
// gradient (Sec. 3.2, Eq. 2).
//
// SSIM (Wang et al. 2004): 11x11 separable Gaussian window (sigma 1.5), zero padding,
// C1 = 0.01^2, C2 = 0.03^2.  The forward kernel computes the five local moments of each 16x16
// output tile from a 26x26 LDS tile (two separable passes), the SSIM map and its three partial
// derivatives (w.r.t. the local mean, E[x^2] and E[xy]) and deterministic per-block sums.  The
// backward kernel correlates the three partial maps with the same window and combines them with
// the L1 sign into dL/dI and d(lambda (1 - SSIM))/dI.
#include "cgv2r_device.h"
#include "cgv2r_kernels.h"

namespace cgv2 {

constexpr int kR = 5;
constexpr int kSide = kTile + 2 * kR;  // 26
constexpr float kC1 = 0.0001f, kC2 = 0.0009f;

struct Win { float g[11]; };

// Block -> (tile x, tile y, plane).  Hardware sends block b to XCD b % 8; XCD x takes the column band
// [x * band, (x + 1) * band) of every plane, row by row, so the halos that neighbouring tiles share
// (left/right and above/below) are read through one L2.  Blocks past the right edge do nothing.
struct LossGrid {
  int tx, ty, band;
};

__device__ __forceinline__ bool loss_tile(const LossGrid& lg, int& bx, int& by, int& vc) {
  const uint32_t b = blockIdx.x;
  const uint32_t x = b % 8u, k = b / 8u;
  const uint32_t per_plane = (uint32_t)(lg.band * lg.ty);
  vc = (int)(k / per_plane);
  const uint32_t r = k % per_plane;
  by = (int)(r / (uint32_t)lg.band);
  bx = (int)(x * (uint32_t)lg.band + r % (uint32_t)lg.band);
  return bx < lg.tx;
}

__device__ __forceinline__ float at(const float* p, int W, int H, int x, int y) {
  return (x >= 0 && x < W && y >= 0 && y < H) ? p[(int64_t)y * W + x] : 0.f;
}

__global__ __launch_bounds__(256) void k_ssim_fwd(const float* __restrict__ img, const float* __restrict__ tgt, int W,
                                                  int H, Win win, LossGrid lg, float* __restrict__ maps,
                                                  double* __restrict__ partial) {
  __shared__ float sx[kSide][kSide], sy[kSide][kSide];
  __shared__ float hs[5][kSide][kTile];
  __shared__ double red[2][4];
  int bx, by, vc;  // vc = v * 3 + channel
  if (!loss_tile(lg, bx, by, vc)) return;
  const int64_t HW = (int64_t)W * H;
  const float* X = img + vc * HW;
  const float* Y = tgt + vc * HW;
  const int ox = bx * kTile - kR, oy = by * kTile - kR;
  for (int k = threadIdx.x; k < kSide * kSide; k += 256) {
    const int ly = k / kSide, lx = k % kSide;
    sx[ly][lx] = at(X, W, H, ox + lx, oy + ly);
    sy[ly][lx] = at(Y, W, H, ox + lx, oy + ly);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kSide * kTile; k += 256) {
    const int ly = k / kTile, lx = k % kTile;
    float m0 = 0, m1 = 0, m2 = 0, m3 = 0, m4 = 0;
#pragma unroll
    for (int a = 0; a < 11; ++a) {
      const float xv = sx[ly][lx + a], yv = sy[ly][lx + a], g = win.g[a];
      m0 = fmaf(g, xv, m0);
      m1 = fmaf(g, yv, m1);
      m2 = fmaf(g, xv * xv, m2);
      m3 = fmaf(g, yv * yv, m3);
      m4 = fmaf(g, xv * yv, m4);
    }
    hs[0][ly][lx] = m0; hs[1][ly][lx] = m1; hs[2][ly][lx] = m2; hs[3][ly][lx] = m3; hs[4][ly][lx] = m4;
  }
  __syncthreads();
  const int lx = threadIdx.x % kTile, ly = threadIdx.x / kTile;
  float mx = 0, my = 0, exx = 0, eyy = 0, exy = 0;
#pragma unroll
  for (int b = 0; b < 11; ++b) {
    const float g = win.g[b];
    mx = fmaf(g, hs[0][ly + b][lx], mx);
    my = fmaf(g, hs[1][ly + b][lx], my);
    exx = fmaf(g, hs[2][ly + b][lx], exx);
    eyy = fmaf(g, hs[3][ly + b][lx], eyy);
    exy = fmaf(g, hs[4][ly + b][lx], exy);
  }
  const int px = bx * kTile + lx, py = by * kTile + ly;
  double m_sum = 0, l1_sum = 0;
  if (px < W && py < H) {
    const float sxx = exx - mx * mx, syy = eyy - my * my, sxy = exy - mx * my;
    const float A1 = 2.f * mx * my + kC1, A2 = 2.f * sxy + kC2;
    const float B1 = mx * mx + my * my + kC1, B2 = sxx + syy + kC2;
    const float iB = 1.f / (B1 * B2);
    const float m = A1 * A2 * iB;
    const int64_t p = (int64_t)py * W + px;
    float* mp = maps + (int64_t)vc * 3 * HW + p;
    mp[0] = 2.f * my * (A2 - A1) * iB - 2.f * m * mx * (1.f / B1 - 1.f / B2);
    mp[HW] = -m / B2;
    mp[2 * HW] = 2.f * A1 * iB;
    m_sum = m;
    l1_sum = fabsf(sx[ly + kR][lx + kR] - sy[ly + kR][lx + kR]);
  }
  // per-block sums in FP64, fixed order: butterfly within each wave, then the four waves in order
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    m_sum += __shfl_xor(m_sum, o, 64);
    l1_sum += __shfl_xor(l1_sum, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = m_sum;
    red[1][threadIdx.x >> 6] = l1_sum;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int64_t blk = ((int64_t)vc * lg.ty + by) * lg.tx + bx;
    partial[2 * blk] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    partial[2 * blk + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  }
}

__global__ __launch_bounds__(256) void k_ssim_bwd(const float* __restrict__ img, const float* __restrict__ tgt, int W,
                                                  int H, Win win, LossGrid lg, float lambda,
                                                  const float* __restrict__ maps, float* __restrict__ d_img,
                                                  float* __restrict__ d_ssim) {
  __shared__ float sm[3][kSide][kSide];
  __shared__ float hs[3][kSide][kTile];
  int bx, by, vc;
  if (!loss_tile(lg, bx, by, vc)) return;
  const int64_t HW = (int64_t)W * H;
  const float* Mp = maps + (int64_t)vc * 3 * HW;
  const int ox = bx * kTile - kR, oy = by * kTile - kR;
  for (int k = threadIdx.x; k < kSide * kSide; k += 256) {
    const int ly = k / kSide, lx = k % kSide;
    sm[0][ly][lx] = at(Mp, W, H, ox + lx, oy + ly);
    sm[1][ly][lx] = at(Mp + HW, W, H, ox + lx, oy + ly);
    sm[2][ly][lx] = at(Mp + 2 * HW, W, H, ox + lx, oy + ly);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kSide * kTile; k += 256) {
    const int ly = k / kTile, lx = k % kTile;
    float m0 = 0, m1 = 0, m2 = 0;
#pragma unroll
    for (int a = 0; a < 11; ++a) {
      const float g = win.g[a];
      m0 = fmaf(g, sm[0][ly][lx + a], m0);
      m1 = fmaf(g, sm[1][ly][lx + a], m1);
      m2 = fmaf(g, sm[2][ly][lx + a], m2);
    }
    hs[0][ly][lx] = m0; hs[1][ly][lx] = m1; hs[2][ly][lx] = m2;
  }
  __syncthreads();
  const int lx = threadIdx.x % kTile, ly = threadIdx.x / kTile;
  const int px = bx * kTile + lx, py = by * kTile + ly;
  if (!(px < W && py < H)) return;
  float s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
  for (int b = 0; b < 11; ++b) {
    const float g = win.g[b];
    s0 = fmaf(g, hs[0][ly + b][lx], s0);
    s1 = fmaf(g, hs[1][ly + b][lx], s1);
    s2 = fmaf(g, hs[2][ly + b][lx], s2);
  }
  const int64_t p = (int64_t)vc * HW + (int64_t)py * W + px;
  const float xv = img[p], yv = tgt[p];
  const float ninv = 1.f / (3.f * (float)HW);
  const float dssim = ninv * (s0 + 2.f * xv * s1 + yv * s2);
  const float d = xv - yv;
  const float sgn = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
  d_ssim[p] = -lambda * dssim;
  d_img[p] = (1.f - lambda) * sgn * ninv - lambda * dssim;
}

__global__ __launch_bounds__(256) void k_loss_final(const double* __restrict__ partial, int64_t blocks_per_view,
                                                    int V, int64_t HW, float lambda, float* __restrict__ loss) {
  __shared__ double red[2][256];
  for (int v = 0; v < V; ++v) {
    // fixed summation order per thread; unrolled so that eight loads are in flight
    double a = 0, b = 0;
    const double2* pv = (const double2*)partial + v * blocks_per_view;
#pragma unroll 8
    for (int64_t k = threadIdx.x; k < blocks_per_view; k += 256) {
      const double2 q = pv[k];
      a += q.x;
      b += q.y;
    }
    red[0][threadIdx.x] = a;
    red[1][threadIdx.x] = b;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) {
        red[0][threadIdx.x] += red[0][threadIdx.x + off];
        red[1][threadIdx.x] += red[1][threadIdx.x + off];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const double ssim = red[0][0] / (3.0 * HW), l1 = red[1][0] / (3.0 * HW);
      loss[3 * v] = (float)((1.0 - lambda) * l1 + lambda * (1.0 - ssim));
      loss[3 * v + 1] = (float)l1;
      loss[3 * v + 2] = (float)ssim;
    }
    __syncthreads();
  }
}

}  // namespace cgv2

size_t cgv2_loss_ws_layout(int W, int H, int V, size_t* off) {
  const int64_t bx = (W + 15) / 16, by = (H + 15) / 16;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o += (bytes + 255) & ~(size_t)255; return r; };
  off[0] = take(sizeof(float) * 9 * (size_t)W * H * V);     // partial maps [V][3][3][H][W]
  off[1] = take(sizeof(double) * 2 * (size_t)(bx * by * 3 * V));
  return o;
}

hipError_t cgv2_launch_loss(const float* img, const float* tgt, int V, int W, int H, float lambda, float* d_img,
                            float* d_ssim, float* loss, void* ws, hipStream_t st) {
  size_t off[kLossOffs];
  cgv2_loss_ws_layout(W, H, V, off);
  float* maps = (float*)((char*)ws + off[0]);
  double* partial = (double*)((char*)ws + off[1]);
  cgv2::Win win;
  double g[11], gs = 0;
  for (int a = -5; a <= 5; ++a) { g[a + 5] = exp(-(double)(a * a) / (2 * 1.5 * 1.5)); gs += g[a + 5]; }
  for (int a = 0; a < 11; ++a) win.g[a] = (float)(g[a] / gs);
  cgv2::LossGrid lg;
  lg.tx = (W + 15) / 16;
  lg.ty = (H + 15) / 16;
  lg.band = (lg.tx + 7) / 8;
  const unsigned blocks = (unsigned)(8 * lg.band * lg.ty * 3 * V);
  hipLaunchKernelGGL(cgv2::k_ssim_fwd, dim3(blocks), dim3(256), 0, st, img, tgt, W, H, win, lg, maps, partial);
  hipLaunchKernelGGL(cgv2::k_ssim_bwd, dim3(blocks), dim3(256), 0, st, img, tgt, W, H, win, lg, lambda, maps, d_img,
                     d_ssim);
  hipLaunchKernelGGL(cgv2::k_loss_final, dim3(1), dim3(256), 0, st, partial, (int64_t)lg.tx * lg.ty * 3, V,
                     (int64_t)W * H, lambda, loss);
  return hipGetLastError();
}
