// Photometric loss of CityGaussianV2 Sec. 3.1: L = (1 - lambda) L1 + lambda (1 - SSIM), with the
// SSIM-only part of the gradient kept apart as the source of the decomposed densification
// gradient (Sec. 3.2, Eq. 2).
//
// SSIM (Wang et al. 2004): 11x11 separable Gaussian window (sigma 1.5), zero padding,
// C1 = 0.01^2, C2 = 0.03^2.  Both kernels run one wave per strip of 64 columns x kStripH rows of one
// image plane and walk down the strip: each input row (the 64 columns and a 5-column halo on either
// side) goes through LDS once, its 11-tap horizontal sums enter a ring of the last 11 rows held in
// registers, and each new row completes the vertical sums of one output row -- the only recomputation
// is the 10-row halo at the strip's top.  The forward kernel computes the five local moments, the SSIM
// map and its three partial derivatives (w.r.t. the local mean, E[x^2] and E[xy]) and deterministic
// per-wave sums; the backward kernel correlates the three partial maps with the same window and
// combines them with the L1 sign into dL/dI and d(lambda (1 - SSIM))/dI.
#include "cgv2r_device.h"
#include "cgv2r_kernels.h"

namespace cgv2 {

constexpr int kR = 5;
constexpr int kTaps = 2 * kR + 1;       // 11
constexpr int kStripW = 64;             // output columns per wave (one per lane)
constexpr int kAhead = 2;               // rows loaded ahead of the one in use (queue slot = row % 2)
constexpr int kLoops = 2;               // row loop iterations of 22 rows after the first 11
constexpr int kInRows = kTaps + 2 * kTaps * kLoops;  // 55 input rows per strip
constexpr int kStripH = kInRows - 2 * kR;            // 45 output rows per wave
constexpr int kRowW = kStripW + 2 * kR;
constexpr float kC1 = 0.0001f, kC2 = 0.0009f;

struct Win { float g[kTaps]; };

// Block -> (strip column, strip row, plane vc = v * 3 + channel).
struct StripGrid {
  int nx, ny;
};

// Hardware sends workgroup b to XCD b % 8: XCD x takes the x-th contiguous eighth of the strips (row-major
// over strip columns, then strip rows, then planes), so the halo columns and rows that neighbouring
// strips share are fetched into one L2.  Blocks past the last full round of 8 map to themselves.
// Returns the strip index (the slot of its per-wave sums).
__device__ __forceinline__ int strip_of_block(const StripGrid& sg, int& x0, int& y0, int& vc) {
  const uint32_t nb = gridDim.x, full = nb - nb % 8u, bb = blockIdx.x;
  const int b = (int)(bb < full ? (bb % 8u) * (full / 8u) + bb / 8u : bb);
  const int r = b / sg.nx;
  x0 = (b - r * sg.nx) * kStripW;
  y0 = (r % sg.ny) * kStripH;
  vc = r / sg.ny;
  return b;
}

// Orders a wave's own LDS writes and reads (the workgroup is that one wave, and a wave's LDS operations
// execute in program order): a compiler barrier only.  __syncthreads() would also wait for every
// outstanding global store of the wave, putting the output rows' store latency on the row loop.
__device__ __forceinline__ void wave_lds_order() {
  __builtin_amdgcn_sched_barrier(0);  // also keeps the scheduler from hoisting later rows' loads (registers)
  __builtin_amdgcn_wave_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Loads and stores through buffer resources: an offset past the plane's end (kDrop) reads 0 (the zero
// padding of the window) and drops a store (an output outside the image), so the row loop has no
// branches and its only waits are for the loads of the row it is about to use, not for earlier stores.
constexpr uint32_t kDrop = 0xfffffff0u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const float* base, int64_t floats) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), (short)0, (int)(floats * 4), 0x00020000);
}
__device__ __forceinline__ float load_or_zero(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
}
__device__ __forceinline__ void store_or_drop(__amdgpu_buffer_rsrc_t r, float v, uint32_t byte_off) {
  // the builtin stores a 32-bit integer: pass the float's bits, not its value
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, byte_off, 0, 0);
}

// Byte offsets of row yy at columns x0 - 5 + lane (a) and x0 + 59 + lane for lane < 10 (b), kDrop
// outside the image (or for a row past the strip, live = false).
__device__ __forceinline__ void row_offsets(int W, int H, int x0, int yy, int lane, bool live, uint32_t& a,
                                            uint32_t& b) {
  const bool row = live && yy >= 0 && yy < H;
  const int c0 = x0 - kR + lane, c1 = x0 - kR + kStripW + lane;
  a = (row && c0 >= 0 && c0 < W) ? (uint32_t)((int64_t)yy * W + c0) * 4u : kDrop;
  b = (row && lane < 2 * kR && c1 < W) ? (uint32_t)((int64_t)yy * W + c1) * 4u : kDrop;
}

// Vertical sum of ring slot values for the output whose newest input row sits in slot j (oldest first).
template <int N, int J>
__device__ __forceinline__ void vsum(const float (&ring)[kTaps][N], const Win& win, float (&o)[N]) {
#pragma unroll
  for (int q = 0; q < N; ++q) o[q] = 0.f;
#pragma unroll
  for (int b = 0; b < kTaps; ++b) {
    const int k = (J + 1 + b) % kTaps;
#pragma unroll
    for (int q = 0; q < N; ++q) o[q] = fmaf(win.g[b], ring[k][q], o[q]);
  }
}

struct FwdStrip {
  __amdgpu_buffer_rsrc_t rx, ry, rm;
  int W, H, x0, y0, lane;
  int64_t HW;
  float xa[kAhead], xb[kAhead], ya[kAhead], yb[kAhead];  // the next kAhead rows, oldest first
  float ring[kTaps][5];  // horizontal sums of the last 11 input rows, slot = row % 11
  float cx[kTaps], cy[kTaps];  // the lane's own column of those rows
  double m_sum, l1_sum;
};

// Loads input row rn of the strip into queue slot Q.
template <int Q>
__device__ __forceinline__ void fwd_load(FwdStrip& f, int rn) {
  uint32_t oa, ob;
  row_offsets(f.W, f.H, f.x0, f.y0 - kR + rn, f.lane, rn < kInRows, oa, ob);
  f.xa[Q] = load_or_zero(f.rx, oa);
  f.xb[Q] = load_or_zero(f.rx, ob);
  f.ya[Q] = load_or_zero(f.ry, oa);
  f.yb[Q] = load_or_zero(f.ry, ob);
}

template <int J, int Q>
__device__ __forceinline__ void fwd_row(FwdStrip& f, float* sx, float* sy, const Win& win, int r) {
  // r = input row index within the strip (y0 - 5 + r): ring slot J = r % 11, queue slot Q = r % 2
  wave_lds_order();  // the previous row is no longer read
  sx[f.lane] = f.xa[Q];
  sy[f.lane] = f.ya[Q];
  if (f.lane < 2 * kR) {
    sx[kStripW + f.lane] = f.xb[Q];
    sy[kStripW + f.lane] = f.yb[Q];
  }
  wave_lds_order();
  fwd_load<Q>(f, r + kAhead);  // the slot is free again: the row two ahead
  float m0 = 0, m1 = 0, m2 = 0, m3 = 0, m4 = 0;
#pragma unroll
  for (int a = 0; a < kTaps; ++a) {
    const float xv = sx[f.lane + a], yv = sy[f.lane + a], g = win.g[a];
    m0 = fmaf(g, xv, m0);
    m1 = fmaf(g, yv, m1);
    m2 = fmaf(g, xv * xv, m2);
    m3 = fmaf(g, yv * yv, m3);
    m4 = fmaf(g, xv * yv, m4);
  }
  f.ring[J][0] = m0; f.ring[J][1] = m1; f.ring[J][2] = m2; f.ring[J][3] = m3; f.ring[J][4] = m4;
  f.cx[J] = sx[f.lane + kR];
  f.cy[J] = sy[f.lane + kR];
}

// Output row y0 + r - 10 from the ring (its newest input row in slot J).
template <int J>
__device__ __forceinline__ void fwd_out(FwdStrip& f, const Win& win, int r) {
  float v[5];
  vsum<5, J>(f.ring, win, v);
  const float mx = v[0], my = v[1], exx = v[2], eyy = v[3], exy = v[4];
  const int px = f.x0 + f.lane, py = f.y0 + r - 2 * kR;
  const bool in = px < f.W && py < f.H;
  const float sxx = exx - mx * mx, syy = eyy - my * my, sxy = exy - mx * my;
  const float A1 = 2.f * mx * my + kC1, A2 = 2.f * sxy + kC2;
  const float B1 = mx * mx + my * my + kC1, B2 = sxx + syy + kC2;
  // single-precision reciprocals (1 ulp) in place of IEEE divisions
  const float iB1 = __builtin_amdgcn_rcpf(B1), iB2 = __builtin_amdgcn_rcpf(B2);
  const float iB = iB1 * iB2;
  const float m = A1 * A2 * iB;
  const uint32_t o = (uint32_t)((int64_t)py * f.W + px) * 4u, hw = (uint32_t)f.HW * 4u;
  store_or_drop(f.rm, 2.f * my * (A2 - A1) * iB - 2.f * m * mx * (iB1 - iB2), in ? o : kDrop);
  store_or_drop(f.rm, -m * iB2, in ? o + hw : kDrop);
  store_or_drop(f.rm, 2.f * A1 * iB, in ? o + 2u * hw : kDrop);
  // the centre pixel is input row r - 5: slot J + 6 (mod 11)
  constexpr int kc = (J + kR + 1) % kTaps;
  f.m_sum += in ? (double)m : 0.0;
  f.l1_sum += in ? (double)fabsf(f.cx[kc] - f.cy[kc]) : 0.0;
}

template <int J, int Q>
__device__ __forceinline__ void fwd_step(FwdStrip& f, float* sx, float* sy, const Win& win, int r, bool out) {
  fwd_row<J, Q>(f, sx, sy, win, r);
  if (out) fwd_out<J>(f, win, r);
}

__global__ __launch_bounds__(64) void k_ssim_fwd(const float* __restrict__ img, const float* __restrict__ tgt, int W,
                                                 int H, Win win, StripGrid sg, float* __restrict__ maps,
                                                 double* __restrict__ partial) {
  __shared__ float sx[kRowW], sy[kRowW];
  FwdStrip f;
  int vc;
  const int strip = strip_of_block(sg, f.x0, f.y0, vc);
  f.W = W;
  f.H = H;
  f.lane = (int)threadIdx.x;
  f.HW = (int64_t)W * H;
  f.rx = plane_rsrc(img + vc * f.HW, f.HW);
  f.ry = plane_rsrc(tgt + vc * f.HW, f.HW);
  f.rm = plane_rsrc(maps + (int64_t)vc * 3 * f.HW, 3 * f.HW);
  f.m_sum = f.l1_sum = 0.0;
  fwd_load<0>(f, 0);
  fwd_load<1>(f, 1);
  // rows 0..10 fill the ring (the first output comes with row 10), then 22 rows per iteration, one output
  // each; the ring slot is row % 11 and the queue slot row % 2, both fixed at every unrolled position
  fwd_step<0, 0>(f, sx, sy, win, 0, false);
  fwd_step<1, 1>(f, sx, sy, win, 1, false);
  fwd_step<2, 0>(f, sx, sy, win, 2, false);
  fwd_step<3, 1>(f, sx, sy, win, 3, false);
  fwd_step<4, 0>(f, sx, sy, win, 4, false);
  fwd_step<5, 1>(f, sx, sy, win, 5, false);
  fwd_step<6, 0>(f, sx, sy, win, 6, false);
  fwd_step<7, 1>(f, sx, sy, win, 7, false);
  fwd_step<8, 0>(f, sx, sy, win, 8, false);
  fwd_step<9, 1>(f, sx, sy, win, 9, false);
  fwd_step<10, 0>(f, sx, sy, win, 10, true);
#pragma nounroll
  for (int r0 = kTaps; r0 < kInRows; r0 += 2 * kTaps) {
    fwd_step<0, 1>(f, sx, sy, win, r0 + 0, true);
    fwd_step<1, 0>(f, sx, sy, win, r0 + 1, true);
    fwd_step<2, 1>(f, sx, sy, win, r0 + 2, true);
    fwd_step<3, 0>(f, sx, sy, win, r0 + 3, true);
    fwd_step<4, 1>(f, sx, sy, win, r0 + 4, true);
    fwd_step<5, 0>(f, sx, sy, win, r0 + 5, true);
    fwd_step<6, 1>(f, sx, sy, win, r0 + 6, true);
    fwd_step<7, 0>(f, sx, sy, win, r0 + 7, true);
    fwd_step<8, 1>(f, sx, sy, win, r0 + 8, true);
    fwd_step<9, 0>(f, sx, sy, win, r0 + 9, true);
    fwd_step<10, 1>(f, sx, sy, win, r0 + 10, true);
    fwd_step<0, 0>(f, sx, sy, win, r0 + 11, true);
    fwd_step<1, 1>(f, sx, sy, win, r0 + 12, true);
    fwd_step<2, 0>(f, sx, sy, win, r0 + 13, true);
    fwd_step<3, 1>(f, sx, sy, win, r0 + 14, true);
    fwd_step<4, 0>(f, sx, sy, win, r0 + 15, true);
    fwd_step<5, 1>(f, sx, sy, win, r0 + 16, true);
    fwd_step<6, 0>(f, sx, sy, win, r0 + 17, true);
    fwd_step<7, 1>(f, sx, sy, win, r0 + 18, true);
    fwd_step<8, 0>(f, sx, sy, win, r0 + 19, true);
    fwd_step<9, 1>(f, sx, sy, win, r0 + 20, true);
    fwd_step<10, 0>(f, sx, sy, win, r0 + 21, true);
  }
  // per-wave sums in FP64, fixed order (butterfly)
  double m_sum = f.m_sum, l1_sum = f.l1_sum;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    m_sum += __shfl_xor(m_sum, o, 64);
    l1_sum += __shfl_xor(l1_sum, o, 64);
  }
  if (f.lane == 0) {
    partial[2 * (int64_t)strip] = m_sum;
    partial[2 * (int64_t)strip + 1] = l1_sum;
  }
}

struct BwdStrip {
  __amdgpu_buffer_rsrc_t rm, rx, ry, rs, ri;
  int W, H, x0, y0, lane;
  int64_t HW;
  float ninv, lambda;
  float va[kAhead][3], vb[kAhead][3];  // the next kAhead rows of the three maps, oldest first
  float xv[kAhead], yv[kAhead];        // image and target at those rows' output pixels
  float ring[kTaps][3];
};

// Loads input row rn of the strip (three maps) and the image / target at its output pixel into slot k.
template <int k>
__device__ __forceinline__ void bwd_load(BwdStrip& f, int rn) {
  uint32_t oa, ob;
  row_offsets(f.W, f.H, f.x0, f.y0 - kR + rn, f.lane, rn < kInRows, oa, ob);
  const uint32_t hw = (uint32_t)f.HW * 4u;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    f.va[k][q] = load_or_zero(f.rm, oa == kDrop ? kDrop : oa + (uint32_t)q * hw);
    f.vb[k][q] = load_or_zero(f.rm, ob == kDrop ? kDrop : ob + (uint32_t)q * hw);
  }
  const int px = f.x0 + f.lane, pyn = f.y0 + rn - 2 * kR;
  const bool ok = rn >= 2 * kR && rn < kInRows && px < f.W && pyn < f.H;
  const uint32_t on = ok ? (uint32_t)((int64_t)pyn * f.W + px) * 4u : kDrop;
  f.xv[k] = load_or_zero(f.rx, on);
  f.yv[k] = load_or_zero(f.ry, on);
}

template <int J, int Q>
__device__ __forceinline__ void bwd_step(BwdStrip& f, float (*sm)[kRowW], const Win& win, int r, bool out) {
  wave_lds_order();
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    sm[q][f.lane] = f.va[Q][q];
    if (f.lane < 2 * kR) sm[q][kStripW + f.lane] = f.vb[Q][q];
  }
  wave_lds_order();
  const float xc = f.xv[Q], yc = f.yv[Q];  // this row's output pixel
  bwd_load<Q>(f, r + kAhead);
  float m0 = 0, m1 = 0, m2 = 0;
#pragma unroll
  for (int a = 0; a < kTaps; ++a) {
    const float g = win.g[a];
    m0 = fmaf(g, sm[0][f.lane + a], m0);
    m1 = fmaf(g, sm[1][f.lane + a], m1);
    m2 = fmaf(g, sm[2][f.lane + a], m2);
  }
  f.ring[J][0] = m0; f.ring[J][1] = m1; f.ring[J][2] = m2;
  if (!out) return;
  float sv[3];
  vsum<3, J>(f.ring, win, sv);
  const int px = f.x0 + f.lane, py = f.y0 + r - 2 * kR;
  const bool in = px < f.W && py < f.H;
  const uint32_t o = in ? (uint32_t)((int64_t)py * f.W + px) * 4u : kDrop;
  const float dssim = f.ninv * (sv[0] + 2.f * xc * sv[1] + yc * sv[2]);
  const float d = xc - yc;
  const float sgn = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
  store_or_drop(f.rs, -f.lambda * dssim, o);
  store_or_drop(f.ri, (1.f - f.lambda) * sgn * f.ninv - f.lambda * dssim, o);
}

__device__ __noinline__ void loss_final(const double* __restrict__ partial, int64_t blocks_per_view, int V, int64_t HW,
                                        float lambda, float* __restrict__ loss);

__global__ __launch_bounds__(64) void k_ssim_bwd(const float* __restrict__ img, const float* __restrict__ tgt, int W,
                                                 int H, Win win, StripGrid sg, float lambda,
                                                 const float* __restrict__ maps, float* __restrict__ d_img,
                                                 float* __restrict__ d_ssim, const double* __restrict__ partial,
                                                 int V, float* __restrict__ loss) {
  __shared__ float sm[3][kRowW];
  if (blockIdx.x == 0) loss_final(partial, (int64_t)sg.nx * sg.ny * 3, V, (int64_t)W * H, lambda, loss);
  BwdStrip f;
  int vc;
  strip_of_block(sg, f.x0, f.y0, vc);
  f.W = W;
  f.H = H;
  f.lane = (int)threadIdx.x;
  f.HW = (int64_t)W * H;
  f.ninv = 1.f / (3.f * (float)f.HW);
  f.lambda = lambda;
  f.rm = plane_rsrc(maps + (int64_t)vc * 3 * f.HW, 3 * f.HW);
  f.rx = plane_rsrc(img + vc * f.HW, f.HW);
  f.ry = plane_rsrc(tgt + vc * f.HW, f.HW);
  f.rs = plane_rsrc(d_ssim + vc * f.HW, f.HW);
  f.ri = plane_rsrc(d_img + vc * f.HW, f.HW);
  bwd_load<0>(f, 0);
  bwd_load<1>(f, 1);
  bwd_step<0, 0>(f, sm, win, 0, false);
  bwd_step<1, 1>(f, sm, win, 1, false);
  bwd_step<2, 0>(f, sm, win, 2, false);
  bwd_step<3, 1>(f, sm, win, 3, false);
  bwd_step<4, 0>(f, sm, win, 4, false);
  bwd_step<5, 1>(f, sm, win, 5, false);
  bwd_step<6, 0>(f, sm, win, 6, false);
  bwd_step<7, 1>(f, sm, win, 7, false);
  bwd_step<8, 0>(f, sm, win, 8, false);
  bwd_step<9, 1>(f, sm, win, 9, false);
  bwd_step<10, 0>(f, sm, win, 10, true);
#pragma nounroll
  for (int r0 = kTaps; r0 < kInRows; r0 += 2 * kTaps) {
    bwd_step<0, 1>(f, sm, win, r0 + 0, true);
    bwd_step<1, 0>(f, sm, win, r0 + 1, true);
    bwd_step<2, 1>(f, sm, win, r0 + 2, true);
    bwd_step<3, 0>(f, sm, win, r0 + 3, true);
    bwd_step<4, 1>(f, sm, win, r0 + 4, true);
    bwd_step<5, 0>(f, sm, win, r0 + 5, true);
    bwd_step<6, 1>(f, sm, win, r0 + 6, true);
    bwd_step<7, 0>(f, sm, win, r0 + 7, true);
    bwd_step<8, 1>(f, sm, win, r0 + 8, true);
    bwd_step<9, 0>(f, sm, win, r0 + 9, true);
    bwd_step<10, 1>(f, sm, win, r0 + 10, true);
    bwd_step<0, 0>(f, sm, win, r0 + 11, true);
    bwd_step<1, 1>(f, sm, win, r0 + 12, true);
    bwd_step<2, 0>(f, sm, win, r0 + 13, true);
    bwd_step<3, 1>(f, sm, win, r0 + 14, true);
    bwd_step<4, 0>(f, sm, win, r0 + 15, true);
    bwd_step<5, 1>(f, sm, win, r0 + 16, true);
    bwd_step<6, 0>(f, sm, win, r0 + 17, true);
    bwd_step<7, 1>(f, sm, win, r0 + 18, true);
    bwd_step<8, 0>(f, sm, win, r0 + 19, true);
    bwd_step<9, 1>(f, sm, win, r0 + 20, true);
    bwd_step<10, 0>(f, sm, win, r0 + 21, true);
  }
}

// The loss values of every view from the forward's per-wave sums, in a fixed order: run by the first
// workgroup of k_ssim_bwd (the forward has completed by then).
__device__ __noinline__ void loss_final(const double* __restrict__ partial, int64_t blocks_per_view, int V, int64_t HW,
                                        float lambda, float* __restrict__ loss) {
  const int lane = (int)threadIdx.x;
  for (int v = 0; v < V; ++v) {
    double a = 0, b = 0;
    const double2* pv = (const double2*)partial + v * blocks_per_view;
#pragma unroll 4
    for (int64_t k = lane; k < blocks_per_view; k += 64) {
      const double2 q = pv[k];
      a += q.x;
      b += q.y;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      a += __shfl_xor(a, o, 64);
      b += __shfl_xor(b, o, 64);
    }
    if (lane == 0) {
      const double ssim = a / (3.0 * HW), l1 = b / (3.0 * HW);
      loss[3 * v] = (float)((1.0 - lambda) * l1 + lambda * (1.0 - ssim));
      loss[3 * v + 1] = (float)l1;
      loss[3 * v + 2] = (float)ssim;
    }
  }
}

}  // namespace cgv2

size_t cgv2_loss_ws_layout(int W, int H, int V, size_t* off) {
  const int64_t nx = (W + cgv2::kStripW - 1) / cgv2::kStripW, ny = (H + cgv2::kStripH - 1) / cgv2::kStripH;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o += (bytes + 255) & ~(size_t)255; return r; };
  off[0] = take(sizeof(float) * 9 * (size_t)W * H * V);     // partial maps [V][3][3][H][W]
  off[1] = take(sizeof(double) * 2 * (size_t)(nx * ny * 3 * V));  // per-wave sums
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
  cgv2::StripGrid sg;
  sg.nx = (W + cgv2::kStripW - 1) / cgv2::kStripW;
  sg.ny = (H + cgv2::kStripH - 1) / cgv2::kStripH;
  const unsigned blocks = (unsigned)(sg.nx * sg.ny * 3 * V);
  hipLaunchKernelGGL(cgv2::k_ssim_fwd, dim3(blocks), dim3(64), 0, st, img, tgt, W, H, win, sg, maps, partial);
  hipLaunchKernelGGL(cgv2::k_ssim_bwd, dim3(blocks), dim3(64), 0, st, img, tgt, W, H, win, sg, lambda, maps, d_img,
                     d_ssim, partial, V, loss);
  return hipGetLastError();
}
