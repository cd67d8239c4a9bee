// Tile renderer: forward (Eq. 1 alpha blending of CityGaussianV2 Sec. 3.1, with the depth,
// median-depth and normal renders of Sec. 3.2 / 5.1) and its reverse.
//
// One 64-lane wave per 16x16 tile; each lane owns a 2x2 pixel quad, so every surfel record read
// from LDS (a broadcast) feeds four pixels.  Records of the tile list are staged 64 at a time
// into LDS, one per lane, converting the centre to tile-relative coordinates exactly
// ((cx_hi - tile_x0) + cx_lo).  The wave leaves the list as soon as every pixel has stopped
// (ballot).  The reverse walks each pixel's list from its checkpointed 'last' entry downwards,
// recovers T by division, sums the per-surfel gradients of its four pixels in registers, reduces
// them over the wave and adds them with one set of float atomics per (surfel, tile).
#include "cgv2r_device.h"
#include "cgv2r_kernels.h"

namespace cgv2 {

// LDS record fields (tile-relative centre first)
enum : int { L_CX = 0, L_CY, L_A11, L_A12, L_A21, L_A22, L_W0, L_W1, L_W2, L_ZC, L_OP, L_R, L_G, L_B, L_NX, L_NY,
             L_NZ, L_ZW, L_ID, L_N };

struct RenderArgs {
  const float* rec;
  const uint32_t* ids;
  const uint32_t* ranges;
  const int32_t* status;
  CamPack cams;
  int64_t n;
  int tiles_x, tiles_y, tiles;
  cgv2_image img;
  unsigned long long* counters;
};

__device__ __forceinline__ void stage_record(float (*s)[64], int lane, const float* rec, int64_t vn, int64_t n,
                                             uint32_t id, float ox, float oy) {
  // an id outside [0, n) (never produced by the binning) stages a zero-opacity record
  const bool valid = (int64_t)id < n;
  const float4* r = (const float4*)(rec + (size_t)(vn + (valid ? id : 0u)) * kRec);
  float4 r0 = r[0], r1 = r[1], r2 = r[2], r3 = r[3], r4 = r[4];
  if (!valid) { r3.x = 0.f; id = 0u; }
  s[L_CX][lane] = (r0.x - ox) + r0.z;
  s[L_CY][lane] = (r0.y - oy) + r0.w;
  s[L_A11][lane] = r1.x; s[L_A12][lane] = r1.y; s[L_A21][lane] = r1.z; s[L_A22][lane] = r1.w;
  s[L_W0][lane] = r2.x; s[L_W1][lane] = r2.y; s[L_W2][lane] = r2.z; s[L_ZC][lane] = r2.w;
  s[L_OP][lane] = r3.x; s[L_R][lane] = r3.y; s[L_G][lane] = r3.z; s[L_B][lane] = r3.w;
  s[L_NX][lane] = r4.x; s[L_NY][lane] = r4.y; s[L_NZ][lane] = r4.z;
  s[L_ZW][lane] = r2.w * r2.x;
  s[L_ID][lane] = __uint_as_float(id);
}

template <bool kCount>
__global__ __launch_bounds__(64) void k_render_fwd(RenderArgs a) {
  __shared__ float s[L_N][64];
  const uint32_t b = xcd_remap(blockIdx.x, gridDim.x);
  const int lv = (int)(b / (uint32_t)a.tiles);
  const int v = a.cams.v0 + lv;
  const int t = (int)(b % (uint32_t)a.tiles);
  if (*a.status != 0) return;
  const int tx = t % a.tiles_x, ty = t / a.tiles_x;
  const DevCam& c = a.cams.c[lv];
  const int W = c.W, H = c.H;
  const int lane = threadIdx.x;
  const int qx = lane & 7, qy = lane >> 3;
  const int ox = tx * kTile, oy = ty * kTile;
  const uint32_t start = a.ranges[(int64_t)v * a.tiles + t], end = a.ranges[(int64_t)v * a.tiles + t + 1];
  const int64_t vn = (int64_t)v * a.n;

  float T[4], C[4][3], D[4], Dm[4], N[4][3];
  uint32_t last[4], med[4];
  bool done[4];
  float lx[4], ly[4];
  unsigned long long n_eval = 0, n_con = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int px = ox + 2 * qx + (k & 1), py = oy + 2 * qy + (k >> 1);
    lx[k] = (float)(2 * qx + (k & 1)) + 0.5f;
    ly[k] = (float)(2 * qy + (k >> 1)) + 0.5f;
    done[k] = !(px < W && py < H);
    T[k] = 1.f; D[k] = 0.f; Dm[k] = 0.f; last[k] = start; med[k] = 0xffffffffu;
    C[k][0] = C[k][1] = C[k][2] = 0.f;
    N[k][0] = N[k][1] = N[k][2] = 0.f;
  }
  const float fox = (float)ox, foy = (float)oy;
  for (uint32_t base = start; base < end; base += 64) {
    const bool lane_done = done[0] && done[1] && done[2] && done[3];
    if (__ballot(!lane_done) == 0) break;
    const uint32_t idx = base + lane;
    if (idx < end) stage_record(s, lane, a.rec, vn, a.n, a.ids[idx], fox, foy);
    __syncthreads();
    const int cnt = (int)min(64u, end - base);
    for (int j = 0; j < cnt; ++j) {
      const float cx = s[L_CX][j], cy = s[L_CY][j];
      const float a11 = s[L_A11][j], a12 = s[L_A12][j], a21 = s[L_A21][j], a22 = s[L_A22][j];
      const float w0 = s[L_W0][j], w1 = s[L_W1][j], w2 = s[L_W2][j], op = s[L_OP][j];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        PairEval e;
        eval_pair(lx[k] - cx, ly[k] - cy, a11, a12, a21, a22, w0, w1, w2, op, e);
        if (kCount && !done[k]) ++n_eval;
        if (!done[k] && e.alpha >= kAlphaMin) {
          const float Tn = T[k] * (1.f - e.alpha);
          if (Tn < kTmin) {
            done[k] = true;
          } else {
            if (kCount) ++n_con;
            const float zf = e.is3d ? s[L_ZW][j] * __builtin_amdgcn_rcpf(e.w) : s[L_ZC][j];
            const float wgt = e.alpha * T[k];
            C[k][0] = fmaf(wgt, s[L_R][j], C[k][0]);
            C[k][1] = fmaf(wgt, s[L_G][j], C[k][1]);
            C[k][2] = fmaf(wgt, s[L_B][j], C[k][2]);
            N[k][0] = fmaf(wgt, s[L_NX][j], N[k][0]);
            N[k][1] = fmaf(wgt, s[L_NY][j], N[k][1]);
            N[k][2] = fmaf(wgt, s[L_NZ][j], N[k][2]);
            D[k] = fmaf(wgt, zf, D[k]);
            if (T[k] > 0.5f) { Dm[k] = zf; med[k] = base + (uint32_t)j; }
            T[k] = Tn;
            last[k] = base + (uint32_t)j + 1u;
          }
        }
      }
      if ((j & 15) == 15) {
        const bool ld = done[0] && done[1] && done[2] && done[3];
        if (__ballot(!ld) == 0) break;
      }
    }
    __syncthreads();
  }
  if (kCount) {
    // pairs the reverse pass walks: list entries before 'last'
    unsigned long long n_bwd = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int px = ox + 2 * qx + (k & 1), py = oy + 2 * qy + (k >> 1);
      if (px < W && py < H) n_bwd += last[k] - start;
    }
    atomicAdd(a.counters + 0, n_eval);
    atomicAdd(a.counters + 1, n_con);
    atomicAdd(a.counters + 2, n_bwd);
    return;
  }
  const int64_t HW = (int64_t)W * H;
  const cgv2_image& im = a.img;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int px = ox + 2 * qx + (k & 1), py = oy + 2 * qy + (k >> 1);
    if (!(px < W && py < H)) continue;
    const int64_t p = (int64_t)py * W + px;
    if (im.rgb) {
      float* o = im.rgb + (int64_t)v * 3 * HW + p;
      o[0] = fmaf(T[k], c.bg[0], C[k][0]);
      o[HW] = fmaf(T[k], c.bg[1], C[k][1]);
      o[2 * HW] = fmaf(T[k], c.bg[2], C[k][2]);
    }
    if (im.normal) {
      float* o = im.normal + (int64_t)v * 3 * HW + p;
      o[0] = N[k][0]; o[HW] = N[k][1]; o[2 * HW] = N[k][2];
    }
    const int64_t vp = (int64_t)v * HW + p;
    if (im.depth) im.depth[vp] = D[k];
    if (im.depth_med) im.depth_med[vp] = Dm[k];
    if (im.alpha) im.alpha[vp] = 1.f - T[k];
    if (im.T_final) im.T_final[vp] = T[k];
    if (im.last) im.last[vp] = last[k];
    if (im.med) im.med[vp] = med[k];
  }
}

struct BwdArgs {
  RenderArgs r;
  cgv2_image_grad up;
  float* rg;  // [V][kGradFields][n]
};

__device__ __forceinline__ float ldg0(const float* p, int64_t i) { return p ? p[i] : 0.f; }

__global__ __launch_bounds__(64) void k_render_bwd(BwdArgs A) {
  __shared__ float s[L_N][64];
  const RenderArgs& a = A.r;
  const uint32_t b = xcd_remap(blockIdx.x, gridDim.x);
  const int lv = (int)(b / (uint32_t)a.tiles);
  const int v = a.cams.v0 + lv;
  const int t = (int)(b % (uint32_t)a.tiles);
  if (*a.status != 0) return;
  const int tx = t % a.tiles_x, ty = t / a.tiles_x;
  const DevCam& c = a.cams.c[lv];
  const int W = c.W, H = c.H;
  const int lane = threadIdx.x;
  const int qx = lane & 7, qy = lane >> 3;
  const int ox = tx * kTile, oy = ty * kTile;
  const uint32_t start = a.ranges[(int64_t)v * a.tiles + t], end = a.ranges[(int64_t)v * a.tiles + t + 1];
  const int64_t vn = (int64_t)v * a.n;
  const int64_t HW = (int64_t)W * H;
  float* rg = A.rg + (int64_t)v * kGradFields * a.n;

  float lx[4], ly[4], T[4], Tf[4], SC[4][3], SD[4], SN[4][3];
  float GC[4][3], GS[4][3], GN[4][3], GD[4], GM[4], GA[4];
  uint32_t last[4], med[4];
  uint32_t hi = start;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int px = ox + 2 * qx + (k & 1), py = oy + 2 * qy + (k >> 1);
    lx[k] = (float)(2 * qx + (k & 1)) + 0.5f;
    ly[k] = (float)(2 * qy + (k >> 1)) + 0.5f;
    const bool in = px < W && py < H;
    const int64_t p = in ? (int64_t)py * W + px : 0;
    const int64_t vp = (int64_t)v * HW + p;
    const int64_t v3 = (int64_t)v * 3 * HW + p;
    last[k] = in ? min(max(a.img.last[vp], start), end) : start;
    med[k] = in ? a.img.med[vp] : 0xffffffffu;
    Tf[k] = in ? a.img.T_final[vp] : 1.f;
    T[k] = Tf[k];
    for (int ch = 0; ch < 3; ++ch) {
      GC[k][ch] = in ? ldg0(A.up.d_rgb, v3 + ch * HW) : 0.f;
      GS[k][ch] = in ? ldg0(A.up.d_rgb_ssim, v3 + ch * HW) : 0.f;
      GN[k][ch] = in ? ldg0(A.up.d_normal, v3 + ch * HW) : 0.f;
      SC[k][ch] = Tf[k] * c.bg[ch];
      SN[k][ch] = 0.f;
    }
    GD[k] = in ? ldg0(A.up.d_depth, vp) : 0.f;
    GM[k] = in ? ldg0(A.up.d_depth_med, vp) : 0.f;
    GA[k] = in ? ldg0(A.up.d_alpha, vp) : 0.f;
    SD[k] = 0.f;
    hi = max(hi, last[k]);
  }
  // wave max of 'last'
  for (int off = 1; off < 64; off <<= 1) hi = max(hi, __shfl_xor(hi, off));
  const float fox = (float)ox, foy = (float)oy;

  for (uint32_t top = hi; top > start;) {
    const uint32_t lo = top - start > 64u ? top - 64u : start;
    const uint32_t idx = lo + lane;
    if (idx < top) stage_record(s, lane, a.rec, vn, a.n, a.ids[idx], fox, foy);
    __syncthreads();
    for (int j = (int)(top - lo) - 1; j >= 0; --j) {
      const uint32_t e_idx = lo + (uint32_t)j;
      const float cx = s[L_CX][j], cy = s[L_CY][j];
      const float a11 = s[L_A11][j], a12 = s[L_A12][j], a21 = s[L_A21][j], a22 = s[L_A22][j];
      const float w0 = s[L_W0][j], w1 = s[L_W1][j], w2 = s[L_W2][j], op = s[L_OP][j];
      const float zc = s[L_ZC][j], zw = s[L_ZW][j];
      const float cr = s[L_R][j], cg = s[L_G][j], cb = s[L_B][j];
      const float nx = s[L_NX][j], ny = s[L_NY][j], nz = s[L_NZ][j];
      float acc[kGradFields];
#pragma unroll
      for (int f = 0; f < kGradFields; ++f) acc[f] = 0.f;
      bool any = false;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (e_idx >= last[k]) continue;
        const float xr = lx[k] - cx, yr = ly[k] - cy;
        PairEval e;
        eval_pair(xr, yr, a11, a12, a21, a22, w0, w1, w2, op, e);
        if (e.alpha < kAlphaMin) continue;
        any = true;
        const float rom = __builtin_amdgcn_rcpf(1.f - e.alpha);
        const float Tn = T[k];            // transmittance after this fragment
        const float Ti = Tn * rom;        // ... and before it
        const float wgt = e.alpha * Ti;
        const float iw = __builtin_amdgcn_rcpf(e.w);
        const float zf = e.is3d ? zw * iw : zc;
        float dA = GC[k][0] * (Tn * cr - SC[k][0]) + GC[k][1] * (Tn * cg - SC[k][1]) + GC[k][2] * (Tn * cb - SC[k][2]);
        dA += GN[k][0] * (Tn * nx - SN[k][0]) + GN[k][1] * (Tn * ny - SN[k][1]) + GN[k][2] * (Tn * nz - SN[k][2]);
        dA += GD[k] * (Tn * zf - SD[k]) + GA[k] * Tf[k];
        dA *= rom;
        float dS = GS[k][0] * (Tn * cr - SC[k][0]) + GS[k][1] * (Tn * cg - SC[k][1]) + GS[k][2] * (Tn * cb - SC[k][2]);
        dS *= rom;
        acc[G_R] = fmaf(GC[k][0], wgt, acc[G_R]);
        acc[G_G] = fmaf(GC[k][1], wgt, acc[G_G]);
        acc[G_B] = fmaf(GC[k][2], wgt, acc[G_B]);
        acc[G_NX] = fmaf(GN[k][0], wgt, acc[G_NX]);
        acc[G_NY] = fmaf(GN[k][1], wgt, acc[G_NY]);
        acc[G_NZ] = fmaf(GN[k][2], wgt, acc[G_NZ]);
        const float dz = GD[k] * wgt + (e_idx == med[k] ? GM[k] : 0.f);
        SC[k][0] = fmaf(wgt, cr, SC[k][0]);
        SC[k][1] = fmaf(wgt, cg, SC[k][1]);
        SC[k][2] = fmaf(wgt, cb, SC[k][2]);
        SN[k][0] = fmaf(wgt, nx, SN[k][0]);
        SN[k][1] = fmaf(wgt, ny, SN[k][1]);
        SN[k][2] = fmaf(wgt, nz, SN[k][2]);
        SD[k] = fmaf(wgt, zf, SD[k]);
        T[k] = Ti;
        float dr = 0.f, drs = 0.f;
        if (!(e.araw > kAlphaMax)) {
          acc[G_OP] = fmaf(dA, e.G, acc[G_OP]);
          dr = -0.5f * e.araw * dA;
          drs = -0.5f * e.araw * dS;
        }
        float dxr, dyr, dsx, dsy;
        if (e.is3d) {
          const float iww = __builtin_amdgcn_rcpf(e.ww);
          const float q1 = 2.f * e.P1 * iww, q2 = 2.f * e.P2 * iww, qw = -2.f * e.rho * iw;
          const float gP1 = dr * q1, gP2 = dr * q2;
          const float gw = dr * qw - dz * zf * iw;
          acc[G_A11] = fmaf(gP1, xr, acc[G_A11]);
          acc[G_A12] = fmaf(gP1, yr, acc[G_A12]);
          acc[G_A21] = fmaf(gP2, xr, acc[G_A21]);
          acc[G_A22] = fmaf(gP2, yr, acc[G_A22]);
          acc[G_W0] += gw + dz * zc * iw;
          acc[G_W1] = fmaf(gw, xr, acc[G_W1]);
          acc[G_W2] = fmaf(gw, yr, acc[G_W2]);
          acc[G_ZC] = fmaf(dz, w0 * iw, acc[G_ZC]);
          dxr = gP1 * a11 + gP2 * a21 + gw * w1;
          dyr = gP1 * a12 + gP2 * a22 + gw * w2;
          const float sP1 = drs * q1, sP2 = drs * q2, sw = drs * qw;
          dsx = sP1 * a11 + sP2 * a21 + sw * w1;
          dsy = sP1 * a12 + sP2 * a22 + sw * w2;
        } else {
          dxr = 4.f * dr * xr;
          dyr = 4.f * dr * yr;
          acc[G_ZC] += dz;
          dsx = 4.f * drs * xr;
          dsy = 4.f * drs * yr;
        }
        acc[G_CX] -= dxr;
        acc[G_CY] -= dyr;
        acc[G_SCX] -= dsx;
        acc[G_SCY] -= dsy;
      }
      if (__ballot(any) != 0) {
        const uint32_t id = __float_as_uint(s[L_ID][j]);
#pragma unroll
        for (int f = 0; f < kGradFields; ++f) {
          const float tot = wave_sum(acc[f]);
          if (lane == 0) atomicAdd(rg + (int64_t)f * a.n + id, tot);
        }
      }
    }
    __syncthreads();
    top = lo;
  }
}

__global__ __launch_bounds__(256) void k_zero_visible(const uint8_t* __restrict__ flags, int64_t n, float* rg,
                                                     int v0) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int v = v0 + (int)blockIdx.y;
  if (i >= n) return;
  if (!(flags[(int64_t)v * n + i] & CGV2_F_VISIBLE)) return;
  float* r = rg + (int64_t)v * kGradFields * n + i;
#pragma unroll
  for (int f = 0; f < kGradFields; ++f) r[(int64_t)f * n] = 0.f;
}

}  // namespace cgv2

static cgv2::RenderArgs make_args(const cgv2_proj& p, const cgv2_bins& b, const cgv2::CamPack& cams, int64_t n,
                                  int tiles_x, int tiles_y, const cgv2_image* img, unsigned long long* counters) {
  cgv2::RenderArgs a;
  a.rec = p.rec;
  a.ids = b.ids;
  a.ranges = b.ranges;
  a.status = b.status;
  a.cams = cams;
  a.n = n;
  a.tiles_x = tiles_x;
  a.tiles_y = tiles_y;
  a.tiles = tiles_x * tiles_y;
  if (img) a.img = *img; else a.img = cgv2_image{};
  a.counters = counters;
  return a;
}

hipError_t cgv2_launch_render_fwd(const cgv2_proj& p, const cgv2_bins& b, const cgv2::CamPack& cams, int64_t n,
                                  int tiles_x, int tiles_y, const cgv2_image& img, hipStream_t st) {
  cgv2::RenderArgs a = make_args(p, b, cams, n, tiles_x, tiles_y, &img, nullptr);
  const unsigned grid = (unsigned)((int64_t)cams.count * a.tiles);
  hipLaunchKernelGGL(cgv2::k_render_fwd<false>, dim3(grid), dim3(64), 0, st, a);
  return hipGetLastError();
}

hipError_t cgv2_launch_render_count(const cgv2_proj& p, const cgv2_bins& b, const cgv2::CamPack& cams, int64_t n, int tiles_x, int tiles_y, unsigned long long* counters,
                                    hipStream_t st) {
  cgv2::RenderArgs a = make_args(p, b, cams, n, tiles_x, tiles_y, nullptr, counters);
  const unsigned grid = (unsigned)((int64_t)cams.count * a.tiles);
  hipLaunchKernelGGL(cgv2::k_render_fwd<true>, dim3(grid), dim3(64), 0, st, a);
  return hipGetLastError();
}

hipError_t cgv2_launch_render_bwd(const cgv2_proj& p, const cgv2_bins& b, const cgv2::CamPack& cams, int64_t n,
                                  int tiles_x, int tiles_y, const cgv2_image& img, const cgv2_image_grad& up,
                                  float* rg, hipStream_t st) {
  if (n > 0) {
    hipLaunchKernelGGL(cgv2::k_zero_visible, dim3((unsigned)((n + 255) / 256), (unsigned)cams.count), dim3(256), 0,
                       st, p.flags, n, rg, cams.v0);
  }
  cgv2::BwdArgs A;
  A.r = make_args(p, b, cams, n, tiles_x, tiles_y, &img, nullptr);
  A.up = up;
  A.rg = rg;
  const unsigned grid = (unsigned)((int64_t)cams.count * A.r.tiles);
  hipLaunchKernelGGL(cgv2::k_render_bwd, dim3(grid), dim3(64), 0, st, A);
  return hipGetLastError();
}
