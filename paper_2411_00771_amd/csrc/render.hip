// Tile renderer: forward (Eq. 1 alpha blending of CityGaussianV2 Sec. 3.1, with the depth,
// median-depth and normal renders of Sec. 3.2 / 5.1) and its reverse.
//
// One 64-lane wave per 16x16 tile; each lane owns a 2x2 pixel quad.  The records of a tile list
// are staged 64 at a time into LDS (one per lane, as five float4), converting the centre to
// tile-relative coordinates exactly ((cx_hi - tile_x0) + cx_lo), pre-scaling the homography
// numerator by 1/sqrt(2) (so rho/2 comes out directly) and replacing the opacity by log2(o) and
// 1/o.  Every staged record is read back as float4 broadcasts and feeds four pixels; within a
// quad the homography terms of the neighbouring pixels are one add away.  The wave leaves the
// list as soon as every pixel has stopped (ballot).
//
// The reverse walks each pixel's list from its checkpointed 'last' entry downwards, recovers T
// by division, sums the per-surfel gradients of its four pixels in registers, reduces them over
// the wave with DPP row operations and adds them once per (surfel, tile) with float atomics.
#include "cgv2r_device.h"
#include "cgv2r_kernels.h"

#include <algorithm>

namespace cgv2 {

constexpr float kInvSqrt2 = 0.70710678118654752440f;
constexpr float kLog2e = 1.44269504088896340736f;

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

// LDS record, five float4:
//   q0 = (cx, cy, a11 / sqrt2, a12 / sqrt2)     q1 = (a21 / sqrt2, a22 / sqrt2, w0, w1)
//   q2 = (w2, log2 o, z_c, z_c * w0)           q3 = (r, g, b, id)      q4 = (nx, ny, nz, 1 / o)
__device__ __forceinline__ void stage_record(float4 (*s)[5], int lane, const float* rec, int64_t vn, int64_t n,
                                             uint32_t id, float ox, float oy) {
  // an id outside [0, n) (never produced by the binning) stages a zero-opacity record
  const bool valid = (int64_t)id < n;
  const float4* r = (const float4*)(rec + (size_t)(vn + (valid ? id : 0u)) * kRec);
  const float4 r0 = r[0], r1 = r[1], r2 = r[2], r3 = r[3], r4 = r[4];
  s[lane][0] = make_float4((r0.x - ox) + r0.z, (r0.y - oy) + r0.w, r1.x * kInvSqrt2, r1.y * kInvSqrt2);
  s[lane][1] = make_float4(r1.z * kInvSqrt2, r1.w * kInvSqrt2, r2.x, r2.y);
  s[lane][2] = make_float4(r2.z, valid ? log2f(r3.x) : -INFINITY, r2.w, r2.w * r2.x);
  s[lane][3] = make_float4(r3.y, r3.z, r3.w, __uint_as_float(valid ? id : 0u));
  s[lane][4] = make_float4(r4.x, r4.y, r4.z, valid ? 1.f / r3.x : 0.f);
}

// Evaluation of one staged surfel at the four pixels of a quad, shared by the forward and the
// reverse so that both take bit-identical decisions.  Pixel k sits at (xr[k & 1], yr[k >> 1])
// relative to the projected centre.  rho is half the Mahalanobis-type distance:
// rho = min(rho_3d, rho_2d) / 2, alpha_raw = o exp(-rho).
struct Quad {
  float xr[2], yr[2];
  float P1[4], P2[4], w[4], iw[4], rho[4], araw[4], alpha[4];
  bool is3d[4];
};

__device__ __forceinline__ void eval_quad(float lx0, float ly0, const float4 q0, const float4 q1, const float4 q2,
                                          Quad& e) {
  const float a11 = q0.z, a12 = q0.w, a21 = q1.x, a22 = q1.y, w0 = q1.z, w1 = q1.w, w2 = q2.x, lo = q2.y;
  e.xr[0] = lx0 - q0.x;
  e.yr[0] = ly0 - q0.y;
  e.xr[1] = e.xr[0] + 1.f;
  e.yr[1] = e.yr[0] + 1.f;
  const float p1 = fmaf(a11, e.xr[0], a12 * e.yr[0]);
  const float p2 = fmaf(a21, e.xr[0], a22 * e.yr[0]);
  const float wb = fmaf(w1, e.xr[0], fmaf(w2, e.yr[0], w0));
  e.P1[0] = p1; e.P1[1] = p1 + a11; e.P1[2] = p1 + a12; e.P1[3] = e.P1[1] + a12;
  e.P2[0] = p2; e.P2[1] = p2 + a21; e.P2[2] = p2 + a22; e.P2[3] = e.P2[1] + a22;
  e.w[0] = wb; e.w[1] = wb + w1; e.w[2] = wb + w2; e.w[3] = e.w[1] + w2;
  const float xx[2] = {e.xr[0] * e.xr[0], e.xr[1] * e.xr[1]};
  const float yy[2] = {e.yr[0] * e.yr[0], e.yr[1] * e.yr[1]};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float r2 = xx[k & 1] + yy[k >> 1];
    const float nn = fmaf(e.P1[k], e.P1[k], e.P2[k] * e.P2[k]);
    // w == 0: the ray runs parallel to the plane; rcp gives inf (or NaN for nn == 0) and the
    // comparison below then selects the screen filter
    e.iw[k] = __builtin_amdgcn_rcpf(e.w[k]);
    const float r3 = nn * (e.iw[k] * e.iw[k]);
    e.is3d[k] = r3 <= r2;
    e.rho[k] = e.is3d[k] ? r3 : r2;
    e.araw[k] = __builtin_amdgcn_exp2f(fmaf(e.rho[k], -kLog2e, lo));
    e.alpha[k] = fminf(kAlphaMax, e.araw[k]);
  }
}

template <bool kCount>
__global__ __launch_bounds__(64) void k_render_fwd(RenderArgs a) {
  __shared__ float4 s[64][5];
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
  unsigned long long n_eval = 0, n_con = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int px = ox + 2 * qx + (k & 1), py = oy + 2 * qy + (k >> 1);
    done[k] = !(px < W && py < H);
    T[k] = 1.f; D[k] = 0.f; Dm[k] = 0.f; last[k] = start; med[k] = 0xffffffffu;
    C[k][0] = C[k][1] = C[k][2] = 0.f;
    N[k][0] = N[k][1] = N[k][2] = 0.f;
  }
  const float lx0 = (float)(2 * qx) + 0.5f, ly0 = (float)(2 * qy) + 0.5f;
  const float fox = (float)ox, foy = (float)oy;
  for (uint32_t base = start; base < end; base += 64) {
    if (__ballot(!(done[0] && done[1] && done[2] && done[3])) == 0) break;
    const uint32_t idx = base + lane;
    if (idx < end) stage_record(s, lane, a.rec, vn, a.n, a.ids[idx], fox, foy);
    __syncthreads();
    const int cnt = (int)min(64u, end - base);
    for (int j = 0; j < cnt; ++j) {
      const float4 q0 = s[j][0], q1 = s[j][1], q2 = s[j][2], q3 = s[j][3], q4 = s[j][4];
      Quad e;
      eval_quad(lx0, ly0, q0, q1, q2, e);
      const uint32_t idx1 = base + (uint32_t)j + 1u;
      bool take4[4];
      bool any = false;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (kCount && !done[k]) ++n_eval;
        take4[k] = !done[k] && e.alpha[k] >= kAlphaMin;
        any = any || take4[k];
      }
      // wave-uniform skip when no pixel of the tile takes this surfel; otherwise branch-free
      if (__ballot(any) == 0) continue;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        // a contribution is a zero-weight no-op for pixels that skip or stop here
        const bool take = take4[k];
        const float a = take ? e.alpha[k] : 0.f;
        const float Tn = T[k] * (1.f - a);
        const bool stop = take && Tn < kTmin;
        done[k] = done[k] || stop;
        const bool upd = take && !stop;
        if (kCount && upd) ++n_con;
        const float wgt = upd ? a * T[k] : 0.f;
        const float zf = e.is3d[k] ? q2.w * e.iw[k] : q2.z;
        C[k][0] = fmaf(wgt, q3.x, C[k][0]);
        C[k][1] = fmaf(wgt, q3.y, C[k][1]);
        C[k][2] = fmaf(wgt, q3.z, C[k][2]);
        N[k][0] = fmaf(wgt, q4.x, N[k][0]);
        N[k][1] = fmaf(wgt, q4.y, N[k][1]);
        N[k][2] = fmaf(wgt, q4.z, N[k][2]);
        D[k] = fmaf(wgt, zf, D[k]);
        const bool m = upd && T[k] > 0.5f;
        Dm[k] = m ? zf : Dm[k];
        med[k] = m ? idx1 - 1u : med[k];
        last[k] = upd ? idx1 : last[k];
        T[k] = upd ? Tn : T[k];
      }
      if ((j & 15) == 15) {
        if (__ballot(!(done[0] && done[1] && done[2] && done[3])) == 0) break;
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

// kGeom: depth, median-depth, normal or alpha upstream gradients are present.  Without them (the
// photometric-loss-only case) their per-pixel state, terms and five of the reductions drop out.
template <bool kGeom>
__global__ __launch_bounds__(64) void k_render_bwd(BwdArgs A) {
  __shared__ float4 s[64][5];
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

  float T[4], Tf[4], SC[4][3], SD[4], SN[4][3];
  float GC[4][3], GS[4][3], GN[4][3], GD[4], GM[4], GA[4];
  uint32_t last[4], med[4];
  uint32_t hi = start;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int px = ox + 2 * qx + (k & 1), py = oy + 2 * qy + (k >> 1);
    const bool in = px < W && py < H;
    const int64_t p = in ? (int64_t)py * W + px : 0;
    const int64_t vp = (int64_t)v * HW + p;
    const int64_t v3 = (int64_t)v * 3 * HW + p;
    last[k] = in ? min(max(a.img.last[vp], start), end) : start;
    med[k] = in ? a.img.med[vp] : 0xffffffffu;
    Tf[k] = in ? a.img.T_final[vp] : 1.f;
    T[k] = Tf[k];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      GC[k][ch] = in ? ldg0(A.up.d_rgb, v3 + ch * HW) : 0.f;
      GS[k][ch] = in ? ldg0(A.up.d_rgb_ssim, v3 + ch * HW) : 0.f;
      GN[k][ch] = kGeom && in ? ldg0(A.up.d_normal, v3 + ch * HW) : 0.f;
      SC[k][ch] = Tf[k] * c.bg[ch];
      SN[k][ch] = 0.f;
    }
    GD[k] = kGeom && in ? ldg0(A.up.d_depth, vp) : 0.f;
    GM[k] = kGeom && in ? ldg0(A.up.d_depth_med, vp) : 0.f;
    GA[k] = kGeom && in ? ldg0(A.up.d_alpha, vp) : 0.f;
    SD[k] = 0.f;
    hi = max(hi, last[k]);
  }
  // wave max of 'last'
  for (int off = 1; off < 64; off <<= 1) hi = max(hi, __shfl_xor(hi, off));
  const float lx0 = (float)(2 * qx) + 0.5f, ly0 = (float)(2 * qy) + 0.5f;
  const float fox = (float)ox, foy = (float)oy;

  for (uint32_t top = hi; top > start;) {
    const uint32_t lo = top - start > 64u ? top - 64u : start;
    const uint32_t idx = lo + lane;
    if (idx < top) stage_record(s, lane, a.rec, vn, a.n, a.ids[idx], fox, foy);
    __syncthreads();
    for (int j = (int)(top - lo) - 1; j >= 0; --j) {
      const uint32_t e_idx = lo + (uint32_t)j;
      const float4 q0 = s[j][0], q1 = s[j][1], q2 = s[j][2];
      Quad e;
      eval_quad(lx0, ly0, q0, q1, q2, e);
      bool con[4];
      bool any = false;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        con[k] = e_idx < last[k] && e.alpha[k] >= kAlphaMin;
        any = any || con[k];
      }
      if (__ballot(any) == 0) continue;
      const float4 q3 = s[j][3], q4 = s[j][4];
      const float a11 = q0.z, a12 = q0.w, a21 = q1.x, a22 = q1.y, w0 = q1.z, w1 = q1.w, w2 = q2.x;
      const float zc = q2.z, zw = q2.w, io = q4.w;
      float acc[kGradFields];
#pragma unroll
      for (int f = 0; f < kGradFields; ++f) acc[f] = 0.f;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        // branch-free: pixels without a contribution here get al = 0, dA = 0 and keep T
        const float xr = e.xr[k & 1], yr = e.yr[k >> 1];
        const float al = con[k] ? e.alpha[k] : 0.f;
        const float rom = __builtin_amdgcn_rcpf(1.f - al);
        const float Tn = T[k];            // transmittance after this fragment
        const float Ti = Tn * rom;        // ... and before it
        const float wgt = al * Ti;
        const float iw = e.iw[k];
        const float zf = e.is3d[k] ? zw * iw : zc;
        const float dcr = Tn * q3.x - SC[k][0], dcg = Tn * q3.y - SC[k][1], dcb = Tn * q3.z - SC[k][2];
        float dA = fmaf(GC[k][0], dcr, fmaf(GC[k][1], dcg, GC[k][2] * dcb));
        float dS = fmaf(GS[k][0], dcr, fmaf(GS[k][1], dcg, GS[k][2] * dcb));
        if (kGeom) {
          dA = fmaf(GN[k][0], Tn * q4.x - SN[k][0], dA);
          dA = fmaf(GN[k][1], Tn * q4.y - SN[k][1], dA);
          dA = fmaf(GN[k][2], Tn * q4.z - SN[k][2], dA);
          dA = fmaf(GD[k], Tn * zf - SD[k], dA);
          dA = fmaf(GA[k], Tf[k], dA);
        }
        // the 0.99 clamp blocks the path to o and rho; non-contributing pixels pass nothing
        const bool live = con[k] && !(e.araw[k] > kAlphaMax);
        dA = live ? dA * rom : 0.f;
        dS = live ? dS * rom : 0.f;
        acc[G_R] = fmaf(GC[k][0], wgt, acc[G_R]);
        acc[G_G] = fmaf(GC[k][1], wgt, acc[G_G]);
        acc[G_B] = fmaf(GC[k][2], wgt, acc[G_B]);
        SC[k][0] = fmaf(wgt, q3.x, SC[k][0]);
        SC[k][1] = fmaf(wgt, q3.y, SC[k][1]);
        SC[k][2] = fmaf(wgt, q3.z, SC[k][2]);
        float dz = 0.f;
        if (kGeom) {
          acc[G_NX] = fmaf(GN[k][0], wgt, acc[G_NX]);
          acc[G_NY] = fmaf(GN[k][1], wgt, acc[G_NY]);
          acc[G_NZ] = fmaf(GN[k][2], wgt, acc[G_NZ]);
          dz = fmaf(GD[k], wgt, con[k] && e_idx == med[k] ? GM[k] : 0.f);
          SN[k][0] = fmaf(wgt, q4.x, SN[k][0]);
          SN[k][1] = fmaf(wgt, q4.y, SN[k][1]);
          SN[k][2] = fmaf(wgt, q4.z, SN[k][2]);
          SD[k] = fmaf(wgt, zf, SD[k]);
        }
        T[k] = Ti;
        // alpha_raw = o exp(-rho): d alpha_raw / d rho = -alpha_raw
        const float dr = -e.araw[k] * dA;
        const float drs = -e.araw[k] * dS;
        acc[G_OP] = fmaf(dA, e.araw[k] * io, acc[G_OP]);
        float dxr, dyr, dsx, dsy;
        if (e.is3d[k]) {
          const float iww = iw * iw;
          const float q1v = 2.f * e.P1[k] * iww, q2v = 2.f * e.P2[k] * iww, qw = -2.f * e.rho[k] * iw;
          const float gP1 = dr * q1v, gP2 = dr * q2v;
          const float gw = kGeom ? fmaf(dr, qw, -dz * zf * iw) : dr * qw;
          acc[G_A11] = fmaf(gP1, xr, acc[G_A11]);
          acc[G_A12] = fmaf(gP1, yr, acc[G_A12]);
          acc[G_A21] = fmaf(gP2, xr, acc[G_A21]);
          acc[G_A22] = fmaf(gP2, yr, acc[G_A22]);
          acc[G_W0] += kGeom ? fmaf(dz * zc, iw, gw) : gw;
          acc[G_W1] = fmaf(gw, xr, acc[G_W1]);
          acc[G_W2] = fmaf(gw, yr, acc[G_W2]);
          if (kGeom) acc[G_ZC] = fmaf(dz, w0 * iw, acc[G_ZC]);
          dxr = fmaf(gP1, a11, fmaf(gP2, a21, gw * w1));
          dyr = fmaf(gP1, a12, fmaf(gP2, a22, gw * w2));
          const float sP1 = drs * q1v, sP2 = drs * q2v, sw = drs * qw;
          dsx = fmaf(sP1, a11, fmaf(sP2, a21, sw * w1));
          dsy = fmaf(sP1, a12, fmaf(sP2, a22, sw * w2));
        } else {
          dxr = 2.f * dr * xr;
          dyr = 2.f * dr * yr;
          if (kGeom) acc[G_ZC] += dz;
          dsx = 2.f * drs * xr;
          dsy = 2.f * drs * yr;
        }
        acc[G_CX] -= dxr;
        acc[G_CY] -= dyr;
        acc[G_SCX] -= dsx;
        acc[G_SCY] -= dsy;
      }
      // slots 0..15 (fields G_CX..G_ZC) by reduce-scatter: one atomic instruction, one lane per field
      float red[16];
#pragma unroll
      for (int f = 0; f < 16; ++f) red[f] = acc[f];
      const float tot = reduce16_scatter(red);
      const int slot = reduce16_index(lane);
      if ((lane & 12) == 0 && (kGeom || slot != G_ZC)) {
        const uint32_t id = __float_as_uint(q3.w);
        // the staged numerator coefficients carry 1/sqrt(2)
        const bool anum = slot >= G_A11 && slot <= G_A22;
        atomicAdd(rg + (int64_t)slot * a.n + id, anum ? tot * kInvSqrt2 : tot);
      }
      if (kGeom) {
        const float nx = wave_sum_lane63(acc[G_NX]), ny = wave_sum_lane63(acc[G_NY]),
                    nz = wave_sum_lane63(acc[G_NZ]);
        if (lane == 63) {
          const uint32_t id = __float_as_uint(q3.w);
          atomicAdd(rg + (int64_t)G_NX * a.n + id, nx);
          atomicAdd(rg + (int64_t)G_NY * a.n + id, ny);
          atomicAdd(rg + (int64_t)G_NZ * a.n + id, nz);
        }
      }
    }
    __syncthreads();
    top = lo;
  }
}

// Clears the record gradients of the surfels in view v's visible list (the atomics add into them).
__global__ __launch_bounds__(256) void k_zero_visible(const uint32_t* __restrict__ visible,
                                                     const uint32_t* __restrict__ vstart, int64_t n, float* rg,
                                                     int v0) {
  const int v = v0 + (int)blockIdx.y;
  const uint32_t e0 = vstart[v], e1 = vstart[v + 1];
  float* r = rg + (int64_t)v * kGradFields * n;
  for (uint32_t e = e0 + blockIdx.x * blockDim.x + threadIdx.x; e < e1; e += gridDim.x * blockDim.x) {
    const uint32_t i = visible[e];
#pragma unroll
    for (int f = 0; f < kGradFields; ++f) r[(int64_t)f * n + i] = 0.f;
  }
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

hipError_t cgv2_launch_render_count(const cgv2_proj& p, const cgv2_bins& b, const cgv2::CamPack& cams, int64_t n,
                                    int tiles_x, int tiles_y, unsigned long long* counters, hipStream_t st) {
  cgv2::RenderArgs a = make_args(p, b, cams, n, tiles_x, tiles_y, nullptr, counters);
  const unsigned grid = (unsigned)((int64_t)cams.count * a.tiles);
  hipLaunchKernelGGL(cgv2::k_render_fwd<true>, dim3(grid), dim3(64), 0, st, a);
  return hipGetLastError();
}

hipError_t cgv2_launch_render_bwd(const cgv2_proj& p, const cgv2_bins& b, const cgv2::CamPack& cams, int64_t n,
                                  int tiles_x, int tiles_y, const cgv2_image& img, const cgv2_image_grad& up,
                                  float* rg, hipStream_t st) {
  if (n > 0) {
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(cgv2::k_zero_visible, dim3(blocks, (unsigned)cams.count), dim3(256), 0, st, p.visible,
                       p.visible_start, n, rg, cams.v0);
  }
  cgv2::BwdArgs A;
  A.r = make_args(p, b, cams, n, tiles_x, tiles_y, &img, nullptr);
  A.up = up;
  A.rg = rg;
  const unsigned grid = (unsigned)((int64_t)cams.count * A.r.tiles);
  const bool geom = up.d_depth || up.d_depth_med || up.d_normal || up.d_alpha;
  if (geom) hipLaunchKernelGGL(cgv2::k_render_bwd<true>, dim3(grid), dim3(64), 0, st, A);
  else hipLaunchKernelGGL(cgv2::k_render_bwd<false>, dim3(grid), dim3(64), 0, st, A);
  return hipGetLastError();
}
