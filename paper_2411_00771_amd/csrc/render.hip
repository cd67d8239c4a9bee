// Tile renderer: forward (Eq. 1 alpha blending of CityGaussianV2 Sec. 3.1, with the depth,
// median-depth and normal renders of Sec. 3.2 / 5.1) and its reverse.
//
// One 64-lane wave per 16x16 tile.  Lane (x, y) = (lane & 7, lane >> 3) owns one pixel in each 8x8
// quadrant of the tile: (x, y), (x + 8, y), (x, y + 8) and (x + 8, y + 8).  The records of a tile
// list are staged 64 at a time into LDS (one per lane, as five float4), converting the centre to
// tile-relative coordinates exactly ((cx_hi - tile_x0) + cx_lo), pre-scaling the homography
// numerator by 1/sqrt(2) (so rho/2 comes out directly), replacing the opacity by log2(o) and 1/o,
// and reducing the surfel's pixel rect to a 4-bit mask of the quadrants it reaches, less those its
// alpha >= 1/255 region (an ellipse, plus the screen-filter disc) misses.  A quadrant outside the mask
// is skipped wave-uniformly, as is a quadrant whose pixels have all stopped; within a quadrant the
// evaluation is branch-free, and the homography terms of a lane's four pixels are one add apart.
//
// The reverse walks each pixel's list from its checkpointed 'last' entry downwards, recovers T by
// division, sums the per-surfel gradients of its four pixels in registers, reduces them over the
// wave with a reduce-scatter (row swaps + DPP) and adds them with one atomic instruction per
// (surfel, tile).
#include "cgv2r_device.h"
#include "cgv2r_kernels.h"

#include <algorithm>

namespace cgv2 {

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
  float* cws;   // contribution mode: [V][n] pairs (sum of alpha^gamma T^(1-gamma), pixel count)
  float gamma;
  const uint32_t* order;  // launch order of this view chunk (heaviest tiles first), or null
  uint32_t n_q, n_h;      // the first n_q tiles of 'order' run as four quadrant blocks, the next n_h as two halves
};

// Block -> (local view, tile) index and quadrant subset.  Without a launch order: the XCD-aware spatial
// mapping, whole tiles.  With one (the bin_sort's heaviest-first order; bounded, so a stale order cannot
// leave the launch), the n_q heaviest tiles run as four single-quadrant blocks each (blocks [0, 4 n_q)),
// the next n_h as two halves (top 0x3, bottom 0xc; the following 2 n_h blocks), the rest whole; the
// launch has 3 n_q + n_h blocks more than tiles.
__device__ __forceinline__ uint32_t tile_of_block(const RenderArgs& a, uint32_t& sub) {
  const uint32_t bid = blockIdx.x, tiles = gridDim.x - 3u * a.n_q - a.n_h;
  sub = 0xfu;
  if (!a.order) return xcd_remap(bid, tiles);
  uint32_t i;
  if (bid < 4u * a.n_q) {
    i = bid >> 2;
    sub = 1u << (bid & 3u);
  } else if (bid < 4u * a.n_q + 2u * a.n_h) {
    const uint32_t r = bid - 4u * a.n_q;
    i = a.n_q + (r >> 1);
    sub = (r & 1u) ? 0xcu : 0x3u;
  } else {
    i = bid - 3u * a.n_q - a.n_h;
  }
  const uint32_t b = a.order[i];
  return b < tiles ? b : tiles - 1u;
}

// LDS record, five float4 (the quadrant masks of the 64 staged entries travel as wave ballots):
//   q0 = (cx, cy, a11 / sqrt2, a12 / sqrt2)     q1 = (a21 / sqrt2, a22 / sqrt2, w0, w1)
//   q2 = (w2, log2 o, z_c, z_c * w0)           q3 = (r, g, b, id)      q4 = (nx, ny, nz, 1 / o)
struct Stage {
  float4 q[64][5];
};

// The 4-bit quadrant masks of the 64 staged entries as nibbles in scalar registers: entry j's mask is
// bits 4 (j % 16) .. 4 (j % 16) + 3 of w[j / 16].  Built with one OR reduction over each row of 16 lanes
// (DPP row shifts) and four lane reads per half; reading one entry's mask is then a shift and a mask.
template <int kCtrl>
__device__ __forceinline__ uint32_t dpp_or_in(uint32_t v) {
  return v | (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kCtrl, 0xf, 0xf, false);
}
struct QuadBits {
  uint64_t w[4];
  __device__ __forceinline__ void from_lanes(uint32_t m) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t sh = 4u * (lane & 7u);
    uint32_t lo = (lane & 8u) ? 0u : (m & 0xfu) << sh, hi = (lane & 8u) ? (m & 0xfu) << sh : 0u;
    lo = dpp_or_in<0x111>(lo);  // row_shr:1
    hi = dpp_or_in<0x111>(hi);
    lo = dpp_or_in<0x112>(lo);  // row_shr:2
    hi = dpp_or_in<0x112>(hi);
    lo = dpp_or_in<0x114>(lo);  // row_shr:4
    hi = dpp_or_in<0x114>(hi);
    lo = dpp_or_in<0x118>(lo);  // row_shr:8: lane 15 of each row holds the row's OR
    hi = dpp_or_in<0x118>(hi);
#pragma unroll
    for (int r = 0; r < 4; ++r)
      w[r] = (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)hi, 16 * r + 15) << 32 |
             (uint32_t)__builtin_amdgcn_readlane((int)lo, 16 * r + 15);
  }
  // the nibbles of entries 16 i .. 16 i + 15 (i wave-uniform)
  __device__ __forceinline__ uint64_t word(int i) const { return i == 0 ? w[0] : i == 1 ? w[1] : i == 2 ? w[2] : w[3]; }
};

// Quadrants (bits of 'm') in which some pixel sample can reach alpha >= 1/255 (reach_setup / reach_cell).
__device__ __forceinline__ uint32_t reach_quadrants(uint32_t m, const float4& q0, const float4& q1, float w2, float k2) {
  Reach r;
  reach_setup(q0.z, q0.w, q1.x, q1.y, q1.z, q1.w, w2, k2, r);
  uint32_t out = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (((m >> k) & 1u) && reach_cell(r, q0.x, q0.y, 8 * (k & 1), 8 * (k >> 1), 8)) out |= 1u << k;
  return out;
}

// Returns the entry's quadrant mask.  qmask (optional): the forward's per-entry mask of quadrants with a
// contributing pixel, ANDed in; without it the quadrants the surfel cannot reach are dropped by
// reach_quadrants.
__device__ __forceinline__ uint32_t stage_record(Stage& s, int lane, const float* rec, int64_t vn, int64_t n,
                                                 uint32_t id, int ox, int oy, const uint8_t* qmask, uint32_t idx) {
  // an entry no pixel of the forward took reaches no quadrant here: its record is not read at all
  const uint32_t qm = qmask ? qmask[idx] : 0xfu;
  if (qm == 0u) return 0u;
  // an id outside [0, n) (never produced by the binning) stages a record that reaches no quadrant
  const bool valid = (int64_t)id < n;
  const float4* r = (const float4*)(rec + (size_t)(vn + (valid ? id : 0u)) * kRec);
  const float4 r0 = r[0], r1 = r[1], r2 = r[2], r3 = r[3], r4 = r[4], r5 = r[5];
  const float fox = (float)ox, foy = (float)oy;
  const float4 q0 = make_float4((r0.x - fox) + r0.z, (r0.y - foy) + r0.w, r1.x * kInvSqrt2, r1.y * kInvSqrt2);
  const float4 q1 = make_float4(r1.z * kInvSqrt2, r1.w * kInvSqrt2, r2.x, r2.y);
  s.q[lane][0] = q0;
  s.q[lane][1] = q1;
  s.q[lane][2] = make_float4(r2.z, valid ? log2f(r3.x) : -INFINITY, r2.w, r2.w * r2.x);
  s.q[lane][3] = make_float4(r3.y, r3.z, r3.w, __uint_as_float(valid ? id : 0u));
  s.q[lane][4] = make_float4(r4.x, r4.y, r4.z, valid ? 1.f / r3.x : 0.f);
  // pixel rect relative to the tile origin
  const uint32_t px = __float_as_uint(r5.x), py = __float_as_uint(r5.y);
  const int i0 = (int)(px & 0xffffu) - ox, i1 = (int)(px >> 16) - ox;
  const int j0 = (int)(py & 0xffffu) - oy, j1 = (int)(py >> 16) - oy;
  uint32_t m = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int x0 = 8 * (k & 1), y0 = 8 * (k >> 1);
    if (i0 <= x0 + 7 && i1 >= x0 && j0 <= y0 + 7 && j1 >= y0) m |= 1u << k;
  }
  if (qmask) m &= qm;
  else if (m) m = reach_quadrants(m, q0, q1, r2.z, r4.w);
  return valid ? m : 0u;
}

// Per-surfel terms of a lane at its quadrant-0 pixel; pixel k sits at (xr0 + 8 (k & 1), yr0 + 8 (k >> 1))
// relative to the projected centre (xr1 = xr0 + 8, yr1 = yr0 + 8).
// (c1x, c1y, c2x, c2y, cwx, cwy) are the coefficients of x' and y' in P1, P2 and w: a pixel 8 columns or
// rows further adds 8 times them (exact in FP32, so one FMA per term).
struct LaneTerms {
  float xr0, yr0, xr1, yr1, p1, p2, wb, c1x, c1y, c2x, c2y, cwx, cwy;
};

__device__ __forceinline__ void lane_terms(float lx0, float ly0, const float4& q0, const float4& q1, const float4& q2,
                                           LaneTerms& t) {
  t.xr0 = lx0 - q0.x;
  t.yr0 = ly0 - q0.y;
  t.xr1 = t.xr0 + 8.f;
  t.yr1 = t.yr0 + 8.f;
  t.p1 = fmaf(q0.z, t.xr0, q0.w * t.yr0);
  t.p2 = fmaf(q1.x, t.xr0, q1.y * t.yr0);
  t.wb = fmaf(q1.w, t.xr0, fmaf(q2.x, t.yr0, q1.z));
  t.c1x = q0.z;
  t.c1y = q0.w;
  t.c2x = q1.x;
  t.c2y = q1.y;
  t.cwx = q1.w;
  t.cwy = q2.x;
}

// Evaluation of one staged surfel at pixel k of a lane, shared by the forward and the reverse so that
// both take bit-identical decisions.  rho is half the Mahalanobis-type distance:
// rho = min(rho_3d, rho_2d) / 2, alpha_raw = o exp(-rho).
struct Px {
  float xr, yr, P1, P2, w, iw, rho, arg, araw, alpha;
  bool is3d;
};

template <int k>
__device__ __forceinline__ void eval_px(const LaneTerms& t, float lo, Px& e) {
  e.xr = (k & 1) ? t.xr1 : t.xr0;
  e.yr = (k >> 1) ? t.yr1 : t.yr0;
  e.P1 = t.p1;
  e.P2 = t.p2;
  e.w = t.wb;
  if (k & 1) {
    e.P1 = fmaf(8.f, t.c1x, e.P1);
    e.P2 = fmaf(8.f, t.c2x, e.P2);
    e.w = fmaf(8.f, t.cwx, e.w);
  }
  if (k >> 1) {
    e.P1 = fmaf(8.f, t.c1y, e.P1);
    e.P2 = fmaf(8.f, t.c2y, e.P2);
    e.w = fmaf(8.f, t.cwy, e.w);
  }
  const float r2 = fmaf(e.xr, e.xr, e.yr * e.yr);
  const float nn = fmaf(e.P1, e.P1, e.P2 * e.P2);
  // w == 0: the ray runs parallel to the plane; rcp gives inf (or NaN for nn == 0) and the
  // comparison below then selects the screen filter
  e.iw = __builtin_amdgcn_rcpf(e.w);
  const float r3 = nn * (e.iw * e.iw);
  e.is3d = r3 <= r2;
  e.rho = e.is3d ? r3 : r2;
  e.arg = fmaf(e.rho, -kLog2e, lo);  // log2(alpha_raw)
  e.araw = __builtin_amdgcn_exp2f(e.arg);
  e.alpha = fminf(kAlphaMax, e.araw);
}

__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// T carries the pixel's state in its sign: T > 0 while the pixel runs (T >= 1e-4 then), -T once it has
// stopped (or lies outside the image); the transmittance itself is |T|.  'last' holds the index of the
// last entry blended (start - 1 before the first); the image stores last + 1.
struct FwdState {
  float T, C[3], D, Dm, N[3];
  uint32_t last, med;
};

// The entry index as a per-lane register, for the selects of 'last' and 'med' (which cannot take it from
// a scalar register next to their lane mask).
__device__ __forceinline__ uint32_t lane_copy(uint32_t x) {
  uint32_t v;
  asm("v_mov_b32 %0, %1" : "=v"(v) : "s"(x));
  return v;
}

// Returns false when no pixel of the quadrant takes the entry (wave-uniform); true otherwise, which
// covers every entry with a contributing fragment (a superset is all the reverse pass needs).
// kContrib: also add the fragment's alpha^gamma T^(1-gamma) (T in front of it) and 1 to csum / ccnt.
constexpr float kLog2AlphaMax = -0.014499569695115089f;  // log2(0.99)

template <bool kContrib>
__device__ __forceinline__ bool fwd_px(const Px& e, const float4& q2, const float4& q3, const float4& q4,
                                       uint32_t e_idx, FwdState& f, unsigned long long& n_con, float gamma,
                                       float& csum, float& ccnt) {
  // wave-uniform skip when no pixel of the quadrant takes this surfel; otherwise branch-free: a
  // contribution is a zero-weight no-op for pixels that skip or stop here
  const bool take = f.T > 0.f && e.alpha >= kAlphaMin;
  if (__ballot(take) == 0) return false;
  // Tn is used only where the pixel takes the entry
  const float Tn = f.T * (1.f - e.alpha);
  const bool upd = take && !(Tn < kTmin);
  n_con += upd ? 1u : 0u;
  if (kContrib) {
    // log2(alpha) = min(log2(alpha_raw), log2(0.99))
    const float la = fminf(e.arg, kLog2AlphaMax);
    const float c = __builtin_amdgcn_exp2f(fmaf(gamma, la, (1.f - gamma) * __builtin_amdgcn_logf(f.T)));
    csum += upd ? c : 0.f;
    ccnt += upd ? 1.f : 0.f;
  }
  const float wgt = upd ? e.alpha * f.T : 0.f;
  const float zf = e.is3d ? q2.w * e.iw : q2.z;
  f.C[0] = fmaf(wgt, q3.x, f.C[0]);
  f.C[1] = fmaf(wgt, q3.y, f.C[1]);
  f.C[2] = fmaf(wgt, q3.z, f.C[2]);
  f.N[0] = fmaf(wgt, q4.x, f.N[0]);
  f.N[1] = fmaf(wgt, q4.y, f.N[1]);
  f.N[2] = fmaf(wgt, q4.z, f.N[2]);
  f.D = fmaf(wgt, zf, f.D);
  const bool m = upd && f.T > 0.5f;
  f.Dm = m ? zf : f.Dm;
  f.med = m ? e_idx : f.med;
  f.last = upd ? e_idx : f.last;
  // a pixel that takes the entry but would fall below 1e-4 stops in front of it
  f.T = upd ? Tn : (take ? -f.T : f.T);
  return true;
}

// Quadrants (of the subset kSub) with a running pixel (wave-uniform bit mask).
template <uint32_t kSub>
__device__ __forceinline__ uint32_t live_quadrants(const FwdState (&f)[4]) {
  uint32_t m = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if ((kSub >> k) & 1u) m |= (__ballot(f[k].T > 0.f) != 0 ? 1u : 0u) << k;
  return m;
}

// Forward of the quadrants kSub of one tile (bit k: 8x8 quadrant k).  kSub = 0xf is the whole tile, a lane
// holding one pixel in each quadrant; a heavy tile runs as two halves (0x3, 0xc) or four single quadrants
// in separate waves.  Every subset runs the per-quadrant arithmetic of the whole tile (eval_px<k> from
// the lane terms at the quadrant-0 pixel), so the decisions do not depend on the split.  The reverse
// pass's per-entry quadrant bits go to img.qmask: a plain byte store for a whole tile, an atomic OR on
// the entry's word for a split one (its waves share the byte, which is cleared before the launch).
// kCount: instead of images, count the (pixel, list entry) pairs of the method (every entry a running
// pixel meets, quadrant mask or not), the contributing pairs, and the pairs the reverse walks.
// kContrib: instead of images, add each surfel's contribution sums (Sec. 3.3, Eq. 3) of this view into
// a.cws, one wave reduction and one atomic pair per (surfel, tile or split block).
template <bool kCount, bool kMask, bool kContrib, uint32_t kSub>
__device__ __forceinline__ void render_fwd_tile(const RenderArgs& a, Stage& s, uint32_t b) {
  const int lv = (int)(b / (uint32_t)a.tiles);
  const int v = a.cams.v0 + lv;
  const int t = (int)(b % (uint32_t)a.tiles);
  const int tx = t % a.tiles_x, ty = t / a.tiles_x;
  const DevCam& c = a.cams.c[lv];
  const int W = c.W, H = c.H;
  const int lane = threadIdx.x;
  const int lx = lane & 7, ly = lane >> 3;
  const int ox = tx * kTile, oy = ty * kTile;
  const uint32_t start = a.ranges[(int64_t)v * a.tiles + t], end = a.ranges[(int64_t)v * a.tiles + t + 1];
  const int64_t vn = (int64_t)v * a.n;

  FwdState f[4];
  unsigned long long n_eval = 0, n_con = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int px = ox + lx + 8 * (k & 1), py = oy + ly + 8 * (k >> 1);
    f[k].T = ((kSub >> k) & 1u) && px < W && py < H ? 1.f : -1.f;
    f[k].D = 0.f;
    f[k].Dm = 0.f;
    f[k].last = start - 1u;
    f[k].med = 0xffffffffu;
    f[k].C[0] = f[k].C[1] = f[k].C[2] = 0.f;
    f[k].N[0] = f[k].N[1] = f[k].N[2] = 0.f;
  }
  const float lx0 = (float)lx + 0.5f, ly0 = (float)ly + 0.5f;
  uint8_t* qmask = kMask ? a.img.qmask : nullptr;
  uint32_t qlive = live_quadrants<kSub>(f);
  // the list ids of the next chunk are loaded one chunk ahead: staging then waits on one load round trip
  // (the records) instead of two
  uint32_t nid = start + lane < end ? a.ids[start + lane] : 0u;
  for (uint32_t base = start; base < end && qlive != 0; base += 64) {
    const uint32_t idx = base + lane;
    const uint32_t id = nid;
    QuadBits qb;
    qb.from_lanes(idx < end ? stage_record(s, lane, a.rec, vn, a.n, id, ox, oy, nullptr, 0) : 0u);
    nid = idx + 64u < end ? a.ids[idx + 64u] : 0u;
    __syncthreads();
    const int cnt = (int)min(64u, end - base);
    int reached = cnt;  // entries of this chunk the wave evaluated
    // bit j of cq[k]: quadrant k had a taking pixel at entry base + j (scalar registers)
    uint64_t cq[4] = {0, 0, 0, 0};
    uint64_t cur = qb.w[0];  // entry j's nibble in bits 0-3
    for (int j = 0; j < cnt; ++j) {
      if (kCount) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if ((kSub >> k) & 1u) n_eval += f[k].T > 0.f ? 1u : 0u;
      }
      const uint32_t m = (uint32_t)cur & 0xfu & qlive;
      cur >>= 4;
      if (m != 0) {
        const float4 q0 = s.q[j][0], q1 = s.q[j][1], q2 = s.q[j][2], q3 = s.q[j][3], q4 = s.q[j][4];
        LaneTerms lt;
        lane_terms(lx0, ly0, q0, q1, q2, lt);
        const uint32_t e_idx = lane_copy(base + (uint32_t)j);
        float csum = 0.f, ccnt = 0.f;
        bool took = false;
        Px e[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          if (!((kSub >> k) & 1u)) continue;
          // (evaluated where it is used: the compiler sinks each pixel's evaluation into its branch)
          if (k == 0) eval_px<0>(lt, q2.y, e[0]);
          if (k == 1) eval_px<1>(lt, q2.y, e[1]);
          if (k == 2) eval_px<2>(lt, q2.y, e[2]);
          if (k == 3) eval_px<3>(lt, q2.y, e[3]);
          if (((m >> k) & 1u) && fwd_px<kContrib>(e[k], q2, q3, q4, e_idx, f[k], n_con, a.gamma, csum, ccnt)) {
            took = true;
            if (kMask) cq[k] |= 1ull << j;
          }
        }
        if (kContrib && took) {
          const float ts = wave_sum_lane63(csum), tc = wave_sum_lane63(ccnt);
          if (lane == 63 && tc > 0.f) {
            float* w = a.cws + 2 * (vn + (int64_t)__float_as_uint(q3.w));
            atomicAdd(w, ts);
            atomicAdd(w + 1, tc);
          }
        }
      }
      if ((j & 15) == 15) {
        qlive = live_quadrants<kSub>(f);
        if (qlive == 0) {
          reached = j + 1;
          break;
        }
        cur = qb.word((j + 1) >> 4);
      }
    }
    // entries past 'reached' lie beyond every pixel's 'last': the reverse pass never reads them
    if (kMask && lane < reached) {
      const uint32_t bits = (uint32_t)((cq[0] >> lane) & 1u) | (uint32_t)((cq[1] >> lane) & 1u) << 1 |
                            (uint32_t)((cq[2] >> lane) & 1u) << 2 | (uint32_t)((cq[3] >> lane) & 1u) << 3;
      if (kSub == 0xfu) qmask[idx] = (uint8_t)bits;
      else if (bits) atomicOr((uint32_t*)(qmask + (idx & ~3u)), bits << (8u * (idx & 3u)));
    }
    qlive = live_quadrants<kSub>(f);
    __syncthreads();
  }
  if (kContrib) return;
  if (kCount) {
    unsigned long long n_bwd = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int px = ox + lx + 8 * (k & 1), py = oy + ly + 8 * (k >> 1);
      if (((kSub >> k) & 1u) && px < W && py < H) n_bwd += f[k].last + 1u - start;
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
    const int px = ox + lx + 8 * (k & 1), py = oy + ly + 8 * (k >> 1);
    if (!((kSub >> k) & 1u) || !(px < W && py < H)) continue;
    const int64_t p = (int64_t)py * W + px;
    const float T = fabsf(f[k].T);
    if (im.rgb) {
      float* o = im.rgb + (int64_t)v * 3 * HW + p;
      o[0] = fmaf(T, c.bg[0], f[k].C[0]);
      o[HW] = fmaf(T, c.bg[1], f[k].C[1]);
      o[2 * HW] = fmaf(T, c.bg[2], f[k].C[2]);
    }
    if (im.normal) {
      float* o = im.normal + (int64_t)v * 3 * HW + p;
      o[0] = f[k].N[0];
      o[HW] = f[k].N[1];
      o[2 * HW] = f[k].N[2];
    }
    const int64_t vp = (int64_t)v * HW + p;
    if (im.depth) im.depth[vp] = f[k].D;
    if (im.depth_med) im.depth_med[vp] = f[k].Dm;
    if (im.alpha) im.alpha[vp] = 1.f - T;
    if (im.T_final) im.T_final[vp] = T;
    if (im.last) im.last[vp] = f[k].last + 1u;
    if (im.med) im.med[vp] = f[k].med;
  }
}

template <bool kCount, bool kMask, bool kContrib>
__global__ __launch_bounds__(64) void k_render_fwd(RenderArgs a) {
  __shared__ Stage s;
  uint32_t sub;
  const uint32_t b = tile_of_block(a, sub);
  if (*a.status != 0) return;
  switch (sub) {
    case 0x1u: render_fwd_tile<kCount, kMask, kContrib, 0x1u>(a, s, b); break;
    case 0x2u: render_fwd_tile<kCount, kMask, kContrib, 0x2u>(a, s, b); break;
    case 0x4u: render_fwd_tile<kCount, kMask, kContrib, 0x4u>(a, s, b); break;
    case 0x8u: render_fwd_tile<kCount, kMask, kContrib, 0x8u>(a, s, b); break;
    case 0x3u: render_fwd_tile<kCount, kMask, kContrib, 0x3u>(a, s, b); break;
    case 0xcu: render_fwd_tile<kCount, kMask, kContrib, 0xcu>(a, s, b); break;
    default: render_fwd_tile<kCount, kMask, kContrib, 0xfu>(a, s, b); break;
  }
}

struct BwdArgs {
  RenderArgs r;
  cgv2_image_grad up;
  RecGrads rg;
};

__device__ __forceinline__ float ldg0(const float* p, int64_t i) { return p ? p[i] : 0.f; }

// Per-pixel state of the reverse walk.  The upstream gradients are held multiplied by -2 (exact), which
// makes 2 d rho come out of the chain directly (rho is half the distance, and d alpha_raw / d rho =
// -alpha_raw); the fields that take them linearly (colour, normal, opacity) are scaled back once per
// (surfel, tile) at the atomics.  Instead of the colour (normal, depth) sums of the fragments behind,
// the walk keeps their dot products with the upstream gradients: sA for the total upstream, sS for the
// SSIM-only one; the background (and the alpha-image term) starts them.
struct BwdState {
  float T, sA, sS, GC[3], GS[3], GN[3], GD2, GD, GM;
  uint32_t last, med;
};

// Pixel (px, py) of view v: its checkpoint (T, last, median id) and upstream gradients.
template <bool kGeom>
__device__ __forceinline__ void bwd_init(const BwdArgs& A, const DevCam& c, int v, int px, int py, uint32_t start,
                                         uint32_t end, BwdState& p) {
  const int W = c.W, H = c.H;
  const int64_t HW = (int64_t)W * H;
  const bool in = px < W && py < H;
  const int64_t pp = in ? (int64_t)py * W + px : 0;
  const int64_t vp = (int64_t)v * HW + pp;
  const int64_t v3 = (int64_t)v * 3 * HW + pp;
  p.last = in ? min(max(A.r.img.last[vp], start), end) : start;
  p.med = in ? A.r.img.med[vp] : 0xffffffffu;
  const float Tf = in ? A.r.img.T_final[vp] : 1.f;
  p.T = Tf;
  float bA = 0.f, bS = 0.f;
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    p.GC[ch] = -2.f * (in ? ldg0(A.up.d_rgb, v3 + ch * HW) : 0.f);
    p.GS[ch] = -2.f * (in ? ldg0(A.up.d_rgb_ssim, v3 + ch * HW) : 0.f);
    p.GN[ch] = -2.f * (kGeom && in ? ldg0(A.up.d_normal, v3 + ch * HW) : 0.f);
    bA = fmaf(p.GC[ch], c.bg[ch], bA);
    bS = fmaf(p.GS[ch], c.bg[ch], bS);
  }
  p.GD = kGeom && in ? ldg0(A.up.d_depth, vp) : 0.f;
  p.GM = kGeom && in ? ldg0(A.up.d_depth_med, vp) : 0.f;
  p.GD2 = -2.f * p.GD;
  // alpha = 1 - T_final: d alpha / d alpha_i = T_final / (1 - alpha_i), the same factor as the blend terms
  const float GA = kGeom && in ? ldg0(A.up.d_alpha, vp) : 0.f;
  p.sA = fmaf(2.f * GA, Tf, Tf * bA);
  p.sS = Tf * bS;
}

// One pixel's share of the record gradients of a staged surfel.  Branch-free: a pixel that does not
// take this surfel (entry at or past its 'last', or alpha below 1/255) adds zero and keeps its T.
// acc[G_OP] collects 2 d rho (the opacity gradient is -alpha_raw d rho / o, formed at the atomics);
// acc[G_R..G_B] and the normal sums collect -2 times their gradients.
template <int k, bool kGeom>
__device__ __forceinline__ void bwd_px(const LaneTerms& lt, const float4& q0, const float4& q1, const float4& q2,
                                       const float4& q3, const float4& q4, uint32_t e_idx, BwdState& p,
                                       float (&acc)[kGradFields], bool& any) {
  Px e;
  eval_px<k>(lt, q2.y, e);
  const bool con = e_idx < p.last && e.alpha >= kAlphaMin;
  // for a quadrant without a contributing pixel every update below is the identity
  if (__ballot(con) == 0) return;
  any = true;  // wave-uniform: some pixel takes the entry
  const float a11 = q0.z, a12 = q0.w, a21 = q1.x, a22 = q1.y, w0 = q1.z, w1 = q1.w, w2 = q2.x;
  const float zc = q2.z, zw = q2.w;
  const float al = con ? e.alpha : 0.f;
  const float rom = __builtin_amdgcn_rcpf(1.f - al);
  const float ar = al * rom;  // alpha / (1 - alpha)
  // upstream . (this fragment's attributes), for the total and the SSIM-only upstream
  float g = fmaf(p.GC[0], q3.x, fmaf(p.GC[1], q3.y, p.GC[2] * q3.z));
  const float gs = fmaf(p.GS[0], q3.x, fmaf(p.GS[1], q3.y, p.GS[2] * q3.z));
  float zf = 0.f;
  if (kGeom) {
    zf = e.is3d ? zw * e.iw : zc;
    g = fmaf(p.GN[0], q4.x, g);
    g = fmaf(p.GN[1], q4.y, g);
    g = fmaf(p.GN[2], q4.z, g);
    g = fmaf(p.GD2, zf, g);
  }
  // Tn = the transmittance after this fragment (its last use is the step back to the one in front, so
  // the step writes in place)
  const float Tn = p.T;
  // 2 (1 - alpha) dL/dalpha: what lies behind minus T in front times this fragment's attributes
  const float nA = fmaf(-Tn, g, p.sA);
  const float nS = fmaf(-Tn, gs, p.sS);
  const float wgt = Tn * ar;  // alpha T_i
  p.T = Tn * rom;             // T_i, in front of it
  p.sA = fmaf(wgt, g, p.sA);
  p.sS = fmaf(wgt, gs, p.sS);
  // d alpha / d alpha_raw / (1 - alpha): the 0.99 clamp blocks the path to o and rho; below it alpha is
  // alpha_raw, and a pixel that does not take the entry has al = 0
  const float rA = e.araw > kAlphaMax ? 0.f : ar;
  acc[G_R] = fmaf(p.GC[0], wgt, acc[G_R]);
  acc[G_G] = fmaf(p.GC[1], wgt, acc[G_G]);
  acc[G_B] = fmaf(p.GC[2], wgt, acc[G_B]);
  float dz = 0.f;
  if (kGeom) {
    acc[G_NX] = fmaf(p.GN[0], wgt, acc[G_NX]);
    acc[G_NY] = fmaf(p.GN[1], wgt, acc[G_NY]);
    acc[G_NZ] = fmaf(p.GN[2], wgt, acc[G_NZ]);
    dz = fmaf(p.GD, wgt, con && e_idx == p.med ? p.GM : 0.f);
  }
  // -2 d rho of either upstream
  const float ndr = rA * nA;
  const float nds = rA * nS;
  acc[G_OP] -= ndr;
  // (vx, vy) = d rho / d(x', y') / 2: the centre gradient of either upstream is -2 d rho * (vx, vy)
  float vx, vy;
  if (e.is3d) {
    // rho = |P|^2 / (2 w^2) with P = (P1, P2), so d rho = (P . dP) / w^2 - 2 rho dw / w
    const float iw = e.iw, iww = iw * iw;
    const float u1 = e.P1 * iww, u2 = e.P2 * iww, uw = e.rho * iw;
    const float nP1 = ndr * u1, nP2 = ndr * u2;
    // the intersection depth z_c w0 / w also depends on w
    const float dzw = kGeom ? dz * zf * iw : 0.f;
    const float gw = kGeom ? fmaf(ndr, uw, -dzw) : ndr * uw;
    acc[G_A11] = fmaf(-nP1, e.xr, acc[G_A11]);
    acc[G_A12] = fmaf(-nP1, e.yr, acc[G_A12]);
    acc[G_A21] = fmaf(-nP2, e.xr, acc[G_A21]);
    acc[G_A22] = fmaf(-nP2, e.yr, acc[G_A22]);
    acc[G_W0] += kGeom ? fmaf(dz * zc, iw, gw) : gw;
    acc[G_W1] = fmaf(gw, e.xr, acc[G_W1]);
    acc[G_W2] = fmaf(gw, e.yr, acc[G_W2]);
    if (kGeom) {
      acc[G_ZC] = fmaf(dz, w0 * iw, acc[G_ZC]);
      acc[G_CX] = fmaf(dzw, w1, acc[G_CX]);
      acc[G_CY] = fmaf(dzw, w2, acc[G_CY]);
    }
    vx = fmaf(u1, a11, fmaf(u2, a21, -uw * w1));
    vy = fmaf(u1, a12, fmaf(u2, a22, -uw * w2));
  } else {
    vx = e.xr;
    vy = e.yr;
    if (kGeom) acc[G_ZC] += dz;
  }
  acc[G_CX] = fmaf(ndr, vx, acc[G_CX]);
  acc[G_CY] = fmaf(ndr, vy, acc[G_CY]);
  acc[G_SCX] = fmaf(nds, vx, acc[G_SCX]);
  acc[G_SCY] = fmaf(nds, vy, acc[G_SCY]);
}

// Factor that turns the reduced value of field 'slot' into its record gradient: the staged numerator
// coefficients carry 1/sqrt(2), the colour fields -2.  (The opacity field, 2 d rho, takes -1 / (2 o) of
// its surfel instead.)
__device__ __forceinline__ float slot_scale(int slot) {
  if (slot >= G_A11 && slot <= G_A22) return kInvSqrt2;
  return slot >= G_R && slot <= G_B ? -0.5f : 1.f;
}

// Adds one staged entry's wave-summed record gradients (acc of every lane) into (view, surfel) 'id':
// fields G_CX..G_ZC by reduce-scatter (one atomic instruction, one lane per field), the normals (kGeom)
// from lane 63.  sc = slot_scale of the lane's field.
template <bool kGeom>
__device__ __forceinline__ void bwd_commit(float (&acc)[kGradFields], int lane, int slot, float sc, float io,
                                           float* rgv, float* rgn, uint32_t id) {
  float red[16];
#pragma unroll
  for (int f = 0; f < 16; ++f) red[f] = acc[f];
  const float tot = reduce16_scatter(red);
  if ((lane & 12) == 0 && (kGeom || slot != G_ZC))
    atomicAdd(rgv + (int64_t)id * kGradRow + slot, tot * (slot == G_OP ? -0.5f * io : sc));
  if (kGeom) {
    const float nx = wave_sum_lane63(acc[G_NX]), ny = wave_sum_lane63(acc[G_NY]), nz = wave_sum_lane63(acc[G_NZ]);
    if (lane == 63) {
      float* w = rgn + (int64_t)id * kGradNrm;
      atomicAdd(w, -0.5f * nx);
      atomicAdd(w + 1, -0.5f * ny);
      atomicAdd(w + 2, -0.5f * nz);
    }
  }
}

// Reverse pass over the quadrants kSub of one tile (as render_fwd_tile): each entry's record gradients
// summed over the block's pixels and added per (surfel, tile or split block).
// kGeom: depth, median-depth, normal or alpha upstream gradients are present.  Without them (the
// photometric-loss-only case) their per-pixel state, terms and four of the reductions drop out.
template <bool kGeom, uint32_t kSub>
__device__ __forceinline__ void render_bwd_tile(const BwdArgs& A, Stage& s, uint32_t b) {
  const RenderArgs& a = A.r;
  const int lv = (int)(b / (uint32_t)a.tiles);
  const int v = a.cams.v0 + lv;
  const int t = (int)(b % (uint32_t)a.tiles);
  const int tx = t % a.tiles_x, ty = t / a.tiles_x;
  const DevCam& c = a.cams.c[lv];
  const int lane = threadIdx.x;
  const int lx = lane & 7, ly = lane >> 3;
  const int ox = tx * kTile, oy = ty * kTile;
  const uint32_t start = a.ranges[(int64_t)v * a.tiles + t], end = a.ranges[(int64_t)v * a.tiles + t + 1];
  const int64_t vn = (int64_t)v * a.n;
  float* rgv = A.rg.row + (int64_t)v * a.n * kGradRow;
  float* rgn = A.rg.nrm + (int64_t)v * a.n * kGradNrm;

  BwdState p[4];
  // per-quadrant wave maxima of 'last': quadrant k has nothing to walk at or above qhi[k]
  uint32_t qhi[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    qhi[k] = start;
    if (!((kSub >> k) & 1u)) continue;
    bwd_init<kGeom>(A, c, v, ox + lx + 8 * (k & 1), oy + ly + 8 * (k >> 1), start, end, p[k]);
    uint32_t h = p[k].last;
    for (int off = 1; off < 64; off <<= 1) h = max(h, __shfl_xor(h, off));
    qhi[k] = uniform(h);
  }
  const uint32_t hi = max(max(qhi[0], qhi[1]), max(qhi[2], qhi[3]));
  const float lx0 = (float)lx + 0.5f, ly0 = (float)ly + 0.5f;
  const int slot = reduce16_index(lane);
  const float sc = slot_scale(slot);

  // the list ids of the next (lower) chunk are loaded one chunk ahead, as in the forward
  uint32_t nlo = hi - start > 64u ? hi - 64u : start;
  uint32_t nid = nlo + lane < hi ? a.ids[nlo + lane] : 0u;
  for (uint32_t top = hi; top > start;) {
    const uint32_t lo = nlo;
    const uint32_t idx = lo + lane;
    const uint32_t id = nid;
    QuadBits qb;
    {
      // the subset's quadrants, each only below its walk bound
      uint32_t allow = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) allow |= (((kSub >> k) & 1u) && idx < qhi[k] ? 1u : 0u) << k;
      qb.from_lanes(idx < top ? stage_record(s, lane, a.rec, vn, a.n, id, ox, oy, a.img.qmask, idx) & allow : 0u);
    }
    nlo = lo - start > 64u ? lo - 64u : start;
    nid = nlo + lane < lo ? a.ids[nlo + lane] : 0u;
    __syncthreads();
    const int j0 = (int)(top - lo) - 1;
    uint64_t cur = qb.word(j0 >> 4) << (4 * (15 - (j0 & 15)));  // entry j's nibble in bits 60-63
    for (int j = (int)(top - lo) - 1; j >= 0; --j) {
      const uint32_t e_idx = lo + (uint32_t)j;
      if ((j & 15) == 15) cur = qb.word(j >> 4);
      const uint32_t m = (uint32_t)(cur >> 60);  // quadrant bits, kSub and the quadrants' walk bounds applied
      cur <<= 4;
      if (m == 0) continue;
      const float4 q0 = s.q[j][0], q1 = s.q[j][1], q2 = s.q[j][2], q3 = s.q[j][3], q4 = s.q[j][4];
      LaneTerms lt;
      lane_terms(lx0, ly0, q0, q1, q2, lt);
      float acc[kGradFields];
#pragma unroll
      for (int f = 0; f < kGradFields; ++f) acc[f] = 0.f;
      bool any = false;
      if ((kSub & 1u) && (m & 1u)) bwd_px<0, kGeom>(lt, q0, q1, q2, q3, q4, e_idx, p[0], acc, any);
      if ((kSub & 2u) && (m & 2u)) bwd_px<1, kGeom>(lt, q0, q1, q2, q3, q4, e_idx, p[1], acc, any);
      if ((kSub & 4u) && (m & 4u)) bwd_px<2, kGeom>(lt, q0, q1, q2, q3, q4, e_idx, p[2], acc, any);
      if ((kSub & 8u) && (m & 8u)) bwd_px<3, kGeom>(lt, q0, q1, q2, q3, q4, e_idx, p[3], acc, any);
      if (!any) continue;
      bwd_commit<kGeom>(acc, lane, slot, sc, q4.w, rgv, rgn, __float_as_uint(q3.w));
    }
    __syncthreads();
    top = lo;
  }
}

template <bool kGeom>
__global__ __launch_bounds__(64) void k_render_bwd(BwdArgs A) {
  __shared__ Stage s;
  uint32_t sub;
  const uint32_t b = tile_of_block(A.r, sub);
  if (*A.r.status != 0) return;
  switch (sub) {
    case 0x1u: render_bwd_tile<kGeom, 0x1u>(A, s, b); break;
    case 0x2u: render_bwd_tile<kGeom, 0x2u>(A, s, b); break;
    case 0x4u: render_bwd_tile<kGeom, 0x4u>(A, s, b); break;
    case 0x8u: render_bwd_tile<kGeom, 0x8u>(A, s, b); break;
    case 0x3u: render_bwd_tile<kGeom, 0x3u>(A, s, b); break;
    case 0xcu: render_bwd_tile<kGeom, 0xcu>(A, s, b); break;
    default: render_bwd_tile<kGeom, 0xfu>(A, s, b); break;
  }
}

// Clears the record gradients of the surfels in view v's visible list (the atomics add into them).
__global__ __launch_bounds__(256) void k_zero_visible(const uint32_t* __restrict__ visible,
                                                     const uint32_t* __restrict__ vstart, int64_t n, RecGrads rg,
                                                     int v0) {
  const int v = v0 + (int)blockIdx.y;
  const uint32_t e0 = vstart[v], e1 = vstart[v + 1];
  const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
  for (uint32_t e = e0 + blockIdx.x * blockDim.x + threadIdx.x; e < e1; e += gridDim.x * blockDim.x) {
    const int64_t vi = (int64_t)v * n + visible[e];
    float4* r = (float4*)(rg.row + vi * kGradRow);
#pragma unroll
    for (int k = 0; k < 4; ++k) r[k] = z;
    *(float4*)(rg.nrm + vi * kGradNrm) = z;
  }
}

}  // namespace cgv2

// Heavy tiles split over several waves: the 1 / kSplitDiv heaviest of a launch's tiles (at most
// kSplitMax) into four quadrant blocks, the next 1 / kHalfDiv (at most kSplitMax; none for 0) into two
// halves.
#ifndef CGV2_SPLIT_DIV
#define CGV2_SPLIT_DIV 48
#endif
#ifndef CGV2_HALF_DIV
#define CGV2_HALF_DIV 12
#endif
constexpr int kSplitDiv = CGV2_SPLIT_DIV;
constexpr int kHalfDiv = CGV2_HALF_DIV;
constexpr int kSplitMax = 1024;

namespace cgv2 {
// Clears the quadrant-mask bytes of the split tiles' lists (their blocks OR their bits in).
__global__ __launch_bounds__(256) void k_clear_split_qmask(RenderArgs a) {
  if (*a.status != 0) return;  // overflowed bins: ranges may lie beyond the list arrays
  const uint32_t tiles = (uint32_t)a.cams.count * (uint32_t)a.tiles;
  const uint32_t b0 = a.order[blockIdx.x];
  const uint32_t b = b0 < tiles ? b0 : tiles - 1u;
  const int v = a.cams.v0 + (int)(b / (uint32_t)a.tiles), t = (int)(b % (uint32_t)a.tiles);
  const uint32_t start = a.ranges[(int64_t)v * a.tiles + t], end = a.ranges[(int64_t)v * a.tiles + t + 1];
  for (uint32_t e = start + threadIdx.x; e < end; e += blockDim.x) a.img.qmask[e] = 0;
}
}  // namespace cgv2

static cgv2::RenderArgs make_args(const cgv2_proj& p, const cgv2_bins& b, const cgv2::CamPack& cams, int64_t n,
                                  int tiles_x, int tiles_y, const cgv2_image* img, unsigned long long* counters) {
  cgv2::RenderArgs a;
  a.rec = p.rec;
  a.ids = b.ids;
  a.ranges = b.ranges;
  a.order = b.order ? b.order + (int64_t)cams.v0 * tiles_x * tiles_y : nullptr;
  a.status = b.status;
  a.cams = cams;
  a.n = n;
  a.tiles_x = tiles_x;
  a.tiles_y = tiles_y;
  a.tiles = tiles_x * tiles_y;
  if (img) a.img = *img; else a.img = cgv2_image{};
  a.counters = counters;
  a.cws = nullptr;
  a.gamma = 0.f;
  const int64_t all = (int64_t)cams.count * a.tiles;
  a.n_q = a.order ? (uint32_t)std::min<int64_t>(all / kSplitDiv, kSplitMax) : 0u;
  a.n_h = a.order && kHalfDiv > 0 ? (uint32_t)std::min<int64_t>({all / std::max(kHalfDiv, 1), (int64_t)kSplitMax,
                                                                   all - (int64_t)a.n_q})
                                  : 0u;
  return a;
}

hipError_t cgv2_launch_render_fwd(const cgv2_proj& p, const cgv2_bins& b, const cgv2::CamPack& cams, int64_t n,
                                  int tiles_x, int tiles_y, const cgv2_image& img, hipStream_t st) {
  cgv2::RenderArgs a = make_args(p, b, cams, n, tiles_x, tiles_y, &img, nullptr);
  const unsigned grid = (unsigned)((int64_t)cams.count * a.tiles + 3 * a.n_q + a.n_h);
  if (img.qmask && a.n_q + a.n_h)
    hipLaunchKernelGGL(cgv2::k_clear_split_qmask, dim3(a.n_q + a.n_h), dim3(256), 0, st, a);
  if (img.qmask) hipLaunchKernelGGL((cgv2::k_render_fwd<false, true, false>), dim3(grid), dim3(64), 0, st, a);
  else hipLaunchKernelGGL((cgv2::k_render_fwd<false, false, false>), dim3(grid), dim3(64), 0, st, a);
  return hipGetLastError();
}

hipError_t cgv2_launch_render_count(const cgv2_proj& p, const cgv2_bins& b, const cgv2::CamPack& cams, int64_t n,
                                    int tiles_x, int tiles_y, unsigned long long* counters, hipStream_t st) {
  cgv2::RenderArgs a = make_args(p, b, cams, n, tiles_x, tiles_y, nullptr, counters);
  const unsigned grid = (unsigned)((int64_t)cams.count * a.tiles + 3 * a.n_q + a.n_h);
  hipLaunchKernelGGL((cgv2::k_render_fwd<true, false, false>), dim3(grid), dim3(64), 0, st, a);
  return hipGetLastError();
}

hipError_t cgv2_launch_render_bwd(const cgv2_proj& p, const cgv2_bins& b, const cgv2::CamPack& cams, int64_t n,
                                  int tiles_x, int tiles_y, const cgv2_image& img, const cgv2_image_grad& up,
                                  const cgv2::RecGrads& rg, hipStream_t st) {
  if (n > 0) {
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(cgv2::k_zero_visible, dim3(blocks, (unsigned)cams.count), dim3(256), 0, st, p.visible,
                       p.visible_start, n, rg, cams.v0);
  }
  cgv2::BwdArgs A;
  A.r = make_args(p, b, cams, n, tiles_x, tiles_y, &img, nullptr);
  A.up = up;
  A.rg = rg;
  const unsigned grid = (unsigned)((int64_t)cams.count * A.r.tiles + 3 * A.r.n_q + A.r.n_h);
  const bool geom = up.d_depth || up.d_depth_med || up.d_normal || up.d_alpha;
  if (geom) hipLaunchKernelGGL(cgv2::k_render_bwd<true>, dim3(grid), dim3(64), 0, st, A);
  else hipLaunchKernelGGL(cgv2::k_render_bwd<false>, dim3(grid), dim3(64), 0, st, A);
  return hipGetLastError();
}

hipError_t cgv2_launch_contribution(const cgv2_proj& p, const cgv2_bins& b, const cgv2::CamPack& cams, int64_t n,
                                    int tiles_x, int tiles_y, float gamma, float* cws, hipStream_t st) {
  cgv2::RenderArgs a = make_args(p, b, cams, n, tiles_x, tiles_y, nullptr, nullptr);
  a.cws = cws;
  a.gamma = gamma;
  const unsigned grid = (unsigned)((int64_t)cams.count * a.tiles + 3 * a.n_q + a.n_h);
  hipLaunchKernelGGL((cgv2::k_render_fwd<false, false, true>), dim3(grid), dim3(64), 0, st, a);
  return hipGetLastError();
}
