/* cgv2r.h -- C ABI of an MI355X (gfx950) differentiable 2D-Gaussian surfel tile rasterizer.
 *
 * The operations follow CityGaussianV2 (arXiv 2411.00771):
 *   - surfels {mu, tangents t_u, t_v, scales (s_u, s_v), opacity, SH features} of the 2DGS
 *     model (Sec. 3.1, "2D Gaussian Splatting" paragraph);
 *   - colour by front-to-back alpha blending (Sec. 3.1, Eq. 1), plus the depth (Sec. 3.2;
 *     median depth, Sec. 5.1) and normal (Sec. 3.1) renders the losses need;
 *   - the decomposed (SSIM-only) densification gradient (Sec. 3.2, Eq. 2) and the
 *     elongation rate eta = min(s_u, s_v) / max(s_u, s_v) (Sec. 3.2).
 *
 * Conventions shared by every call
 *   - Array pointers are DEVICE pointers owned by the caller, contiguous, 16-byte aligned
 *     (256-byte recommended).  Structs themselves live in host memory and are read during
 *     the call only.  Layouts are planar: field[c][n] for per-surfel data, [V][c][H][W] for
 *     images.
 *   - Every call enqueues work on the given HIP stream (NULL = the null stream) and returns
 *     without synchronising.  The library never allocates device memory, never prints and
 *     never aborts.  Its only state: a thread-local last-HIP-error code, a thread-local record of
 *     which devices are gfx950, and the fixed per-GPU buffer of cgv2_densify_stats_noalloc.
 *   - Every call that launches work first checks that the calling thread's current HIP device is a
 *     gfx950 (CGV2_EUNSUPPORTED otherwise, also when no device is present), after its argument
 *     checks.
 *   - Data layout.  The problem is stated per surfel and per view (Sec. 3.1): a surfel's screen
 *     transform, colour, normal, opacity and cutoff, per-tile lists ordered by depth, per-pixel images.
 *     The buffers below carry exactly that, arranged for the GPU rather than as separate key/value
 *     arrays: one 96-byte record per (view, surfel) holding the projection's outputs (read whole by the
 *     render's staging), the tile lists as sorted ids plus ranges (the sort key is rebuilt from the
 *     record and never stored), and the per-pixel checkpoint of the reverse pass.
 *   - Return value: CGV2_OK or a negative CGV2_E* code.  On an error nothing was enqueued
 *     (CGV2_EHIP: a launch failed; cgv2_last_hip_error() gives the hipError_t).
 *   - Conditions found on the device (intersection overflow) are reported through device
 *     words, never through return codes.
 *   - The V cameras of one call must share width and height.
 *   - Pixel (i, j) is sampled at (i + 0.5, j + 0.5).  Tiles are 16 x 16 pixels, numbered
 *     row-major per view: tile = ty * tiles_x + tx.
 */
#ifndef CGV2R_H
#define CGV2R_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CGV2_OK 0
#define CGV2_EINVAL (-1)      /* null pointer, n < 0, V < 1, sh_degree outside 0..3, W/H <= 0,
                                 more than 65535 tiles per axis, mismatched camera sizes */
#define CGV2_EWORKSPACE (-2)  /* workspace smaller than the matching *_workspace() size */
#define CGV2_EUNSUPPORTED (-3)/* no usable gfx950 device */
#define CGV2_EHIP (-4)        /* a HIP launch failed */

#define CGV2_TILE 16
#define CGV2_REC_FLOATS 24    /* floats per render record, see cgv2_proj */

/* project flags (cgv2_proj.flags) */
#define CGV2_F_VISIBLE 1u     /* tile rect non-empty: the surfel is binned in this view */
#define CGV2_F_NEAR 2u        /* centre depth <= znear */
#define CGV2_F_OPACITY 4u     /* opacity <= 1/255: alpha can never reach the 1/255 skip level */
#define CGV2_F_BEHIND 8u      /* the cutoff disc is not entirely in front of the camera */
#define CGV2_F_NONFINITE 16u  /* NaN/Inf parameter */
#define CGV2_F_LOWPASS 32u    /* the screen low-pass filter wins at the sample nearest the centre
                                 (the sub-pixel case of Sec. 3.2) */

/* Pinhole camera.  World -> camera: Xc = R Xw + t (row-major R; x right, y down, z forward). */
typedef struct {
  int32_t width, height;
  float fx, fy, cx, cy;
  float R[9], t[3];
  float znear;   /* surfels whose centre depth <= znear are culled */
  float bg[3];   /* background colour added with the final transmittance */
} cgv2_camera;

/* Surfel parameters (Sec. 3.1): n surfels, float32.
 *   Geometry planar SoA: mean[3][n]; log_scale[2][n] (s = exp); quat[4][n] (w, x, y, z;
 *   normalised inside; the rotation's columns are t_u, t_v and the surfel normal);
 *   opacity_logit[n] (sigmoid).
 *   Colour as one block per surfel: sh[n][(deg+1)^2][3] real SH coefficients, index l*l + l + m,
 *   colour = max(0, 0.5 + sum f Y) with the Condon-Shortley phase (Y_1^1 = -sqrt(3/4pi) x).  (Only
 *   the surfels visible in a view read their SH, so a per-surfel block is read whole instead of
 *   one cache line per coefficient.) */
typedef struct {
  int64_t n;
  int32_t sh_degree;
  const float *mean, *log_scale, *quat, *opacity_logit, *sh;
} cgv2_surfels;

/* Serving storage of a trained set (Sec. 3.3: SH degree 2 from the start; the appendix's vector-tree
 * quantization: the least important surfels' SH replaced by a codebook row, everything else but the
 * positions in float16).  uint16_t arrays hold IEEE float16 bits (codes and codebook rows excepted).
 *   mean[3][n] float32; log_scale[2][n], quat[4][n], opacity_logit[n] float16;
 *   sh[n_full][(deg+1)^2][3] float16 for the surfels [0, n_full);
 *   code[n - n_full]: codebook row of surfel n_full + j (a row >= codebook_size culls the surfel, as a
 *   non-finite parameter would);
 *   codebook[codebook_size][(deg+1)^2][3] float16.
 * The decoded float32 values go through the projection unchanged: a compact set projects exactly like
 * its decoded float32 copy. */
typedef struct {
  int64_t n, n_full;
  int32_t sh_degree, codebook_size;
  const float* mean;
  const uint16_t *log_scale, *quat, *opacity_logit, *sh, *code, *codebook;
} cgv2_surfels_compact;

/* Per-view projection.  rec[V][n][24] is written for visible surfels only:
 *   0,1  cx_hi, cy_hi   integer part of the projected centre (pixels)
 *   2,3  cx_lo, cy_lo   remainder: centre = hi + lo
 *   4-7  a11 a12 a21 a22  with x' = x - cx, y' = y - cy the ray through (x, y) meets the surfel
 *   8-10 w0 w1 w2        plane at local (u, v) = (a11 x' + a12 y', a21 x' + a22 y') / w,
 *                        w = w0 + w1 x' + w2 y' (the inverse homography, scaled to max |coef| = 1)
 *   11   z_c            centre depth (sort key); intersection depth = z_c w0 / w
 *   12   opacity        13-15 rgb   16-18 camera-space normal (facing the camera)   19 k^2 cutoff
 *   20,21 pixel rect (i0 | i1 << 16), (j0 | j1 << 16) as uint32 bits (inclusive, clamped to the image)
 *   22,23 zero
 * rect[V][n][4] = tx0, ty0, tx1, ty1 (end exclusive; all 0 when not visible); radius[V][n] screen
 * radius in pixels; flags[V][n] CGV2_F_* bits (written for every surfel).
 * visible[V * n], visible_start[V + 1]: written by cgv2_bin_sort; entries visible[visible_start[v] ..
 * visible_start[v + 1]) are the ids of the surfels visible in view v, ascending (the reverse pass walks
 * these lists instead of all n surfels). */
typedef struct {
  float* rec;
  uint16_t* rect;
  float* radius;
  uint8_t* flags;
  uint32_t* visible;
  uint32_t* visible_start;
} cgv2_proj;

/* Tile bins.  ranges[V * tiles + 1]: list of tile t in view v is ids[ranges[v*tiles + t] ..
 * ranges[v*tiles + t + 1]), ordered front to back by (float32 bits of z_c, id).  A surfel is listed in
 * the tiles of its rect where its alpha >= 1/255 region can reach a pixel sample: some point of the
 * tile's pixel-sample box, padded by 1/64 px, has min(rho_3d, rho_2d) <= k^2 (1 + 2e-3) + 2e-3 (every
 * pixel that can blend the surfel keeps it; Sec. 3.1 cutoff).
 * The staging holds one slot per tile of every rect: 'capacity' and *needed count those slots.
 * *status is set to 1 when they exceed 'capacity' (sticky: the library never clears it; the caller
 * zeroes it before the first call).  *needed receives the total number of rect slots of the call.
 * While *status != 0, bins are invalid, render calls write nothing and the caller must rerun with
 * capacity >= *needed.
 * order (optional, [V * tiles]): the render calls' launch order.  When non-NULL, cgv2_bin_sort writes
 * it and the render calls (forward, count, backward, contribution) launch the tiles of each chunk of up
 * to 32 views heaviest first: order[32 c tiles + i] = the i-th tile (local index v' tiles + t within
 * chunk c) by descending log-scale bucket of its list length, ties in index order.  It must come from
 * the same cgv2_bin_sort call as ranges.  NULL: tiles in spatial order.  Results are the same either
 * way, up to the summation order of the backward's atomics. */
typedef struct {
  int64_t capacity;  /* entries in ids (< 2^32 - 1) */
  uint32_t* ids;
  uint32_t* ranges;
  int32_t* status;
  int64_t* needed;
  uint32_t* order;   /* optional launch order, see above */
} cgv2_bins;

/* Rendered images [V][c][H][W] and the backward checkpoint.  rgb (Eq. 1, with T_final * bg),
 * depth = sum w z (not normalised), depth_med (depth of the last fragment whose incoming
 * transmittance exceeds 0.5; 0 if none), normal = sum w n (not normalised), alpha = 1 - T_final.
 * Checkpoint: T_final; last = one past the last contributing list entry; med = list index of
 * the median fragment (0xffffffff if none).  rgb/depth/depth_med/normal/alpha may be NULL;
 * T_final/last/med may be NULL when no backward pass follows.
 * qmask (optional, [bins.capacity], indexed like bins.ids): per tile-list entry, bit k set when some
 * pixel of quadrant k of the tile (k = (x >= 8) + 2 (y >= 8) within the 16x16 tile) takes the entry
 * as a contributing fragment.  Written by cgv2_render_fwd for the entries it reaches; when the
 * backward gets the same pointer it skips the entry/quadrant pairs without a contribution (same
 * result, less work).  One byte per intersection; no per-fragment state. */
typedef struct {
  float *rgb, *depth, *depth_med, *normal, *alpha, *T_final;
  uint32_t *last, *med;
  uint8_t* qmask;
} cgv2_image;

/* Upstream gradients [V][c][H][W]; any may be NULL (= zero).  d_rgb_ssim is the part of d_rgb
 * that comes from the SSIM term (the DGD source of Eq. 2); NULL gives g_view_ssim = 0. */
typedef struct {
  const float *d_rgb, *d_depth, *d_depth_med, *d_normal, *d_alpha;
  const float* d_rgb_ssim;
} cgv2_image_grad;

/* Parameter gradients accumulate (+=) over views and calls: the caller zeroes them.  Each has the
 * layout of its parameter (d_sh[n][(deg+1)^2][3]).
 * g_view_total / g_view_ssim [V][2][n] are overwritten: the gradient w.r.t. a rigid screen
 * translation of the surfel's image (the 2DGS form of the view-space position gradient of
 * Sec. 3.1), in NDC units (pixels * (W/2, H/2)), zero for surfels not visible in the view. */
typedef struct {
  float *d_mean, *d_log_scale, *d_quat, *d_opacity_logit, *d_sh;
  float *g_view_total, *g_view_ssim;
} cgv2_grads;

/* Densification parameters: omega of Eq. 2 (0.9 in Sec. 5.1), elongation threshold eta_min
 * (Sec. 3.2 leaves it open; 0.05 suggested), clone/split threshold on the accumulated
 * average DGD gradient (NDC units). */
typedef struct {
  float omega, eta_min, grad_threshold;
} cgv2_densify_params;

/* Densification state [n], accumulated across calls until the caller resets it.
 * mask bits: 1 high gradient, 2 elongated (eta < eta_min), 4 clone/split candidate
 * (high and not elongated), 8 low-pass dominant in a view of this call.
 * counters[8] (overwritten): visible (summed over views), high, elongated, high & elongated,
 * low-pass & visible (summed over views), candidates, 0, 0.  scale[V]: the Eq. 2 factor used
 * for each view. */
typedef struct {
  float *accum_dgd, *accum_total, *max_radius;
  int32_t* denom;
  uint8_t* mask;
  uint32_t* counters;
  float* scale;
} cgv2_densify_state;

/* Per-surfel projection of n surfels into V views (2DGS surfel model, Sec. 3.1).  Computes the
 * screen transform M = K [R s_u t_u | R s_v t_v | R mu + t] in FP64, SH colour, the normal
 * flipped to face the camera, sigmoid opacity, the cutoff k^2 = 2 ln(255 o) at which alpha
 * reaches 1/255, and the tile rect of the exact conic bound of the k-disc united with the
 * low-pass filter disc of radius k sqrt(2)/2 px (Sec. 3.2).
 * Errors: CGV2_EINVAL (nulls, bad sizes), CGV2_EHIP. */
int cgv2_project(const cgv2_surfels* s, const cgv2_camera* cams, int32_t V, cgv2_proj* proj, void* hip_stream);

/* cgv2_project for a compact set (serving).  Same outputs and rules.  Errors: CGV2_EINVAL (also
 * n_full outside [0, n], codebook_size outside [1, 65536] with n_full < n), CGV2_EHIP. */
int cgv2_project_compact(const cgv2_surfels_compact* s, const cgv2_camera* cams, int32_t V, cgv2_proj* proj,
                         void* hip_stream);

/* Workspace bytes for cgv2_bin_sort with the given capacity, view count, tiles per view and surfel
 * count (0 for invalid arguments). */
size_t cgv2_bin_sort_workspace(int64_t capacity, int32_t V, int32_t tiles_per_view, int64_t n);

/* Tile binning: prefix-sums every surfel's tile count, stages (tile, depth bits, id) per surfel,
 * prefix-sums the per-tile counts into ranges, places the keys in their tiles and sorts every tile's
 * list; depth ties are broken by id, so the order is deterministic and bit-exact.
 * Errors: CGV2_EINVAL, CGV2_EWORKSPACE, CGV2_EHIP. */
int cgv2_bin_sort(const cgv2_proj* proj, const cgv2_camera* cams, int32_t V, int64_t n, cgv2_bins* bins,
                  void* workspace, size_t ws_bytes, void* hip_stream);

/* Forward render (Sec. 3.1, Eq. 1): per pixel, front to back over its tile list,
 * alpha = min(0.99, o exp(-rho/2)) with rho = min(rho_3d, rho_2d) (ray-splat intersection vs
 * screen low-pass filter), entries with alpha < 1/255 skipped, stop before T(1 - alpha) < 1e-4.
 * Errors: CGV2_EINVAL, CGV2_EHIP. */
int cgv2_render_fwd(const cgv2_proj* proj, const cgv2_bins* bins, const cgv2_camera* cams, int32_t V, int64_t n,
                    cgv2_image* img, void* hip_stream);

/* Workspace bytes for cgv2_loss. */
size_t cgv2_loss_workspace(int32_t width, int32_t height, int32_t V);

/* Photometric loss of Sec. 3.1: L = (1 - lambda) mean|I - I*| + lambda (1 - SSIM(I, I*)), SSIM with
 * an 11x11 Gaussian window (sigma 1.5), C1 = 0.01^2, C2 = 0.03^2, zero padding, mean over pixels and
 * channels.  img, target: [V][3][H][W].  Writes d_img = dL/dI, d_img_ssim = d(lambda (1 - SSIM))/dI,
 * and loss[V][3] = {L, mean L1, SSIM}.  Errors: CGV2_EINVAL, CGV2_EWORKSPACE, CGV2_EHIP. */
int cgv2_loss(const float* img, const float* target, int32_t V, int32_t width, int32_t height, float lambda,
              float* d_img, float* d_img_ssim, float* loss, void* workspace, size_t ws_bytes, void* hip_stream);

/* Workspace bytes for cgv2_render_bwd. */
size_t cgv2_render_bwd_workspace(int64_t n, int32_t V);

/* Backward of project + render_fwd.  Traverses each pixel's list in reverse from the checkpoint
 * (T recovered as T_{i+1} / (1 - alpha_i); no per-fragment state is stored), reduces the per-surfel
 * gradients of every tile in registers and adds them atomically, then chains them to the
 * parameters.  Also writes the total and SSIM-only view-space gradients (Eq. 2's inputs).
 * img must hold T_final, last and med of the matching cgv2_render_fwd call.
 * Errors: CGV2_EINVAL, CGV2_EWORKSPACE, CGV2_EHIP. */
int cgv2_render_bwd(const cgv2_surfels* s, const cgv2_proj* proj, const cgv2_bins* bins, const cgv2_camera* cams,
                    int32_t V, const cgv2_image* img, const cgv2_image_grad* up, cgv2_grads* grads,
                    void* workspace, size_t ws_bytes, void* hip_stream);

/* The two stages of cgv2_render_bwd, callable on their own (same stream order, same workspace):
 *
 * cgv2_render_bwd_records: the reverse traversal of Eq. 1 only.  Writes, into the workspace, the
 * gradients of each (view, visible surfel) render record: the 9 screen-transform terms, opacity, colour,
 * the SSIM-only screen-position pair, the intersection depth and the normal (unspecified layout; the
 * workspace must stay untouched until cgv2_project_bwd has read it).
 * Errors: CGV2_EINVAL, CGV2_EWORKSPACE, CGV2_EHIP.
 *
 * cgv2_project_bwd: chains those record gradients to the parameters (d_* of grads, added to) and writes
 * both view-space gradients of every view.  proj, cams and V must be those of the records call.
 * Errors: CGV2_EINVAL, CGV2_EWORKSPACE, CGV2_EHIP. */
int cgv2_render_bwd_records(const cgv2_proj* proj, const cgv2_bins* bins, const cgv2_camera* cams, int32_t V,
                            int64_t n, const cgv2_image* img, const cgv2_image_grad* up, void* workspace,
                            size_t ws_bytes, void* hip_stream);
int cgv2_project_bwd(const cgv2_surfels* s, const cgv2_proj* proj, const cgv2_camera* cams, int32_t V,
                     const void* workspace, size_t ws_bytes, cgv2_grads* grads, void* hip_stream);

/* Zeroes the parameter gradients of grads (d_mean, d_log_scale, d_quat, d_opacity_logit and d_sh of n
 * surfels of SH degree sh_degree, 0-3, with the layouts above; the view-space gradients are left as they
 * are, cgv2_project_bwd overwrites them) before the views of a step add into them, in one launch.
 * Unlike the other calls it also takes arrays that are only 4-byte aligned.
 * Errors: CGV2_EINVAL (for n > 0, an array that is null or not 4-byte aligned), CGV2_EHIP. */
int cgv2_zero_grads(const cgv2_grads* grads, int64_t n, int32_t sh_degree, void* hip_stream);

/* Workspace bytes for cgv2_densify_stats. */
size_t cgv2_densify_workspace(int64_t n, int32_t V);

/* Densification statistics (Sec. 3.2): per view, the DGD factor of Eq. 2,
 * scale = max(omega * sum_vis |g_total| / sum_vis |g_ssim|, 1) (both sums over the surfels visible in
 * the view, so the ratio equals the ratio of the two averages; scale = 1 if the SSIM sum is 0), reduced
 * in a fixed order (deterministic); then accum_dgd += scale |g_ssim|, accum_total += |g_total|,
 * denom += 1, max_radius = max(max_radius, radius) over visible surfels; eta, masks and counters.
 * Errors: CGV2_EINVAL, CGV2_EWORKSPACE, CGV2_EHIP. */
int cgv2_densify_stats(const cgv2_surfels* s, const cgv2_proj* proj, const cgv2_grads* grads, int32_t V,
                       const cgv2_densify_params* prm, cgv2_densify_state* st, void* workspace, size_t ws_bytes,
                       void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): cgv2_densify_stats with its workspace taken from a fixed buffer the
 * library holds on each GPU (CGV2_NOALLOC_SCRATCH_BYTES, reserved when the library's code is loaded on
 * the device and held until the process ends).  Same arguments, rules and results as
 * cgv2_densify_stats; the caller still passes every input and output.  Allocates nothing.  Every call
 * on one GPU shares that GPU's buffer, so calls that overlap on one GPU (other streams, other threads)
 * race: order them.  The buffer needs no clearing (each call writes what it reads).
 * Errors: CGV2_EINVAL as cgv2_densify_stats; CGV2_EWORKSPACE when cgv2_densify_workspace(n, V) exceeds
 * CGV2_NOALLOC_SCRATCH_BYTES (above about 75 M surfels at 8 views, 28 M at 32); CGV2_EUNSUPPORTED;
 * CGV2_EHIP. */
#define CGV2_NOALLOC_SCRATCH_BYTES (16u << 20)
int cgv2_densify_stats_noalloc(const cgv2_surfels* s, const cgv2_proj* proj, const cgv2_grads* grads, int32_t V,
                               const cgv2_densify_params* prm, cgv2_densify_state* st, void* hip_stream);

/* Counting variant of cgv2_render_fwd for work accounting: counters[3] (device, uint64, added to)
 * receive the (pixel, entry) pairs the forward evaluates, the pairs that contribute, and the pairs
 * the reverse pass walks (entries before each pixel's 'last').  Same rules as the render; writes no
 * image.  Errors: CGV2_EINVAL, CGV2_EHIP. */
int cgv2_render_count(const cgv2_proj* proj, const cgv2_bins* bins, const cgv2_camera* cams, int32_t V,
                      int64_t n, uint64_t* counters, void* hip_stream);

/* Workspace bytes for cgv2_contribution. */
size_t cgv2_contribution_workspace(int64_t n, int32_t V);

/* Contribution of each surfel (Sec. 3.3, Eq. 3) in each of the V views of the call: over the pixels P at
 * which the surfel is blended (the decisions of cgv2_render_fwd), C = (1/|P|) sum alpha^gamma
 * T^(1-gamma) with T the transmittance in front of it; C = 0 when P is empty.  Any output may be NULL:
 *   c_view [V][n] receives C per view;
 *   c_sum  [n]    accumulates (+=) the sum of C over the V views (Eq. 4 averages over the block's views:
 *                 divide by their number; the caller zeroes it);
 *   pixels [V][n] receives |P| (u32).
 * proj, bins, cams, V and n as for cgv2_render_fwd (bins must be valid).
 * Errors: CGV2_EINVAL, CGV2_EWORKSPACE, CGV2_EHIP. */
int cgv2_contribution(const cgv2_proj* proj, const cgv2_bins* bins, const cgv2_camera* cams, int32_t V, int64_t n,
                      float gamma, float* c_view, float* c_sum, uint32_t* pixels, void* workspace, size_t ws_bytes,
                      void* hip_stream);

/* Workspace bytes for cgv2_trim_mask. */
size_t cgv2_trim_workspace(int64_t n);

/* Trimming of Sec. 3.3: *bound (device) = the floor(ratio (n - 1))-th smallest of c[0 .. n) (0-based;
 * c >= 0, found exactly by radix selection on the float bits), mask[i] = 1 when c[i] <= *bound, else
 * 0, and *removed (device, u32) = the number of ones.  ratio in [0, 1], n >= 1.
 * Errors: CGV2_EINVAL, CGV2_EWORKSPACE, CGV2_EHIP. */
int cgv2_trim_mask(const float* c, int64_t n, float ratio, float* bound, uint8_t* mask, uint32_t* removed,
                   void* workspace, size_t ws_bytes, void* hip_stream);

/* Densification action.  Sec. 3.2 fixes which surfels are densified (the candidate bit 4 of
 * cgv2_densify_state.mask: DGD high gradient and not elongated) and Sec. 3.3 which are removed (the
 * cgv2_trim_mask mask); what a candidate becomes follows the 3DGS / 2DGS training the method builds on:
 * a clone (an identical copy) when max(s_u, s_v) <= dense_scale, else a split into two children drawn
 * from the surfel's own Gaussian, child c at mu + s_u z_c0 t_u + s_v z_c1 t_v with both scales divided
 * by split_shrink and rotation, opacity and SH copied; a split surfel itself is removed. */
typedef struct {
  float dense_scale;   /* clone / split boundary on the larger scale (scene units) */
  float min_opacity;   /* surfels with sigmoid(logit) < min_opacity are removed too (0 disables) */
  float split_shrink;  /* scale divisor of split children (1.6 in 3DGS) */
} cgv2_action_params;

/* Output surfel set of cgv2_densify_apply: the layouts of cgv2_surfels with n = the capacity (stride of
 * the planar arrays; sh[n][(deg+1)^2][3]).  Must not overlap the input set. */
typedef struct {
  int64_t n;
  int32_t sh_degree;
  float *mean, *log_scale, *quat, *opacity_logit, *sh;
} cgv2_surfels_out;

/* Workspace bytes for cgv2_densify_plan. */
size_t cgv2_densify_plan_workspace(int64_t n);

/* Plans the densification action of n surfels (n < 2^30).  Decisions are taken in FP64 on the float32
 * parameters, in this order: remove when remove[i] != 0 (remove may be NULL) or sigmoid(logit) <
 * min_opacity; else keep when bit 4 of mask[i] is clear; else clone when max(exp(log_scale)) <=
 * dense_scale; else split.  Outputs (device):
 *   actions[n]  0 keep, 1 clone, 2 split, 3 remove;
 *   dst[2][n]   dst[0][i] = output slot of surfel i itself (keep, clone), dst[1][i] = first output slot
 *               of its new surfel(s) (clone: 1, split: 2), 0xffffffff where none.  The output holds the
 *               survivors in id order, then the new surfels in id order of their source;
 *   counts[5]   (int64) keep, clone, split, removed, output size = keep + 2 clone + 2 split.
 * Errors: CGV2_EINVAL, CGV2_EWORKSPACE, CGV2_EHIP. */
int cgv2_densify_plan(const cgv2_surfels* s, const uint8_t* mask, const uint8_t* remove, const cgv2_action_params* prm,
                      uint8_t* actions, uint32_t* dst, int64_t* counts, void* workspace, size_t ws_bytes,
                      void* hip_stream);

/* Applies a plan of cgv2_densify_plan (same s, actions, dst, counts): writes the new surfel set into out
 * (out->n >= counts[4] is the caller's to ensure, e.g. by reading counts first; slots beyond out->n
 * are dropped, never written out of bounds) and src[out->n] (device, u32): for each output slot,
 * (source id << 2) | kind with kind 0 survivor, 1 clone copy, 2 split child 0, 3 split child 1 (the
 * map cgv2_densify_gather re-lays other per-surfel arrays by).  z[n][2][2] (device, float32) holds the
 * offsets of the two children of surfel i (standard-normal draws, read for split surfels only).
 * Survivors and copies are bit-exact copies; a child's mean and log-scales are evaluated in FP64 and
 * rounded once.  Only prm->split_shrink is read.  Errors: CGV2_EINVAL, CGV2_EHIP. */
int cgv2_densify_apply(const cgv2_surfels* s, const uint8_t* actions, const uint32_t* dst, const int64_t* counts,
                       const float* z, const cgv2_action_params* prm, const cgv2_surfels_out* out, uint32_t* src,
                       void* hip_stream);

/* Re-lays a per-surfel float field of n surfels (channels C; blocked = 0: field[C][n] -> out[C][out_n],
 * blocked = 1: field[n][C] -> out[out_n][C]) by the map src of cgv2_densify_apply.  zero_new = 1
 * writes 0 into the new slots (copies and children: fresh optimiser moments), 0 copies the source.
 * Errors: CGV2_EINVAL, CGV2_EHIP. */
int cgv2_densify_gather(const float* field, int64_t n, int32_t channels, int32_t blocked, const uint32_t* src,
                        const int64_t* counts, int32_t zero_new, float* out, int64_t out_n, void* hip_stream);

/* Workspace bytes for cgv2_visibility_count (the views' FP64 camera table). */
size_t cgv2_visibility_workspace(int32_t V);

/* Visible frequency of m ground-truth points (Sec. 4, crop-volume estimate of the evaluation protocol):
 * count[i] += the number of the V views in which point i's visible mask is set (the caller zeroes count
 * first).  Each point is a small isotropic Gaussian: its footprint is the image of the sphere of radius
 * 'radius' (scene units) around it, hulled with a disc of filter_px pixels around its projected centre;
 * it is visible when its centre depth exceeds znear and a pixel sample (i + 0.5, j + 0.5) of the view
 * lies in the footprint's bounding box (no occlusion test; a sphere reaching the camera plane, depth <=
 * radius, is visible).  All decisions in FP64.  points[3][m] (device, float32); cams: V host structs,
 * each with its own width and height and znear > 0 (bg unused).  Any point order gives the same
 * counts; spatially coherent order (e.g. scan or tile order) is much faster, since whole workgroups of
 * neighbouring points then skip a view or count it at once.
 * Errors: CGV2_EINVAL (m < 0, V < 1, radius < 0, filter_px < 0, a camera without positive size, focal
 * lengths or znear), CGV2_EWORKSPACE, CGV2_EHIP. */
int cgv2_visibility_count(const float* points, int64_t m, const cgv2_camera* cams, int32_t V, float radius,
                          float filter_px, uint32_t* count, void* workspace, size_t ws_bytes, void* hip_stream);

/* Workspace bytes for cgv2_crop_volume. */
size_t cgv2_crop_workspace(int64_t m);

/* Crop statistics of Sec. 4 from the visible frequencies: keep[i] = count[i] >= tau; for the kept
 * points, (x, y, h) = T p with T (host, 3x4 row-major, FP64) the ground transform: ground[2][m] (device,
 * FP64, stride m) receives (x, y) of the kept points in id order in its first *kept columns (for the
 * alpha shape), hrange[2] (device, FP64) = min and max h over them (NaN when none is kept), *kept
 * (device, int64) their number.  Errors: CGV2_EINVAL, CGV2_EWORKSPACE, CGV2_EHIP. */
int cgv2_crop_volume(const float* points, int64_t m, const uint32_t* count, uint32_t tau, const double* T,
                     uint8_t* keep, double* ground, double* hrange, int64_t* kept, void* workspace, size_t ws_bytes,
                     void* hip_stream);

/* ---- building the serving storage (see cgv2_surfels_compact) ---------------------------------------
 * x[*][D] below is any float32 array of D-vectors (e.g. cgv2_surfels.sh, D = 3 (deg+1)^2) and rows[m]
 * (device, u32) selects the vectors taken part, each < the number of vectors in x.  D must be one of
 * 1-4, 9-12, 25-28, 45-48 (the SH sizes of degrees 0-3, padded to whole 4-wide MFMA steps). */

/* Workspace bytes for cgv2_compact_order. */
size_t cgv2_compact_order_workspace(int64_t n);

/* Stable partition of n surfels by quantize[n] (0 = keep its SH, else = replace it by a codeword):
 * order[n] (device, u32) = source id of each storage slot, kept surfels first, both groups in id order;
 * *n_full (device, int64) = number kept.  Errors: CGV2_EINVAL, CGV2_EWORKSPACE, CGV2_EHIP. */
int cgv2_compact_order(const uint8_t* quantize, int64_t n, uint32_t* order, int64_t* n_full, void* workspace,
                       size_t ws_bytes, void* hip_stream);

/* Codebook start for K codewords: codebook[j] = x[rows[floor(j m / K)]] (m >= 1).
 * Errors: CGV2_EINVAL, CGV2_EHIP. */
int cgv2_vq_init(const float* x, int32_t D, const uint32_t* rows, int64_t m, int32_t K, float* codebook,
                 void* hip_stream);

/* Workspace bytes for cgv2_vq_assign. */
size_t cgv2_vq_assign_workspace(int32_t K);

/* Nearest codeword (squared Euclidean distance) of each selected vector: code[m] (device, u16) = argmin_j
 * |x - c_j|^2 over codebook[K][D] (float32), evaluated as |c_j|^2 - 2 x.c_j in FP32 on the matrix cores;
 * equal values go to the smaller index.  half_codebook = 1 measures against the float16 rounding of each
 * codeword (the stored one).  K in [1, 65536].  Errors: CGV2_EINVAL, CGV2_EWORKSPACE, CGV2_EHIP. */
int cgv2_vq_assign(const float* x, int32_t D, const uint32_t* rows, int64_t m, const float* codebook, int32_t K,
                   int32_t half_codebook, uint16_t* code, void* workspace, size_t ws_bytes, void* hip_stream);

/* Workspace bytes for cgv2_vq_update. */
size_t cgv2_vq_update_workspace(int32_t K, int32_t D);

/* Lloyd update: every codeword with members becomes their mean (FP64 sums, rounded once), one without
 * keeps its value; counts[K] (device, u32) receives the member counts.  codebook is read and written.
 * Errors: CGV2_EINVAL, CGV2_EWORKSPACE, CGV2_EHIP. */
int cgv2_vq_update(const float* x, int32_t D, const uint32_t* rows, int64_t m, const uint16_t* code, int32_t K,
                   float* codebook, uint32_t* counts, void* workspace, size_t ws_bytes, void* hip_stream);

/* Destination of cgv2_compact_write: the arrays of cgv2_surfels_compact (float16 as uint16_t bits) for
 * n = the input's n: mean[3][n], log_scale[2][n], quat[4][n], opacity_logit[n], sh[n][(deg+1)^2][3] (the
 * first *n_full rows are written), codebook[K][(deg+1)^2][3]. */
typedef struct {
  int64_t n;
  int32_t sh_degree;
  float* mean;
  uint16_t *log_scale, *quat, *opacity_logit, *sh, *codebook;
} cgv2_compact_out;

/* Writes the stored arrays of s in the slot order of cgv2_compact_order (order, n_full as it left them):
 * positions copied, everything else rounded to float16 (nearest, ties to even), the SH of the kept slots
 * and the K codewords of codebook[K][(deg+1)^2][3] (float32; may be NULL with K = 0).  The codes of the
 * quantized slots are cgv2_vq_assign's output over rows = order + n_full.
 * Errors: CGV2_EINVAL, CGV2_EHIP. */
int cgv2_compact_write(const cgv2_surfels* s, const uint32_t* order, const int64_t* n_full, const float* codebook,
                       int32_t K, const cgv2_compact_out* out, void* hip_stream);

/* Error string for a CGV2_E* code; thread-local hipError_t of the last failing launch. */
const char* cgv2_strerror(int code);
int cgv2_last_hip_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CGV2R_H */
