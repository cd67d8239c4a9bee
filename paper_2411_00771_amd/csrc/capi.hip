// C ABI of the surfel rasterizer: argument validation, workspace sizing, camera packing and the
// launch sequence of each call.  Nothing here allocates, prints or synchronises.
#include <string.h>

#include "cgv2r_device.h"
#include "cgv2r_kernels.h"

namespace {

thread_local int g_last_hip = 0;

int hip_status(hipError_t e) {
  if (e == hipSuccess) return CGV2_OK;
  g_last_hip = (int)e;
  return CGV2_EHIP;
}

// The library carries gfx950 code only.  A call can launch when the calling thread's current HIP device
// is a gfx950; the answer is kept per device for the calling thread (device properties do not change).
int device_check() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return CGV2_EUNSUPPORTED;
  thread_local signed char known[64] = {0};
  if (dev < 64 && known[dev]) return known[dev] > 0 ? CGV2_OK : CGV2_EUNSUPPORTED;
  hipDeviceProp_t prop;
  const bool ok = hipGetDeviceProperties(&prop, dev) == hipSuccess && strncmp(prop.gcnArchName, "gfx950", 6) == 0;
  if (dev < 64) known[dev] = ok ? 1 : -1;
  return ok ? CGV2_OK : CGV2_EUNSUPPORTED;
}

bool cams_ok(const cgv2_camera* c, int32_t V) {
  if (!c || V < 1) return false;
  for (int v = 0; v < V; ++v) {
    if (c[v].width <= 0 || c[v].height <= 0) return false;
    if (c[v].width != c[0].width || c[v].height != c[0].height) return false;
    if ((c[v].width + CGV2_TILE - 1) / CGV2_TILE > 65535 || (c[v].height + CGV2_TILE - 1) / CGV2_TILE > 65535)
      return false;
  }
  return true;
}

bool surfels_ok(const cgv2_surfels* s) {
  return s && s->n >= 0 && s->n < (int64_t)0xffffffff && s->sh_degree >= 0 && s->sh_degree <= 3 &&
         (s->n == 0 || (s->mean && s->log_scale && s->quat && s->opacity_logit && s->sh));
}

// the densification action packs source ids into 30 bits
bool action_surfels_ok(const cgv2_surfels* s) { return surfels_ok(s) && s->n < ((int64_t)1 << 30); }

bool proj_ok(const cgv2_proj* p) {
  return p && p->rec && p->rect && p->radius && p->flags && p->visible && p->visible_start;
}

bool bins_ok(const cgv2_bins* b) {
  return b && b->capacity >= 0 && b->capacity < (int64_t)0xffffffff && b->ranges && b->status && b->needed &&
         (b->capacity == 0 || b->ids);
}

cgv2::CamPack pack(const cgv2_camera* c, int v0, int count) {
  cgv2::CamPack p;
  memset(&p, 0, sizeof(p));
  for (int k = 0; k < count; ++k) {
    const cgv2_camera& s = c[v0 + k];
    cgv2::DevCam& d = p.c[k];
    d.W = s.width; d.H = s.height;
    d.fx = s.fx; d.fy = s.fy; d.cx = s.cx; d.cy = s.cy;
    memcpy(d.R, s.R, sizeof(d.R));
    memcpy(d.t, s.t, sizeof(d.t));
    d.znear = s.znear;
    memcpy(d.bg, s.bg, sizeof(d.bg));
  }
  p.v0 = v0;
  p.count = count;
  return p;
}

inline int tiles_x(const cgv2_camera* c) { return (c[0].width + CGV2_TILE - 1) / CGV2_TILE; }
inline int tiles_y(const cgv2_camera* c) { return (c[0].height + CGV2_TILE - 1) / CGV2_TILE; }

cgv2::RecGrads rec_grads(void* workspace, int64_t n, int32_t V) {
  cgv2::RecGrads rg;
  rg.row = (float*)workspace;
  rg.nrm = rg.row + (size_t)cgv2::kGradRow * (size_t)n * (size_t)V;
  return rg;
}

int bwd_records(const cgv2_proj* proj, const cgv2_bins* bins, const cgv2_camera* cams, int32_t V, int64_t n,
                const cgv2_image* img, const cgv2_image_grad* up, void* workspace, hipStream_t st) {
  const int tx = tiles_x(cams), ty = tiles_y(cams);
  const cgv2::RecGrads rg = rec_grads(workspace, n, V);
  for (int v0 = 0; v0 < V; v0 += cgv2::kMaxViews) {
    const int cnt = V - v0 < cgv2::kMaxViews ? V - v0 : cgv2::kMaxViews;
    const int rc = hip_status(cgv2_launch_render_bwd(*proj, *bins, pack(cams, v0, cnt), n, tx, ty, *img, *up, rg, st));
    if (rc) return rc;
  }
  return CGV2_OK;
}

int bwd_project(const cgv2_surfels* s, const cgv2_proj* proj, const cgv2_camera* cams, int32_t V,
                const void* workspace, cgv2_grads* g, hipStream_t st) {
  const cgv2::RecGrads rg = rec_grads(const_cast<void*>(workspace), s->n, V);
  for (int v0 = 0; v0 < V; v0 += cgv2::kMaxViews) {
    const int cnt = V - v0 < cgv2::kMaxViews ? V - v0 : cgv2::kMaxViews;
    const int rc = hip_status(cgv2_launch_project_bwd(*s, pack(cams, v0, cnt), *proj, rg, *g, st));
    if (rc) return rc;
  }
  return CGV2_OK;
}

bool records_args_ok(const cgv2_proj* proj, const cgv2_bins* bins, const cgv2_camera* cams, int32_t V, int64_t n,
                     const cgv2_image* img, const cgv2_image_grad* up) {
  return proj_ok(proj) && bins_ok(bins) && cams_ok(cams, V) && img && up && n >= 0 && img->T_final && img->last &&
         img->med;
}

bool project_args_ok(const cgv2_surfels* s, const cgv2_proj* proj, const cgv2_camera* cams, int32_t V,
                     const cgv2_grads* g) {
  if (!surfels_ok(s) || !proj_ok(proj) || !cams_ok(cams, V) || !g) return false;
  return s->n == 0 || (g->d_mean && g->d_log_scale && g->d_quat && g->d_opacity_logit && g->d_sh);
}


}  // namespace

extern "C" {

const char* cgv2_strerror(int code) {
  switch (code) {
    case CGV2_OK: return "ok";
    case CGV2_EINVAL: return "invalid argument";
    case CGV2_EWORKSPACE: return "workspace too small";
    case CGV2_EUNSUPPORTED: return "unsupported device";
    case CGV2_EHIP: return "HIP launch failed";
    default: return "unknown error";
  }
}

int cgv2_last_hip_error(void) { return g_last_hip; }

int cgv2_project_compact(const cgv2_surfels_compact* s, const cgv2_camera* cams, int32_t V, cgv2_proj* proj,
                         void* stream) {
  if (!s || s->n < 0 || s->n >= (int64_t)0xffffffff || s->sh_degree < 0 || s->sh_degree > 3 || !cams_ok(cams, V) ||
      !proj_ok(proj) || s->n_full < 0 || s->n_full > s->n)
    return CGV2_EINVAL;
  if (s->n > 0 && (!s->mean || !s->log_scale || !s->quat || !s->opacity_logit)) return CGV2_EINVAL;
  if (s->n_full > 0 && !s->sh) return CGV2_EINVAL;
  if (s->n_full < s->n && (!s->code || !s->codebook || s->codebook_size < 1 || s->codebook_size > 65536))
    return CGV2_EINVAL;
  if (const int dv = device_check()) return dv;
  for (int v0 = 0; v0 < V; v0 += cgv2::kMaxViews) {
    const int cnt = V - v0 < cgv2::kMaxViews ? V - v0 : cgv2::kMaxViews;
    const int rc = hip_status(cgv2_launch_project_compact(*s, pack(cams, v0, cnt), *proj, (hipStream_t)stream));
    if (rc) return rc;
  }
  return CGV2_OK;
}

int cgv2_project(const cgv2_surfels* s, const cgv2_camera* cams, int32_t V, cgv2_proj* proj, void* stream) {
  if (!surfels_ok(s) || !cams_ok(cams, V) || !proj_ok(proj)) return CGV2_EINVAL;
  if (const int dv = device_check()) return dv;
  for (int v0 = 0; v0 < V; v0 += cgv2::kMaxViews) {
    const int cnt = V - v0 < cgv2::kMaxViews ? V - v0 : cgv2::kMaxViews;
    const int rc = hip_status(cgv2_launch_project(*s, pack(cams, v0, cnt), *proj, (hipStream_t)stream));
    if (rc) return rc;
  }
  return CGV2_OK;
}

size_t cgv2_bin_sort_workspace(int64_t capacity, int32_t V, int32_t tiles_per_view, int64_t n) {
  if (capacity < 0 || V < 1 || tiles_per_view < 1 || n < 0) return 0;
  size_t off[kBinsortOffs];
  return cgv2_binsort_ws_layout(capacity, V, tiles_per_view, n, off);
}

int cgv2_bin_sort(const cgv2_proj* proj, const cgv2_camera* cams, int32_t V, int64_t n, cgv2_bins* bins,
                  void* workspace, size_t ws_bytes, void* stream) {
  if (!cams_ok(cams, V) || !proj_ok(proj) || !bins_ok(bins) || n < 0 || !workspace)
    return CGV2_EINVAL;
  if ((int64_t)V * n >= (int64_t)0xffffffff) return CGV2_EINVAL;
  const int tx = tiles_x(cams), ty = tiles_y(cams);
  if ((int64_t)V * tx * ty >= (int64_t)0x7fffffff) return CGV2_EINVAL;
  if (ws_bytes < cgv2_bin_sort_workspace(bins->capacity, V, tx * ty, n)) return CGV2_EWORKSPACE;
  if (const int dv = device_check()) return dv;
  return hip_status(cgv2_launch_bin_sort(*proj, n, V, tx, ty, *bins, workspace, (hipStream_t)stream));
}

int cgv2_render_fwd(const cgv2_proj* proj, const cgv2_bins* bins, const cgv2_camera* cams, int32_t V, int64_t n,
                    cgv2_image* img, void* stream) {
  if (!proj_ok(proj) || !bins_ok(bins) || !cams_ok(cams, V) || !img || n < 0) return CGV2_EINVAL;
  const int tx = tiles_x(cams), ty = tiles_y(cams);
  if (const int dv = device_check()) return dv;
  for (int v0 = 0; v0 < V; v0 += cgv2::kMaxViews) {
    const int cnt = V - v0 < cgv2::kMaxViews ? V - v0 : cgv2::kMaxViews;
    const int rc = hip_status(cgv2_launch_render_fwd(*proj, *bins, pack(cams, v0, cnt), n, tx, ty, *img,
                                                     (hipStream_t)stream));
    if (rc) return rc;
  }
  return CGV2_OK;
}

int cgv2_render_count(const cgv2_proj* proj, const cgv2_bins* bins, const cgv2_camera* cams, int32_t V, int64_t n,
                      uint64_t* counters, void* stream) {
  if (!proj_ok(proj) || !bins_ok(bins) || !cams_ok(cams, V) || !counters || n < 0) return CGV2_EINVAL;
  const int tx = tiles_x(cams), ty = tiles_y(cams);
  if (const int dv = device_check()) return dv;
  for (int v0 = 0; v0 < V; v0 += cgv2::kMaxViews) {
    const int cnt = V - v0 < cgv2::kMaxViews ? V - v0 : cgv2::kMaxViews;
    const int rc = hip_status(cgv2_launch_render_count(*proj, *bins, pack(cams, v0, cnt), n, tx, ty,
                                                       (unsigned long long*)counters, (hipStream_t)stream));
    if (rc) return rc;
  }
  return CGV2_OK;
}

size_t cgv2_loss_workspace(int32_t width, int32_t height, int32_t V) {
  if (width <= 0 || height <= 0 || V < 1) return 0;
  size_t off[kLossOffs];
  return cgv2_loss_ws_layout(width, height, V, off);
}

int cgv2_loss(const float* img, const float* target, int32_t V, int32_t width, int32_t height, float lambda,
              float* d_img, float* d_img_ssim, float* loss, void* workspace, size_t ws_bytes, void* stream) {
  if (!img || !target || !d_img || !d_img_ssim || !loss || !workspace || V < 1 || width <= 0 || height <= 0)
    return CGV2_EINVAL;
  if ((int64_t)V * 3 > 65535) return CGV2_EINVAL;
  if (ws_bytes < cgv2_loss_workspace(width, height, V)) return CGV2_EWORKSPACE;
  if (const int dv = device_check()) return dv;
  return hip_status(
      cgv2_launch_loss(img, target, V, width, height, lambda, d_img, d_img_ssim, loss, workspace, (hipStream_t)stream));
}

size_t cgv2_render_bwd_workspace(int64_t n, int32_t V) {
  if (n < 0 || V < 1) return 0;
  return ((size_t)(cgv2::kGradRow + cgv2::kGradNrm) * sizeof(float) * (size_t)n * (size_t)V + 255) & ~(size_t)255;
}

int cgv2_render_bwd(const cgv2_surfels* s, const cgv2_proj* proj, const cgv2_bins* bins, const cgv2_camera* cams,
                    int32_t V, const cgv2_image* img, const cgv2_image_grad* up, cgv2_grads* g, void* workspace,
                    size_t ws_bytes, void* stream) {
  if (!project_args_ok(s, proj, cams, V, g) || !records_args_ok(proj, bins, cams, V, s->n, img, up))
    return CGV2_EINVAL;
  if (!workspace || ws_bytes < cgv2_render_bwd_workspace(s->n, V)) return workspace ? CGV2_EWORKSPACE : CGV2_EINVAL;
  if (const int dv = device_check()) return dv;
  const int rc = bwd_records(proj, bins, cams, V, s->n, img, up, workspace, (hipStream_t)stream);
  return rc ? rc : bwd_project(s, proj, cams, V, workspace, g, (hipStream_t)stream);
}

int cgv2_render_bwd_records(const cgv2_proj* proj, const cgv2_bins* bins, const cgv2_camera* cams, int32_t V,
                            int64_t n, const cgv2_image* img, const cgv2_image_grad* up, void* workspace,
                            size_t ws_bytes, void* stream) {
  if (!records_args_ok(proj, bins, cams, V, n, img, up)) return CGV2_EINVAL;
  if (!workspace || ws_bytes < cgv2_render_bwd_workspace(n, V)) return workspace ? CGV2_EWORKSPACE : CGV2_EINVAL;
  if (const int dv = device_check()) return dv;
  return bwd_records(proj, bins, cams, V, n, img, up, workspace, (hipStream_t)stream);
}

int cgv2_project_bwd(const cgv2_surfels* s, const cgv2_proj* proj, const cgv2_camera* cams, int32_t V,
                     const void* workspace, size_t ws_bytes, cgv2_grads* g, void* stream) {
  if (!project_args_ok(s, proj, cams, V, g)) return CGV2_EINVAL;
  if (!workspace || ws_bytes < cgv2_render_bwd_workspace(s->n, V)) return workspace ? CGV2_EWORKSPACE : CGV2_EINVAL;
  if (const int dv = device_check()) return dv;
  return bwd_project(s, proj, cams, V, workspace, g, (hipStream_t)stream);
}

int cgv2_zero_grads(const cgv2_grads* g, int64_t n, int32_t sh_degree, void* stream) {
  if (!g || n < 0 || sh_degree < 0 || sh_degree > 3) return CGV2_EINVAL;
  if (n > 0 && (!g->d_mean || !g->d_log_scale || !g->d_quat || !g->d_opacity_logit || !g->d_sh)) return CGV2_EINVAL;
  const float* ps[5] = {g->d_mean, g->d_log_scale, g->d_quat, g->d_opacity_logit, g->d_sh};
  for (const float* p : ps)
    if ((uintptr_t)p & 3u) return CGV2_EINVAL;
  if (const int dv = device_check()) return dv;
  return hip_status(cgv2_launch_zero_grads(*g, n, sh_degree, (hipStream_t)stream));
}

size_t cgv2_densify_workspace(int64_t n, int32_t V) {
  if (n < 0 || V < 1) return 0;
  size_t off[kDensifyOffs];
  return cgv2_densify_ws_layout(n, V, off);
}

int cgv2_densify_stats(const cgv2_surfels* s, const cgv2_proj* proj, const cgv2_grads* g, int32_t V,
                       const cgv2_densify_params* prm, cgv2_densify_state* st, void* workspace, size_t ws_bytes,
                       void* stream) {
  if (!surfels_ok(s) || !proj || !proj->flags || !proj->radius || !g || !g->g_view_total || !prm || !st ||
      V < 1 || V > 64)
    return CGV2_EINVAL;
  if (!st->accum_dgd || !st->accum_total || !st->max_radius || !st->denom || !st->mask || !st->counters)
    return CGV2_EINVAL;
  if (!workspace || ws_bytes < cgv2_densify_workspace(s->n, V)) return workspace ? CGV2_EWORKSPACE : CGV2_EINVAL;
  if (const int dv = device_check()) return dv;
  return hip_status(cgv2_launch_densify(*s, *proj, *g, V, *prm, *st, workspace, (hipStream_t)stream));
}

int cgv2_densify_stats_noalloc(const cgv2_surfels* s, const cgv2_proj* proj, const cgv2_grads* g, int32_t V,
                               const cgv2_densify_params* prm, cgv2_densify_state* st, void* stream) {
  if (!surfels_ok(s) || !proj || !proj->flags || !proj->radius || !g || !g->g_view_total || !prm || !st ||
      V < 1 || V > 64)
    return CGV2_EINVAL;
  if (!st->accum_dgd || !st->accum_total || !st->max_radius || !st->denom || !st->mask || !st->counters)
    return CGV2_EINVAL;
  if (cgv2_densify_workspace(s->n, V) > (size_t)CGV2_NOALLOC_SCRATCH_BYTES) return CGV2_EWORKSPACE;
  if (const int dv = device_check()) return dv;
  void* scratch = nullptr;
  if (const int rc = hip_status(cgv2_densify_scratch(&scratch))) return rc;
  return hip_status(cgv2_launch_densify(*s, *proj, *g, V, *prm, *st, scratch, (hipStream_t)stream));
}

size_t cgv2_contribution_workspace(int64_t n, int32_t V) {
  if (n < 0 || V < 1) return 0;
  return cgv2_contribution_ws_layout(n, V);
}

int cgv2_contribution(const cgv2_proj* proj, const cgv2_bins* bins, const cgv2_camera* cams, int32_t V, int64_t n,
                      float gamma, float* c_view, float* c_sum, uint32_t* pixels, void* workspace, size_t ws_bytes,
                      void* stream) {
  if (!proj_ok(proj) || !bins_ok(bins) || !cams_ok(cams, V) || n < 0 || !(gamma >= 0.f && gamma <= 1.f))
    return CGV2_EINVAL;
  if (!workspace || ws_bytes < cgv2_contribution_workspace(n, V)) return workspace ? CGV2_EWORKSPACE : CGV2_EINVAL;
  if (const int dv = device_check()) return dv;
  if (n == 0) return CGV2_OK;
  const hipStream_t st = (hipStream_t)stream;
  const int tx = tiles_x(cams), ty = tiles_y(cams);
  for (int v0 = 0; v0 < V; v0 += cgv2::kMaxViews) {
    const int cnt = V - v0 < cgv2::kMaxViews ? V - v0 : cgv2::kMaxViews;
    const cgv2::CamPack cp = pack(cams, v0, cnt);
    int rc = hip_status(cgv2_launch_contribution_final(*proj, cp, n, V, workspace, true, nullptr, nullptr, nullptr, st));
    if (rc) return rc;
    rc = hip_status(cgv2_launch_contribution(*proj, *bins, cp, n, tx, ty, gamma, (float*)workspace, st));
    if (rc) return rc;
  }
  return hip_status(cgv2_launch_contribution_final(*proj, pack(cams, 0, V < cgv2::kMaxViews ? V : cgv2::kMaxViews), n,
                                                   V, workspace, false, c_view, c_sum, pixels, st));
}

size_t cgv2_trim_workspace(int64_t n) {
  if (n < 1) return 0;
  size_t off[kTrimOffs];
  return cgv2_trim_ws_layout(n, off);
}

int cgv2_trim_mask(const float* c, int64_t n, float ratio, float* bound, uint8_t* mask, uint32_t* removed,
                   void* workspace, size_t ws_bytes, void* stream) {
  if (!c || !mask || n < 1 || !(ratio >= 0.f && ratio <= 1.f) || n > 0xffffffffLL) return CGV2_EINVAL;
  if (!workspace || ws_bytes < cgv2_trim_workspace(n)) return workspace ? CGV2_EWORKSPACE : CGV2_EINVAL;
  if (const int dv = device_check()) return dv;
  const uint32_t k = (uint32_t)floor((double)ratio * (double)(n - 1));
  return hip_status(cgv2_launch_trim(c, n, k, bound, mask, removed, workspace, (hipStream_t)stream));
}

size_t cgv2_densify_plan_workspace(int64_t n) {
  if (n < 0) return 0;
  size_t off[kActionOffs];
  return cgv2_action_ws_layout(n, off);
}

int cgv2_densify_plan(const cgv2_surfels* s, const uint8_t* mask, const uint8_t* remove, const cgv2_action_params* prm,
                      uint8_t* actions, uint32_t* dst, int64_t* counts, void* workspace, size_t ws_bytes,
                      void* stream) {
  if (!action_surfels_ok(s) || !prm || !counts || (s->n > 0 && (!mask || !actions || !dst))) return CGV2_EINVAL;
  if (!(prm->dense_scale >= 0.f) || !(prm->min_opacity >= 0.f && prm->min_opacity <= 1.f)) return CGV2_EINVAL;
  if (!workspace || ws_bytes < cgv2_densify_plan_workspace(s->n)) return workspace ? CGV2_EWORKSPACE : CGV2_EINVAL;
  if (const int dv = device_check()) return dv;
  return hip_status(cgv2_launch_densify_plan(*s, mask, remove, *prm, actions, dst, counts, workspace,
                                             (hipStream_t)stream));
}

int cgv2_densify_apply(const cgv2_surfels* s, const uint8_t* actions, const uint32_t* dst, const int64_t* counts,
                       const float* z, const cgv2_action_params* prm, const cgv2_surfels_out* out, uint32_t* src,
                       void* stream) {
  if (!action_surfels_ok(s) || !prm || !counts || !out || !(prm->split_shrink > 0.f)) return CGV2_EINVAL;
  if (out->n < 0 || out->n >= ((int64_t)1 << 31) || out->sh_degree != s->sh_degree) return CGV2_EINVAL;
  if (s->n > 0 && (!actions || !dst || !z)) return CGV2_EINVAL;
  if (out->n > 0 && (!out->mean || !out->log_scale || !out->quat || !out->opacity_logit || !out->sh || !src))
    return CGV2_EINVAL;
  if (const int dv = device_check()) return dv;
  return hip_status(cgv2_launch_densify_apply(*s, actions, dst, counts, z, *prm, *out, src, (hipStream_t)stream));
}

int cgv2_densify_gather(const float* field, int64_t n, int32_t channels, int32_t blocked, const uint32_t* src,
                        const int64_t* counts, int32_t zero_new, float* out, int64_t out_n, void* stream) {
  if (n < 0 || n >= ((int64_t)1 << 30) || out_n < 0 || out_n >= ((int64_t)1 << 31) || channels < 1 || !counts ||
      (blocked != 0 && blocked != 1))
    return CGV2_EINVAL;
  if (n > 0 && out_n > 0 && (!field || !src || !out)) return CGV2_EINVAL;
  if (const int dv = device_check()) return dv;
  return hip_status(cgv2_launch_densify_gather(field, n, channels, blocked, src, counts, zero_new ? 1 : 0, out, out_n,
                                               (hipStream_t)stream));
}

size_t cgv2_visibility_workspace(int32_t V) { return V < 1 ? 0 : cgv2_vis_ws_layout(V); }

int cgv2_visibility_count(const float* points, int64_t m, const cgv2_camera* cams, int32_t V, float radius,
                          float filter_px, uint32_t* count, void* workspace, size_t ws_bytes, void* stream) {
  if (m < 0 || V < 1 || !cams || !(radius >= 0.f) || !(filter_px >= 0.f) || (m > 0 && (!points || !count)))
    return CGV2_EINVAL;
  for (int v = 0; v < V; ++v)
    if (cams[v].width <= 0 || cams[v].height <= 0 || !(cams[v].fx > 0.f) || !(cams[v].fy > 0.f) ||
        !(cams[v].znear > 0.f))
      return CGV2_EINVAL;
  if (!workspace || ws_bytes < cgv2_visibility_workspace(V)) return workspace ? CGV2_EWORKSPACE : CGV2_EINVAL;
  if (const int dv = device_check()) return dv;
  const hipStream_t st = (hipStream_t)stream;
  for (int v0 = 0; v0 < V; v0 += cgv2::kMaxViews) {
    const int cnt = V - v0 < cgv2::kMaxViews ? V - v0 : cgv2::kMaxViews;
    const int rc = hip_status(cgv2_launch_vis_table(pack(cams, v0, cnt), V, radius, filter_px, workspace, st));
    if (rc) return rc;
  }
  return hip_status(cgv2_launch_vis_count(points, m, V, radius, filter_px, count, workspace, st));
}

size_t cgv2_crop_workspace(int64_t m) {
  if (m < 0) return 0;
  size_t off[kCropOffs];
  return cgv2_crop_ws_layout(m, off);
}

int cgv2_crop_volume(const float* points, int64_t m, const uint32_t* count, uint32_t tau, const double* T,
                     uint8_t* keep, double* ground, double* hrange, int64_t* kept, void* workspace, size_t ws_bytes,
                     void* stream) {
  if (m < 0 || m >= ((int64_t)1 << 32) || !T || !hrange || !kept ||
      (m > 0 && (!points || !count || !keep || !ground)))
    return CGV2_EINVAL;
  if (!workspace || ws_bytes < cgv2_crop_workspace(m)) return workspace ? CGV2_EWORKSPACE : CGV2_EINVAL;
  if (const int dv = device_check()) return dv;
  return hip_status(cgv2_launch_crop(points, m, count, tau, T, keep, ground, hrange, kept, workspace,
                                     (hipStream_t)stream));
}

size_t cgv2_compact_order_workspace(int64_t n) { return n < 0 ? 0 : cgv2_part_ws_layout(n); }

int cgv2_compact_order(const uint8_t* quantize, int64_t n, uint32_t* order, int64_t* n_full, void* workspace,
                       size_t ws_bytes, void* stream) {
  if (n < 0 || n >= (int64_t)0xffffffff || !n_full || (n > 0 && (!quantize || !order))) return CGV2_EINVAL;
  if (!workspace || ws_bytes < cgv2_compact_order_workspace(n)) return workspace ? CGV2_EWORKSPACE : CGV2_EINVAL;
  if (const int dv = device_check()) return dv;
  return hip_status(cgv2_launch_compact_order(quantize, n, order, n_full, workspace, (hipStream_t)stream));
}

static bool vq_dim_ok(int32_t D) {
  const int DP = (D + 3) & ~3;
  return D >= 1 && (DP == 4 || DP == 12 || DP == 28 || DP == 48);
}

int cgv2_vq_init(const float* x, int32_t D, const uint32_t* rows, int64_t m, int32_t K, float* codebook,
                 void* stream) {
  if (!vq_dim_ok(D) || m < 1 || K < 1 || K > 65536 || !x || !rows || !codebook) return CGV2_EINVAL;
  if (const int dv = device_check()) return dv;
  return hip_status(cgv2_launch_vq_init(x, D, rows, m, K, codebook, (hipStream_t)stream));
}

size_t cgv2_vq_assign_workspace(int32_t K) { return K < 1 ? 0 : cgv2_vq_assign_ws_layout(K); }

int cgv2_vq_assign(const float* x, int32_t D, const uint32_t* rows, int64_t m, const float* codebook, int32_t K,
                   int32_t half_codebook, uint16_t* code, void* workspace, size_t ws_bytes, void* stream) {
  if (!vq_dim_ok(D) || m < 0 || K < 1 || K > 65536 || !codebook || (m > 0 && (!x || !rows || !code)))
    return CGV2_EINVAL;
  if (!workspace || ws_bytes < cgv2_vq_assign_workspace(K)) return workspace ? CGV2_EWORKSPACE : CGV2_EINVAL;
  if (const int dv = device_check()) return dv;
  return hip_status(cgv2_launch_vq_assign(x, D, rows, m, codebook, K, half_codebook ? 1 : 0, code, workspace,
                                          (hipStream_t)stream));
}

size_t cgv2_vq_update_workspace(int32_t K, int32_t D) { return (K < 1 || D < 1) ? 0 : cgv2_vq_update_ws_layout(K, D); }

int cgv2_vq_update(const float* x, int32_t D, const uint32_t* rows, int64_t m, const uint16_t* code, int32_t K,
                   float* codebook, uint32_t* counts, void* workspace, size_t ws_bytes, void* stream) {
  if (!vq_dim_ok(D) || m < 0 || K < 1 || K > 65536 || !codebook || !counts || (m > 0 && (!x || !rows || !code)))
    return CGV2_EINVAL;
  if (!workspace || ws_bytes < cgv2_vq_update_workspace(K, D)) return workspace ? CGV2_EWORKSPACE : CGV2_EINVAL;
  if (const int dv = device_check()) return dv;
  return hip_status(cgv2_launch_vq_update(x, D, rows, m, code, K, codebook, counts, workspace, (hipStream_t)stream));
}

int cgv2_compact_write(const cgv2_surfels* s, const uint32_t* order, const int64_t* n_full, const float* codebook,
                       int32_t K, const cgv2_compact_out* out, void* stream) {
  if (!surfels_ok(s) || !n_full || !out || out->n != s->n || out->sh_degree != s->sh_degree || K < 0 || K > 65536 ||
      (K > 0 && (!codebook || !out->codebook)))
    return CGV2_EINVAL;
  if (s->n > 0 && (!order || !out->mean || !out->log_scale || !out->quat || !out->opacity_logit || !out->sh))
    return CGV2_EINVAL;
  if (const int dv = device_check()) return dv;
  return hip_status(cgv2_launch_compact_write(*s, order, n_full, codebook, K, *out, (hipStream_t)stream));
}

}  // extern "C"
