// Host-side launchers of the gfx950 kernels (one per source file); the C ABI in capi.hip
// validates arguments and calls these.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/cgv2r.h"

#include "cgv2r_device.h"

hipError_t cgv2_launch_project(const cgv2_surfels& s, const cgv2::CamPack& cams, const cgv2_proj& p, hipStream_t st);
hipError_t cgv2_launch_project_compact(const cgv2_surfels_compact& s, const cgv2::CamPack& cams, const cgv2_proj& p,
                                      hipStream_t st);
hipError_t cgv2_launch_project_bwd(const cgv2_surfels& s, const cgv2::CamPack& cams, const cgv2_proj& p,
                                   const cgv2::RecGrads& rg, const cgv2_grads& g, hipStream_t st);
hipError_t cgv2_launch_zero_grads(const cgv2_grads& g, int64_t n, int sh_degree, hipStream_t st);

// Workspace layouts: each fills off[0 .. k*Offs) with byte offsets and returns the total size.
constexpr int kBinsortOffs = 11, kLossOffs = 2, kDensifyOffs = 2, kTrimOffs = 3, kActionOffs = 2, kCropOffs = 2;

size_t cgv2_binsort_ws_layout(int64_t capacity, int V, int tiles, int64_t n, size_t* off);
hipError_t cgv2_launch_bin_sort(const cgv2_proj& p, int64_t n, int V, int tiles_x, int tiles_y, const cgv2_bins& b,
                                void* ws, hipStream_t st);

hipError_t cgv2_launch_render_fwd(const cgv2_proj& p, const cgv2_bins& b, const cgv2::CamPack& cams, int64_t n,
                                  int tiles_x, int tiles_y, const cgv2_image& img, hipStream_t st);
hipError_t cgv2_launch_render_count(const cgv2_proj& p, const cgv2_bins& b, const cgv2::CamPack& cams, int64_t n,
                                    int tiles_x, int tiles_y, unsigned long long* counters, hipStream_t st);
hipError_t cgv2_launch_render_bwd(const cgv2_proj& p, const cgv2_bins& b, const cgv2::CamPack& cams, int64_t n,
                                  int tiles_x, int tiles_y, const cgv2_image& img, const cgv2_image_grad& up,
                                  const cgv2::RecGrads& rg, hipStream_t st);

size_t cgv2_loss_ws_layout(int W, int H, int V, size_t* off);
hipError_t cgv2_launch_loss(const float* img, const float* tgt, int V, int W, int H, float lambda, float* d_img,
                            float* d_ssim, float* loss, void* ws, hipStream_t st);

size_t cgv2_densify_ws_layout(int64_t n, int V, size_t* off);
hipError_t cgv2_launch_densify(const cgv2_surfels& s, const cgv2_proj& p, const cgv2_grads& g, int V,
                               const cgv2_densify_params& prm, const cgv2_densify_state& st, void* ws,
                               hipStream_t stream);
// the calling thread's current device's copy of the fixed buffer of cgv2_densify_stats_noalloc
// (CGV2_NOALLOC_SCRATCH_BYTES); its address is looked up on the first call on each device
hipError_t cgv2_densify_scratch(void** ptr);

// contribution-based trimming (render.hip: the traversal; trim.hip: the rest)
hipError_t cgv2_launch_contribution(const cgv2_proj& p, const cgv2_bins& b, const cgv2::CamPack& cams, int64_t n,
                                    int tiles_x, int tiles_y, float gamma, float* cws, hipStream_t st);
size_t cgv2_contribution_ws_layout(int64_t n, int V);
// zero = true: clear the pairs of the chunk's visible surfels; false: finalise every view of the call
hipError_t cgv2_launch_contribution_final(const cgv2_proj& p, const cgv2::CamPack& cams, int64_t n, int V_total,
                                          void* ws, bool zero, float* c_view, float* c_sum, uint32_t* pixels,
                                          hipStream_t st);
size_t cgv2_trim_ws_layout(int64_t n, size_t* off);
hipError_t cgv2_launch_trim(const float* c, int64_t n, uint32_t k, float* bound, uint8_t* mask, uint32_t* removed,
                            void* ws, hipStream_t st);

// densification action (action.hip)
size_t cgv2_action_ws_layout(int64_t n, size_t* off);
hipError_t cgv2_launch_densify_plan(const cgv2_surfels& s, const uint8_t* mask, const uint8_t* remove,
                                    const cgv2_action_params& prm, uint8_t* actions, uint32_t* dst, int64_t* counts,
                                    void* ws, hipStream_t st);
hipError_t cgv2_launch_densify_apply(const cgv2_surfels& s, const uint8_t* actions, const uint32_t* dst,
                                     const int64_t* counts, const float* z, const cgv2_action_params& prm,
                                     const cgv2_surfels_out& out, uint32_t* src, hipStream_t st);
hipError_t cgv2_launch_densify_gather(const float* f, int64_t n, int C, int blocked, const uint32_t* src,
                                      const int64_t* counts, int zero_new, float* out, int64_t cap, hipStream_t st);

// visibility-frequency crop volume (crop.hip)
constexpr int kVisMaxViews = 4096;  // views per k_vis_count launch (its LDS list of edge views)
size_t cgv2_vis_ws_layout(int V);
hipError_t cgv2_launch_vis_table(const cgv2::CamPack& cams, int V, double rho, double rf, void* ws, hipStream_t st);
hipError_t cgv2_launch_vis_count(const float* pts, int64_t m, int V, double rho, double rf, uint32_t* count,
                                 void* ws, hipStream_t st);
size_t cgv2_crop_ws_layout(int64_t m, size_t* off);
hipError_t cgv2_launch_crop(const float* pts, int64_t m, const uint32_t* count, uint32_t tau, const double* T,
                            uint8_t* keep, double* ground, double* hrange, int64_t* kept, void* ws, hipStream_t st);

// serving storage: partition, vector quantization, float16 packing (vq.hip)
size_t cgv2_part_ws_layout(int64_t n);
hipError_t cgv2_launch_compact_order(const uint8_t* q, int64_t n, uint32_t* order, int64_t* n_full, void* ws,
                                     hipStream_t st);
hipError_t cgv2_launch_vq_init(const float* x, int D, const uint32_t* rows, int64_t m, int K, float* cb,
                               hipStream_t st);
size_t cgv2_vq_assign_ws_layout(int K);
hipError_t cgv2_launch_vq_assign(const float* x, int D, const uint32_t* rows, int64_t m, const float* cb, int K,
                                 int half_cb, uint16_t* code, void* ws, hipStream_t st);
size_t cgv2_vq_update_ws_layout(int K, int D);
hipError_t cgv2_launch_vq_update(const float* x, int D, const uint32_t* rows, int64_t m, const uint16_t* code, int K,
                                 float* cb, uint32_t* counts, void* ws, hipStream_t st);
hipError_t cgv2_launch_compact_write(const cgv2_surfels& s, const uint32_t* order, const int64_t* n_full,
                                     const float* cb, int K, const cgv2_compact_out& out, hipStream_t st);
