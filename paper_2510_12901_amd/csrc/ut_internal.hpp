// ut_internal.hpp -- launchers shared between the kernel files and the C-ABI layer.
#pragma once

#include "ut_device.hpp"

namespace ut {

// Plain fill kernels (used instead of hipMemsetAsync so the calls stay graph-capturable).
hipError_t fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t st);
hipError_t fill_u64(uint64_t* p, uint64_t v, size_t n, hipStream_t st);
hipError_t fill_f64(double* p, double v, size_t n, hipStream_t st);

hipError_t launch_project(const ut_gaussians& g, const SensorK& s, const double abk[3],
                          const ut_projected& out, hipStream_t st);

// Workspace carve-up of the binning stage: the count part depends on the particle count
// only; the pair part (tile keys, value scratch, histograms of the pair sort) on the pair
// total P, so it can be reserved after ut_bin_count has reported P.
struct CountWorkspace {
  uint32_t *dkA, *dkB, *dvA, *dvB;   // depth sort keys / values, ping-pong [n]
  uint64_t* offs;                    // [n + 1] counts in depth order -> exclusive offsets
  uint64_t* total;                   // pair total
  uint32_t* scount;                  // [n] super-tile count per particle (index order)
  uint32_t* m_dev;                   // number of visible particles
  uint32_t* hist;                    // the depth sort's digit offsets, look-back words, tickets
  uint64_t* scan_aux;                // block sums of the device scans
  size_t bytes;
};
struct PairWorkspace {
  uint32_t *tkA, *tkB, *tv;          // pair tile keys ping-pong, pair value scratch [P]
  uint32_t* hist;                    // the pair sort's digit offsets, look-back words, tickets
  uint32_t* n_dev;                   // pair count on the device (the device-count sort)
  size_t bytes;
};
CountWorkspace count_workspace(void* base, int n);
PairWorkspace pair_workspace(void* base, uint64_t n_pairs);

hipError_t launch_bin_count(const ut_projected& p, int n, const SensorK& s, CountWorkspace& ws, hipStream_t st);
hipError_t launch_bin_sort(const ut_projected& p, int n, const SensorK& s, CountWorkspace& ws,
                           PairWorkspace& pw, uint64_t n_pairs, const ut_bin_lists& bins, hipStream_t st);
hipError_t launch_bin_sort_device(const ut_projected& p, int n, const SensorK& s, CountWorkspace& ws,
                                  PairWorkspace& pw, uint64_t max_pairs, const ut_bin_lists& bins,
                                  uint32_t* overflow, hipStream_t st);
hipError_t launch_tile_lists_count(const ut_projected& p, const SensorK& s, const ut_bin_lists& bins,
                                   const ut_tile_lists& lists, hipStream_t st);
hipError_t launch_tile_lists_fill(const ut_projected& p, const SensorK& s, const ut_bin_lists& bins,
                                  const ut_tile_lists& lists, hipStream_t st);

struct RenderParamsK {
  double alpha_min, alpha_max, t_min, log_alpha_min;
};

hipError_t launch_composite(const ut_projected& p, const ut_bin_lists& bins, const SensorK& s,
                            const RenderParamsK& prm, const ut_render_out& out, int max_tile_rays,
                            hipStream_t st);

// Batched compositing over several requests.
struct BatchItemK {
  SensorK s;
  const RecordG* rec;
  const uint2* trect;
  const uint32_t* gauss;    // super-tile bins
  const uint32_t* ranges;
  ut_render_out out;
  int n_tiles;
  int tile_base;   // prefix over items of n_tiles
};
// Items of one batch in four groups (bit 0: moving sensor, bit 1: LiDAR units), each group's
// items contiguous from first[g] in the device item array.
struct BatchGroups {
  int first[4], count[4], tiles[4];
};
hipError_t launch_composite_batch(const BatchItemK* items_dev, const BatchGroups& groups, uint32_t* counter,
                                  const RenderParamsK& prm, int n_workgroups, hipStream_t st);

hipError_t launch_backward(const ut_gaussians& g, const ut_projected& p, const ut_bin_lists& bins,
                           const SensorK& s, const RenderParamsK& prm, const ut_render_out& fwd,
                           const ut_upstream& up, double* acc, const ut_gaussian_grads& grads,
                           int max_tile_rays, hipStream_t st);

// Radix sort of (key, value) pairs, shared by the binning and the spatial order.
size_t radix_ws_bytes(size_t n_max);
size_t radix_tiles(size_t n_max);
size_t radix_clear_words();
hipError_t radix_sort(uint32_t* kA, uint32_t* kB, uint32_t* vA, uint32_t* vB, size_t n_max,
                      const uint32_t* n_dev, int bits, uint32_t* ws, hipStream_t st,
                      uint32_t** k_res, uint32_t** v_res, bool ws_clear = false);

size_t spatial_order_ws_bytes(int n);
hipError_t launch_spatial_order(const ut_gaussians& g, uint32_t* perm, void* ws, hipStream_t st);
hipError_t launch_gather_rows(const float* src, const uint32_t* perm, float* dst, int rows, int n, hipStream_t st);

hipError_t launch_actor_transform(const ut_gaussians& g, const int32_t* actor, const ut_actor_pose* poses,
                                  int n_act, float* mean_w, float* quat_w, hipStream_t st);
hipError_t launch_actor_backward(const ut_gaussians& g, const int32_t* actor, const ut_actor_pose* poses,
                                 int n_act, const float* dmw, const float* dqw, float* dmean, float* dquat,
                                 double* d_pose, hipStream_t st);

}  // namespace ut
