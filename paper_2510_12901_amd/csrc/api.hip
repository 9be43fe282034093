// api.hip -- the extern "C" boundary (include/utrast.h): argument checks, sensor set-up on
// the host (Alg. 1 tiling, ray mask and summed-area table of Appendix B), kernel launches.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "host_tables.hpp"
#include "ut_internal.hpp"

using namespace ut;

namespace {

hipStream_t as_stream(ut_stream s) { return reinterpret_cast<hipStream_t>(s); }

ut_status from_hip(hipError_t e) { return e == hipSuccess ? UT_OK : UT_ERR_DEVICE; }

int camera_tiles_x(const ut_sensor* s) { return (s->width + UT_CAMERA_TILE - 1) / UT_CAMERA_TILE; }
int camera_tiles_y(const ut_sensor* s) { return (s->height + UT_CAMERA_TILE - 1) / UT_CAMERA_TILE; }

using ut_host::gaussians_ok;
using ut_host::params_ok;
using ut_host::sensor_ok;
using ut_host::table_layout;
using ut_host::TableLayout;
static_assert(ut_host::kUnitTiles == kUnitTilesMax, "unit width of the host tables and the kernels");

// Unit quaternion (w, x, y, z) of a (float32, near-orthonormal) rotation matrix, from the
// largest of the four diagonal combinations for conditioning.
void rotation_quaternion(const float Rf[9], double q[4]) {
  double m[9];
  for (int i = 0; i < 9; ++i) m[i] = Rf[i];
  const double tr = m[0] + m[4] + m[8];
  const double c[4] = {1 + tr, 1 + m[0] - m[4] - m[8], 1 - m[0] + m[4] - m[8], 1 - m[0] - m[4] + m[8]};
  int b = 0;
  for (int i = 1; i < 4; ++i)
    if (c[i] > c[b]) b = i;
  const double r = std::sqrt(c[b]), h = 0.5 / r;
  switch (b) {
    case 0: q[0] = 0.5 * r; q[1] = (m[7] - m[5]) * h; q[2] = (m[2] - m[6]) * h; q[3] = (m[3] - m[1]) * h; break;
    case 1: q[1] = 0.5 * r; q[0] = (m[7] - m[5]) * h; q[2] = (m[1] + m[3]) * h; q[3] = (m[2] + m[6]) * h; break;
    case 2: q[2] = 0.5 * r; q[0] = (m[2] - m[6]) * h; q[1] = (m[1] + m[3]) * h; q[3] = (m[5] + m[7]) * h; break;
    default: q[3] = 0.5 * r; q[0] = (m[3] - m[1]) * h; q[1] = (m[2] + m[6]) * h; q[2] = (m[5] + m[7]) * h; break;
  }
  const double n = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int i = 0; i < 4; ++i) q[i] /= n;
}

SensorK make_sensor_k(const ut_sensor* s) {
  SensorK k;
  std::memset(&k, 0, sizeof k);
  k.kind = s->kind;
  for (int i = 0; i < 9; ++i) k.R[i] = s->R_sw[i];
  for (int i = 0; i < 3; ++i) { k.o[i] = s->origin[i]; k.of[i] = s->origin[i]; }
  k.near_ = s->near_;
  k.ray_dir = s->ray_dir;
  if (s->kind == UT_LIDAR) {
    k.n_beams = s->n_beams; k.n_az = s->n_az; k.n_phi = s->n_phi; k.n_theta = s->n_theta;
    k.cull = s->cull; k.cull_az = s->cull_az; k.cull_el = s->cull_el;
    k.tiles_x = s->n_theta; k.tiles_y = s->n_phi;
    const TableLayout t = table_layout(s->n_phi, s->cull ? s->cull_az : 0, s->cull ? s->cull_el : 0,
                                       s->n_phi * s->n_theta);
    char* base = static_cast<char*>(s->tables);
    k.bounds = reinterpret_cast<const double*>(base + t.bounds);
    k.beam_start = reinterpret_cast<const int*>(base + t.beam_start);
    k.sat = reinterpret_cast<const int*>(base + t.sat);
    k.units = reinterpret_cast<const int4*>(base + t.units);
    k.n_units = s->n_units;
    k.unit_rays = s->unit_rays;
    k.units_wide = k.units + (size_t)s->n_phi * s->n_theta;
    k.n_units_wide = s->n_units_wide;
    k.n_rays = (long long)s->n_beams * s->n_az;
    k.div_tan = s->beam_divergence > 0 ? std::tan(0.5 * s->beam_divergence) : 0.0;
  } else {
    k.width = s->width; k.height = s->height;
    k.tiles_x = camera_tiles_x(s); k.tiles_y = camera_tiles_y(s);
    k.fx = s->fx; k.fy = s->fy; k.cx = s->cx; k.cy = s->cy;
    for (int i = 0; i < 4; ++i) k.k[i] = s->k[i];
    k.theta_max = s->theta_max;
    k.n_rays = (long long)s->width * s->height;
  }
  k.super_h = ut_host::super_rows(s->kind);
  k.super_x = (k.tiles_x + kSuper - 1) / kSuper;
  k.super_y = (k.tiles_y + k.super_h - 1) / k.super_h;
  if (s->moving) {
    k.moving = 1;
    k.rs_iters = s->rs_iters;
    k.ray_org = s->ray_org;
    for (int i = 0; i < 3; ++i) k.o1[i] = s->origin1[i];
    rotation_quaternion(s->R_sw, k.q0);
    rotation_quaternion(s->R_sw1, k.q1);
    double dot = 0;
    for (int i = 0; i < 4; ++i) dot += k.q0[i] * k.q1[i];
    if (dot < 0) {   // the shorter arc
      for (int i = 0; i < 4; ++i) k.q1[i] = -k.q1[i];
      dot = -dot;
    }
    k.slerp_th = dot < 1.0 - 1e-12 ? std::acos(std::min(dot, 1.0)) : 0.0;
    k.slerp_isin = k.slerp_th > 0 ? 1.0 / std::sin(k.slerp_th) : 0.0;
  }
  return k;
}

RenderParamsK make_params(const ut_render_params* p) {
  RenderParamsK k;
  k.alpha_min = p->alpha_min;
  k.alpha_max = p->alpha_max;
  k.t_min = p->t_min;
  k.log_alpha_min = std::log(p->alpha_min);
  return k;
}


bool projected_ok(const ut_projected* p, int n) {
  return p && (n == 0 || (p->records && p->rect && p->trect && p->key && p->count)) && p->n_culled;
}

}  // namespace

extern "C" {

const char* ut_status_str(ut_status s) {
  switch (s) {
    case UT_OK: return "ok";
    case UT_ERR_ARG: return "invalid argument";
    case UT_ERR_CAPACITY: return "tile-list capacity or workspace exceeded";
    case UT_ERR_DEVICE: return "HIP device error";
    case UT_ERR_UNSUPPORTED: return "unsupported configuration";
  }
  return "unknown status";
}

int32_t ut_record_bytes(void) { return UT_RECORD_BYTES; }

// Alg. 1 (host_tables.hpp).
ut_status ut_lidar_tiling(const float* beam_elev, int32_t n_beams, int32_t n_az, int32_t n_phi,
                          int32_t M, double* bounds, int32_t* beam_start, int32_t* n_theta) {
  return ut_host::lidar_tiling(beam_elev, n_beams, n_az, n_phi, M, bounds, beam_start, n_theta);
}

ut_status ut_sensor_table_bytes(const ut_sensor* s, size_t* bytes) {
  if (!s || !bytes) return UT_ERR_ARG;
  if (s->kind != UT_LIDAR) { *bytes = 0; return UT_OK; }
  if (s->n_phi <= 0 || s->n_phi > UT_MAX_ELEV_TILES || (s->cull && (s->cull_az <= 0 || s->cull_el <= 0)) ||
      !s->beam_elev_host)
    return UT_ERR_ARG;
  // the unit table is sized by the tile count, which Alg. 1 fixes
  std::vector<double> bounds(s->n_phi + 1);
  std::vector<int32_t> bstart(s->n_phi + 1);
  int32_t nth = 0;
  const ut_status st = ut_lidar_tiling(s->beam_elev_host, s->n_beams, s->n_az, s->n_phi, s->max_per_tile,
                                       bounds.data(), bstart.data(), &nth);
  if (st != UT_OK) return st;
  *bytes = table_layout(s->n_phi, s->cull ? s->cull_az : 0, s->cull ? s->cull_el : 0, s->n_phi * nth).total;
  return UT_OK;
}

ut_status ut_sensor_build(ut_sensor* s, ut_stream stream) {
  if (!s) return UT_ERR_ARG;
  if (s->kind != UT_LIDAR) {
    if (s->kind != UT_PINHOLE && s->kind != UT_FISHEYE && s->kind != UT_ORTHO) return UT_ERR_ARG;
    if (s->width <= 0 || s->height <= 0) return UT_ERR_ARG;
    s->max_tile_rays = UT_CAMERA_TILE * UT_CAMERA_TILE;
    return UT_OK;
  }
  if (!s->beam_elev_host || !s->tables || s->n_beams <= 0 || s->n_az <= 0) return UT_ERR_ARG;
  size_t bytes = 0;
  ut_status st = ut_sensor_table_bytes(s, &bytes);
  if (st != UT_OK) return st;
  const int NP = s->n_phi;
  std::vector<double> bounds(NP + 1);
  std::vector<int32_t> bstart(NP + 1);
  int32_t nth = 0;
  st = ut_lidar_tiling(s->beam_elev_host, s->n_beams, s->n_az, NP, s->max_per_tile, bounds.data(), bstart.data(), &nth);
  if (st != UT_OK) return st;
  const int max_rays = ut_host::max_tile_rays(bstart.data(), NP, s->n_az, nth);
  if (max_rays > UT_MAX_LIDAR_TILE_RAYS) return UT_ERR_UNSUPPORTED;
  const TableLayout t = table_layout(NP, s->cull ? s->cull_az : 0, s->cull ? s->cull_el : 0, NP * nth);
  std::vector<char> host(t.total, 0);
  std::memcpy(host.data() + t.bounds, bounds.data(), sizeof(double) * (NP + 1));
  std::memcpy(host.data() + t.beam_start, bstart.data(), sizeof(int32_t) * (NP + 1));
  const int unit_rays = ut_host::unit_width(max_rays);
  int32_t* units = reinterpret_cast<int32_t*>(host.data() + t.units);
  const int n_units = unit_rays > 0 ? ut_host::build_units(bstart.data(), NP, s->n_az, nth, unit_rays, units) : 0;
  const int n_units_wide =
      unit_rays > 0 ? ut_host::build_units(bstart.data(), NP, s->n_az, nth, 256, units + 4 * (size_t)NP * nth) : 0;
  if (s->cull)
    ut_host::ray_sat(s->beam_elev_host, s->n_beams, s->n_az, bounds.data(), NP, s->cull_az, s->cull_el,
                     reinterpret_cast<int32_t*>(host.data() + t.sat));
  hipError_t e = hipMemcpyAsync(s->tables, host.data(), t.total, hipMemcpyHostToDevice, as_stream(stream));
  if (e == hipSuccess) e = hipStreamSynchronize(as_stream(stream));
  if (e != hipSuccess) return UT_ERR_DEVICE;
  s->n_theta = nth;
  s->max_tile_rays = max_rays;
  s->n_units = n_units;
  s->unit_rays = unit_rays;
  s->n_units_wide = n_units_wide;
  return UT_OK;
}

int32_t ut_sensor_tiles(const ut_sensor* s) {
  if (!s) return 0;
  if (s->kind == UT_LIDAR) return s->n_phi * s->n_theta;
  return camera_tiles_x(s) * camera_tiles_y(s);
}

int32_t ut_sensor_super_tiles(const ut_sensor* s) {
  if (!s) return 0;
  const int tx = s->kind == UT_LIDAR ? s->n_theta : camera_tiles_x(s);
  const int ty = s->kind == UT_LIDAR ? s->n_phi : camera_tiles_y(s);
  const int sh = ut_host::super_rows(s->kind);
  return ((tx + kSuper - 1) / kSuper) * ((ty + sh - 1) / sh);
}

int64_t ut_sensor_rays(const ut_sensor* s) {
  if (!s) return 0;
  if (s->kind == UT_LIDAR) return (int64_t)s->n_beams * s->n_az;
  return (int64_t)s->width * s->height;
}

ut_status ut_project(const ut_gaussians* g, const ut_sensor* s, const double* ut_abk, ut_projected* out,
                     ut_stream stream) {
  if (!gaussians_ok(g) || !sensor_ok(s) || !ut_abk || !projected_ok(out, g ? g->n : 0)) return UT_ERR_ARG;
  const SensorK k = make_sensor_k(s);
  return from_hip(launch_project(*g, k, ut_abk, *out, as_stream(stream)));
}

size_t ut_count_workspace_bytes(int32_t n_gaussians) { return count_workspace(nullptr, n_gaussians).bytes; }

size_t ut_pair_workspace_bytes(uint64_t n_pairs) { return pair_workspace(nullptr, n_pairs).bytes; }

size_t ut_workspace_bytes(uint64_t max_pairs, int32_t n_tiles, int32_t n_gaussians) {
  (void)n_tiles;
  return ut_count_workspace_bytes(n_gaussians) + ut_pair_workspace_bytes(max_pairs);
}

ut_status ut_bin_count(const ut_projected* p, int32_t n, const ut_sensor* s, void* ws, size_t ws_bytes,
                       uint64_t* n_pairs_host, ut_stream stream) {
  if (n < 0 || !projected_ok(p, n) || !sensor_ok(s) || !ws) return UT_ERR_ARG;
  CountWorkspace w = count_workspace(ws, n);
  if (w.bytes > ws_bytes) return UT_ERR_CAPACITY;
  const SensorK k = make_sensor_k(s);
  hipError_t e = launch_bin_count(*p, n, k, w, as_stream(stream));
  if (e == hipSuccess && n_pairs_host)
    e = hipMemcpyAsync(n_pairs_host, w.total, sizeof(uint64_t), hipMemcpyDeviceToHost, as_stream(stream));
  return from_hip(e);
}

ut_status ut_bin_sort(const ut_projected* p, int32_t n, const ut_sensor* s, void* ws, size_t ws_bytes,
                      void* pair_ws, size_t pair_ws_bytes, uint64_t n_pairs, ut_bin_lists* bins,
                      ut_stream stream) {
  if (n < 0 || !projected_ok(p, n) || !sensor_ok(s) || !ws || !bins || !bins->ranges ||
      (n_pairs > 0 && (!bins->gauss || !pair_ws)))
    return UT_ERR_ARG;
  if (n_pairs > bins->max_pairs || n_pairs >= 0xFFFFFFFFull) return UT_ERR_CAPACITY;
  CountWorkspace w = count_workspace(ws, n);
  PairWorkspace pw = pair_workspace(pair_ws, n_pairs);
  if (w.bytes > ws_bytes || (n_pairs > 0 && pw.bytes > pair_ws_bytes)) return UT_ERR_CAPACITY;
  const SensorK k = make_sensor_k(s);
  return from_hip(launch_bin_sort(*p, n, k, w, pw, n_pairs, *bins, as_stream(stream)));
}

ut_status ut_bin_sort_device(const ut_projected* p, int32_t n, const ut_sensor* s, void* ws, size_t ws_bytes,
                             void* pair_ws, size_t pair_ws_bytes, uint64_t max_pairs, ut_bin_lists* bins,
                             uint32_t* overflow, ut_stream stream) {
  if (n < 0 || !projected_ok(p, n) || !sensor_ok(s) || !ws || !bins || !bins->ranges ||
      (max_pairs > 0 && (!bins->gauss || !pair_ws)))
    return UT_ERR_ARG;
  if (max_pairs > bins->max_pairs || max_pairs >= (1ull << 30)) return UT_ERR_CAPACITY;
  CountWorkspace w = count_workspace(ws, n);
  PairWorkspace pw = pair_workspace(pair_ws, max_pairs);
  if (w.bytes > ws_bytes || (max_pairs > 0 && pw.bytes > pair_ws_bytes)) return UT_ERR_CAPACITY;
  const SensorK k = make_sensor_k(s);
  return from_hip(launch_bin_sort_device(*p, n, k, w, pw, max_pairs, *bins, overflow, as_stream(stream)));
}

ut_status ut_bin_and_sort(const ut_projected* p, int32_t n, const ut_sensor* s, void* ws, size_t ws_bytes,
                          ut_bin_lists* bins, uint64_t* n_pairs, ut_stream stream) {
  uint64_t P = 0;
  ut_status st = ut_bin_count(p, n, s, ws, ws_bytes, &P, stream);
  if (st != UT_OK) return st;
  if (hipStreamSynchronize(as_stream(stream)) != hipSuccess) return UT_ERR_DEVICE;
  if (n_pairs) *n_pairs = P;
  const size_t cb = ut_count_workspace_bytes(n);
  char* pair_ws = static_cast<char*>(ws) + cb;
  return ut_bin_sort(p, n, s, ws, cb, pair_ws, ws_bytes - cb, P, bins, stream);
}

static bool bins_ok(const ut_bin_lists* b) { return b && b->ranges && (b->gauss || b->max_pairs == 0); }

ut_status ut_tile_lists_count(const ut_projected* p, const ut_sensor* s, const ut_bin_lists* bins,
                              ut_tile_lists* lists, uint64_t* n_pairs_host, ut_stream stream) {
  if (!p || !p->trect || !sensor_ok(s) || !bins_ok(bins) || !lists || !lists->ranges || !lists->n_pairs_dev)
    return UT_ERR_ARG;
  const SensorK k = make_sensor_k(s);
  hipError_t e = launch_tile_lists_count(*p, k, *bins, *lists, as_stream(stream));
  if (e == hipSuccess && n_pairs_host)
    e = hipMemcpyAsync(n_pairs_host, lists->n_pairs_dev, sizeof(uint64_t), hipMemcpyDeviceToHost, as_stream(stream));
  return from_hip(e);
}

ut_status ut_tile_lists_fill(const ut_projected* p, const ut_sensor* s, const ut_bin_lists* bins,
                             ut_tile_lists* lists, ut_stream stream) {
  if (!p || !p->trect || !sensor_ok(s) || !bins_ok(bins) || !lists || !lists->ranges || !lists->gauss)
    return UT_ERR_ARG;
  const SensorK k = make_sensor_k(s);
  return from_hip(launch_tile_lists_fill(*p, k, *bins, *lists, as_stream(stream)));
}

static ut_status composite_common(const ut_projected* p, const ut_bin_lists* bins, const ut_sensor* s,
                                  const ut_render_params* prm, ut_render_out* out, ut_stream stream) {
  if (!p || !p->records || !p->trect || !bins_ok(bins) || !sensor_ok(s) || !params_ok(prm) || !out ||
      !out->feat || !out->depth || !out->alpha)
    return UT_ERR_ARG;
  const SensorK k = make_sensor_k(s);
  return from_hip(launch_composite(*p, *bins, k, make_params(prm), *out, s->max_tile_rays, as_stream(stream)));
}

ut_status ut_composite_camera(const ut_projected* p, const ut_bin_lists* bins, const ut_sensor* s,
                              const ut_render_params* prm, ut_render_out* out, ut_stream stream) {
  if (!s || s->kind == UT_LIDAR) return UT_ERR_ARG;
  return composite_common(p, bins, s, prm, out, stream);
}

ut_status ut_composite_lidar(const ut_projected* p, const ut_bin_lists* bins, const ut_sensor* s,
                             const ut_render_params* prm, ut_render_out* out, ut_stream stream) {
  if (!s || s->kind != UT_LIDAR) return UT_ERR_ARG;
  return composite_common(p, bins, s, prm, out, stream);
}

size_t ut_backward_workspace_bytes(int32_t n_gaussians) {
  return (size_t)UT_ACC_FLOATS * sizeof(double) * (size_t)(n_gaussians > 0 ? n_gaussians : 1);
}

ut_status ut_composite_backward(const ut_gaussians* g, const ut_projected* p, const ut_bin_lists* bins,
                                const ut_sensor* s, const ut_render_params* prm, const ut_render_out* fwd,
                                const ut_upstream* up, void* acc_ws, size_t acc_ws_bytes,
                                ut_gaussian_grads* grads, ut_stream stream) {
  if (!gaussians_ok(g) || !p || !p->records || !p->trect || !bins_ok(bins) || !sensor_ok(s) || !params_ok(prm) ||
      !fwd || !fwd->feat || !fwd->t_final || !fwd->n_proc || !fwd->tile_end || !up || !acc_ws || !grads || !grads->mean ||
      !grads->quat || !grads->log_scale || !grads->opacity_logit || !grads->feat)
    return UT_ERR_ARG;
  if (acc_ws_bytes < ut_backward_workspace_bytes(g->n)) return UT_ERR_CAPACITY;
  if (s->max_tile_rays > 256) return UT_ERR_UNSUPPORTED;   // the adjoint runs one lane per ray of a tile
  const SensorK k = make_sensor_k(s);
  return from_hip(launch_backward(*g, *p, *bins, k, make_params(prm), *fwd, *up, static_cast<double*>(acc_ws),
                                  *grads, s->max_tile_rays, as_stream(stream)));
}

}  // extern "C"

// ---------------------------------------------------------------------------------- batch
namespace {

__global__ void k_write_item(BatchItemK item, BatchItemK* dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = item;
}

// The batch queue (four work counters, then the device copies of the items) at the start of
// a workspace of ut_batch_workspace_bytes(n_items) bytes.  The items are written by small
// kernels and the counters cleared by a fill kernel, so the whole call stays graph-capturable.
ut_status enqueue_batch(const ut_batch_item* items, int32_t n_items, const ut_render_params* prm, void* queue_ws,
                        int32_t n_workgroups, hipStream_t st) {
  uint32_t* counter = static_cast<uint32_t*>(queue_ws);
  BatchItemK* dev = reinterpret_cast<BatchItemK*>(static_cast<char*>(queue_ws) + 256);
  for (int i = 0; i < n_items; ++i) {
    const ut_batch_item& it = items[i];
    if (!it.proj || !it.proj->records || !it.proj->trect || !bins_ok(it.bins) || !sensor_ok(it.sensor) || !it.out ||
        !it.out->feat || !it.out->depth || !it.out->alpha)
      return UT_ERR_ARG;
    if (it.sensor->max_tile_rays > 256) return UT_ERR_UNSUPPORTED;   // one lane per ray of a 256-lane group
  }
  // items in four groups, each its own launch: static or moving sensor (the per-ray
  // origins of a moving sensor would otherwise cost every static pair registers), tiles or LiDAR
  // units (several azimuth tiles per 256-lane workgroup)
  BatchGroups grp;
  std::memset(&grp, 0, sizeof grp);
  int slot = 0;
  for (int gi = 0; gi < 4; ++gi) {
    const bool moving = (gi & 1) != 0, unit = (gi & 2) != 0;
    grp.first[gi] = slot;
    int total = 0;
    for (int i = 0; i < n_items; ++i) {
      const ut_batch_item& it = items[i];
      const bool it_unit = it.sensor->kind == UT_LIDAR && it.sensor->n_units_wide > 0;
      if ((it.sensor->moving != 0) != moving || it_unit != unit) continue;
      BatchItemK k;
      std::memset(&k, 0, sizeof k);
      k.s = make_sensor_k(it.sensor);
      if (unit) {   // this item's workgroups take the 256-lane units
        k.s.units = k.s.units_wide;
        k.s.n_units = k.s.n_units_wide;
        k.s.unit_rays = 256;
      }
      k.rec = reinterpret_cast<const RecordG*>(it.proj->records);
      k.trect = reinterpret_cast<const uint2*>(it.proj->trect);
      k.gauss = it.bins->gauss;
      k.ranges = it.bins->ranges;
      k.out = *it.out;
      k.n_tiles = unit ? k.s.n_units : ut_sensor_tiles(it.sensor);
      k.tile_base = total;
      total += k.n_tiles;
      hipLaunchKernelGGL(k_write_item, dim3(1), dim3(64), 0, st, k, dev + slot);
      ++slot;
    }
    grp.count[gi] = slot - grp.first[gi];
    grp.tiles[gi] = total;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return UT_ERR_DEVICE;
  return from_hip(launch_composite_batch(dev, grp, counter, make_params(prm), n_workgroups, st));
}

// Library-owned queue memory of ut_composite_batch_noalloc: one copy per device, for up to
// UT_BATCH_NOALLOC_MAX_ITEMS items, alive until the process ends.  In host code the array's
// name stands for a host-side shadow, not a device address: its device address is looked up
// once per device (hipGetSymbolAddress with that device current) and only that address is
// handed to kernels.
constexpr size_t kBatchScratchBytes = 256 + sizeof(BatchItemK) * (size_t)UT_BATCH_NOALLOC_MAX_ITEMS;
static __device__ __align__(256) unsigned char scratch[kBatchScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

ut_status batch_scratch_ptr(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return UT_ERR_DEVICE;
  if (dev >= kMaxDevices) return UT_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return UT_ERR_DEVICE;
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return UT_OK;
}

}  // namespace

extern "C" {

size_t ut_batch_workspace_bytes(int32_t n_items) {
  return 256 + sizeof(BatchItemK) * (size_t)(n_items > 0 ? n_items : 1);
}

ut_status ut_composite_batch(const ut_batch_item* items, int32_t n_items, const ut_render_params* prm,
                             void* queue_ws, size_t ws_bytes, int32_t n_workgroups, ut_stream stream) {
  if (!items || n_items <= 0 || !params_ok(prm) || !queue_ws || n_workgroups < 0) return UT_ERR_ARG;
  if (ws_bytes < ut_batch_workspace_bytes(n_items)) return UT_ERR_CAPACITY;
  return enqueue_batch(items, n_items, prm, queue_ws, n_workgroups, as_stream(stream));
}

ut_status ut_composite_batch_noalloc(const ut_batch_item* items, int32_t n_items, const ut_render_params* prm,
                                     int32_t n_workgroups, ut_stream stream) {
  if (!items || n_items <= 0 || !params_ok(prm) || n_workgroups < 0) return UT_ERR_ARG;
  if (n_items > UT_BATCH_NOALLOC_MAX_ITEMS) return UT_ERR_CAPACITY;
  void* ws = nullptr;
  const ut_status st = batch_scratch_ptr(&ws);
  if (st != UT_OK) return st;
  return enqueue_batch(items, n_items, prm, ws, n_workgroups, as_stream(stream));
}

ut_status ut_actor_transform(const ut_gaussians* g, const int32_t* actor, const ut_actor_pose* poses,
                             int32_t n_actors, float* mean_world, float* quat_world, ut_stream stream) {
  if (!g || g->n < 0 || n_actors < 0 || (n_actors > 0 && !poses)) return UT_ERR_ARG;
  if (g->n > 0 && (!g->mean || !g->quat || !actor || !mean_world || !quat_world)) return UT_ERR_ARG;
  return from_hip(launch_actor_transform(*g, actor, poses, n_actors, mean_world, quat_world, as_stream(stream)));
}

ut_status ut_actor_transform_backward(const ut_gaussians* g, const int32_t* actor,
                                      const ut_actor_pose* poses, int32_t n_actors,
                                      const float* d_mean_world, const float* d_quat_world,
                                      float* d_mean, float* d_quat, double* d_pose, ut_stream stream) {
  if (!g || g->n < 0 || n_actors < 0 || (n_actors > 0 && !poses)) return UT_ERR_ARG;
  if (g->n > 0 && (!g->mean || !g->quat || !actor || !d_mean_world || !d_quat_world || !d_mean || !d_quat))
    return UT_ERR_ARG;
  return from_hip(launch_actor_backward(*g, actor, poses, n_actors, d_mean_world, d_quat_world, d_mean, d_quat,
                                        d_pose, as_stream(stream)));
}

size_t ut_spatial_order_workspace_bytes(int32_t n_gaussians) { return spatial_order_ws_bytes(n_gaussians); }

ut_status ut_spatial_order(const ut_gaussians* g, uint32_t* perm, void* ws, size_t ws_bytes, ut_stream stream) {
  if (!g || g->n < 0 || (g->n > 0 && (!g->mean || !perm || !ws))) return UT_ERR_ARG;
  if (g->n > 0 && ws_bytes < spatial_order_ws_bytes(g->n)) return UT_ERR_CAPACITY;
  return from_hip(launch_spatial_order(*g, perm, ws, as_stream(stream)));
}

ut_status ut_gather_gaussians(const ut_gaussians* src, const uint32_t* perm, float* mean, float* quat,
                              float* log_scale, float* opacity_logit, float* feat, ut_stream stream) {
  if (!gaussians_ok(src)) return UT_ERR_ARG;
  const int n = src->n;
  if (n > 0 && (!perm || !mean || !quat || !log_scale || !opacity_logit || !feat)) return UT_ERR_ARG;
  const int K = (src->sh_degree + 1) * (src->sh_degree + 1);
  hipStream_t st = as_stream(stream);
  hipError_t e = launch_gather_rows(src->mean, perm, mean, 3, n, st);
  if (e == hipSuccess) e = launch_gather_rows(src->quat, perm, quat, 4, n, st);
  if (e == hipSuccess) e = launch_gather_rows(src->log_scale, perm, log_scale, 3, n, st);
  if (e == hipSuccess) e = launch_gather_rows(src->opacity_logit, perm, opacity_logit, 1, n, st);
  if (e == hipSuccess) e = launch_gather_rows(src->feat, perm, feat, 3 * K, n, st);
  return from_hip(e);
}

}  // extern "C"
