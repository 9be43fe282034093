// host_tables.hpp -- host-side sensor set-up and argument checks of the C-ABI, in plain C++
// (no HIP): Alg. 1 elevation tiling, the ray mask and summed-area table of Appendix B, the
// LiDAR compositing units, the byte layout of the device tables, and the validity checks of
// sensors, particles and render parameters.  api.hip uses them; a sanitizer build of a small
// host driver exercises them without a GPU.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <vector>

#include "utrast.h"

namespace ut_host {

constexpr int kSuperTile = UT_SUPER_TILE;
// Tile rows of a LiDAR super-tile (cameras: UT_SUPER_TILE).  Fewer rows shorten the bin each
// LiDAR tile filters its list from, but add pairs, and past 256 super-tiles a second radix
// pass of the pair sort.  On the 300k-particle 128 x 2048 scan: 2 rows, bins 2.6x the tile
// lists instead of 7x, compositing -13%, pair sort +60 us; 4 rows, compositing 202 -> 177 us,
// one more radix pass (+15 us), and the multi-sensor frame about 1% slower.  The square
// super-tile is kept.
constexpr int kLidarSuperRows = UT_SUPER_TILE;
inline int super_rows(int kind) { return kind == UT_LIDAR ? kLidarSuperRows : kSuperTile; }
constexpr int kUnitTiles = 4;         // tiles of a LiDAR compositing unit at most
constexpr double kPiHost = 3.14159265358979323846;

// Byte layout of the LiDAR device tables (bounds, beam_start, sat, units), 256-byte aligned.
struct TableLayout {
  size_t bounds, beam_start, sat, units, total;
};
inline TableLayout table_layout(int n_phi, int cull_az, int cull_el, int n_tiles) {
  auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
  TableLayout t;
  t.bounds = 0;
  t.beam_start = al(sizeof(double) * (size_t)(n_phi + 1));
  t.sat = t.beam_start + al(sizeof(int) * (size_t)(n_phi + 1));
  t.units = t.sat + al(sizeof(int) * (size_t)(cull_az + 1) * (size_t)(cull_el + 1));
  // two unit lists of up to n_tiles units each: for the single-request kernel (unit_rays lanes)
  // and for the batched kernel's 256-lane workgroups
  t.total = t.units + al(2 * 4 * sizeof(int) * (size_t)(n_tiles > 0 ? n_tiles : 1));
  return t;
}

// Alg. 1.  Histogram of per-ray elevations (each beam counts n_az rays) over r = 400 bins
// spanning [min, max] elevation; a boundary sits at the upper edge of every bin where the
// cumulative count reaches b/N_phi of the total (tested while it holds, so one bin can place
// several boundaries); N_theta = ceil(max rays of an elevation tile / M).
inline ut_status lidar_tiling(const float* beam_elev, int32_t n_beams, int32_t n_az, int32_t n_phi, int32_t M,
                              double* bounds, int32_t* beam_start, int32_t* n_theta) {
  if (!beam_elev || !bounds || !beam_start || !n_theta || n_beams <= 0 || n_az <= 0 || n_phi <= 0 ||
      n_phi > UT_MAX_ELEV_TILES || M <= 0)
    return UT_ERR_ARG;
  for (int b = 1; b < n_beams; ++b)
    if (!(beam_elev[b] >= beam_elev[b - 1])) return UT_ERR_ARG;
  const int r_bins = 400;
  const double lo = beam_elev[0], hi = beam_elev[n_beams - 1];
  if (!(hi > lo) || !std::isfinite(lo) || !std::isfinite(hi)) return UT_ERR_ARG;
  const double w = (hi - lo) / r_bins;
  std::vector<long long> cum(r_bins, 0);
  for (int b = 0; b < n_beams; ++b) {
    int bin = (int)std::floor(((double)beam_elev[b] - lo) / w);
    bin = std::min(std::max(bin, 0), r_bins - 1);
    cum[bin] += n_az;
  }
  for (int i = 1; i < r_bins; ++i) cum[i] += cum[i - 1];
  const long long total = cum[r_bins - 1];
  int placed = 0;
  bounds[0] = lo;
  for (int i = 0; i < r_bins && placed < n_phi; ++i)
    while (placed < n_phi && cum[i] * (long long)n_phi >= (long long)(placed + 1) * total) {
      ++placed;
      bounds[placed] = lo + (i + 1) * w;
    }
  long long most = 0;
  int b = 0;
  for (int k = 0; k < n_phi; ++k) {
    beam_start[k] = b;
    if (k == n_phi - 1) b = n_beams;
    else
      while (b < n_beams && (double)beam_elev[b] < bounds[k + 1]) ++b;
    most = std::max(most, (long long)(b - beam_start[k]) * n_az);
  }
  beam_start[n_phi] = n_beams;
  const long long nth = (most + M - 1) / M;
  if (nth <= 0 || nth > 0x7FFF) return UT_ERR_UNSUPPORTED;   // tile rects pack 16-bit columns
  *n_theta = (int32_t)nth;
  return UT_OK;
}

// First azimuth step of azimuth tile j of n_theta over n_az steps.
inline int az_start(int j, int n_az, int n_theta) { return (int)(((long long)j * n_az + n_theta - 1) / n_theta); }

// Largest ray count of one tile.
inline int max_tile_rays(const int32_t* beam_start, int n_phi, int n_az, int n_theta) {
  int max_beams = 0;
  for (int k = 0; k < n_phi; ++k) max_beams = std::max(max_beams, beam_start[k + 1] - beam_start[k]);
  int max_az = 0;
  for (int j = 0; j < n_theta; ++j) max_az = std::max(max_az, az_start(j + 1, n_az, n_theta) - az_start(j, n_az, n_theta));
  return max_beams * max_az;
}

// Ray mask over (cull_az azimuth cells over 360 deg) x (cull_el elevation cells over
// [bounds[0], bounds[n_phi]]) and its summed-area table sat[(cull_az + 1) * (cull_el + 1)]
// (zero-initialised by the caller): sat[i][j] = occupied cells with az < i and el < j.
inline void ray_sat(const float* beam_elev, int n_beams, int n_az, const double* bounds, int n_phi, int cull_az,
                    int cull_el, int32_t* sat) {
  const int CA = cull_az, CE = cull_el;
  std::vector<uint8_t> mask((size_t)CA * CE, 0);
  const double e0 = bounds[0], span = bounds[n_phi] - bounds[0];
  for (int b = 0; b < n_beams; ++b) {
    int ce = (int)std::floor(((double)beam_elev[b] - e0) * CE / span);
    ce = std::min(std::max(ce, 0), CE - 1);
    for (int a = 0; a < n_az; ++a) mask[(size_t)((long long)a * CA / n_az) * CE + ce] = 1;
  }
  const size_t W = (size_t)CE + 1;
  for (int i = 1; i <= CA; ++i) {
    int32_t row = 0;
    for (int j = 1; j <= CE; ++j) {
      row += mask[(size_t)(i - 1) * CE + (j - 1)];
      sat[i * W + j] = sat[(i - 1) * W + j] + row;
    }
  }
}

// Compositing units: greedy runs of adjacent azimuth tiles of one elevation tile inside one
// super-tile column (so one bin serves the whole unit), at most kUnitTiles long, while the
// rays fit unit_rays lanes.  units[4 * u] = (elevation tile, first tile, end tile, rays);
// room for n_phi * n_theta units.  Returns the unit count.
inline int build_units(const int32_t* beam_start, int n_phi, int n_az, int n_theta, int unit_rays, int32_t* units) {
  int n = 0;
  for (int k = 0; k < n_phi; ++k) {
    const long long nb = beam_start[k + 1] - beam_start[k];
    for (int c0 = 0; c0 < n_theta; c0 += kSuperTile) {
      const int c1 = std::min(c0 + kSuperTile, n_theta);
      for (int j0 = c0; j0 < c1;) {
        int j1 = j0 + 1;
        while (j1 < c1 && j1 - j0 < kUnitTiles &&
               nb * (az_start(j1 + 1, n_az, n_theta) - az_start(j0, n_az, n_theta)) <= unit_rays)
          ++j1;
        units[4 * n + 0] = k;
        units[4 * n + 1] = j0;
        units[4 * n + 2] = j1;
        units[4 * n + 3] = (int32_t)(nb * (az_start(j1, n_az, n_theta) - az_start(j0, n_az, n_theta)));
        ++n;
        j0 = j1;
      }
    }
  }
  return n;
}

// The workgroup width of a LiDAR's units: the smallest of 64, 128, 256 that holds its largest
// tile, 0 when none does (its tiles are then composited one per workgroup).
inline int unit_width(int max_rays) {
  for (int cap : {64, 128, 256})
    if (max_rays <= cap) return cap;
  return 0;
}

inline bool sensor_ok(const ut_sensor* s) {
  if (!s || !s->ray_dir) return false;
  if (s->moving && (!s->ray_org || s->rs_iters < 1 || s->rs_iters > 64 || s->kind == UT_ORTHO)) return false;
  if (!(s->beam_divergence >= 0 && s->beam_divergence < kPiHost)) return false;
  if (s->beam_divergence > 0 && s->kind != UT_LIDAR) return false;
  if (s->kind == UT_LIDAR)
    return s->n_beams > 0 && s->n_az > 0 && s->n_phi > 0 && s->n_phi <= UT_MAX_ELEV_TILES &&
           s->n_theta > 0 && s->tables && s->max_tile_rays > 0 && s->max_tile_rays <= UT_MAX_LIDAR_TILE_RAYS &&
           s->n_units >= 0 && (long long)s->n_units <= (long long)s->n_phi * s->n_theta &&
           s->n_units_wide >= 0 && (long long)s->n_units_wide <= (long long)s->n_phi * s->n_theta &&
           (s->unit_rays == 0 || ((s->unit_rays == 64 || s->unit_rays == 128 || s->unit_rays == 256) &&
                                  s->unit_rays >= s->max_tile_rays)) &&
           (!s->cull || (s->cull_az > 0 && s->cull_el > 0));
  if (s->kind == UT_PINHOLE || s->kind == UT_FISHEYE || s->kind == UT_ORTHO)
    return s->width > 0 && s->height > 0;
  return false;
}

inline bool gaussians_ok(const ut_gaussians* g) {
  return g && g->n >= 0 && g->sh_degree >= 0 && g->sh_degree <= 3 &&
         (g->feat_kind == UT_FEAT_CAMERA || g->feat_kind == UT_FEAT_LIDAR) &&
         (g->n == 0 || (g->mean && g->quat && g->log_scale && g->opacity_logit && g->feat));
}

inline bool params_ok(const ut_render_params* p) {
  return p && p->alpha_min > 0 && p->alpha_max >= p->alpha_min && p->alpha_max < 1 && p->t_min >= 0;
}

}  // namespace ut_host
