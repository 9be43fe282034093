// Host-side set-up code of the C-ABI (host_tables.hpp) under AddressSanitizer and
// UndefinedBehaviorSanitizer: Alg. 1 tiling, ray mask + summed-area table, compositing units
// and the argument checks, over seeded random LiDAR definitions and edge cases.  Prints "ok"
// and exits 0 when every invariant holds; any sanitizer finding aborts.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "host_tables.hpp"

#define CHECK(c)                                                      \
  do {                                                                \
    if (!(c)) {                                                       \
      std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
      std::exit(1);                                                   \
    }                                                                 \
  } while (0)

static void one_lidar(std::mt19937& rng, int n_beams, int n_az, int n_phi, int M, bool dups) {
  std::uniform_real_distribution<float> U(-0.44f, 0.26f);
  std::vector<float> be(n_beams);
  for (auto& x : be) x = U(rng);
  if (dups && n_beams > 2) be[1] = be[0];
  std::sort(be.begin(), be.end());
  if (n_beams > 1 && be.front() == be.back()) be.back() += 0.01f;
  std::vector<double> bounds(n_phi + 1);
  std::vector<int32_t> bstart(n_phi + 1);
  int32_t nth = 0;
  const ut_status st = ut_host::lidar_tiling(be.data(), n_beams, n_az, n_phi, M, bounds.data(), bstart.data(), &nth);
  if (n_beams < 2) { CHECK(st == UT_ERR_ARG); return; }
  if (st != UT_OK) { CHECK(st == UT_ERR_UNSUPPORTED); return; }
  CHECK(nth > 0);
  for (int k = 0; k < n_phi; ++k) CHECK(bounds[k] <= bounds[k + 1] && bstart[k] <= bstart[k + 1]);
  CHECK(bstart[0] == 0 && bstart[n_phi] == n_beams);
  const int mr = ut_host::max_tile_rays(bstart.data(), n_phi, n_az, nth);
  CHECK(mr > 0);
  const int w = ut_host::unit_width(mr);
  if (w > 0) {
    std::vector<int32_t> units(4 * (size_t)n_phi * nth);
    const int nu = ut_host::build_units(bstart.data(), n_phi, n_az, nth, w, units.data());
    CHECK(nu > 0 && nu <= n_phi * nth);
    std::vector<int> seen((size_t)n_phi * nth, 0);
    for (int u = 0; u < nu; ++u) {
      const int k = units[4 * u], j0 = units[4 * u + 1], j1 = units[4 * u + 2], rays = units[4 * u + 3];
      CHECK(k >= 0 && k < n_phi && j0 >= 0 && j0 < j1 && j1 <= nth && j1 - j0 <= ut_host::kUnitTiles);
      CHECK(j0 / ut_host::kSuperTile == (j1 - 1) / ut_host::kSuperTile);
      CHECK(rays <= w);
      for (int j = j0; j < j1; ++j) seen[(size_t)k * nth + j] += 1;
    }
    for (int v : seen) CHECK(v == 1);
    // the 256-lane packing for the batched kernel partitions the tiles too, in fewer units
    const int nw = ut_host::build_units(bstart.data(), n_phi, n_az, nth, 256, units.data());
    CHECK(nw > 0 && nw <= nu);
    std::fill(seen.begin(), seen.end(), 0);
    for (int u = 0; u < nw; ++u) {
      const int k = units[4 * u], j0 = units[4 * u + 1], j1 = units[4 * u + 2];
      CHECK(units[4 * u + 3] <= 256 && j1 - j0 <= ut_host::kUnitTiles);
      for (int j = j0; j < j1; ++j) seen[(size_t)k * nth + j] += 1;
    }
    for (int v : seen) CHECK(v == 1);
  }
  const int CA = 1 + (int)(rng() % 1600), CE = 1 + (int)(rng() % (8 * n_phi));
  std::vector<int32_t> sat((size_t)(CA + 1) * (CE + 1), 0);
  ut_host::ray_sat(be.data(), n_beams, n_az, bounds.data(), n_phi, CA, CE, sat.data());
  // the table's total is the number of occupied cells, and it never decreases along a row
  const int32_t total = sat[(size_t)CA * (CE + 1) + CE];
  CHECK(total > 0 && total <= CA * CE);
  for (int i = 1; i <= CA; ++i)
    for (int j = 1; j <= CE; ++j) CHECK(sat[(size_t)i * (CE + 1) + j] >= sat[(size_t)i * (CE + 1) + j - 1]);
}

int main() {
  std::mt19937 rng(7);
  const int beams[] = {1, 2, 3, 8, 17, 64, 128, 256};
  const int azs[] = {1, 7, 512, 2048};
  const int Ms[] = {1, 7, 32, 64, 512};
  for (int nb : beams)
    for (int na : azs)
      for (int M : Ms) {
        const int np = 1 + (int)(rng() % std::min(nb + 3, (int)UT_MAX_ELEV_TILES));
        one_lidar(rng, nb, na, np, M, (rng() & 1) != 0);
      }
  one_lidar(rng, 128, 2048, UT_MAX_ELEV_TILES, 32, false);
  // argument checks
  float be[3] = {0.1f, 0.0f, 0.2f};   // unsorted
  double bounds[5];
  int32_t bs[5], nth = 0;
  CHECK(ut_host::lidar_tiling(be, 3, 16, 2, 8, bounds, bs, &nth) == UT_ERR_ARG);
  CHECK(ut_host::lidar_tiling(nullptr, 3, 16, 2, 8, bounds, bs, &nth) == UT_ERR_ARG);
  float flat[3] = {0.1f, 0.1f, 0.1f};
  CHECK(ut_host::lidar_tiling(flat, 3, 16, 2, 8, bounds, bs, &nth) == UT_ERR_ARG);
  float nanb[3] = {0.0f, 0.1f, __builtin_nanf("")};
  CHECK(ut_host::lidar_tiling(nanb, 3, 16, 2, 8, bounds, bs, &nth) == UT_ERR_ARG);
  float ok3[3] = {0.0f, 0.1f, 0.2f};
  CHECK(ut_host::lidar_tiling(ok3, 3, 16, UT_MAX_ELEV_TILES + 1, 8, bounds, bs, &nth) == UT_ERR_ARG);
  CHECK(ut_host::lidar_tiling(ok3, 3, 16, 2, 0, bounds, bs, &nth) == UT_ERR_ARG);
  CHECK(ut_host::lidar_tiling(ok3, 3, 1 << 20, 2, 1, bounds, bs, &nth) == UT_ERR_UNSUPPORTED);
  ut_sensor s;
  std::memset(&s, 0, sizeof s);
  CHECK(!ut_host::sensor_ok(nullptr) && !ut_host::sensor_ok(&s));
  float dummy[3];
  s.ray_dir = dummy;
  s.kind = UT_PINHOLE;
  CHECK(!ut_host::sensor_ok(&s));
  s.width = 16; s.height = 16;
  CHECK(ut_host::sensor_ok(&s));
  s.beam_divergence = 0.01;
  CHECK(!ut_host::sensor_ok(&s));   // divergence is LiDAR-only
  s.beam_divergence = 0; s.moving = 1;
  CHECK(!ut_host::sensor_ok(&s));   // moving without ray origins
  s.moving = 0; s.kind = 9;
  CHECK(!ut_host::sensor_ok(&s));
  s.kind = UT_LIDAR; s.n_beams = 4; s.n_az = 8; s.n_phi = 2; s.n_theta = 2; s.tables = dummy;
  s.max_tile_rays = 16; s.unit_rays = 64; s.n_units = 4;
  CHECK(ut_host::sensor_ok(&s));
  s.unit_rays = 32;
  CHECK(!ut_host::sensor_ok(&s));
  s.unit_rays = 64; s.n_units = 5;
  CHECK(!ut_host::sensor_ok(&s));
  ut_gaussians g;
  std::memset(&g, 0, sizeof g);
  CHECK(ut_host::gaussians_ok(&g));   // empty set
  g.n = 3;
  CHECK(!ut_host::gaussians_ok(&g));
  g.n = 0; g.sh_degree = 4;
  CHECK(!ut_host::gaussians_ok(&g));
  ut_render_params p{1.0 / 255, 0.99, 1e-4};
  CHECK(ut_host::params_ok(&p));
  p.alpha_max = 1.0;
  CHECK(!ut_host::params_ok(&p) && !ut_host::params_ok(nullptr));
  std::puts("ok");
  return 0;
}
