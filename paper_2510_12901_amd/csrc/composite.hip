// composite.hip -- per-ray front-to-back compositing (Eq. 1) over tile lists.
//
// One workgroup per tile, one lane per ray.  The workgroup streams its super-tile bin and
// keeps the entries whose rect contains the tile (ballot + popcount per wavefront, wave
// counts combined in LDS); these form the tile's exact (depth, index) list.  Of those it
// appends to an LDS ring only the entries that can reach alpha_min on at least one ray of
// the tile (the tile-cone test below), stages batches of their 128-byte records in LDS
// (gathered cooperatively as 16-byte chunks), and every lane walks the batch for its own ray.
// A lane that reaches T < t_min stops (its wavefront stops when all 64 lanes have), and the
// workgroup stops once every lane is done.  LiDAR tiles are composited in units of a few
// adjacent azimuth tiles per workgroup: the unit keeps the bin entries that meet any of its
// tiles, with per-tile list positions, and each ray walks only its own tile's entries.
//
// Per (ray, particle), from the record's response quadric B = Sigma^{-1}, B v and v^T B v
// (v = mu - o): d^T B d from the ray's six quadratic monomials, d^T B v, and
// num = v^T B v d^T B d - (d^T B v)^2; the pair is rejected when num > cut d^T B d (alpha
// cannot reach alpha_min), else t* = d^T B v / d^T B d, D^2 = num / d^T B d (records of very
// thin particles take D^2 from the residual u = v - t* d instead) and rho = exp(-D^2/2) --
// all float64 with explicit FMAs, so no contraction flag can change the arithmetic between
// the plain and the batched kernel, or between forward and adjoint.
#include "ut_cone.hpp"
#include "ut_internal.hpp"

namespace ut {
namespace {

// Camera tiles (16 x 16 rays) and the batched kernel (any tile of up to 256 rays) run BLOCK
// threads with RPL rays per lane and stage BATCH records per step.
constexpr int kCamBlock = 256, kCamRpl = 1, kCamBatch = 128;
static_assert(kCamBlock * kCamRpl >= 256, "batched tiles (up to 256 rays) must fit one workgroup");

// BLOCK threads, RPL rays per lane: one workgroup covers up to BLOCK * RPL rays.  Records are
// staged BATCH at a time; the ring of candidate indices holds a batch plus one refill step of
// BLOCK entries.  Keeping LDS per workgroup small lets the register count, not LDS, set the
// occupancy.
template <int BLOCK, int RPL, int BATCH>
struct CompositeShared {
  static_assert(BATCH >= 32 && (BATCH & (BATCH - 1)) == 0, "batch must be a power of two");
  static constexpr int kBatch = BATCH;
  static constexpr uint32_t kRing = BATCH + BLOCK <= 2 * BATCH ? 2 * BATCH : 4 * BATCH;
  static_assert(BATCH + BLOCK <= (int)kRing, "ring must hold a batch plus one refill step");
  Record rec[BATCH];
  uint32_t rpos[BATCH];    // position of each staged record in the tile's list
  uint32_t rbin[BATCH];    // ... and in the super-tile bin
  uint32_t cand[kRing];    // ring of candidate particle indices ...
  uint32_t cpos[kRing];    // ... their positions in the tile's list ...
  uint32_t cbin[kRing];    // ... and in the super-tile bin
  uint32_t tend;           // the tile's bin end for the adjoint
  uint2 wcnt[BLOCK / 64];  // per wavefront: (rect hits, kept entries) of one refill step
  double red[4][BLOCK / 64];
  double etab[32];         // LDS copy of kExp2Frac for the response's exponential
  TileCone cone;
};

// What a LiDAR unit (several azimuth tiles in one workgroup) adds: per candidate the tiles of
// the unit its rect covers (bit t = tile j0 + t), per candidate and staged record its position
// in each of those tiles' lists, per tile the staged slots of its entries, the list entries
// seen so far and the adjoint's bin end.
template <int BLOCK, int BATCH>
struct UnitShared {
  static constexpr uint32_t kRing = CompositeShared<BLOCK, 1, BATCH>::kRing;
  uint32_t cposT[kRing][kUnitTilesMax];
  uint32_t rposT[BATCH][kUnitTilesMax];
  uint8_t cmask[kRing];
  uint32_t wcntT[BLOCK / 64][kUnitTilesMax];
  uint8_t tlist[kUnitTilesMax][BATCH];   // per tile: the staged slots of its list entries, in order
  uint32_t nhT[kUnitTilesMax];
  uint32_t tendT[kUnitTilesMax];
};

// TILE_END: track each ray's bin end and write the tile's (adjoint state); the batched serving
// path, which never feeds an adjoint, leaves it out and keeps those registers.
// UNIT: `tile` is a LiDAR unit (s.units): the rays of its g tiles share the workgroup, the
// candidates are the bin entries meeting any of the g tiles, and each ray evaluates only the
// entries that cover its own tile, in the same order -- exactly its tile's list.  List
// positions (n_proc) and bin ends (tile_end) are kept per tile.  us is used only for UNIT.
template <int BLOCK, int RPL, int BATCH, bool STATS = false, bool MOVING = false, bool TILE_END = true,
          bool UNIT = false>
__device__ __forceinline__ void composite_tile(const SensorK& s, const RecordG* __restrict__ rec,
                                               const uint2* __restrict__ trect,
                                               const uint32_t* __restrict__ bgauss,
                                               const uint32_t* __restrict__ branges, int tile, int n_super,
                                               const RenderParamsK& prm, const ut_render_out& out,
                                               CompositeShared<BLOCK, RPL, BATCH>& sm,
                                               UnitShared<BLOCK, BATCH>* us = nullptr) {
  static_assert(!UNIT || RPL == 1, "a unit runs one ray per lane");
  static_assert(!UNIT || BATCH <= BLOCK, "a unit's per-tile lists give each staged slot its own thread");
  constexpr int kBatch = BATCH;
  constexpr uint32_t kRing = CompositeShared<BLOCK, RPL, BATCH>::kRing - 1;
  int tx, ty, sid, j0 = 0, gt = 1;
  if constexpr (UNIT) {
    const int4 u = s.units[tile];
    ty = u.x;
    j0 = u.y;
    gt = u.z - u.y;
    tx = j0;
    sid = (ty / s.super_h) * s.super_x + j0 / kSuper;
  } else {
    tx = tile % s.tiles_x;
    ty = tile / s.tiles_x;
    sid = super_of_tile(tile, s);
  }
  const uint32_t start = branges[sid], end = branges[n_super + sid];
  int tl[RPL];        // UNIT: the ray's tile relative to j0
  long long ray[RPL];
  double dx[RPL], dy[RPL], dz[RPL], T[RPL], f0[RPL], f1[RPL], f2[RPL], dep[RPL];
  double ex[RPL], ey[RPL], ez[RPL];   // moving sensor: ray origin minus the sensor origin
  double emax = 0.0;
  uint32_t nproc[RPL], nbin[RPL], nvisit[RPL], npass[RPL];
  bool rdone[RPL];
  bool done = true;
  double sx = 0, sy = 0, sz = 0;
#pragma unroll
  for (int k = 0; k < RPL; ++k) {
    tl[k] = 0;
    if constexpr (UNIT) ray[k] = unit_ray(s, s.units[tile], threadIdx.x + k * BLOCK, &tl[k]);
    else ray[k] = tile_ray(s, tile, threadIdx.x + k * BLOCK);
    dx[k] = dy[k] = dz[k] = 0;
    if (ray[k] >= 0) {
      dx[k] = s.ray_dir[ray[k]];
      dy[k] = s.ray_dir[s.n_rays + ray[k]];
      dz[k] = s.ray_dir[2 * s.n_rays + ray[k]];
    }
    rdone[k] = !(ray[k] >= 0 && (dx[k] != 0 || dy[k] != 0 || dz[k] != 0));
    done = done && rdone[k];
    ex[k] = ey[k] = ez[k] = 0;
    if constexpr (MOVING) {
      if (!rdone[k]) {
        ex[k] = (double)s.ray_org[ray[k]] - s.o[0];
        ey[k] = (double)s.ray_org[s.n_rays + ray[k]] - s.o[1];
        ez[k] = (double)s.ray_org[2 * s.n_rays + ray[k]] - s.o[2];
      }
    }
    T[k] = 1.0;
    f0[k] = f1[k] = f2[k] = dep[k] = 0;
    nproc[k] = nbin[k] = nvisit[k] = npass[k] = 0;
    if (!rdone[k]) {
      const double il = rcp_f64(__builtin_sqrt(__builtin_fma(dx[k], dx[k], __builtin_fma(dy[k], dy[k], dz[k] * dz[k]))));
      sx = __builtin_fma(dx[k], il, sx);
      sy = __builtin_fma(dy[k], il, sy);
      sz = __builtin_fma(dz[k], il, sz);
    }
  }
  RayQ rq[RPL];
#pragma unroll
  for (int k = 0; k < RPL; ++k) rq[k] = ray_q(dx[k], dy[k], dz[k]);
  const int lane = __lane_id(), wave = threadIdx.x >> 6;
  const unsigned long long lt = (1ull << lane) - 1ull;
  if (threadIdx.x < 32) sm.etab[threadIdx.x] = kExp2Frac[threadIdx.x];
  if constexpr (UNIT) {
    if (threadIdx.x < kUnitTilesMax) us->nhT[threadIdx.x] = 0, us->tendT[threadIdx.x] = 0;
  }

  // bounding cone of the tile's rays (identical in every lane: built from block reductions)
  double ux, uy, uz, sn;
  tile_cone_axis<BLOCK>(sx, sy, sz, sm.red, wave, lane, ux, uy, uz, sn);
  double cmin = 1.0;
#pragma unroll
  for (int k = 0; k < RPL; ++k)
    if (!rdone[k]) cmin = fmin(cmin, cone_cos(ux, uy, uz, dx[k], dy[k], dz[k]));
  double etx = 0, ety = 0, etz = 0;
  if constexpr (MOVING) {
    // reference origin of the tile: the mean ray origin; spread: the largest distance from it
    double cx = 0, cy = 0, cz = 0, cnt = 0;
#pragma unroll
    for (int k = 0; k < RPL; ++k)
      if (!rdone[k]) cx += ex[k], cy += ey[k], cz += ez[k], cnt += 1.0;
    cnt = block_reduce<BLOCK>(cnt, false, sm.red[3], wave, lane);
    cx = block_reduce<BLOCK>(cx, false, sm.red[0], wave, lane);
    cy = block_reduce<BLOCK>(cy, false, sm.red[1], wave, lane);
    cz = block_reduce<BLOCK>(cz, false, sm.red[2], wave, lane);
    if (cnt > 0) etx = cx / cnt, ety = cy / cnt, etz = cz / cnt;
    emax = 0.0;
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
      if (rdone[k]) continue;
      const double fx = ex[k] - etx, fy = ey[k] - ety, fz = ez[k] - etz;
      emax = fmax(emax, __builtin_sqrt(__builtin_fma(fx, fx, __builtin_fma(fy, fy, fz * fz))));
    }
    emax = -block_reduce<BLOCK>(-emax, true, sm.red[0], wave, lane);
  }
  tile_cone_finish<BLOCK>(cmin, sn, ux, uy, uz, sm.red, wave, lane, sm.cone, emax, etx, ety, etz);
  const bool cull = sm.cone.on != 0;

  uint32_t pos = start, head = 0, n_cand = 0, n_hits = 0;   // uniform across the workgroup

  for (;;) {
    if (__syncthreads_and(done)) break;
    // refill the candidate ring with this tile's list entries that pass the tile-cone test
    while (n_cand < (uint32_t)kBatch && pos < end) {
      const uint32_t j = pos + threadIdx.x;
      uint32_t g = 0;
      bool hit = false;
      uint32_t tmask = 0;   // UNIT: tiles of the unit the entry's rect covers
      if (j < end) {
        g = bgauss[j];
        if constexpr (UNIT) {
          const uint2 r = trect[g];
          if (rect_meets_unit(r, ty, j0, j0 + gt, s))
            for (int t = 0; t < gt; ++t) tmask |= rect_covers(r, j0 + t, ty, s) ? 1u << t : 0u;
          hit = tmask != 0;
        } else {
          hit = rect_covers(trect[g], tx, ty, s);
        }
      }
      const bool keep = hit && !(cull && cone_rejects<MOVING>(rec + g, sm.cone, prm.log_alpha_min));
      const unsigned long long mh = __ballot(hit), mk = __ballot(keep);
      if (lane == 0) sm.wcnt[wave] = make_uint2((uint32_t)__popcll(mh), (uint32_t)__popcll(mk));
      if constexpr (UNIT) {
        // per tile of the unit: how many of this step's entries its list gains, per wavefront
        for (int t = 0; t < gt; ++t) {
          const unsigned long long mt = __ballot((tmask >> t) & 1u);
          if (lane == 0) us->wcntT[wave][t] = (uint32_t)__popcll(mt);
        }
      }
      __syncthreads();
      uint32_t hb = 0, kb = 0, ht = 0, kt = 0;
#pragma unroll
      for (int w = 0; w < BLOCK / 64; ++w) {
        const uint2 c = sm.wcnt[w];
        if (w < wave) hb += c.x, kb += c.y;
        ht += c.x, kt += c.y;
      }
      const uint32_t slot = (head + n_cand + kb + (uint32_t)__popcll(mk & lt)) & kRing;
      if (keep) {
        sm.cand[slot] = g;
        sm.cpos[slot] = n_hits + hb + (uint32_t)__popcll(mh & lt);
        if constexpr (TILE_END) sm.cbin[slot] = j;
      }
      uint32_t step_t = 0;   // UNIT, thread t < gt: entries tile t's list gains in this step
      if constexpr (UNIT) {
        // the entry's position in each covered tile's list (entries the cone drops count too)
        for (int t = 0; t < gt; ++t) {
          const unsigned long long mt = __ballot((tmask >> t) & 1u);
          if (keep && ((tmask >> t) & 1u)) {
            uint32_t base = us->nhT[t];
            for (int w = 0; w < wave; ++w) base += us->wcntT[w][t];
            us->cposT[slot][t] = base + (uint32_t)__popcll(mt & lt);
          }
        }
        if (keep) us->cmask[slot] = (uint8_t)tmask;
        if ((int)threadIdx.x < gt)
          for (int w = 0; w < BLOCK / 64; ++w) step_t += us->wcntT[w][threadIdx.x];
      }
      n_cand += kt;
      n_hits += ht;
      pos += BLOCK;
      __syncthreads();
      if constexpr (UNIT) {
        if ((int)threadIdx.x < gt) us->nhT[threadIdx.x] += step_t;
      }
    }
    if (n_cand == 0) break;
    const uint32_t cnt = min(n_cand, (uint32_t)kBatch);
    // stage the batch: the float64 chunks as plain copies, then per record its features
    // widened to float64 (two uniform loops instead of one with a divergent chunk)
    for (uint32_t c = threadIdx.x; c < cnt * kFeatChunk; c += BLOCK) {
      const uint32_t j = c / kFeatChunk, part = c - j * kFeatChunk;
      const uint32_t g = sm.cand[(head + j) & kRing];
      reinterpret_cast<uint4*>(sm.rec + j)[part] = reinterpret_cast<const uint4*>(rec + g)[part];
    }
    for (uint32_t j = threadIdx.x; j < cnt; j += BLOCK) {
      const uint32_t slot = (head + j) & kRing;
      const uint32_t g = sm.cand[slot];
      const uint4 x = reinterpret_cast<const uint4*>(rec + g)[kFeatChunk];
      sm.rec[j].feat[0] = (double)__uint_as_float(x.x);
      sm.rec[j].feat[1] = (double)__uint_as_float(x.y);
      sm.rec[j].feat[2] = (double)__uint_as_float(x.z);
      sm.rpos[j] = sm.cpos[slot];
      if constexpr (TILE_END) sm.rbin[j] = sm.cbin[slot];
      if constexpr (UNIT) {
        const uint32_t m = us->cmask[slot];
        for (int t = 0; t < gt; ++t)
          if ((m >> t) & 1u) us->rposT[j][t] = us->cposT[slot][t];
      }
    }
    if constexpr (UNIT) {
      // per tile of the unit, the staged slots of its entries in list order (slot j is thread
      // j's: a batch never exceeds the workgroup), so each ray walks only its own tile's entries
      const uint32_t jt = threadIdx.x;
      const uint32_t mt = jt < cnt ? (uint32_t)us->cmask[(head + jt) & kRing] : 0u;
      unsigned long long bt[kUnitTilesMax];
#pragma unroll
      for (int t = 0; t < kUnitTilesMax; ++t) {
        bt[t] = __ballot(t < gt && ((mt >> t) & 1u));
        if (lane == 0) us->wcntT[wave][t] = (uint32_t)__popcll(bt[t]);
      }
      __syncthreads();
#pragma unroll
      for (int t = 0; t < kUnitTilesMax; ++t) {
        if (t < gt && ((mt >> t) & 1u)) {
          uint32_t p = (uint32_t)__popcll(bt[t] & lt);
          for (int w = 0; w < wave; ++w) p += us->wcntT[w][t];
          us->tlist[t][p] = (uint8_t)jt;
        }
      }
    }
    __syncthreads();
    if constexpr (UNIT) {
      if (!done) {
        // LiDAR units: the longest units set the launch time and run alone at the end, so each
        // ray takes two of its tile's entries per step (two independent float64 chains), then
        // composites them in list order; the second is evaluated even when the first ends the ray
        const int t = tl[0];
        uint32_t n_t = 0;
        for (int w = 0; w < BLOCK / 64; ++w) n_t += us->wcntT[w][t];
        auto resp = [&](const Record& r, double& tau, double& alpha, bool& pass) -> bool {
          Centre cv;
          if constexpr (MOVING) cv = pair_centre(r, ex[0], ey[0], ez[0]);
          else cv = record_centre(r);
          PairResp pr;
          pass = pair_eval<Record, false>(r, cv, rq[0], MOVING ? ex[0] : 0.0, MOVING ? ey[0] : 0.0,
                                          MOVING ? ez[0] : 0.0, cut_threshold(r.log_sigma, prm.log_alpha_min), pr);
          tau = pr.tau;
          alpha = __builtin_fmin(pair_alpha(r, pr, sm.etab), prm.alpha_max);
          return pass && tau >= s.near_ && alpha >= prm.alpha_min;
        };
        auto add = [&](const Record& r, double tau, double alpha, uint32_t j) {
          const double w = alpha * T[0];
          f0[0] = __builtin_fma(w, r.feat[0], f0[0]);
          f1[0] = __builtin_fma(w, r.feat[1], f1[0]);
          f2[0] = __builtin_fma(w, r.feat[2], f2[0]);
          dep[0] = __builtin_fma(w, tau, dep[0]);
          T[0] = T[0] * (1.0 - alpha);
          if (T[0] < prm.t_min) {
            rdone[0] = true;
            nproc[0] = us->rposT[j][t] + 1;
            if constexpr (TILE_END) nbin[0] = sm.rbin[j] + 1;
          }
        };
        for (uint32_t p = 0; p < n_t; p += 2) {
          const bool two = p + 1 < n_t;
          const uint32_t ja = us->tlist[t][p], jb = two ? us->tlist[t][p + 1] : ja;
          const Record& ra = sm.rec[ja];
          const Record& rb = sm.rec[jb];
          double taua, alpa, taub, alpb;
          bool passa, passb;
          const bool hita = resp(ra, taua, alpa, passa);
          const bool hitb = resp(rb, taub, alpb, passb);
          if constexpr (STATS) ++nvisit[0], npass[0] += passa ? 1u : 0u;
          if (hita) add(ra, taua, alpa, ja);
          if (rdone[0] || !two) break;
          if constexpr (STATS) ++nvisit[0], npass[0] += passb ? 1u : 0u;
          if (hitb) add(rb, taub, alpb, jb);
          if (rdone[0]) break;
        }
        done = rdone[0];
      }
    } else if (!done) {
      for (uint32_t j = 0; j < cnt; ++j) {
        const Record& r = sm.rec[j];
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
          if (rdone[k]) continue;
          Centre cv;
          if constexpr (MOVING) cv = pair_centre(r, ex[k], ey[k], ez[k]);
          else cv = record_centre(r);
          if constexpr (STATS) ++nvisit[k];
          // the response is evaluated for every visited pair and the three skip tests are taken
          // together: one branch per pair instead of three (the pre-test passes ~90% of pairs)
          PairResp pr;
          const bool pass = pair_eval(r, cv, rq[k], MOVING ? ex[k] : 0.0, MOVING ? ey[k] : 0.0, MOVING ? ez[k] : 0.0,
                                      cut_threshold(r.log_sigma, prm.log_alpha_min), pr);
          if constexpr (STATS) npass[k] += pass ? 1u : 0u;
          const double tau = pr.tau;
          const double alpha = __builtin_fmin(pair_alpha(r, pr, sm.etab), prm.alpha_max);
          if (!(pass && tau >= s.near_ && alpha >= prm.alpha_min)) continue;
          const double w = alpha * T[k];
          f0[k] = __builtin_fma(w, r.feat[0], f0[k]);
          f1[k] = __builtin_fma(w, r.feat[1], f1[k]);
          f2[k] = __builtin_fma(w, r.feat[2], f2[k]);
          dep[k] = __builtin_fma(w, tau, dep[k]);
          T[k] = T[k] * (1.0 - alpha);
          if (T[k] < prm.t_min) {
            rdone[k] = true;
            // list entries up to and including the terminating one
            nproc[k] = sm.rpos[j] + 1;
            if constexpr (TILE_END) nbin[k] = sm.rbin[j] + 1;   // bin entries up to and including it
          }
        }
        bool all = true;
#pragma unroll
        for (int k = 0; k < RPL; ++k) all = all && rdone[k];
        if (all) {
          done = true;
          break;
        }
      }
    }
    head = (head + cnt) & kRing;
    n_cand -= cnt;
  }
  // a ray still open here has visited the whole list of its tile
  if constexpr (UNIT) __syncthreads();   // the per-tile list lengths are final
#pragma unroll
  for (int k = 0; k < RPL; ++k)
    if (!rdone[k]) {
      if constexpr (UNIT) nproc[k] = us->nhT[tl[k]];
      else nproc[k] = n_hits;
      nbin[k] = end;
    }
  if (UNIT && TILE_END && out.tile_end) {
    // per tile of the unit: the largest bin end of its rays
#pragma unroll
    for (int k = 0; k < RPL; ++k)
      if (ray[k] >= 0 && nproc[k] > 0) atomicMax(&us->tendT[tl[k]], nbin[k]);
    __syncthreads();
    if ((int)threadIdx.x < gt) out.tile_end[ty * s.tiles_x + j0 + threadIdx.x] = us->tendT[threadIdx.x];
  } else if (TILE_END && out.tile_end) {   // uniform: the adjoint walks the bin back from the largest end
    uint32_t m = 0;
#pragma unroll
    for (int k = 0; k < RPL; ++k) m = nproc[k] > 0 && nbin[k] > m ? nbin[k] : m;
    if (threadIdx.x == 0) sm.tend = 0;
    __syncthreads();
    if (m > 0) atomicMax(&sm.tend, m);
    __syncthreads();
    if (threadIdx.x == 0) out.tile_end[tile] = sm.tend;
  }
#pragma unroll
  for (int k = 0; k < RPL; ++k) {
    if (ray[k] < 0) continue;
    const long long R = s.n_rays, id = ray[k];
    out.feat[id] = (float)f0[k];
    out.feat[R + id] = (float)f1[k];
    out.feat[2 * R + id] = (float)f2[k];
    out.depth[id] = (float)dep[k];
    out.alpha[id] = (float)(1.0 - T[k]);
    if (out.t_final) out.t_final[id] = T[k];
    if (out.n_proc) out.n_proc[id] = nproc[k];
    if constexpr (STATS) {
      if (out.n_visit) out.n_visit[id] = nvisit[k];
      if (out.n_pass) out.n_pass[id] = npass[k];
    }
    if (s.kind == UT_LIDAR && out.drop) out.drop[id] = (float)(1.0 / (1.0 + exp(-(f2[k] - f1[k]))));
  }
}

// Consecutive workgroup ids land on different XCDs (round-robin over 8); give each XCD a
// contiguous run of tiles so neighbouring tiles share records in that XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int n_tiles) {
  const int per = (n_tiles + 7) / 8;
  const int t = (b & 7) * per + (b >> 3);
  return t < n_tiles ? t : -1;
}

// Register budget: one ray per lane keeps the ray, its six quadratic monomials and the
// accumulators in 128 VGPRs (4 waves per SIMD) with no spill in the pair loop; two rays per
// lane take 3 waves.
template <int BLOCK, int RPL, int BATCH, bool STATS, bool MOVING>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(RPL == 1 ? 4 : 3))) void k_composite(SensorK s, const RecordG* __restrict__ rec,
                                                      const uint2* __restrict__ trect,
                                                      const uint32_t* __restrict__ bgauss,
                                                      const uint32_t* __restrict__ branges, int n_tiles,
                                                      RenderParamsK prm, ut_render_out out) {
  __shared__ CompositeShared<BLOCK, RPL, BATCH> sm;
  const int tile = super_major_tile(blockIdx.x, s);
  if (tile < 0) return;
  composite_tile<BLOCK, RPL, BATCH, STATS, MOVING>(s, rec, trect, bgauss, branges, tile, s.super_x * s.super_y, prm, out, sm);
}

// LiDAR compositing over units of adjacent azimuth tiles (one ray per lane, unit_rays lanes).
template <int BLOCK, bool STATS, bool MOVING>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(BLOCK == 128 || MOVING ? 3 : 4))) void k_composite_unit(
    SensorK s, const RecordG* __restrict__ rec, const uint2* __restrict__ trect, const uint32_t* __restrict__ bgauss,
    const uint32_t* __restrict__ branges, RenderParamsK prm, ut_render_out out) {
  constexpr int kBatchU = BLOCK == 64 ? 32 : 128;   // 64 lanes: small LDS for 4 waves per SIMD
  __shared__ CompositeShared<BLOCK, 1, kBatchU> sm;
  __shared__ UnitShared<BLOCK, kBatchU> us;
  const int unit = xcd_tile(blockIdx.x, s.n_units);
  if (unit < 0) return;
  composite_tile<BLOCK, 1, kBatchU, STATS, MOVING, true, true>(s, rec, trect, bgauss, branges, unit,
                                                               s.super_x * s.super_y, prm, out, sm, &us);
}

// Persistent batched compositing: workgroups pull (request, tile) items from a counter.  Static
// and moving sensors run in separate launches (MOVING), so each keeps the register budget of
// its single-request kernel; LiDAR requests run their 256-lane units in launches of their own
// (UNIT).
template <bool MOVING, bool UNIT>
__global__ __launch_bounds__(kCamBlock) __attribute__((amdgpu_waves_per_eu(3))) void k_composite_batch(
    const BatchItemK* __restrict__ items, int n_items, int total_tiles, uint32_t* counter, RenderParamsK prm) {
  __shared__ CompositeShared<kCamBlock, kCamRpl, kCamBatch> sm;
  __shared__ UnitShared<kCamBlock, kCamBatch> us_mem;
  UnitShared<kCamBlock, kCamBatch>* us = UNIT ? &us_mem : nullptr;
  __shared__ uint32_t s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1u);
    __syncthreads();
    // uniform by construction; saying so lets the item's sensor description live in SGPRs
    const uint32_t w = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (w >= (uint32_t)total_tiles) break;
    int it = 0;
    while (it + 1 < n_items && (uint32_t)items[it + 1].tile_base <= w) ++it;
    const BatchItemK& I = items[it];
    composite_tile<kCamBlock, kCamRpl, kCamBatch, false, MOVING, false, UNIT>(
        I.s, I.rec, I.trect, I.gauss, I.ranges, (int)(w - I.tile_base), I.s.super_x * I.s.super_y, prm, I.out, sm, us);
  }
}

// The same items with one workgroup per (request, tile) item and no loop: the grid is the
// batch's item count and the hardware dispatcher is the queue.  Without the persistent loop the
// kernel keeps the single-request kernel's register budget (4 waves per SIMD, no spill; 3 for
// LiDAR units, whose two-entry walk needs a few more registers), where the looping kernel needs
// 168 VGPRs (3 waves).
template <bool MOVING, bool UNIT>
__global__ __launch_bounds__(kCamBlock) __attribute__((amdgpu_waves_per_eu(UNIT ? 3 : 4))) void k_composite_batch_direct(
    const BatchItemK* __restrict__ items, int n_items, RenderParamsK prm) {
  __shared__ CompositeShared<kCamBlock, kCamRpl, kCamBatch> sm;
  __shared__ UnitShared<kCamBlock, kCamBatch> us_mem;
  UnitShared<kCamBlock, kCamBatch>* us = UNIT ? &us_mem : nullptr;
  const uint32_t w = blockIdx.x;
  int it = 0;
  while (it + 1 < n_items && (uint32_t)items[it + 1].tile_base <= w) ++it;
  const BatchItemK& I = items[it];
  composite_tile<kCamBlock, kCamRpl, kCamBatch, false, MOVING, false, UNIT>(
      I.s, I.rec, I.trect, I.gauss, I.ranges, (int)(w - I.tile_base), I.s.super_x * I.s.super_y, prm, I.out, sm, us);
}

}  // namespace

hipError_t launch_composite(const ut_projected& p, const ut_bin_lists& bins, const SensorK& s,
                            const RenderParamsK& prm, const ut_render_out& out, int max_tile_rays,
                            hipStream_t st) {
  const int n_tiles = s.tiles_x * s.tiles_y;
  if (n_tiles == 0) return hipSuccess;
  const int grid = super_tile_slots(s.super_x, s.super_y, s.super_h);
  const RecordG* rec = reinterpret_cast<const RecordG*>(p.records);
  const uint2* tr = reinterpret_cast<const uint2*>(p.trect);
  const bool stats = out.n_visit != nullptr || out.n_pass != nullptr;
  const bool mv = s.moving != 0;
#define UT_LAUNCH_COMPOSITE_V(B, R, N, ST, MV)                                                                \
  hipLaunchKernelGGL((k_composite<B, R, N, ST, MV>), dim3(grid), dim3(B), 0, st, s, rec, tr, bins.gauss,      \
                     bins.ranges, n_tiles, prm, out)
#define UT_LAUNCH_COMPOSITE(B, R, N)                        \
  do {                                                      \
    if (stats) {                                            \
      if (mv) UT_LAUNCH_COMPOSITE_V(B, R, N, true, true);   \
      else UT_LAUNCH_COMPOSITE_V(B, R, N, true, false);     \
    } else {                                                \
      if (mv) UT_LAUNCH_COMPOSITE_V(B, R, N, false, true);  \
      else UT_LAUNCH_COMPOSITE_V(B, R, N, false, false);    \
    }                                                       \
  } while (0)
  if (s.kind == UT_LIDAR && s.n_units > 0 && s.unit_rays >= max_tile_rays) {
    // LiDAR units: several azimuth tiles per workgroup, one ray per lane
    const int ugrid = 8 * ((s.n_units + 7) / 8);
#define UT_LAUNCH_UNIT(B)                                                                                     \
  do {                                                                                                        \
    if (stats) {                                                                                              \
      if (mv) hipLaunchKernelGGL((k_composite_unit<B, true, true>), dim3(ugrid), dim3(B), 0, st, s, rec, tr,  \
                                 bins.gauss, bins.ranges, prm, out);                                          \
      else hipLaunchKernelGGL((k_composite_unit<B, true, false>), dim3(ugrid), dim3(B), 0, st, s, rec, tr,    \
                              bins.gauss, bins.ranges, prm, out);                                             \
    } else {                                                                                                  \
      if (mv) hipLaunchKernelGGL((k_composite_unit<B, false, true>), dim3(ugrid), dim3(B), 0, st, s, rec, tr, \
                                 bins.gauss, bins.ranges, prm, out);                                          \
      else hipLaunchKernelGGL((k_composite_unit<B, false, false>), dim3(ugrid), dim3(B), 0, st, s, rec, tr,   \
                              bins.gauss, bins.ranges, prm, out);                                             \
    }                                                                                                         \
  } while (0)
    if (s.unit_rays == 64) UT_LAUNCH_UNIT(64);
    else if (s.unit_rays == 128) UT_LAUNCH_UNIT(128);
    else UT_LAUNCH_UNIT(256);
#undef UT_LAUNCH_UNIT
  } else if (s.kind == UT_LIDAR && max_tile_rays > 256)
    UT_LAUNCH_COMPOSITE(256, 2, 256);   // LiDAR tiles of up to 512 rays: two rays per lane
  else if (s.kind != UT_LIDAR || max_tile_rays > 128)
    UT_LAUNCH_COMPOSITE(kCamBlock, kCamRpl, kCamBatch);
  else if (max_tile_rays > 64)
    UT_LAUNCH_COMPOSITE(128, 1, 128);
  else
    UT_LAUNCH_COMPOSITE(64, 1, 64);
#undef UT_LAUNCH_COMPOSITE
#undef UT_LAUNCH_COMPOSITE_V
  return hipGetLastError();
}

hipError_t launch_composite_batch(const BatchItemK* items_dev, const BatchGroups& grp, uint32_t* counter,
                                  const RenderParamsK& prm, int n_workgroups, hipStream_t st) {
  if (n_workgroups <= 0) {
    // one workgroup per (request, tile) item: the hardware dispatcher hands them out in order
#define UT_LAUNCH_DIRECT(G, MV, UN)                                                                             \
  if (grp.tiles[G] > 0)                                                                                         \
  hipLaunchKernelGGL((k_composite_batch_direct<MV, UN>), dim3(grp.tiles[G]), dim3(kCamBlock), 0, st,             \
                     items_dev + grp.first[G], grp.count[G], prm)
    UT_LAUNCH_DIRECT(0, false, false);
    UT_LAUNCH_DIRECT(1, true, false);
    UT_LAUNCH_DIRECT(2, false, true);
    UT_LAUNCH_DIRECT(3, true, true);
#undef UT_LAUNCH_DIRECT
    return hipGetLastError();
  }
  hipError_t e = fill_u32(counter, 0u, 4, st);
  if (e != hipSuccess) return e;
#define UT_LAUNCH_BATCH(G, MV, UN)                                                                              \
  if (grp.tiles[G] > 0)                                                                                         \
  hipLaunchKernelGGL((k_composite_batch<MV, UN>), dim3(n_workgroups), dim3(kCamBlock), 0, st, items_dev + grp.first[G], \
                     grp.count[G], grp.tiles[G], counter + (G), prm)
  UT_LAUNCH_BATCH(0, false, false);
  UT_LAUNCH_BATCH(1, true, false);
  UT_LAUNCH_BATCH(2, false, true);
  UT_LAUNCH_BATCH(3, true, true);
#undef UT_LAUNCH_BATCH
  return hipGetLastError();
}

}  // namespace ut
