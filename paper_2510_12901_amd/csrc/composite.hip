// composite.hip -- per-ray front-to-back compositing (Eq. 1) over tile lists.
//
// One workgroup per tile, one lane per ray.  The workgroup streams its super-tile bin,
// keeps the entries whose rect contains the tile (ballot + popcount per wavefront, wave
// counts combined in LDS, appended in order to an LDS ring of candidate indices), and
// stages batches of BLOCK candidates' records (96 B each, gathered cooperatively as
// 16-byte chunks) in LDS; every lane then walks the batch for its own ray.  The candidate
// order is the tile's exact (depth, index) list.  A lane that reaches T < t_min stops (its
// wavefront stops when all 64 lanes have), and the workgroup stops once every lane is done.
//
// Per (ray, particle): w = M d, t* = a.w / w.w, r = a - t* w, D^2 = r.r (see Record),
// rho = exp(-D^2/2) -- all float64 with explicit FMAs (no contraction flags can change
// the arithmetic between the plain and the batched kernel, or between forward and adjoint).
#include "ut_internal.hpp"

namespace ut {
namespace {

// Camera tiles (16 x 16 rays) and the batched kernel (any tile of up to 256 rays) run BLOCK
// threads with RPL rays per lane and stage BATCH records per step.
constexpr int kCamBlock = 256, kCamRpl = 1, kCamBatch = 128;
static_assert(kCamBlock * kCamRpl >= UT_MAX_LIDAR_TILE_RAYS, "batched tiles must fit one workgroup");

// BLOCK threads, RPL rays per lane: one workgroup covers up to BLOCK * RPL rays.  Records are
// staged BATCH at a time; the ring of candidate indices holds a batch plus one refill step of
// BLOCK entries.  Keeping LDS per workgroup small lets the register count, not LDS, set the
// occupancy.
template <int BLOCK, int RPL, int BATCH>
struct CompositeShared {
  static_assert(BATCH >= 64 && (BATCH & (BATCH - 1)) == 0, "batch must be a power of two");
  static constexpr int kBatch = BATCH;
  static constexpr uint32_t kRing = BATCH + BLOCK <= 2 * BATCH ? 2 * BATCH : 4 * BATCH;
  static_assert(BATCH + BLOCK <= (int)kRing, "ring must hold a batch plus one refill step");
  Record rec[BATCH];
  uint32_t cand[kRing];   // ring of candidate particle indices
  uint32_t wcnt[BLOCK / 64];
};

template <int BLOCK, int RPL, int BATCH>
__device__ __forceinline__ void composite_tile(const SensorK& s, const Record* __restrict__ rec,
                                               const uint2* __restrict__ trect,
                                               const uint32_t* __restrict__ bgauss,
                                               const uint32_t* __restrict__ branges, int tile, int n_super,
                                               const RenderParamsK& prm, const ut_render_out& out,
                                               CompositeShared<BLOCK, RPL, BATCH>& sm) {
  constexpr int kBatch = BATCH;
  constexpr uint32_t kRing = CompositeShared<BLOCK, RPL, BATCH>::kRing - 1;
  const int tx = tile % s.tiles_x, ty = tile / s.tiles_x;
  const int sid = super_of_tile(tile, s);
  const uint32_t start = branges[sid], end = branges[n_super + sid];
  long long ray[RPL];
  double dx[RPL], dy[RPL], dz[RPL], T[RPL], f0[RPL], f1[RPL], f2[RPL], dep[RPL];
  uint32_t nproc[RPL];
  bool rdone[RPL];
  bool done = true;
#pragma unroll
  for (int k = 0; k < RPL; ++k) {
    ray[k] = tile_ray(s, tile, threadIdx.x + k * BLOCK);
    dx[k] = dy[k] = dz[k] = 0;
    if (ray[k] >= 0) {
      dx[k] = s.ray_dir[ray[k]];
      dy[k] = s.ray_dir[s.n_rays + ray[k]];
      dz[k] = s.ray_dir[2 * s.n_rays + ray[k]];
    }
    rdone[k] = !(ray[k] >= 0 && (dx[k] != 0 || dy[k] != 0 || dz[k] != 0));
    done = done && rdone[k];
    T[k] = 1.0;
    f0[k] = f1[k] = f2[k] = dep[k] = 0;
    nproc[k] = 0;
  }
  const int lane = __lane_id(), wave = threadIdx.x >> 6;
  const unsigned long long lt = (1ull << lane) - 1ull;
  uint32_t pos = start, head = 0, n_cand = 0, list_base = 0;   // uniform across the workgroup

  for (;;) {
    if (__syncthreads_and(done)) break;
    // refill the candidate ring with this tile's entries of the super-tile bin
    while (n_cand < (uint32_t)kBatch && pos < end) {
      const uint32_t j = pos + threadIdx.x;
      uint32_t g = 0;
      bool hit = false;
      if (j < end) {
        g = bgauss[j];
        hit = rect_covers(trect[g], tx, ty, s);
      }
      const unsigned long long m = __ballot(hit);
      if (lane == 0) sm.wcnt[wave] = (uint32_t)__popcll(m);
      __syncthreads();
      uint32_t before = 0, total = 0;
#pragma unroll
      for (int w = 0; w < BLOCK / 64; ++w) {
        const uint32_t c = sm.wcnt[w];
        if (w < wave) before += c;
        total += c;
      }
      if (hit) sm.cand[(head + n_cand + before + (uint32_t)__popcll(m & lt)) & kRing] = g;
      n_cand += total;
      pos += BLOCK;
      __syncthreads();
    }
    if (n_cand == 0) break;
    const uint32_t cnt = min(n_cand, (uint32_t)kBatch);
    for (uint32_t c = threadIdx.x; c < cnt * kRecordChunks; c += BLOCK) {
      const uint32_t j = c / kRecordChunks, part = c - j * kRecordChunks;
      const uint32_t g = sm.cand[(head + j) & kRing];
      uint4 v = reinterpret_cast<const uint4*>(rec + g)[part];
      if (part == kRecordChunks - 1) {   // bytes 112..127: feat[2], log_sigma, aux
        const double cut = cut_threshold(__uint_as_float(v.y), prm.log_alpha_min);
        v.z = (uint32_t)__double2loint(cut);
        v.w = (uint32_t)__double2hiint(cut);
      }
      reinterpret_cast<uint4*>(sm.rec + j)[part] = v;
    }
    __syncthreads();
    if (!done) {
      for (uint32_t j = 0; j < cnt; ++j) {
        const Record& r = sm.rec[j];
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
          if (rdone[k]) continue;
          const PairGeom q = pair_geometry(r, dx[k], dy[k], dz[k]);
          if (pair_cut(q, r.aux)) continue;
          const PairResp pr = pair_response(r, q);
          const double tau = pr.tau;
          if (tau < s.near_) continue;
          const double rho = exp_f64(-0.5 * pr.D2);
          const double a = r.sigma * rho;
          const double alpha = a > prm.alpha_max ? prm.alpha_max : a;
          if (alpha < prm.alpha_min) continue;
          const double w = alpha * T[k];
          f0[k] = __builtin_fma(w, (double)r.feat[0], f0[k]);
          f1[k] = __builtin_fma(w, (double)r.feat[1], f1[k]);
          f2[k] = __builtin_fma(w, (double)r.feat[2], f2[k]);
          dep[k] = __builtin_fma(w, tau, dep[k]);
          T[k] = T[k] * (1.0 - alpha);
          if (T[k] < prm.t_min) {
            rdone[k] = true;
            nproc[k] = list_base + j + 1;   // entries up to and including the terminating one
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
    list_base += cnt;
  }
  // a ray still open here has visited the whole list of its tile
#pragma unroll
  for (int k = 0; k < RPL; ++k)
    if (!rdone[k]) nproc[k] = list_base;
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

template <int BLOCK, int RPL, int BATCH>
__global__ __launch_bounds__(BLOCK) void k_composite(SensorK s, const Record* __restrict__ rec,
                                                      const uint2* __restrict__ trect,
                                                      const uint32_t* __restrict__ bgauss,
                                                      const uint32_t* __restrict__ branges, int n_tiles,
                                                      RenderParamsK prm, ut_render_out out) {
  __shared__ CompositeShared<BLOCK, RPL, BATCH> sm;
  const int tile = xcd_tile(blockIdx.x, n_tiles);
  if (tile < 0) return;
  composite_tile<BLOCK, RPL, BATCH>(s, rec, trect, bgauss, branges, tile, s.super_x * s.super_y, prm, out, sm);
}

// Persistent batched compositing: workgroups pull (request, tile) items from a counter.
__global__ __launch_bounds__(kCamBlock) void k_composite_batch(const BatchItemK* __restrict__ items, int n_items,
                                                          int total_tiles, uint32_t* counter,
                                                          RenderParamsK prm) {
  __shared__ CompositeShared<kCamBlock, kCamRpl, kCamBatch> sm;
  __shared__ uint32_t s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1u);
    __syncthreads();
    const uint32_t w = s_item;
    __syncthreads();
    if (w >= (uint32_t)total_tiles) break;
    int it = 0;
    while (it + 1 < n_items && (uint32_t)items[it + 1].tile_base <= w) ++it;
    const BatchItemK& I = items[it];
    composite_tile<kCamBlock, kCamRpl, kCamBatch>(I.s, I.rec, I.trect, I.gauss, I.ranges, (int)(w - I.tile_base),
                        I.s.super_x * I.s.super_y, prm, I.out, sm);
  }
}

}  // namespace

hipError_t launch_composite(const ut_projected& p, const ut_bin_lists& bins, const SensorK& s,
                            const RenderParamsK& prm, const ut_render_out& out, int max_tile_rays,
                            hipStream_t st) {
  const int n_tiles = s.tiles_x * s.tiles_y;
  if (n_tiles == 0) return hipSuccess;
  const int grid = 8 * ((n_tiles + 7) / 8);
  const Record* rec = reinterpret_cast<const Record*>(p.records);
  const uint2* tr = reinterpret_cast<const uint2*>(p.trect);
  if (s.kind != UT_LIDAR || max_tile_rays > 128)
    hipLaunchKernelGGL((k_composite<kCamBlock, kCamRpl, kCamBatch>), dim3(grid), dim3(kCamBlock), 0, st, s, rec, tr, bins.gauss, bins.ranges, n_tiles, prm, out);
  else if (max_tile_rays > 64)
    hipLaunchKernelGGL((k_composite<128, 1, 128>), dim3(grid), dim3(128), 0, st, s, rec, tr, bins.gauss, bins.ranges, n_tiles, prm, out);
  else
    hipLaunchKernelGGL((k_composite<64, 1, 64>), dim3(grid), dim3(64), 0, st, s, rec, tr, bins.gauss, bins.ranges, n_tiles, prm, out);
  return hipGetLastError();
}

hipError_t launch_composite_batch(const BatchItemK* items_dev, int n_items, int total_tiles,
                                  uint32_t* counter, const RenderParamsK& prm, int n_workgroups,
                                  hipStream_t st) {
  hipError_t e = fill_u32(counter, 0u, 1, st);
  if (e != hipSuccess || total_tiles == 0) return e;
  hipLaunchKernelGGL(k_composite_batch, dim3(n_workgroups), dim3(kCamBlock), 0, st, items_dev, n_items, total_tiles,
                     counter, prm);
  return hipGetLastError();
}

}  // namespace ut
