// composite.hip -- per-ray front-to-back compositing (Eq. 1) over tile lists.
//
// One workgroup per tile, one lane per ray.  The tile's sorted list is streamed through
// LDS in batches of BLOCK records (96 B each, gathered cooperatively as 16-byte chunks so
// neighbouring lanes read neighbouring bytes); every lane then walks the batch for its
// own ray.  A lane that reaches T < t_min stops (its wavefront stops when all 64 lanes
// have), and the workgroup stops streaming once every lane is done.
//
// Per (ray, particle): v = mu - o, Bd = B d, t* = v.Bd / d.Bd, u = v - t* d,
// D^2 = u.B u, rho = exp(-D^2/2) -- all float64 with explicit FMAs (no contraction
// flags can change the arithmetic between the plain and the batched kernel).
#include "ut_internal.hpp"

namespace ut {
namespace {

template <int BLOCK>
__device__ __forceinline__ void composite_tile(const SensorK& s, const Record* __restrict__ rec,
                                               const uint32_t* __restrict__ gauss,
                                               const uint32_t* __restrict__ ranges, int tile, int n_tiles,
                                               const RenderParamsK& prm, const ut_render_out& out,
                                               Record* sh) {
  const uint32_t start = ranges[tile], end = ranges[n_tiles + tile];
  const long long ray = tile_ray(s, tile, threadIdx.x);
  const double ox = s.o[0], oy = s.o[1], oz = s.o[2];
  double dx = 0, dy = 0, dz = 0;
  if (ray >= 0) {
    dx = s.ray_dir[ray];
    dy = s.ray_dir[s.n_rays + ray];
    dz = s.ray_dir[2 * s.n_rays + ray];
  }
  bool done = !(ray >= 0 && (dx != 0 || dy != 0 || dz != 0));
  double T = 1.0, f0 = 0, f1 = 0, f2 = 0, dep = 0;
  uint32_t nproc = 0;
  const double cut_bias = 1e-3 - 2.0 * prm.log_alpha_min;

  for (uint32_t base = start; base < end; base += BLOCK) {
    if (__syncthreads_and(done)) break;
    const uint32_t cnt = min((uint32_t)BLOCK, end - base);
    for (uint32_t c = threadIdx.x; c < cnt * kRecordChunks; c += BLOCK) {
      const uint32_t j = c / kRecordChunks, part = c - j * kRecordChunks;
      const uint32_t g = gauss[base + j];
      reinterpret_cast<uint4*>(sh + j)[part] = reinterpret_cast<const uint4*>(rec + g)[part];
    }
    __syncthreads();
    if (!done) {
      for (uint32_t j = 0; j < cnt; ++j) {
        const Record& r = sh[j];
        nproc = base - start + j + 1;
        const double vx = r.mu[0] - ox, vy = r.mu[1] - oy, vz = r.mu[2] - oz;
        const double b0 = r.b[0], b1 = r.b[1], b2 = r.b[2], b3 = r.b[3], b4 = r.b[4], b5 = r.b[5];
        const double bdx = __builtin_fma(b0, dx, __builtin_fma(b3, dy, b4 * dz));
        const double bdy = __builtin_fma(b3, dx, __builtin_fma(b1, dy, b5 * dz));
        const double bdz = __builtin_fma(b4, dx, __builtin_fma(b5, dy, b2 * dz));
        const double dBd = __builtin_fma(dx, bdx, __builtin_fma(dy, bdy, dz * bdz));
        const double vBd = __builtin_fma(vx, bdx, __builtin_fma(vy, bdy, vz * bdz));
        const double tau = vBd * rcp_f64(dBd);
        const double ux = __builtin_fma(-tau, dx, vx), uy = __builtin_fma(-tau, dy, vy), uz = __builtin_fma(-tau, dz, vz);
        const double bux = __builtin_fma(b0, ux, __builtin_fma(b3, uy, b4 * uz));
        const double buy = __builtin_fma(b3, ux, __builtin_fma(b1, uy, b5 * uz));
        const double buz = __builtin_fma(b4, ux, __builtin_fma(b5, uy, b2 * uz));
        const double D2 = __builtin_fma(ux, bux, __builtin_fma(uy, buy, uz * buz));
        if (tau < s.near_) continue;
        // conservative pre-test: beyond this D^2, sigma rho < alpha_min for certain
        if (D2 > __builtin_fma(2.0, (double)r.log_sigma, cut_bias)) continue;
        const double rho = exp_f64(-0.5 * D2);
        const double a = r.sigma * rho;
        const double alpha = a > prm.alpha_max ? prm.alpha_max : a;
        if (alpha < prm.alpha_min) continue;
        const double w = alpha * T;
        f0 = __builtin_fma(w, (double)r.feat[0], f0);
        f1 = __builtin_fma(w, (double)r.feat[1], f1);
        f2 = __builtin_fma(w, (double)r.feat[2], f2);
        dep = __builtin_fma(w, tau, dep);
        T = T * (1.0 - alpha);
        if (T < prm.t_min) {
          done = true;
          break;
        }
      }
    }
  }
  if (ray >= 0) {
    const long long R = s.n_rays;
    out.feat[ray] = (float)f0;
    out.feat[R + ray] = (float)f1;
    out.feat[2 * R + ray] = (float)f2;
    out.depth[ray] = (float)dep;
    out.alpha[ray] = (float)(1.0 - T);
    if (out.t_final) out.t_final[ray] = T;
    if (out.n_proc) out.n_proc[ray] = nproc;
    if (s.kind == UT_LIDAR && out.drop) out.drop[ray] = (float)(1.0 / (1.0 + exp(-(f2 - f1))));
  }
}

// Consecutive workgroup ids land on different XCDs (round-robin over 8); give each XCD a
// contiguous run of tiles so neighbouring tiles share records in that XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int n_tiles) {
  const int per = (n_tiles + 7) / 8;
  const int t = (b & 7) * per + (b >> 3);
  return t < n_tiles ? t : -1;
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_composite(SensorK s, const Record* __restrict__ rec,
                                                      const uint32_t* __restrict__ gauss,
                                                      const uint32_t* __restrict__ ranges, int n_tiles,
                                                      RenderParamsK prm, ut_render_out out) {
  __shared__ Record sh[BLOCK];
  const int tile = xcd_tile(blockIdx.x, n_tiles);
  if (tile < 0) return;
  composite_tile<BLOCK>(s, rec, gauss, ranges, tile, n_tiles, prm, out, sh);
}

// Persistent batched compositing: workgroups pull (request, tile) items from a counter.
__global__ __launch_bounds__(256) void k_composite_batch(const BatchItemK* __restrict__ items, int n_items,
                                                          int total_tiles, uint32_t* counter,
                                                          RenderParamsK prm) {
  __shared__ Record sh[256];
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
    composite_tile<256>(I.s, I.rec, I.gauss, I.ranges, (int)(w - I.tile_base), I.n_tiles, prm, I.out, sh);
  }
}

}  // namespace

hipError_t launch_composite(const ut_projected& p, const ut_tile_lists& lists, const SensorK& s,
                            const RenderParamsK& prm, const ut_render_out& out, int max_tile_rays,
                            hipStream_t st) {
  const int n_tiles = s.tiles_x * s.tiles_y;
  if (n_tiles == 0) return hipSuccess;
  const int grid = 8 * ((n_tiles + 7) / 8);
  const Record* rec = reinterpret_cast<const Record*>(p.records);
  if (s.kind != UT_LIDAR || max_tile_rays > 128)
    hipLaunchKernelGGL(k_composite<256>, dim3(grid), dim3(256), 0, st, s, rec, lists.gauss, lists.ranges, n_tiles, prm, out);
  else if (max_tile_rays > 64)
    hipLaunchKernelGGL(k_composite<128>, dim3(grid), dim3(128), 0, st, s, rec, lists.gauss, lists.ranges, n_tiles, prm, out);
  else
    hipLaunchKernelGGL(k_composite<64>, dim3(grid), dim3(64), 0, st, s, rec, lists.gauss, lists.ranges, n_tiles, prm, out);
  return hipGetLastError();
}

hipError_t launch_composite_batch(const BatchItemK* items_dev, int n_items, int total_tiles,
                                  uint32_t* counter, const RenderParamsK& prm, int n_workgroups,
                                  hipStream_t st) {
  hipError_t e = fill_u32(counter, 0u, 1, st);
  if (e != hipSuccess || total_tiles == 0) return e;
  hipLaunchKernelGGL(k_composite_batch, dim3(n_workgroups), dim3(256), 0, st, items_dev, n_items, total_tiles,
                     counter, prm);
  return hipGetLastError();
}

}  // namespace ut
