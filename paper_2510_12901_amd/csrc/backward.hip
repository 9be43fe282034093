// backward.hip -- adjoint of the compositing with the forward's discrete structure fixed.
//
// k_backward: one workgroup per tile (same ray mapping as the forward).  The tile's list
// is replayed from the largest n_proc of the workgroup down to 0, in LDS batches.  Each
// lane recomputes its pair exactly as the forward did (same expressions), recovers
// T_i = T_{i+1} / (1 - alpha_i) from the stored final transmittance, and keeps the suffix
// sum S = sum_{j>i} w_j a_j.  Per pair it forms 13 partials (colour 3, ln opacity, mean 3,
// the 6 unique entries of B = Sigma^{-1}); wavefronts whose lanes touched the particle
// reduce all 13 across 64 lanes in one reduce-scatter (17 exchanges) and 13 lanes add them
// into the step's LDS sums (float64 LDS atomics), which reach the SoA accumulators acc[13][n]
// with one float64 atomic per (entry, partial) when the step ends.
// k_chain: one lane per particle, chain rule to (mean, quat, log_scale, logit, SH).
#include "ut_cone.hpp"
#include "ut_internal.hpp"
#include "ut_sh.hpp"

namespace ut {
namespace {

// Lane exchanges of float64 values without LDS: each 32-bit half moves through a DPP lane
// pattern (within rows of 16 lanes) or a gfx950 permlane swap (across rows and halves).
__device__ __forceinline__ uint32_t lo32(double x) { return (uint32_t)__double_as_longlong(x); }
__device__ __forceinline__ uint32_t hi32(double x) { return (uint32_t)((unsigned long long)__double_as_longlong(x) >> 32); }
__device__ __forceinline__ double from32(uint32_t lo, uint32_t hi) {
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
// the value of lane dpp(l) for the pattern CTRL (every lane reads a lane of its own row)
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  return from32((uint32_t)__builtin_amdgcn_update_dpp(0, (int)lo32(x), CTRL, 0xF, 0xF, false),
                (uint32_t)__builtin_amdgcn_update_dpp(0, (int)hi32(x), CTRL, 0xF, 0xF, false));
}
// a (lanes 32..63) <-> b (lanes 0..31): afterwards a + b holds, in lanes 0..31, a summed over
// lanes l and l + 32, and in lanes 32..63 b summed over lanes l - 32 and l
__device__ __forceinline__ double swap32_sum(double a, double b) {
  const auto l = __builtin_amdgcn_permlane32_swap(lo32(a), lo32(b), false, false);
  const auto h = __builtin_amdgcn_permlane32_swap(hi32(a), hi32(b), false, false);
  return from32(l[0], h[0]) + from32(l[1], h[1]);
}
// the same across rows of 16 lanes: a summed over rows 2r and 2r+1 in even rows, b in odd rows
__device__ __forceinline__ double swap16_sum(double a, double b) {
  const auto l = __builtin_amdgcn_permlane16_swap(lo32(a), lo32(b), false, false);
  const auto h = __builtin_amdgcn_permlane16_swap(hi32(a), hi32(b), false, false);
  return from32(l[0], h[0]) + from32(l[1], h[1]);
}
constexpr int kDppRowRor8 = 0x128, kDppRowHalfMirror = 0x141, kDppQuad2301 = 0x4E, kDppQuad1032 = 0xB1;

// Sums 16 per-lane values over the 64 lanes of a wavefront: at each step a lane keeps half of
// its partial sums and trades the other half with a lane that differs in one more bit (32 and
// 16: permlane swaps; 8: rotate within the row; 4: mirror within 8 lanes, then the quad sum).
// Afterwards lane l holds the total of value idx = 8 b5 + 4 b4 + 2 b3 + b2 (b_k = bit k of l),
// the same on the 4 lanes of its quad.  Every lane of the wavefront must be active.
__device__ __forceinline__ double wave_reduce_scatter16(const double v[16], int lane, int& idx) {
  const bool b3 = lane & 8, b2 = lane & 4;
  double w[8], x[4], y[2];
#pragma unroll
  for (int k = 0; k < 8; ++k) w[k] = swap32_sum(v[k], v[k + 8]);        // lanes 32..63 keep k + 8
#pragma unroll
  for (int k = 0; k < 4; ++k) x[k] = swap16_sum(w[k], w[k + 4]);        // odd rows keep k + 4
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double send = b3 ? x[k] : x[k + 2], keep = b3 ? x[k + 2] : x[k];
    y[k] = keep + dpp_f64<kDppRowRor8>(send);                           // partner l ^ 8
  }
  double z = (b2 ? y[1] : y[0]) + dpp_f64<kDppRowHalfMirror>(b2 ? y[0] : y[1]);   // partner 7 - l (mod 8)
  z += dpp_f64<kDppQuad2301>(z);
  z += dpp_f64<kDppQuad1032>(z);
  idx = ((lane & 32) ? 8 : 0) + ((lane & 16) ? 4 : 0) + (b3 ? 2 : 0) + (b2 ? 1 : 0);
  return z;
}

template <int BLOCK, bool MOVING>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(MOVING ? 3 : 4))) void k_backward(SensorK s, const RecordG* __restrict__ rec,
                                                     const uint2* __restrict__ trect,
                                                     const uint32_t* __restrict__ bgauss,
                                                     const uint32_t* __restrict__ branges, int n_super,
                                                     RenderParamsK prm, ut_render_out fwd, ut_upstream up,
                                                     double* __restrict__ acc, int n) {
  // a step stages up to kStep list entries; their 13 partials are summed over the workgroup's
  // wavefronts in LDS and leave with one float64 atomic per (entry, partial)
  constexpr int kStep = BLOCK >= 256 ? 128 : BLOCK / 2;
  __shared__ Record sh[kStep];
  __shared__ uint32_t sh_g[kStep];   // kept entries of one step: particle ...
  __shared__ uint32_t sh_j[kStep];   // ... and its position in the tile's list
  __shared__ double sacc[UT_ACC_FLOATS][kStep];
  __shared__ uint2 s_wc[BLOCK / 64];
  __shared__ uint32_t s_max;
  __shared__ double red[4][BLOCK / 64];
  __shared__ TileCone cone;
  const int tile = blockIdx.x;
  const int tx = tile % s.tiles_x, ty = tile / s.tiles_x;
  const int sid = super_of_tile(tile, s);
  const uint32_t bstart = branges[sid], bend = branges[n_super + sid];
  const long long ray = tile_ray(s, tile, threadIdx.x);
  const long long R = s.n_rays;
  double ox = s.o[0], oy = s.o[1], oz = s.o[2];   // this ray's origin (moving sensors: its own)
  double ex = 0, ey = 0, ez = 0;                  // ... minus the sensor origin
  double dx = 0, dy = 0, dz = 0;
  uint32_t np = 0;
  double T = 1.0, gf0 = 0, gf1 = 0, gf2 = 0, gdep = 0, gom = 0;
  if (ray >= 0) {
    dx = s.ray_dir[ray];
    dy = s.ray_dir[R + ray];
    dz = s.ray_dir[2 * R + ray];
    if (dx != 0 || dy != 0 || dz != 0) np = fwd.n_proc[ray];
    T = fwd.t_final[ray];
    if (up.feat) { gf0 = up.feat[ray]; gf1 = up.feat[R + ray]; gf2 = up.feat[2 * R + ray]; }
    if (up.depth) gdep = up.depth[ray];
    if (up.alpha) gom = up.alpha[ray];
    if (up.drop && s.kind == UT_LIDAR) {
      // drop = sigmoid(zeta_2 - zeta_1): d drop / d zeta_2 = p (1 - p) = -d drop / d zeta_1
      const double z1 = fwd.feat[R + ray], z2 = fwd.feat[2 * R + ray];
      const double p = 1.0 / (1.0 + exp(-(z2 - z1)));
      const double gd = (double)up.drop[ray] * p * (1.0 - p);
      gf1 -= gd;
      gf2 += gd;
    }
  }
  const double Tf = T;
  const double gomTf = gom * Tf;   // the alpha output's upstream term, the same for every pair of the ray
  const RayQ rq = ray_q(dx, dy, dz);
  double S = 0.0;
  const int lane = __lane_id(), wave = threadIdx.x >> 6;
  // the forward's tile cone, rebuilt from the same rays: entries it drops are skipped here too
  const bool has_ray = ray >= 0 && (dx != 0 || dy != 0 || dz != 0);
  constexpr bool mv = MOVING;
  if (mv && has_ray) {
    ox = s.ray_org[ray];
    oy = s.ray_org[R + ray];
    oz = s.ray_org[2 * R + ray];
    ex = ox - s.o[0], ey = oy - s.o[1], ez = oz - s.o[2];
  }
  double emax = 0.0, etx = 0.0, ety = 0.0, etz = 0.0;
  double ux, uy, uz, sn;
  {
    const double il = has_ray ? rcp_f64(__builtin_sqrt(__builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz)))) : 0.0;
    tile_cone_axis<BLOCK>(dx * il, dy * il, dz * il, red, wave, lane, ux, uy, uz, sn);
  }
  if constexpr (mv) {
    // the tile's reference origin (mean ray origin) and the spread around it, as the forward
    const double cnt = block_reduce<BLOCK>(has_ray ? 1.0 : 0.0, false, red[3], wave, lane);
    const double cx = block_reduce<BLOCK>(ex, false, red[0], wave, lane);
    const double cy = block_reduce<BLOCK>(ey, false, red[1], wave, lane);
    const double cz = block_reduce<BLOCK>(ez, false, red[2], wave, lane);
    if (cnt > 0) etx = cx / cnt, ety = cy / cnt, etz = cz / cnt;
    const double fx = ex - etx, fy = ey - ety, fz = ez - etz;
    emax = has_ray ? __builtin_sqrt(__builtin_fma(fx, fx, __builtin_fma(fy, fy, fz * fz))) : 0.0;
    emax = -block_reduce<BLOCK>(-emax, true, red[0], wave, lane);
  }
  tile_cone_finish<BLOCK>(has_ray ? cone_cos(ux, uy, uz, dx, dy, dz) : 1.0, sn, ux, uy, uz, red, wave, lane, cone,
                          emax, etx, ety, etz);
  const bool cull = cone.on != 0;
  if (threadIdx.x == 0) s_max = 0;
  __syncthreads();
  atomicMax(&s_max, np);
  __syncthreads();
  const uint32_t jmax = s_max;
  const unsigned long long lt = (1ull << lane) - 1ull;

  // Walk the super-tile bin backwards from the forward's end for this tile.  Entries whose rect
  // covers the tile form the tile's list; the first jmax of them lie in [bstart, tile_end), so
  // a step's covering entries take the positions just below those of the later steps.  Entries
  // the tile cone rules out are dropped before their records are staged.
  // exclusive bin index; clamped to the bin so that a stale state cannot read past it
  uint32_t cur = jmax > 0 ? min(max(fwd.tile_end[tile], bstart), bend) : bstart;
  uint32_t top = jmax;                                     // list positions below this remain
  while (cur > bstart && top > 0) {
    const uint32_t lo = cur - bstart > (uint32_t)kStep ? cur - kStep : bstart;
    const uint32_t b = lo + threadIdx.x;
    uint32_t g = 0;
    bool hit = false;
    if ((int)threadIdx.x < kStep && b < cur) {
      g = bgauss[b];
      hit = rect_covers(trect[g], tx, ty, s);
    }
    const bool keep = hit && !(cull && cone_rejects<MOVING>(rec + g, cone, prm.log_alpha_min));
    const unsigned long long mh = __ballot(hit), mk = __ballot(keep);
    __syncthreads();   // the previous step's records are no longer read
    if (lane == 0) s_wc[wave] = make_uint2((uint32_t)__popcll(mh), (uint32_t)__popcll(mk));
    __syncthreads();
    uint32_t hb = 0, kb = 0, ht = 0, kt = 0;
#pragma unroll
    for (int w = 0; w < BLOCK / 64; ++w) {
      const uint2 c = s_wc[w];
      if (w < wave) hb += c.x, kb += c.y;
      ht += c.x, kt += c.y;
    }
    if (keep) {
      const uint32_t slot = kb + (uint32_t)__popcll(mk & lt);
      sh_g[slot] = g;
      sh_j[slot] = top - ht + hb + (uint32_t)__popcll(mh & lt);   // position in the tile's list
    }
    __syncthreads();
    const int cnt = (int)kt;
    for (int c = threadIdx.x; c < cnt * kRecordChunks; c += BLOCK) {
      const int j = c / kRecordChunks, part = c - j * kRecordChunks;
      stage_record_chunk(rec + sh_g[j], sh + j, part);
    }
    for (int c = threadIdx.x; c < cnt * UT_ACC_FLOATS; c += BLOCK) sacc[c / cnt][c % cnt] = 0.0;
    __syncthreads();
    top -= ht;
    cur = lo;
    for (int jj = cnt - 1; jj >= 0; --jj) {
      const int j = (int)sh_j[jj];
      if (__ballot(j < (int)np) == 0ull) continue;   // no lane of this wave visited entry j
      const Record& r = sh[jj];
      bool contrib = false;
      double g[UT_ACC_FLOATS];
#pragma unroll
      for (int k = 0; k < UT_ACC_FLOATS; ++k) g[k] = 0.0;
      if (j < (int)np) {
        Centre cv;   // the centre seen from this ray's origin
        if constexpr (mv) cv = pair_centre(r, ex, ey, ez);
        else cv = record_centre(r);
        PairResp pr;
        const bool pass = pair_eval(r, cv, rq, ex, ey, ez, cut_threshold(r.log_sigma, prm.log_alpha_min), pr);
        const double tau = pr.tau;
        if (pass && tau >= s.near_) {
          const double a = pair_alpha(r, pr, kExp2Frac);
          const bool clamped = a > prm.alpha_max;
          const double alpha = clamped ? prm.alpha_max : a;
          if (alpha >= prm.alpha_min) {
            contrib = true;
            const double ioma = rcp_f64(1.0 - alpha);
            const double Ti = T * ioma;
            const double w = alpha * Ti;
            const double ai = __builtin_fma(gf0, r.feat[0], __builtin_fma(gf1, r.feat[1],
                                            __builtin_fma(gf2, r.feat[2], gdep * tau)));
            const double dalpha = __builtin_fma(Ti, ai, (gomTf - S) * ioma);
            S = __builtin_fma(w, ai, S);
            T = Ti;
            g[0] = gf0 * w;
            g[1] = gf1 * w;
            g[2] = gf2 * w;
            const double dtau = gdep * w;
            double dD2 = 0.0;
            if (!clamped) {
              g[3] = dalpha * a;   // dL/d ln sigma: alpha = sigma rho, so d alpha / d ln sigma = alpha
              dD2 = -0.5 * g[3];
            }
            // B d from the record's quadric and B u = B v - t* B d, u = mu - o - t* d (for thin
            // records B u from u itself: the difference cancels like the forward's num)
            double bd[3];
            sym_apply(r.b, dx, dy, dz, bd);
            const double bdx = bd[0], bdy = bd[1], bdz = bd[2];
            // u = mu - o_ray - t* d; the record's v = mu - o (sensor origin) is exact in float64
            // (a difference of two float32 values), and so is v - e = mu - o_ray
            const double ux = (r.v[0] - ex) - tau * dx;
            const double uy = (r.v[1] - ey) - tau * dy;
            const double uz = (r.v[2] - ez) - tau * dz;
            double bux, buy, buz;
            if (record_thin(r)) {
              double bu[3];
              sym_apply(r.b, ux, uy, uz, bu);
              bux = bu[0]; buy = bu[1]; buz = bu[2];
            } else {
              bux = __builtin_fma(-tau, bdx, cv.bv[0]);
              buy = __builtin_fma(-tau, bdy, cv.bv[1]);
              buz = __builtin_fma(-tau, bdz, cv.bv[2]);
            }
            // dL/dmu = 2 dD2 B u + (dtau / d^T B d) B d; dL/dB_kl from u u^T and the tau term
            // (d u^T + u d^T) / 2, factored so each partial is one or two FMAs
            const double t2 = 2.0 * dD2, ti = dtau * pr.idbd;
            const double tdx = ti * dx, tdy = ti * dy, tdz = ti * dz;
            g[4] = __builtin_fma(t2, bux, ti * bdx);
            g[5] = __builtin_fma(t2, buy, ti * bdy);
            g[6] = __builtin_fma(t2, buz, ti * bdz);
            g[7] = ux * __builtin_fma(dD2, ux, tdx);
            g[8] = uy * __builtin_fma(dD2, uy, tdy);
            g[9] = uz * __builtin_fma(dD2, uz, tdz);
            g[10] = __builtin_fma(ux, __builtin_fma(t2, uy, tdy), uy * tdx);
            g[11] = __builtin_fma(ux, __builtin_fma(t2, uz, tdz), uz * tdx);
            g[12] = __builtin_fma(uy, __builtin_fma(t2, uz, tdz), uz * tdy);
          }
        }
      }
      if (__ballot(contrib)) {
        // one reduction for all 13 partials, then one LDS atomic instruction: lane 4k adds sum k
        double v16[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) v16[k] = k < UT_ACC_FLOATS ? g[k] : 0.0;
        int idx;
        const double tot = wave_reduce_scatter16(v16, lane, idx);
        if ((lane & 3) == 0 && idx < UT_ACC_FLOATS && tot != 0.0) atomicAdd(&sacc[idx][jj], tot);
      }
    }
    __syncthreads();
    // the step's sums to the particles' accumulators
    for (int c = threadIdx.x; c < cnt * UT_ACC_FLOATS; c += BLOCK) {
      const int k = c / cnt, jj = c - k * cnt;
      const double v = sacc[k][jj];
      if (v != 0.0) unsafeAtomicAdd(acc + (size_t)k * n + sh_g[jj], v);
    }
  }
}

// DEG is the SH degree as a compile-time constant, so the per-coefficient arrays below are
// indexed statically and stay in registers.  A particle that no pair touched has zero
// accumulators and therefore zero gradients; it only writes the zeros.
template <int DEG>
__global__ __launch_bounds__(256) void k_chain(ut_gaussians g, SensorK s, const double* __restrict__ acc,
                                                ut_gaussian_grads out) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  const int n = g.n;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a[UT_ACC_FLOATS];
  bool touched = false;
#pragma unroll
  for (int k = 0; k < UT_ACC_FLOATS; ++k) {
    a[k] = acc[(size_t)k * n + i];
    touched = touched || a[k] != 0.0;
  }
  if (!touched) {
    for (int c = 0; c < 3; ++c) out.mean[(size_t)c * n + i] = 0.0f;
    for (int c = 0; c < 4; ++c) out.quat[(size_t)c * n + i] = 0.0f;
    for (int c = 0; c < 3; ++c) out.log_scale[(size_t)c * n + i] = 0.0f;
    out.opacity_logit[i] = 0.0f;
#pragma unroll
    for (int k = 0; k < 3 * K; ++k) out.feat[(size_t)k * n + i] = 0.0f;
    return;
  }
  const float q0 = g.quat[i], q1 = g.quat[n + i], q2 = g.quat[2 * n + i], q3 = g.quat[3 * n + i];
  const float l0 = g.log_scale[i], l1 = g.log_scale[n + i], l2 = g.log_scale[2 * n + i];
  const float lg = g.opacity_logit[i];
  const double mx = g.mean[i], my = g.mean[n + i], mz = g.mean[2 * n + i];
  const double qq = (double)q0 * q0 + (double)q1 * q1 + (double)q2 * q2 + (double)q3 * q3;
  const bool ok = isfinite(mx) && isfinite(my) && isfinite(mz) && isfinite(l0) && isfinite(l1) &&
                  isfinite(l2) && isfinite(lg) && isfinite(qq) && qq > 0;
  double dmean[3] = {0, 0, 0}, dq[4] = {0, 0, 0, 0}, dls[3] = {0, 0, 0}, dlogit = 0;
  double dcoef[K][3];
#pragma unroll
  for (int k = 0; k < K; ++k) dcoef[k][0] = dcoef[k][1] = dcoef[k][2] = 0;
  if (ok) {
    const double qn = sqrt(qq), iq = 1.0 / qn;
    const double w = q0 * iq, x = q1 * iq, y = q2 * iq, z = q3 * iq;
    const double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                         2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                         2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
    const double sc[3] = {exp((double)l0), exp((double)l1), exp((double)l2)};
    const double sigma = 1.0 / (1.0 + exp(-(double)lg));
    dlogit = a[3] * (1.0 - sigma);   // a[3] = dL/d ln sigma; d ln sigma / d logit = 1 - sigma
    // unique-entry gradient of B -> full symmetric G
    const double G[9] = {a[7], 0.5 * a[10], 0.5 * a[11], 0.5 * a[10], a[8], 0.5 * a[12], 0.5 * a[11], 0.5 * a[12], a[9]};
    const double vx = mx - s.o[0], vy = my - s.o[1], vz = mz - s.o[2];
    double dR[9];
    if (s.div_tan > 0) {
      // LiDAR beam divergence: B = Sigma_hat^{-1}, Sigma_hat = R S^2 R^T + t^2 (|v|^2 I - v v^T)
      // (t = tan(theta/2), v = mu - o), so dL/dSigma_hat = -B G B =: GS reaches R and S as for
      // a plain covariance, dL/dR = 2 GS R S^2, dL/dlog s_j = 2 s_j^2 (R^T GS R)_jj, and the
      // mean through the smoothing term, t^2 (2 tr(GS) v - 2 GS v).
      const double vv[3] = {vx, vy, vz};
      const double t2 = s.div_tan * s.div_tan, r2 = vx * vx + vy * vy + vz * vz;
      double A[9];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
          double sig = 0;
          for (int j = 0; j < 3; ++j) sig += R[r * 3 + j] * sc[j] * sc[j] * R[c * 3 + j];
          A[r * 3 + c] = sig + t2 * ((r == c ? r2 : 0.0) - vv[r] * vv[c]);
        }
      // B by the adjugate (A is symmetric positive definite: the forward factored it)
      const double c00 = A[4] * A[8] - A[5] * A[7], c01 = A[5] * A[6] - A[3] * A[8], c02 = A[3] * A[7] - A[4] * A[6];
      const double idet = 1.0 / (A[0] * c00 + A[1] * c01 + A[2] * c02);
      const double B[9] = {c00 * idet, (A[2] * A[7] - A[1] * A[8]) * idet, (A[1] * A[5] - A[2] * A[4]) * idet,
                           c01 * idet, (A[0] * A[8] - A[2] * A[6]) * idet, (A[2] * A[3] - A[0] * A[5]) * idet,
                           c02 * idet, (A[1] * A[6] - A[0] * A[7]) * idet, (A[0] * A[4] - A[1] * A[3]) * idet};
      double GB[9], GS[9];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) GB[r * 3 + c] = G[r * 3] * B[c] + G[r * 3 + 1] * B[3 + c] + G[r * 3 + 2] * B[6 + c];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) GS[r * 3 + c] = -(B[r * 3] * GB[c] + B[r * 3 + 1] * GB[3 + c] + B[r * 3 + 2] * GB[6 + c]);
      double SR[9];
      for (int r = 0; r < 3; ++r)
        for (int j = 0; j < 3; ++j) SR[r * 3 + j] = GS[r * 3] * R[j] + GS[r * 3 + 1] * R[3 + j] + GS[r * 3 + 2] * R[6 + j];
      for (int r = 0; r < 3; ++r)
        for (int j = 0; j < 3; ++j) dR[r * 3 + j] = 2.0 * SR[r * 3 + j] * sc[j] * sc[j];
      for (int j = 0; j < 3; ++j) dls[j] = 2.0 * sc[j] * sc[j] * (R[j] * SR[j] + R[3 + j] * SR[3 + j] + R[6 + j] * SR[6 + j]);
      const double tr = GS[0] + GS[4] + GS[8];
      for (int r = 0; r < 3; ++r)
        dmean[r] = 2.0 * t2 * (tr * vv[r] - (GS[r * 3] * vx + GS[r * 3 + 1] * vy + GS[r * 3 + 2] * vz));
    } else {
      // B = R D R^T, D = diag(1/s^2): dL/dR = 2 G R D, dL/dD_jj = (R^T G R)_jj
      double GR[9];
      for (int r = 0; r < 3; ++r)
        for (int j = 0; j < 3; ++j) {
          const double gr = G[r * 3] * R[j] + G[r * 3 + 1] * R[3 + j] + G[r * 3 + 2] * R[6 + j];
          GR[r * 3 + j] = gr;
        }
      for (int r = 0; r < 3; ++r)
        for (int j = 0; j < 3; ++j) dR[r * 3 + j] = 2.0 * GR[r * 3 + j] / (sc[j] * sc[j]);
      for (int j = 0; j < 3; ++j) {
        const double rtgr = R[j] * GR[j] + R[3 + j] * GR[3 + j] + R[6 + j] * GR[6 + j];
        dls[j] = -2.0 * rtgr / (sc[j] * sc[j]);
      }
    }
    // R(q_hat) -> q_hat
    const double dw = 2 * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
    const double dxq = 2 * (y * dR[1] + z * dR[2] + y * dR[3] - 2 * x * dR[4] - w * dR[5] + z * dR[6] + w * dR[7] - 2 * x * dR[8]);
    const double dyq = 2 * (-2 * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] + z * dR[7] - 2 * y * dR[8]);
    const double dzq = 2 * (-2 * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2 * z * dR[4] + y * dR[5] + x * dR[6] + y * dR[7]);
    const double dot = dw * w + dxq * x + dyq * y + dzq * z;
    dq[0] = (dw - w * dot) * iq;
    dq[1] = (dxq - x * dot) * iq;
    dq[2] = (dyq - y * dot) * iq;
    dq[3] = (dzq - z * dot) * iq;
    // features: SH coefficients and the direction's dependence on the mean
    const double len = sqrt(vx * vx + vy * vy + vz * vz);
    double ex = 0, ey = 0, ez = 1;
    if (len > 0) { ex = vx / len; ey = vy / len; ez = vz / len; }
    double Y[16], GY[16][3];
    sh_basis(DEG, ex, ey, ez, Y);
    sh_basis_grad(DEG, ex, ey, ez, GY);
    double ddir[3] = {0, 0, 0};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double dc = a[c];
      if (g.feat_kind == UT_FEAT_CAMERA) {
        double f = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) f += (double)g.feat[(size_t)(k * 3 + c) * n + i] * Y[k];
        if (!(f + 0.5 > 0)) dc = 0;
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        dcoef[k][c] = dc * Y[k];
        const double coef = g.feat[(size_t)(k * 3 + c) * n + i];
        ddir[0] += dc * coef * GY[k][0];
        ddir[1] += dc * coef * GY[k][1];
        ddir[2] += dc * coef * GY[k][2];
      }
    }
    dmean[0] += a[4]; dmean[1] += a[5]; dmean[2] += a[6];
    if (len > 0) {
      const double dd = ddir[0] * ex + ddir[1] * ey + ddir[2] * ez;
      dmean[0] += (ddir[0] - ex * dd) / len;
      dmean[1] += (ddir[1] - ey * dd) / len;
      dmean[2] += (ddir[2] - ez * dd) / len;
    }
  }
  for (int c = 0; c < 3; ++c) out.mean[(size_t)c * n + i] = (float)dmean[c];
  for (int c = 0; c < 4; ++c) out.quat[(size_t)c * n + i] = (float)dq[c];
  for (int c = 0; c < 3; ++c) out.log_scale[(size_t)c * n + i] = (float)dls[c];
  out.opacity_logit[i] = (float)dlogit;
#pragma unroll
  for (int k = 0; k < K; ++k)
    for (int c = 0; c < 3; ++c) out.feat[(size_t)(k * 3 + c) * n + i] = (float)dcoef[k][c];
}

}  // namespace

hipError_t launch_backward(const ut_gaussians& g, const ut_projected& p, const ut_bin_lists& bins,
                           const SensorK& s, const RenderParamsK& prm, const ut_render_out& fwd,
                           const ut_upstream& up, double* acc, const ut_gaussian_grads& grads,
                           int max_tile_rays, hipStream_t st) {
  hipError_t e = fill_f64(acc, 0.0, (size_t)UT_ACC_FLOATS * g.n, st);
  if (e != hipSuccess || g.n == 0) return e;
  const int n_tiles = s.tiles_x * s.tiles_y;
  const RecordG* rec = reinterpret_cast<const RecordG*>(p.records);
  const uint2* tr = reinterpret_cast<const uint2*>(p.trect);
  const int n_super = s.super_x * s.super_y;
  const int grid = n_tiles;
  if (n_tiles > 0) {
#define UT_LAUNCH_BACKWARD(B)                                                                              \
  do {                                                                                                     \
    if (s.moving)                                                                                          \
      hipLaunchKernelGGL((k_backward<B, true>), dim3(grid), dim3(B), 0, st, s, rec, tr, bins.gauss,     \
                         bins.ranges, n_super, prm, fwd, up, acc, g.n);                             \
    else                                                                                                   \
      hipLaunchKernelGGL((k_backward<B, false>), dim3(grid), dim3(B), 0, st, s, rec, tr, bins.gauss,    \
                         bins.ranges, n_super, prm, fwd, up, acc, g.n);                             \
  } while (0)
    if (s.kind != UT_LIDAR || max_tile_rays > 128)
      UT_LAUNCH_BACKWARD(256);
    else if (max_tile_rays > 64)
      UT_LAUNCH_BACKWARD(128);
    else
      UT_LAUNCH_BACKWARD(64);
#undef UT_LAUNCH_BACKWARD
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const dim3 cg((g.n + 255) / 256);
  switch (g.sh_degree) {
    case 0: hipLaunchKernelGGL(k_chain<0>, cg, dim3(256), 0, st, g, s, acc, grads); break;
    case 1: hipLaunchKernelGGL(k_chain<1>, cg, dim3(256), 0, st, g, s, acc, grads); break;
    case 2: hipLaunchKernelGGL(k_chain<2>, cg, dim3(256), 0, st, g, s, acc, grads); break;
    default: hipLaunchKernelGGL(k_chain<3>, cg, dim3(256), 0, st, g, s, acc, grads); break;
  }
  return hipGetLastError();
}

}  // namespace ut
