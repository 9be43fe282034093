// project.hip -- per-particle sigma-point projection (one lane per particle).
//
// Loads are structure-of-arrays and coalesced; the arithmetic is float64 (on gfx950 a
// float64 FMA costs the same issue slot as an unpacked float32 FMA).  Every particle reads
// 11 floats and writes 32 bytes (rects, key, count); a particle that reaches a tile also
// reads its 3K SH floats and writes its 128-byte record.
#include <algorithm>

#include "ut_internal.hpp"
#include "ut_sh.hpp"

namespace ut {
namespace {

// Sensor map of one point in sensor axes: (u, v) and validity (see utrast.h for each model).
template <int KIND>
__device__ __forceinline__ bool project_sensor(const SensorK& s, double x, double y, double z, double& u,
                                               double& v) {
  if constexpr (KIND == UT_PINHOLE) {
    if (!(z > s.near_)) return false;
    const double iz = 1.0 / z;
    u = s.fx * x * iz + s.cx;
    v = s.fy * y * iz + s.cy;
    return true;
  }
  if constexpr (KIND == UT_ORTHO) {
    if (!(z > s.near_)) return false;
    u = s.fx * x + s.cx;
    v = s.fy * y + s.cy;
    return true;
  }
  if constexpr (KIND != UT_FISHEYE && KIND != UT_LIDAR) return false;
  const double rho2 = x * x + y * y;
  const double r = sqrt(rho2 + z * z);
  if (!(r > s.near_)) return false;
  const double rho = sqrt(rho2);
  if constexpr (KIND == UT_FISHEYE) {
    const double theta = atan2(rho, z);
    if (!(theta <= s.theta_max)) return false;
    const double t2 = theta * theta;
    const double td = theta * (1.0 + t2 * (s.k[0] + t2 * (s.k[1] + t2 * (s.k[2] + t2 * s.k[3]))));
    if (rho > 0) {
      const double f = td / rho;
      u = s.cx + s.fx * f * x;
      v = s.cy + s.fy * f * y;
    } else {
      u = s.cx;
      v = s.cy;
    }
    return true;
  }
  // spinning LiDAR (Eq. 3): azimuth in [0, 2 pi), elevation
  double phi = atan2(y, x);
  if (phi < 0) phi += 2 * kPi;
  u = phi;
  v = atan2(z, rho);
  return true;
}

// Sensor map g(x) of one world point.  A moving sensor observes the point at the time of the
// row (camera, t = v / height) or azimuth (LiDAR, t = phi / 2 pi) it falls on: the point is
// projected with the pose at t = 1/2 and then rs_iters - 1 more times with the pose at the
// time of its previous projection (see utrast.h).
template <int KIND, bool MOVING>
__device__ __forceinline__ bool project_point(const SensorK& s, const double xw[3], double& u, double& v) {
  if constexpr (!MOVING) {
    const double dx = xw[0] - s.o[0], dy = xw[1] - s.o[1], dz = xw[2] - s.o[2];
    const double x = s.R[0] * dx + s.R[1] * dy + s.R[2] * dz;
    const double y = s.R[3] * dx + s.R[4] * dy + s.R[5] * dz;
    const double z = s.R[6] * dx + s.R[7] * dy + s.R[8] * dz;
    return project_sensor<KIND>(s, x, y, z, u, v);
  } else {
    double t = 0.5;
    for (int it = 0; it < s.rs_iters; ++it) {
      double q[4], o[3], rel[3], p[3];
      pose_at(s, t, q, o);
      rel[0] = xw[0] - o[0], rel[1] = xw[1] - o[1], rel[2] = xw[2] - o[2];
      quat_rotate(q, rel, p);
      if (!project_sensor<KIND>(s, p[0], p[1], p[2], u, v)) return false;
      if constexpr (KIND == UT_LIDAR) t = u * (0.5 / kPi);
      else t = fmin(fmax(v / s.height, 0.0), 1.0);
    }
    return true;
  }
}

// summed-area-table count over inclusive culling cells [x0,x1] x [y0,y1] (Alg. 2)
__device__ __forceinline__ long sat_count(const SensorK& s, int x0, int x1, int y0, int y1) {
  const long W = s.cull_el + 1;
  const int* S = s.sat;
  return (long)S[(x1 + 1) * W + (y1 + 1)] - S[(long)x0 * W + (y1 + 1)] - S[(x1 + 1) * W + y0] +
         S[(long)x0 * W + y0];
}

// float32 squared distance to the sensor origin, fixed operation order, no contraction
__device__ __forceinline__ uint32_t depth_key(float mx, float my, float mz, const float o[3]) {
#pragma clang fp contract(off)
  const float dx = __fsub_rn(mx, o[0]);
  const float dy = __fsub_rn(my, o[1]);
  const float dz = __fsub_rn(mz, o[2]);
  const float k = __fadd_rn(__fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy)), __fmul_rn(dz, dz));
  return __float_as_uint(k);
}

// Image-axis interval [lo, hi] that contains the pinhole projection f * a / z + c of every point
// of a ball of radius rho around camera-frame (a, z) seen in the (a, z) plane, z > rho: the
// tangents of the viewing angle plus / minus the ball's angular radius.  False when the ball
// reaches 90 degrees off axis (no finite bound).
__device__ __forceinline__ bool pinhole_ball_range(double a, double z, double rho, double f, double c, double& lo,
                                                   double& hi) {
  const double t = a / z;
  const double td = rho / sqrt(fmax(a * a + z * z - rho * rho, 0.0));
  const double dp = 1.0 - t * td, dm = 1.0 + t * td;
  if (!(dp > 0.0) || !(dm > 0.0) || !isfinite(td)) return false;
  lo = f * ((t - td) / dm) + c;
  hi = f * ((t + td) / dp) + c;
  return true;
}

// DEG is the SH degree as a compile-time constant, so the (DEG+1)^2 x 3 coefficient loads are
// unrolled and issued together instead of one dependent loop trip at a time.  KIND is the
// sensor model, so each instantiation carries only its own projection code (the LiDAR and
// fisheye arctangents would otherwise set the register count of every camera).
// LiDAR beam divergence (Sec. 3.2, LiDAR appendix): the particle is smoothed across the beam
// at its range r, Sigma_hat = Sigma + (r tan(theta/2))^2 (I - d d^T) with Sigma = L L^T on
// entry (L = S R^T's transpose, column-scaled rotation), and the opacity is not rescaled.  On
// return L holds the lower Cholesky factor of Sigma_hat, m = L^{-1} and a = m (mu - o), so the
// record's quadric is Sigma_hat^{-1} = m^T m and the compositing response is
// exp(-(x-mu)^T Sigma_hat^{-1} (x-mu) / 2).
// false if Sigma_hat is not numerically positive definite.
__device__ __forceinline__ bool beam_divergence_filter(const SensorK& s, float mx, float my, float mz,
                                                       double L[9], double m[9], double a[3]) {
  const double vx = (double)mx - s.o[0], vy = (double)my - s.o[1], vz = (double)mz - s.o[2];
  const double range = sqrt(vx * vx + vy * vy + vz * vz);
  if (!(range > 0)) return true;
  const double ir = 1.0 / range, d[3] = {vx * ir, vy * ir, vz * ir};
  const double w = range * s.div_tan, w2 = w * w;
  double A[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      A[i * 3 + j] = L[i * 3] * L[j * 3] + L[i * 3 + 1] * L[j * 3 + 1] + L[i * 3 + 2] * L[j * 3 + 2] +
                     w2 * ((i == j ? 1.0 : 0.0) - d[i] * d[j]);
  // Cholesky, column by column
  const double p00 = A[0];
  if (!(p00 > 0)) return false;
  const double l00 = sqrt(p00), l10 = A[3] / l00, l20 = A[6] / l00;
  const double p11 = A[4] - l10 * l10;
  if (!(p11 > 0)) return false;
  const double l11 = sqrt(p11), l21 = (A[7] - l20 * l10) / l11;
  const double p22 = A[8] - l20 * l20 - l21 * l21;
  if (!(p22 > 0)) return false;
  const double l22 = sqrt(p22);
  L[0] = l00; L[1] = 0;   L[2] = 0;
  L[3] = l10; L[4] = l11; L[5] = 0;
  L[6] = l20; L[7] = l21; L[8] = l22;
  // M = L^{-1}, lower triangular
  const double i00 = 1.0 / l00, i11 = 1.0 / l11, i22 = 1.0 / l22;
  const double i10 = -l10 * i00 * i11, i21 = -l21 * i11 * i22, i20 = -(l20 * i00 + l21 * i10) * i22;
  m[0] = i00; m[1] = 0;   m[2] = 0;
  m[3] = i10; m[4] = i11; m[5] = 0;
  m[6] = i20; m[7] = i21; m[8] = i22;
  a[0] = i00 * vx;
  a[1] = __builtin_fma(i10, vx, i11 * vy);
  a[2] = __builtin_fma(i20, vx, __builtin_fma(i21, vy, i22 * vz));
  return true;
}

template <int DEG, int KIND, bool MOVING, bool DIV = false>
__device__ __forceinline__ void project_all(const ut_gaussians& g, const SensorK& s, double ut_a, double ut_b,
                                            double ut_k, RecordG* __restrict__ rec,
                                            int32_t* __restrict__ rect, uint2* __restrict__ trect,
                                            uint32_t* __restrict__ key,
                                            uint32_t* __restrict__ count, float* __restrict__ moments,
                                            uint32_t* __restrict__ n_culled) {
  const int n = g.n;
  uint32_t n_invalid = 0, n_raycull = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    int invalid = 0, raycull = 0;
    const float mx = g.mean[i], my = g.mean[n + i], mz = g.mean[2 * n + i];
    // The UT's first sigma point is the mean: where its projection is invalid (behind a
    // pinhole, outside a fisheye's field of view) the particle is culled as invalid whatever its
    // other parameters, so those are neither loaded nor set up (about half of the particles
    // around a camera).  Outputs are exactly those of the full path.
    double gu0 = 0, gv0 = 0;
    const double mu[3] = {(double)mx, (double)my, (double)mz};
    const bool mean_ok =
        isfinite(mx) && isfinite(my) && isfinite(mz) && project_point<KIND, MOVING>(s, mu, gu0, gv0);
    float q0 = 1.0f, q1 = 0.0f, q2 = 0.0f, q3 = 0.0f, l0 = 0.0f, l1 = 0.0f, l2 = 0.0f, lg = 0.0f;
    if (mean_ok) {
      q0 = g.quat[i]; q1 = g.quat[n + i]; q2 = g.quat[2 * n + i]; q3 = g.quat[3 * n + i];
      l0 = g.log_scale[i]; l1 = g.log_scale[n + i]; l2 = g.log_scale[2 * n + i];
      lg = g.opacity_logit[i];
    }
    const double qq = (double)q0 * q0 + (double)q1 * q1 + (double)q2 * q2 + (double)q3 * q3;
    bool ok = mean_ok && isfinite(l0) && isfinite(l1) && isfinite(l2) && isfinite(lg) && isfinite(qq) && qq > 0;
    RecordG r;
    double M[9], A[3];   // M with M^T M = Sigma^{-1}, and A = M (mu - o)
    double Rm[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, sc[3] = {1, 1, 1};
    if (ok) {
      const double inv = 1.0 / sqrt(qq);
      const double w = q0 * inv, x = q1 * inv, y = q2 * inv, z = q3 * inv;
      Rm[0] = 1 - 2 * (y * y + z * z); Rm[1] = 2 * (x * y - w * z);     Rm[2] = 2 * (x * z + w * y);
      Rm[3] = 2 * (x * y + w * z);     Rm[4] = 1 - 2 * (x * x + z * z); Rm[5] = 2 * (y * z - w * x);
      Rm[6] = 2 * (x * z - w * y);     Rm[7] = 2 * (y * z + w * x);     Rm[8] = 1 - 2 * (x * x + y * y);
      sc[0] = exp((double)l0); sc[1] = exp((double)l1); sc[2] = exp((double)l2);
    }
    // M = S^{-1} R^T and a = M (mu - o); formed where the record is written (so they are not
    // live through the UT), except with beam divergence, whose filter replaces them here
    auto form_m = [&]() {
      const double i0 = 1.0 / sc[0], i1 = 1.0 / sc[1], i2 = 1.0 / sc[2];
      M[0] = Rm[0] * i0; M[1] = Rm[3] * i0; M[2] = Rm[6] * i0;
      M[3] = Rm[1] * i1; M[4] = Rm[4] * i1; M[5] = Rm[7] * i1;
      M[6] = Rm[2] * i2; M[7] = Rm[5] * i2; M[8] = Rm[8] * i2;
      const double vx = (double)mx - s.o[0], vy = (double)my - s.o[1], vz = (double)mz - s.o[2];
      A[0] = __builtin_fma(M[0], vx, __builtin_fma(M[1], vy, M[2] * vz));
      A[1] = __builtin_fma(M[3], vx, __builtin_fma(M[4], vy, M[5] * vz));
      A[2] = __builtin_fma(M[6], vx, __builtin_fma(M[7], vy, M[8] * vz));
    };
    if constexpr (DIV) form_m();
    r.log_sigma = ok ? -log1p(exp(-(double)lg)) : -1e30;   // ln sigmoid(logit)

    // columns of the covariance square root the sigma points step along: column j of R S, or
    // with LiDAR beam divergence the lower Cholesky factor of the smoothed covariance (kept
    // in registers only in that variant)
    double Lc[DIV ? 9 : 1];
    if constexpr (KIND == UT_LIDAR && DIV) {   // launched only for a LiDAR with beam divergence
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int j = 0; j < 3; ++j) Lc[d * 3 + j] = sc[j] * Rm[d * 3 + j];
      if (ok) ok = beam_divergence_filter(s, mx, my, mz, Lc, M, A);
    }
    auto col = [&](int d, int j) -> double {
      if constexpr (DIV) return Lc[d * 3 + j];
      else return sc[j] * Rm[d * 3 + j];
    };

    // Static pinhole, no moments requested: a particle whose sigma points all lie in front of
    // the camera and whose 3-sigma rect certainly misses the image needs no UT.  The sigma
    // points lie within rho = sqrt(3 + lambda) max(s) of the mean, so their projections fall in
    // the interval [lo, hi] of the ball; the UT mean lies in it too and each variance is at most
    // (|W_c0| + 6 W_i) (hi - lo)^2, which bounds the rect's half-extent.  Culling then matches
    // the full path exactly (count 0, empty rect) with a pixel of slack for rounding.
    bool off_image = false;
    if constexpr (KIND == UT_PINHOLE && !MOVING) {
      const double lam = ut_a * ut_a * (3.0 + ut_k) - 3.0;
      const double cpl = 3.0 + lam;
      // convex mean weights (lambda >= 0) and positive focal lengths keep the bound valid
      if (ok && moments == nullptr && lam >= 0.0 && s.fx > 0.0 && s.fy > 0.0) {
        const double rho = sqrt(cpl) * fmax(sc[0], fmax(sc[1], sc[2]));
        const double dx = (double)mx - s.o[0], dy = (double)my - s.o[1], dz = (double)mz - s.o[2];
        const double xc = s.R[0] * dx + s.R[1] * dy + s.R[2] * dz;
        const double yc = s.R[3] * dx + s.R[4] * dy + s.R[5] * dz;
        const double zc = s.R[6] * dx + s.R[7] * dy + s.R[8] * dz;
        double ulo, uhi, vlo, vhi;
        if (zc - rho > s.near_ && pinhole_ball_range(xc, zc, rho, s.fx, s.cx, ulo, uhi) &&
            pinhole_ball_range(yc, zc, rho, s.fy, s.cy, vlo, vhi)) {
          const double wsum = fabs(lam / cpl + 1.0 - ut_a * ut_a + ut_b) + 3.0 / cpl;
          const double k = 3.0 * sqrt(wsum);
          const double eu = k * (uhi - ulo) + 1.0, ev = k * (vhi - vlo) + 1.0;
          const double W = (double)s.tiles_x * UT_CAMERA_TILE, H = (double)s.tiles_y * UT_CAMERA_TILE;
          off_image = uhi + eu < 0.0 || ulo - eu >= W || vhi + ev < 0.0 || vlo - ev >= H;
        }
      }
    }

    // unscented transform over 7 sigma points
    double m0 = 0, m1 = 0, c00 = 0, c01 = 0, c11 = 0;
    if (ok && !off_image) {
      const double lam = ut_a * ut_a * (3.0 + ut_k) - 3.0;
      const double cpl = 3.0 + lam;
      ok = cpl > 0;
      if (ok) {
        const double gam = sqrt(cpl);
        double gu[7], gv[7];
        gu[0] = gu0;   // the mean, projected above
        gv[0] = gv0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          if (!ok) break;
          const double e0 = gam * col(0, j), e1 = gam * col(1, j), e2 = gam * col(2, j);
          const double pp[3] = {mu[0] + e0, mu[1] + e1, mu[2] + e2};
          const double pm[3] = {mu[0] - e0, mu[1] - e1, mu[2] - e2};
          ok = project_point<KIND, MOVING>(s, pp, gu[1 + j], gv[1 + j]) && project_point<KIND, MOVING>(s, pm, gu[4 + j], gv[4 + j]);
        }
        if (ok) {
          if constexpr (KIND == UT_LIDAR) {
#pragma unroll
            for (int k = 1; k < 7; ++k) {
              while (gu[k] - gu[0] > kPi) gu[k] -= 2 * kPi;
              while (gu[k] - gu[0] <= -kPi) gu[k] += 2 * kPi;
            }
          }
          const double wm0 = lam / cpl, wc0 = lam / cpl + 1.0 - ut_a * ut_a + ut_b, wi = 1.0 / (2.0 * cpl);
          m0 = wm0 * gu[0];
          m1 = wm0 * gv[0];
#pragma unroll
          for (int k = 1; k < 7; ++k) { m0 += wi * gu[k]; m1 += wi * gv[k]; }
#pragma unroll
          for (int k = 0; k < 7; ++k) {
            const double w = k == 0 ? wc0 : wi;
            const double du = gu[k] - m0, dv = gv[k] - m1;
            c00 += w * du * du;
            c01 += w * du * dv;
            c11 += w * dv * dv;
          }
          ok = isfinite(c00) && isfinite(c11) && c00 >= 0 && c11 >= 0;
        }
      }
    }
    invalid = !ok;

    int x0 = 0, y0 = 0, x1 = -1, y1 = -1;
    uint32_t cnt = 0;
    if (ok && !off_image) {
      const double eu = 3.0 * sqrt(c00), ev = 3.0 * sqrt(c11);
      if constexpr (KIND != UT_LIDAR) {
        const double T = UT_CAMERA_TILE;
        double fx0 = floor((m0 - eu) / T), fx1 = floor((m0 + eu) / T);
        double fy0 = floor((m1 - ev) / T), fy1 = floor((m1 + ev) / T);
        if (!(fx1 < 0 || fy1 < 0 || fx0 > s.tiles_x - 1 || fy0 > s.tiles_y - 1)) {
          x0 = (int)fmax(fx0, 0.0); y0 = (int)fmax(fy0, 0.0);
          x1 = (int)fmin(fx1, (double)(s.tiles_x - 1)); y1 = (int)fmin(fy1, (double)(s.tiles_y - 1));
          cnt = (uint32_t)((x1 - x0 + 1) * (y1 - y0 + 1));
        }
      } else {
        const double lo = m1 - ev, hi = m1 + ev;
        const int NP = s.n_phi;
        if (!(hi < s.bounds[0] || lo > s.bounds[NP])) {
          int e0 = 0, e1 = 0;
          for (int k = 1; k < NP; ++k) {
            const double tk = s.bounds[k];
            if (tk <= lo) e0 = k;
            if (tk <= hi) e1 = k;
          }
          const double two_pi = 2 * kPi;
          // an extent of at least 2 pi covers every azimuth tile (and keeps the casts in range)
          const bool full_az = eu >= kPi;
          long a0 = full_az ? 0 : (long)floor((m0 - eu) * s.n_theta / two_pi);
          long a1 = full_az ? s.n_theta - 1 : (long)floor((m0 + eu) * s.n_theta / two_pi);
          if (a1 - a0 + 1 >= s.n_theta) { a0 = 0; a1 = s.n_theta - 1; }
          else {
            const long w0 = ((a0 % s.n_theta) + s.n_theta) % s.n_theta;
            a1 = w0 + (a1 - a0);
            a0 = w0;
          }
          x0 = (int)a0; x1 = (int)a1; y0 = e0; y1 = e1;
          cnt = (uint32_t)((x1 - x0 + 1) * (y1 - y0 + 1));
          if (s.cull) {
            // Alg. 2 / Alg. 3: is any ray inside the extent on the denser culling grid?
            const double span = s.bounds[NP] - s.bounds[0];
            const long ca0 = full_az ? 0 : (long)floor((m0 - eu) * s.cull_az / two_pi);
            const long ca1 = full_az ? s.cull_az - 1 : (long)floor((m0 + eu) * s.cull_az / two_pi);
            const int ce0 = (int)fmax(floor((lo - s.bounds[0]) * s.cull_el / span), 0.0);
            const int ce1 = (int)fmin(floor((hi - s.bounds[0]) * s.cull_el / span), (double)(s.cull_el - 1));
            long occ = 0;
            if (ce0 <= ce1) {
              if (ca1 - ca0 + 1 >= s.cull_az) occ = sat_count(s, 0, s.cull_az - 1, ce0, ce1);
              else {
                const long w0 = ((ca0 % s.cull_az) + s.cull_az) % s.cull_az;
                const long w1 = w0 + (ca1 - ca0);
                if (w1 < s.cull_az) occ = sat_count(s, (int)w0, (int)w1, ce0, ce1);
                else occ = sat_count(s, (int)w0, s.cull_az - 1, ce0, ce1) +
                           sat_count(s, 0, (int)(w1 - s.cull_az), ce0, ce1);
              }
            }
            if (occ == 0) { cnt = 0; raycull = 1; }
          }
        }
      }
    }

    // Features and the record only for particles that reach a tile: nothing downstream reads
    // the record of a particle with count 0, and skipping it saves most of the SH loads and
    // record stores (most particles of a scene lie outside any one camera's view).
    if (cnt > 0) {
      // features: SH at the unit direction from the sensor origin to the mean
      double f[3] = {0, 0, 0};
      const double vx = (double)mx - s.o[0], vy = (double)my - s.o[1], vz = (double)mz - s.o[2];
      const double len = sqrt(vx * vx + vy * vy + vz * vz);
      double dx = 0, dy = 0, dz = 1;
      if (len > 0) { const double il = 1.0 / len; dx = vx * il; dy = vy * il; dz = vz * il; }
      double Y[16];
      sh_basis(DEG, dx, dy, dz, Y);
      constexpr int K = (DEG + 1) * (DEG + 1);
      for (int c = 0; c < 3; ++c) {
        double acc = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) acc += (double)g.feat[(size_t)(k * 3 + c) * n + i] * Y[k];
        f[c] = (g.feat_kind == UT_FEAT_CAMERA) ? (acc + 0.5 > 0 ? acc + 0.5 : 0.0) : acc;
      }
      r.feat[0] = (float)f[0]; r.feat[1] = (float)f[1]; r.feat[2] = (float)f[2];
      r.pad = 0.0f;
      if constexpr (!DIV) form_m();
      // the quadric form of the record: B = M^T M, B v = M^T A, v^T B v = A.A
      r.b[0] = __builtin_fma(M[0], M[0], __builtin_fma(M[3], M[3], M[6] * M[6]));
      r.b[1] = __builtin_fma(M[0], M[1], __builtin_fma(M[3], M[4], M[6] * M[7]));
      r.b[2] = __builtin_fma(M[0], M[2], __builtin_fma(M[3], M[5], M[6] * M[8]));
      r.b[3] = __builtin_fma(M[1], M[1], __builtin_fma(M[4], M[4], M[7] * M[7]));
      r.b[4] = __builtin_fma(M[1], M[2], __builtin_fma(M[4], M[5], M[7] * M[8]));
      r.b[5] = __builtin_fma(M[2], M[2], __builtin_fma(M[5], M[5], M[8] * M[8]));
      r.bv[0] = __builtin_fma(M[0], A[0], __builtin_fma(M[3], A[1], M[6] * A[2]));
      r.bv[1] = __builtin_fma(M[1], A[0], __builtin_fma(M[4], A[1], M[7] * A[2]));
      r.bv[2] = __builtin_fma(M[2], A[0], __builtin_fma(M[5], A[1], M[8] * A[2]));
      r.vbv = __builtin_fma(A[0], A[0], __builtin_fma(A[1], A[1], A[2] * A[2]));
      r.v[0] = vx; r.v[1] = vy; r.v[2] = vz;
      const uint4* src = reinterpret_cast<const uint4*>(&r);
      uint4* dst = reinterpret_cast<uint4*>(rec + i);
#pragma unroll
      for (int c = 0; c < kRecordChunks; ++c) dst[c] = src[c];
    }
    rect[i] = x0; rect[n + i] = y0; rect[2 * n + i] = x1; rect[3 * n + i] = y1;
    trect[i] = make_uint2(((uint32_t)x0 & 0xFFFFu) | ((uint32_t)y0 << 16), ((uint32_t)x1 & 0xFFFFu) | ((uint32_t)y1 << 16));
    count[i] = cnt;
    key[i] = depth_key(mx, my, mz, s.of);
    if (moments) {
      moments[i] = (float)m0; moments[n + i] = (float)m1;
      moments[2 * n + i] = (float)c00; moments[3 * n + i] = (float)c01; moments[4 * n + i] = (float)c11;
    }
    n_invalid += invalid;
    n_raycull += raycull;
  }
  // culled counts: wavefront sums, then one atomic per counter per workgroup (every
  // wavefront adding to the same two words serialises in L2 when half the particles are
  // behind the camera)
  __shared__ uint32_t s_cnt[2][4];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    n_invalid += (uint32_t)__shfl_xor(n_invalid, o);
    n_raycull += (uint32_t)__shfl_xor(n_raycull, o);
  }
  if (__lane_id() == 0) {
    s_cnt[0][threadIdx.x >> 6] = n_invalid;
    s_cnt[1][threadIdx.x >> 6] = n_raycull;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t a = s_cnt[0][0] + s_cnt[0][1] + s_cnt[0][2] + s_cnt[0][3];
    const uint32_t b = s_cnt[1][0] + s_cnt[1][1] + s_cnt[1][2] + s_cnt[1][3];
    if (a) atomicAdd(&n_culled[0], a);
    if (b) atomicAdd(&n_culled[1], b);
  }
}

// Occupancy is set per sensor model from measurement: the LiDAR kernel fits 168 VGPRs without
// spilling and runs best at three waves per SIMD; the camera kernels run best at two waves,
// where the compiler keeps all (DEG+1)^2 x 3 coefficient loads in flight (left to itself it
// trades them for a third wave, and the pinhole then takes over twice as long).
template <int DEG, int KIND, bool MOVING, bool DIV>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_project_capped(
    ut_gaussians g, SensorK s, double ut_a, double ut_b, double ut_k, RecordG* __restrict__ rec,
    int32_t* __restrict__ rect, uint2* __restrict__ trect, uint32_t* __restrict__ key,
    uint32_t* __restrict__ count, float* __restrict__ moments, uint32_t* __restrict__ n_culled) {
  project_all<DEG, KIND, MOVING, DIV>(g, s, ut_a, ut_b, ut_k, rec, rect, trect, key, count, moments, n_culled);
}

template <int DEG, int KIND, bool MOVING>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_project(
    ut_gaussians g, SensorK s, double ut_a, double ut_b, double ut_k, RecordG* __restrict__ rec,
    int32_t* __restrict__ rect, uint2* __restrict__ trect, uint32_t* __restrict__ key,
    uint32_t* __restrict__ count, float* __restrict__ moments, uint32_t* __restrict__ n_culled) {
  project_all<DEG, KIND, MOVING>(g, s, ut_a, ut_b, ut_k, rec, rect, trect, key, count, moments, n_culled);
}

}  // namespace

hipError_t launch_project(const ut_gaussians& g, const SensorK& s, const double abk[3],
                          const ut_projected& out, hipStream_t st) {
  hipError_t e = fill_u32(out.n_culled, 0u, 2, st);
  if (e != hipSuccess) return e;
  if (g.n == 0) return hipSuccess;
  const int blocks = std::min((g.n + 255) / 256, 2048);
  RecordG* rec = reinterpret_cast<RecordG*>(out.records);
  uint2* tr = reinterpret_cast<uint2*>(out.trect);
#define UT_LAUNCH_PROJECT(KERNEL, D, K, MV)                                                                \
  hipLaunchKernelGGL((KERNEL<D, K, MV>), dim3(blocks), dim3(256), 0, st, g, s, abk[0], abk[1], abk[2], rec, \
                     out.rect, tr, out.key, out.count, out.moments, out.n_culled)
#define UT_LAUNCH_LIDAR(D, MV)                                                                               \
  do {                                                                                                    \
    if (s.div_tan > 0)                                                                                    \
      hipLaunchKernelGGL((k_project_capped<D, UT_LIDAR, MV, true>), dim3(blocks), dim3(256), 0, st, g, s,  \
                         abk[0], abk[1], abk[2], rec, out.rect, tr, out.key, out.count, out.moments,      \
                         out.n_culled);                                                                   \
    else                                                                                                  \
      hipLaunchKernelGGL((k_project_capped<D, UT_LIDAR, MV, false>), dim3(blocks), dim3(256), 0, st, g, s, \
                         abk[0], abk[1], abk[2], rec, out.rect, tr, out.key, out.count, out.moments,      \
                         out.n_culled);                                                                   \
  } while (0)
#define UT_LAUNCH_PROJECT_MV(KERNEL, D, K)                      \
  do {                                                          \
    if (s.moving) UT_LAUNCH_PROJECT(KERNEL, D, K, true);        \
    else UT_LAUNCH_PROJECT(KERNEL, D, K, false);                \
  } while (0)
#define UT_LAUNCH_PROJECT_KIND(D)                                                    \
  switch (s.kind) {                                                                  \
    case UT_PINHOLE: UT_LAUNCH_PROJECT_MV(k_project, D, UT_PINHOLE); break;          \
    case UT_FISHEYE: UT_LAUNCH_PROJECT_MV(k_project, D, UT_FISHEYE); break;          \
    case UT_LIDAR:                                                                   \
      if (s.moving) UT_LAUNCH_LIDAR(D, true);                                        \
      else UT_LAUNCH_LIDAR(D, false);                                                \
      break;                                                                         \
    default: UT_LAUNCH_PROJECT(k_project, D, UT_ORTHO, false); break;                \
  }
  switch (g.sh_degree) {
    case 0: UT_LAUNCH_PROJECT_KIND(0); break;
    case 1: UT_LAUNCH_PROJECT_KIND(1); break;
    case 2: UT_LAUNCH_PROJECT_KIND(2); break;
    default: UT_LAUNCH_PROJECT_KIND(3); break;
  }
#undef UT_LAUNCH_PROJECT_KIND
#undef UT_LAUNCH_PROJECT_MV
#undef UT_LAUNCH_LIDAR
#undef UT_LAUNCH_PROJECT
  return hipGetLastError();
}

}  // namespace ut
