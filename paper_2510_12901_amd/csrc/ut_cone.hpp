// ut_cone.hpp -- conservative per-tile culling of list entries (device code shared by the
// compositing and its adjoint).
//
// A tile's rays are bounded by a cone (unit axis u, half-angle theta, built from block
// reductions over the tile's actual ray directions).  An entry whose response cannot reach
// alpha_min on any direction of the cone is dropped for the whole tile; every ray of the tile
// would skip it, so results do not change.
#pragma once
#include "ut_device.hpp"

namespace ut {

// Bounding cone of a tile's rays: unit axis u, orthonormal e1, e2 spanning u's complement,
// and cos / sin of twice the half-angle.  `on` is false when the tile has no ray or the cone
// is too wide for the bound below (half-angle > 45 degrees).
struct TileCone {
  double u[3], e1[3], e2[3];
  double cos2t, sin2t;
  // moving sensors: the tile's reference origin relative to the sensor origin, and the
  // largest distance of a ray origin of the tile from that reference
  double et[3], emax;
  int on;
};

template <int BLOCK>
__device__ __forceinline__ double block_reduce(double v, bool is_min, double (&red)[BLOCK / 64], int wave, int lane) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_xor(v, off);
    v = is_min ? (o < v ? o : v) : v + o;
  }
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double r = red[0];
#pragma unroll
  for (int w = 1; w < BLOCK / 64; ++w) r = is_min ? (red[w] < r ? red[w] : r) : r + red[w];
  __syncthreads();
  return r;
}

// cosine of the angle between the unit axis u and a (not necessarily unit) ray direction d
__device__ __forceinline__ double cone_cos(double ux, double uy, double uz, double dx, double dy, double dz) {
  const double l = __builtin_sqrt(__builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz)));
  return __builtin_fma(ux, dx, __builtin_fma(uy, dy, uz * dz)) / l;
}

// Axis of the tile's cone: every thread passes the sum of its rays' unit directions (zero when
// it has none) and receives the normalised block sum u and its length sn (0 = no ray).
template <int BLOCK>
__device__ __forceinline__ void tile_cone_axis(double sx, double sy, double sz, double (&red)[4][BLOCK / 64],
                                               int wave, int lane, double& ux, double& uy, double& uz,
                                               double& sn) {
  sx = block_reduce<BLOCK>(sx, false, red[0], wave, lane);
  sy = block_reduce<BLOCK>(sy, false, red[1], wave, lane);
  sz = block_reduce<BLOCK>(sz, false, red[2], wave, lane);
  sn = __builtin_sqrt(__builtin_fma(sx, sx, __builtin_fma(sy, sy, sz * sz)));
  ux = sx / sn, uy = sy / sn, uz = sz / sn;
}

// Half-angle from the block minimum of cone_cos over all rays (each thread passes its own
// minimum, 1 when it has no ray); thread 0 writes the cone, then the block synchronises.
template <int BLOCK>
__device__ __forceinline__ void tile_cone_finish(double cmin, double sn, double ux, double uy, double uz,
                                                 double (&red)[4][BLOCK / 64], int wave, int lane, TileCone& tc,
                                                 double emax = 0.0, double etx = 0.0, double ety = 0.0,
                                                 double etz = 0.0) {
  cmin = block_reduce<BLOCK>(cmin, true, red[3], wave, lane);
  if (threadIdx.x == 0) {
    tc.emax = emax;
    tc.et[0] = etx, tc.et[1] = ety, tc.et[2] = etz;
    const double ct = cmin - 1e-9;                       // widen for rounding
    tc.on = (sn > 0.0 && ct > 0.7071067811865476) ? 1 : 0;
    const double st = __builtin_sqrt(1.0 - ct * ct);
    tc.cos2t = 2.0 * ct * ct - 1.0;
    tc.sin2t = 2.0 * st * ct;
    tc.u[0] = ux, tc.u[1] = uy, tc.u[2] = uz;
    // e1 = normalise(u x t) with t the coordinate axis least aligned with u; e2 = u x e1
    double t0 = 0, t1 = 0, t2 = 0;
    if (__builtin_fabs(ux) <= __builtin_fabs(uy) && __builtin_fabs(ux) <= __builtin_fabs(uz)) t0 = 1;
    else if (__builtin_fabs(uy) <= __builtin_fabs(uz)) t1 = 1;
    else t2 = 1;
    double e0 = uy * t2 - uz * t1, e1 = uz * t0 - ux * t2, e2 = ux * t1 - uy * t0;
    const double en = __builtin_sqrt(e0 * e0 + e1 * e1 + e2 * e2);
    e0 /= en, e1 /= en, e2 /= en;
    tc.e1[0] = e0, tc.e1[1] = e1, tc.e1[2] = e2;
    tc.e2[0] = uy * e2 - uz * e1, tc.e2[1] = uz * e0 - ux * e2, tc.e2[2] = ux * e1 - uy * e0;
  }
  __syncthreads();
}

// Conservative tile-cone test: true when no unit direction d within the cone can bring the
// particle's response to alpha_min, i.e. h(d) = |a x Md|^2 - cut |Md|^2 > 0 on the whole cone
// (M^T M = Sigma^{-1}, a = M (mu - o); the record's quadric gives h without M).
// With d = cos(phi) u + sin(phi) e, e a unit vector in span(e1, e2) and phi <= theta,
//   h >= cos^2(phi) A - 2 sin(phi) cos(phi) B + sin^2(phi) C,
// where A = h(u), B bounds the mixed term over all e and C is the smallest eigenvalue of the
// form on span(e1, e2).  In psi = 2 phi this is P + Rc cos(psi) - B sin(psi), minimised over
// psi in [0, 2 theta] in closed form.  The threshold carries 0.05 of slack over the per-ray
// cut so that rounding cannot drop an entry that a ray would keep; the dropped entries are
// exactly ones every ray of the tile would skip, so outputs are unchanged.  For a moving
// sensor the rays start from different origins; the threshold grows by their spread.
template <bool MOVING>
__device__ __forceinline__ bool cone_rejects(const RecordG* __restrict__ rp, const TileCone& tc,
                                             double log_alpha_min) {
  double cut = cut_threshold(rp->log_sigma, log_alpha_min);
  double b[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) b[i] = rp->b[i];
  Centre c = record_centre(*rp);
  if constexpr (MOVING) {
    // seen from the tile's reference origin o + et
    c = pair_centre(*rp, tc.et[0], tc.et[1], tc.et[2]);
    // Rays from origins o + et + e, |e| <= emax: the whitened centre moves by M e, with
    // |M e| <= |M|_F emax and |M|_F^2 = trace(B), so the distance to each ray's line is at
    // least the one from the reference origin minus that.
    if (cut < 0.0) return true;   // sigma < alpha_min: no ray reaches it
    const double r = __builtin_sqrt(cut) + __builtin_sqrt(b[0] + b[3] + b[5]) * tc.emax;   // trace(B) = |M|_F^2
    cut = r * r;
  }
  cut += 0.05;
  // h(d) = d^T Q d with Q = (v^T B v - cut) B - (B v)(B v)^T, i.e. |a x Md|^2 - cut |Md|^2
  // for any M with M^T M = B and a = M v; H(i, j) = v_i^T Q v_j over v = (u, e1, e2)
  const double* v[3] = {tc.u, tc.e1, tc.e2};
  double bvk[3][3], p[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    sym_apply(b, v[k][0], v[k][1], v[k][2], bvk[k]);
    p[k] = __builtin_fma(c.bv[0], v[k][0], __builtin_fma(c.bv[1], v[k][1], c.bv[2] * v[k][2]));
  }
  const double s = c.vbv - cut;
  auto H = [&](int i, int j) {
    const double q = __builtin_fma(v[i][0], bvk[j][0], __builtin_fma(v[i][1], bvk[j][1], v[i][2] * bvk[j][2]));
    return __builtin_fma(s, q, -(p[i] * p[j]));
  };
  const double A = H(0, 0), H01 = H(0, 1), H02 = H(0, 2);
  const double H11 = H(1, 1), H12 = H(1, 2), H22 = H(2, 2);
  const double B = __builtin_sqrt(__builtin_fma(H01, H01, H02 * H02));
  const double hd = 0.5 * (H11 - H22);
  const double C = 0.5 * (H11 + H22) - __builtin_sqrt(__builtin_fma(hd, hd, H12 * H12));
  const double P = 0.5 * (A + C), Rc = 0.5 * (A - C);
  const double rad = __builtin_sqrt(__builtin_fma(Rc, Rc, B * B));
  double fmin;
  if (-Rc >= rad * tc.cos2t) {
    fmin = P - rad;   // the minimiser psi* = pi - atan2(B, Rc) lies inside [0, 2 theta]
  } else {
    const double f1 = __builtin_fma(Rc, tc.cos2t, P) - B * tc.sin2t;
    fmin = A < f1 ? A : f1;
  }
  // the cone's quadric (v^T B v - cut) B - B v (B v)^T cancels like num does: thin records
  // are never dropped here (their pairs are decided by the residual form).  Tested last, so
  // the record's loads are not held behind a branch.
  return fmin > 0.0 && !record_thin(*rp);
}

}  // namespace ut
