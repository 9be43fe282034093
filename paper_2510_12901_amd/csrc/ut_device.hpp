// ut_device.hpp -- device-side types and helpers shared by the gfx950 kernels.
//
// Design notes (MI355X / CDNA4):
// * Geometry and accumulation are float64.  On gfx950 a float64 FMA issues at the same
//   rate as an unpacked float32 FMA (packed float32 is disabled at build time), so the
//   compositing loop pays register space and LDS bytes for float64, not VALU cycles.
// * Wave64 everywhere: ballots are 64-bit, reductions run over 64 lanes.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "utrast.h"

namespace ut {

constexpr double kPi = 3.14159265358979323846;

// Tiles are binned in super-tiles of kSuper x kSuper tiles; a tile's exact list is the
// super-tile list filtered by "the particle's rect contains this tile" (order preserved).
constexpr int kSuper = UT_SUPER_TILE;

// Per-particle compositing record written by the projection for one sensor, read
// (gathered) by the compositing and adjoint kernels.  128 bytes = eight 16-byte chunks, so a
// gathered record is one cache line.
// The response along a ray o + t d is a quadric in t: with B = Sigma^{-1} and v = mu - o,
// (t d - v)^T B (t d - v) is smallest at t* = d^T B v / d^T B d, where it equals
// D^2 = (v^T B v d^T B d - (d^T B v)^2) / d^T B d.  B, B v and v^T B v are fixed per particle
// and sensor, so a pair costs the two ray products d^T B d (from the ray's six quadratic
// monomials) and d^T B v.
struct alignas(16) RecordG {
  double b[6];       // B = Sigma^{-1}: b00, b01, b02, b11, b12, b22
  double bv[3];      // B (mu - o), o = sensor origin
  double vbv;        // (mu - o)^T B (mu - o)
  double log_sigma;  // ln(opacity): alpha = exp(ln sigma - D^2 / 2), and the pre-test threshold
  double v[3];       // mu - o itself, for the residual form of thin records (record_thin)
  float feat[3];     // colour or LiDAR features at the particle's SH direction (the outputs' precision)
  float pad;
};
static_assert(sizeof(RecordG) == UT_RECORD_BYTES, "record size must match the ABI");
constexpr int kRecordChunks = UT_RECORD_BYTES / 16;
constexpr int kFeatChunk = 7;   // the chunk holding feat; the seven before it are float64 fields

// The record as the compositing and adjoint kernels keep it in LDS: the same fields with the
// features widened to float64 once, when the record is staged.
struct alignas(16) Record {
  double b[6];
  double bv[3];
  double vbv;
  double log_sigma;
  double v[3];
  double feat[3];
  double pad;
};
static_assert(sizeof(Record) == UT_RECORD_BYTES + 16, "staged record layout");

static_assert(offsetof(RecordG, feat) == kFeatChunk * 16, "chunk map of the record");

// Records whose v^T B v exceeds kThinVbv take the residual form of D^2 (pair_eval).
constexpr double kThinVbv = 1e7;

// Stage chunk `part` of a gathered record into its LDS copy.
__device__ __forceinline__ void stage_record_chunk(const RecordG* __restrict__ src, Record* dst, int part) {
  const uint4 x = reinterpret_cast<const uint4*>(src)[part];
  if (part < kFeatChunk) {
    reinterpret_cast<uint4*>(dst)[part] = x;
  } else {
    dst->feat[0] = (double)__uint_as_float(x.x);
    dst->feat[1] = (double)__uint_as_float(x.y);
    dst->feat[2] = (double)__uint_as_float(x.z);
  }
}

// Sensor description passed to kernels by value.
struct SensorK {
  int kind;
  double R[9];
  double o[3];
  float of[3];
  double near_;
  int width, height, tiles_x, tiles_y;
  double fx, fy, cx, cy, k[4], theta_max;
  int n_beams, n_az, n_phi, n_theta;
  int cull, cull_az, cull_el;
  const double* bounds;     // [n_phi+1]
  const int* beam_start;    // [n_phi+1]
  const int* sat;           // [(cull_az+1)*(cull_el+1)]
  const float* ray_dir;     // [3][R]
  long long n_rays;
  int super_x, super_y;     // super-tile grid
  int super_h;              // tile rows per super-tile (kSuper columns each)
  // moving sensor: unit quaternions of the poses at t = 0 and 1 (shorter arc), the slerp
  // angle and 1 / sin of it (0: the rotations coincide, interpolate linearly), end origin,
  // per-ray origins and the fixed-point iteration count
  int moving, rs_iters;
  double q0[4], q1[4], slerp_th, slerp_isin;
  double o1[3];
  const float* ray_org;     // [3][R]
  double div_tan;           // LiDAR beam divergence: tan(cone angle / 2), 0 = off
  // LiDAR compositing units: runs of adjacent azimuth tiles of one elevation tile inside one
  // super-tile column, (band, first tile, end tile, rays), packed so that a unit holds at
  // most unit_rays rays; one workgroup of unit_rays lanes composites a unit
  const int4* units;
  int n_units, unit_rays;
  const int4* units_wide;   // the same packing for 256 lanes (batched compositing)
  int n_units_wide;
};

// Tiles of a LiDAR compositing unit: at most 4 adjacent tiles, inside one super-tile column.
constexpr int kUnitTilesMax = 4;

// 2^(j/32), j = 0..31, correctly rounded to float64 (evaluated in 60-digit decimal arithmetic).
__constant__ static const double kExp2Frac[32] = {
    0x1.0000000000000p+0, 0x1.059b0d3158574p+0, 0x1.0b5586cf9890fp+0, 0x1.11301d0125b51p+0,
    0x1.172b83c7d517bp+0, 0x1.1d4873168b9aap+0, 0x1.2387a6e756238p+0, 0x1.29e9df51fdee1p+0,
    0x1.306fe0a31b715p+0, 0x1.371a7373aa9cbp+0, 0x1.3dea64c123422p+0, 0x1.44e086061892dp+0,
    0x1.4bfdad5362a27p+0, 0x1.5342b569d4f82p+0, 0x1.5ab07dd485429p+0, 0x1.6247eb03a5585p+0,
    0x1.6a09e667f3bcdp+0, 0x1.71f75e8ec5f74p+0, 0x1.7a11473eb0187p+0, 0x1.82589994cce13p+0,
    0x1.8ace5422aa0dbp+0, 0x1.93737b0cdc5e5p+0, 0x1.9c49182a3f090p+0, 0x1.a5503b23e255dp+0,
    0x1.ae89f995ad3adp+0, 0x1.b7f76f2fb5e47p+0, 0x1.c199bdd85529cp+0, 0x1.cb720dcef9069p+0,
    0x1.d5818dcfba487p+0, 0x1.dfc97337b9b5fp+0, 0x1.ea4afa2a490dap+0, 0x1.f50765b6e4540p+0};

// e^x in float64 for the response (x <= 0; results below the smallest normal flush towards 0).
// Table-driven reduction: x = (32 n + j) ln2/32 + r with |r| <= ln2/64 (Cody-Waite: ln2/32 split
// into a 40-bit head, so k * head is exact, and a tail), e^x = 2^n 2^(j/32) e^r, and e^r by its
// degree-5 Taylor polynomial (truncation < 2.3e-15 relative).  `tab` holds the 32 values of
// kExp2Frac; the compositing passes an LDS copy, the adjoint the constant array itself, and
// both get bit-identical results.
__device__ __forceinline__ double exp_neg(double x, const double* tab) {
  const double kInvLn2x32 = 0x1.71547652b82fep+5;   // 32 / ln 2
  const double kHi = 0x1.62e42fefa2000p-6;          // head of ln 2 / 32
  const double kLo = 0x1.9ef35793c7673p-46;         // ln 2 / 32 - head
  const double k = __builtin_rint(x * kInvLn2x32);
  double r = __builtin_fma(-k, kHi, x);
  r = __builtin_fma(-k, kLo, r);
  const int ki = (int)k;
  double p = __builtin_fma(r, 1.0 / 120.0, 1.0 / 24.0);
  p = __builtin_fma(p, r, 1.0 / 6.0);
  p = __builtin_fma(p, r, 0.5);
  p = __builtin_fma(p, r, 1.0);
  p = __builtin_fma(p, r, 1.0);
  return __builtin_ldexp(p * tab[ki & 31], ki >> 5);
}

// 1/x in float64 from the hardware estimate refined by two Newton steps.
__device__ __forceinline__ double rcp_f64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}

// Pose of a moving sensor at frame time t (the origin linear in t, the rotation slerped
// between the unit quaternions q0 and q1): the world->sensor rotation as a unit quaternion.
__device__ __forceinline__ void pose_at(const SensorK& s, double t, double q[4], double o[3]) {
  double w0 = 1.0 - t, w1 = t;
  if (s.slerp_isin > 0) {
    w0 = sin((1.0 - t) * s.slerp_th) * s.slerp_isin;
    w1 = sin(t * s.slerp_th) * s.slerp_isin;
  }
  double n = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    q[i] = __builtin_fma(w0, s.q0[i], w1 * s.q1[i]);
    n = __builtin_fma(q[i], q[i], n);
  }
  const double in = 1.0 / sqrt(n);
#pragma unroll
  for (int i = 0; i < 4; ++i) q[i] *= in;
#pragma unroll
  for (int i = 0; i < 3; ++i) o[i] = __builtin_fma(1.0 - t, s.o[i], t * s.o1[i]);
}

// R(q) v for a unit quaternion q = (w, u): v + 2 w (u x v) + 2 u x (u x v).
__device__ __forceinline__ void quat_rotate(const double q[4], const double v[3], double r[3]) {
  const double w = q[0], ux = q[1], uy = q[2], uz = q[3];
  const double cx = uy * v[2] - uz * v[1], cy = uz * v[0] - ux * v[2], cz = ux * v[1] - uy * v[0];
  const double dx = uy * cz - uz * cy, dy = uz * cx - ux * cz, dz = ux * cy - uy * cx;
  r[0] = v[0] + 2.0 * (w * cx + dx);
  r[1] = v[1] + 2.0 * (w * cy + dy);
  r[2] = v[2] + 2.0 * (w * cz + dz);
}

// A ray direction with its quadratic monomials (the cross terms doubled), so that
// d^T B d = b00 xx + b11 yy + b22 zz + b01 xy + b02 xz + b12 yz.
struct RayQ {
  double x, y, z;
  double xx, yy, zz, xy, xz, yz;
};

__device__ __forceinline__ RayQ ray_q(double x, double y, double z) {
  RayQ r;
  r.x = x; r.y = y; r.z = z;
  r.xx = x * x; r.yy = y * y; r.zz = z * z;
  r.xy = 2.0 * x * y; r.xz = 2.0 * x * z; r.yz = 2.0 * y * z;
  return r;
}

// B s for a symmetric B stored as its six unique entries.
__device__ __forceinline__ void sym_apply(const double b[6], double sx, double sy, double sz, double o[3]) {
  o[0] = __builtin_fma(b[0], sx, __builtin_fma(b[1], sy, b[2] * sz));
  o[1] = __builtin_fma(b[1], sx, __builtin_fma(b[3], sy, b[4] * sz));
  o[2] = __builtin_fma(b[2], sx, __builtin_fma(b[4], sy, b[5] * sz));
}

// Response geometry of one (ray, particle) pair (Sec. 3, the 3D response replacing the 2D
// splat).  The compositing and the adjoint evaluate it through the same functions, so both
// take identical skip / clamp / stop decisions.
struct PairGeom {
  double dbd;   // d^T B d
  double dbv;   // d^T B v
  double num;   // v^T B v d^T B d - (d^T B v)^2 = D^2 d^T B d
};

// The particle's centre seen from the ray's origin: (B v, v^T B v) from the record for a
// static sensor, pair_centre() for a ray with its own origin.
struct Centre {
  double bv[3];
  double vbv;
};

template <class Rec>
__device__ __forceinline__ Centre record_centre(const Rec& c) {
  Centre q;
  q.bv[0] = c.bv[0]; q.bv[1] = c.bv[1]; q.bv[2] = c.bv[2];
  q.vbv = c.vbv;
  return q;
}

// Centre for a ray whose origin lies e = o_i - o from the record's sensor origin o:
// v_i = v - e, so B v_i = B v - B e and v_i^T B v_i = v^T B v - e^T (2 B v - B e).
template <class Rec>
__device__ __forceinline__ Centre pair_centre(const Rec& c, double ex, double ey, double ez) {
  double be[3];
  sym_apply(c.b, ex, ey, ez, be);
  Centre q;
  q.bv[0] = c.bv[0] - be[0]; q.bv[1] = c.bv[1] - be[1]; q.bv[2] = c.bv[2] - be[2];
  const double s0 = __builtin_fma(2.0, c.bv[0], -be[0]), s1 = __builtin_fma(2.0, c.bv[1], -be[1]),
               s2 = __builtin_fma(2.0, c.bv[2], -be[2]);
  q.vbv = c.vbv - __builtin_fma(ex, s0, __builtin_fma(ey, s1, ez * s2));
  return q;
}

template <class Rec>
__device__ __forceinline__ PairGeom pair_geometry(const Rec& c, const Centre& v, const RayQ& d) {
  PairGeom p;
  p.dbd = __builtin_fma(c.b[0], d.xx, __builtin_fma(c.b[3], d.yy, __builtin_fma(c.b[5], d.zz,
          __builtin_fma(c.b[1], d.xy, __builtin_fma(c.b[2], d.xz, c.b[4] * d.yz)))));
  p.dbv = __builtin_fma(v.bv[0], d.x, __builtin_fma(v.bv[1], d.y, v.bv[2] * d.z));
  p.num = __builtin_fma(v.vbv, p.dbd, -(p.dbv * p.dbv));
  return p;
}

// D^2 threshold of the conservative pre-test: beyond it sigma * rho < alpha_min for certain
// (ln rho = -D^2 / 2, with 1e-3 of slack for rounding).
__device__ __forceinline__ double cut_threshold(double log_sigma, double log_alpha_min) {
  return __builtin_fma(2.0, log_sigma, 1e-3 - 2.0 * log_alpha_min);
}

// True when the pair cannot reach alpha_min: D^2 > cut, tested as num > cut d^T B d.
__device__ __forceinline__ bool pair_cut(const PairGeom& q, double cut) { return q.num > q.dbd * cut; }

struct PairResp {
  double idbd;  // 1 / d^T B d
  double tau;   // t*
  double D2;    // squared Mahalanobis distance at t*
};

__device__ __forceinline__ PairResp pair_response(const PairGeom& q) {
  PairResp r;
  r.idbd = rcp_f64(q.dbd);
  r.tau = q.dbv * r.idbd;
  r.D2 = __builtin_fmax(q.num, 0.0) * r.idbd;
  return r;
}

// Records whose v^T B v exceeds kThinVbv (particles very thin, or small and far, relative to
// their distance) lose about ulp(v^T B v) of D^2 to the cancellation in
// num = v^T B v d^T B d - (d^T B v)^2: 2e-3 in alpha for a disc 1e-4 as thick as it is wide
// at 50 m.  For them D^2 comes from the residual u = v_i - t* d instead, D^2 = u^T B u, whose
// error stays near ulp(|v|) in the whitened frame.  The test reads the record, so it is
// uniform across a wavefront; fewer than 1 in 10^4 records of a typical scene take it.
template <class Rec>
__device__ __forceinline__ bool record_thin(const Rec& c) { return c.vbv > kThinVbv; }

// Response of one (ray, record) pair for a ray whose origin lies e from the record's sensor
// origin (cv = pair_centre(c, e), or record_centre(c) with e = 0).  Returns false when the
// pair cannot reach alpha_min (D^2 > cut); pr holds 1/d^T B d, t* and D^2 either way.  The
// compositing and the adjoint both evaluate pairs here, so their alphas are bit-identical.
// Every active lane of a wavefront evaluates the same record, so the thin test is taken from
// the first active lane as a scalar branch.
// UNIFORM = false: the lanes may hold different records, so the thin test is taken per lane.
template <class Rec, bool UNIFORM = true>
__device__ __forceinline__ bool pair_eval(const Rec& c, const Centre& cv, const RayQ& d, double ex, double ey,
                                          double ez, double cut, PairResp& pr) {
  const PairGeom q = pair_geometry(c, cv, d);
  const bool thin = UNIFORM ? __builtin_amdgcn_readfirstlane((int)record_thin(c)) != 0 : record_thin(c);
  if (__builtin_expect(thin, 0)) {
    pr.idbd = rcp_f64(q.dbd);
    pr.tau = q.dbv * pr.idbd;
    const double ux = __builtin_fma(-pr.tau, d.x, c.v[0] - ex);
    const double uy = __builtin_fma(-pr.tau, d.y, c.v[1] - ey);
    const double uz = __builtin_fma(-pr.tau, d.z, c.v[2] - ez);
    const double cross = __builtin_fma(c.b[1], ux * uy, __builtin_fma(c.b[2], ux * uz, c.b[4] * (uy * uz)));
    const double diag = __builtin_fma(c.b[0], ux * ux, __builtin_fma(c.b[3], uy * uy, c.b[5] * (uz * uz)));
    pr.D2 = __builtin_fmax(__builtin_fma(2.0, cross, diag), 0.0);
    return !(pr.D2 > cut);
  }
  pr = pair_response(q);   // formed before the test, so a caller can select on the result
  return !pair_cut(q, cut);
}

// Unclamped opacity of the pair, sigma * exp(-D^2 / 2), evaluated as exp(ln sigma - D^2 / 2).
template <class Rec>
__device__ __forceinline__ double pair_alpha(const Rec& c, const PairResp& r, const double* tab) {
  return exp_neg(__builtin_fma(-0.5, r.D2, c.log_sigma), tab);
}

// Packed tile rect of a particle: (x0 | y0 << 16, x1 | y1 << 16); LiDAR x1 may exceed
// n_theta - 1 where the rect wraps through azimuth 0.
__device__ __forceinline__ bool rect_covers(uint2 r, int tx, int ty, const SensorK& s) {
  const int x0 = (int)(r.x & 0xFFFFu), y0 = (int)(r.x >> 16), x1 = (int)(r.y & 0xFFFFu), y1 = (int)(r.y >> 16);
  if (ty < y0 || ty > y1) return false;
  if (s.kind != UT_LIDAR) return tx >= x0 && tx <= x1;
  int dx = tx - x0;
  if (dx < 0) dx += s.n_theta;
  return dx <= x1 - x0;
}

// First azimuth step of LiDAR azimuth tile j: ceil(j n_az / N_theta); step a lies in tile
// floor(a N_theta / n_az).
__device__ __forceinline__ int az_start(const SensorK& s, int j) {
  return (int)(((long long)j * s.n_az + s.n_theta - 1) / s.n_theta);
}

// Ray r of LiDAR unit u = (band k, tiles [j0, j1)): the unit's beams times its azimuth steps,
// azimuth fastest; *t receives the ray's tile relative to j0.  Returns -1 past the end.
__device__ __forceinline__ long long unit_ray(const SensorK& s, int4 u, int r, int* t) {
  const int b0 = s.beam_start[u.x], b1 = s.beam_start[u.x + 1];
  const int a0 = az_start(s, u.y), a1 = az_start(s, u.z);
  const int naz = a1 - a0;
  *t = 0;
  if (naz <= 0 || r >= (b1 - b0) * naz) return -1;
  const int a = a0 + r % naz;
  *t = (int)(((long long)a * s.n_theta) / s.n_az) - u.y;
  return (long long)(b0 + r / naz) * s.n_az + a;
}

// Does a packed LiDAR rect cover elevation tile k and some azimuth tile of [j0, j1)
// (j1 <= N_theta)?  The covered azimuth arc starts at x0 and is contiguous modulo N_theta.
__device__ __forceinline__ bool rect_meets_unit(uint2 r, int k, int j0, int j1, const SensorK& s) {
  const int x0 = (int)(r.x & 0xFFFFu), y0 = (int)(r.x >> 16), x1 = (int)(r.y & 0xFFFFu), y1 = (int)(r.y >> 16);
  if (k < y0 || k > y1) return false;
  int dx = j0 - x0;
  if (dx < 0) dx += s.n_theta;
  return dx <= x1 - x0 || (x0 > j0 && x0 < j1);
}

__device__ __forceinline__ int super_of_tile(int tile, const SensorK& s) {
  const int tx = tile % s.tiles_x, ty = tile / s.tiles_x;
  return (ty / s.super_h) * s.super_x + tx / kSuper;
}

// Workgroup b of a grid of super_tile_slots() -> tile: the tiles of super-tile b / slots, row
// by row.  The GPU hands consecutive workgroups to its 8 XCDs in turn, so every super-tile's
// tiles are spread over all XCDs and each XCD gets an even share of every image region.  (Giving
// each XCD whole super-tiles, so that the tiles filtering one bin share that XCD's L2, left
// the XCDs unevenly loaded: the frame's fisheye compositing took 9-11% longer.)  Slots of an
// edge super-tile that lie past the image return -1.
__device__ __forceinline__ int super_major_tile(int b, const SensorK& s) {
  const int slots = kSuper * s.super_h;
  const int sid = b / slots, t = b % slots;
  if (sid >= s.super_x * s.super_y) return -1;
  const int tx = (sid % s.super_x) * kSuper + t % kSuper, ty = (sid / s.super_x) * s.super_h + t / kSuper;
  if (tx >= s.tiles_x || ty >= s.tiles_y) return -1;
  return ty * s.tiles_x + tx;
}
inline int super_tile_slots(int super_x, int super_y, int super_h) { return super_x * super_y * kSuper * super_h; }

// Rays of a tile: camera 16x16 pixel block; LiDAR beams of the elevation tile times the
// azimuth steps a with floor(a N_theta / n_az) == azimuth tile.  Returns -1 past the end.
__device__ __forceinline__ long long tile_ray(const SensorK& s, int tile, int r) {
  if (s.kind != UT_LIDAR) {
    const int tx = tile % s.tiles_x, ty = tile / s.tiles_x;
    const int px = tx * UT_CAMERA_TILE + (r & (UT_CAMERA_TILE - 1));
    const int py = ty * UT_CAMERA_TILE + (r >> 4);
    if (r >= UT_CAMERA_TILE * UT_CAMERA_TILE || px >= s.width || py >= s.height) return -1;
    return (long long)py * s.width + px;
  }
  const int j = tile % s.n_theta, k = tile / s.n_theta;
  const int b0 = s.beam_start[k], b1 = s.beam_start[k + 1];
  const long long A = s.n_az, NT = s.n_theta;
  const int a0 = (int)((j * A + NT - 1) / NT), a1 = (int)(((j + 1) * A + NT - 1) / NT);
  const int naz = a1 - a0;
  if (naz <= 0 || r >= (b1 - b0) * naz) return -1;
  return (long long)(b0 + r / naz) * s.n_az + (a0 + r % naz);
}

}  // namespace ut
