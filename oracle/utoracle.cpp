/*
 * utoracle.cpp -- plain FP64 CPU oracle of the unscented-transform Gaussian rasterizer
 * for cameras and spinning LiDAR (SimULi, arXiv 2510.12901).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark may load this library.  It shares no code, header or table with the
 * GPU library: every step is written out here from the paper (or, where the paper defers
 * to 3DGUT / 3DGRT / 3DGS, from the textbook definition named at the step).  It is slow
 * on purpose: no blocking, fusion or reordering beyond what each definition states.
 *
 * Precision: every quantity is double; the float32 inputs are converted exactly.  The
 * only float32 arithmetic is the depth sort key, which the method defines in float32.
 * Build: -O2 -fno-fast-math -ffp-contract=off (no FMA contraction), OpenMP over
 * independent rays / tiles only.
 *
 * Readings of passages the paper leaves open are marked READING where they are applied.
 */
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include <omp.h>

extern "C" {

/* Particles (Sec. 3.1, "Particle Representation"): float64 copies of the inputs.
 * mean[3][n], quat[4][n] (w,x,y,z; normalised here), log_scale[3][n], opacity_logit[n],
 * feat[K][3][n] with K = (sh_degree+1)^2 coefficients per channel. */
typedef struct {
  const double *mean, *quat, *log_scale, *opacity_logit, *feat;
  int n, sh_degree, feat_kind; /* feat_kind 0 camera colour, 1 LiDAR features */
} orc_gaussians;

/* Sensor.  kind 0 pinhole, 1 equidistant fisheye (k1..k4), 2 spinning LiDAR, 3 orthographic.
 * R_sw world->sensor rows, origin = sensor position (both float32 inputs). */
typedef struct {
  int kind;
  float R_sw[9];
  float origin[3];
  int width, height, tile;
  double fx, fy, cx, cy, k[4], theta_max, near_;
  int n_beams, n_az, n_phi, n_theta;
  const double* elev_bounds; /* [n_phi+1] */
  const int* beam_start;     /* [n_phi+1] first beam of each elevation tile */
  int cull, cull_az, cull_el;
  const int* sat;            /* [(cull_az+1)*(cull_el+1)] summed-area table */
  const float* ray_dir;      /* [3][R] world frame */
  /* Time-dependent sensor (Sec. 3.2 and the appendix on time-dependent effects): moving = 1
   * means the pose (R_sw, origin) holds at frame time t = 0 and (R_sw1, origin1) at t = 1,
   * every ray carries its own origin ray_org[3][R] (and direction), and a projected point is
   * observed at the time of the row (camera) or azimuth (LiDAR) it falls on. */
  int moving;
  float R_sw1[9];
  float origin1[3];
  const float* ray_org;      /* [3][R] world frame, moving sensors only */
  int rs_iters;              /* fixed-point iterations of the time-dependent projection */
  /* LiDAR beam divergence (full angle, radians; 0 = off): the 3D smoothing filter of the
   * appendix on beam divergence (Eq. 6), without its opacity factor. */
  double beam_divergence;
} orc_sensor;

typedef struct {
  double ut_alpha, ut_beta, ut_kappa;
  double alpha_min, alpha_max, t_min;
} orc_params;

typedef struct {
  int* valid;        /* [n] all sigma points projected */
  double* mean2;     /* [2][n] UT mean */
  double* cov2;      /* [3][n] UT covariance (uu, uv, vv) */
  int* rect;         /* [4][n] x0,y0,x1,y1 inclusive tiles (LiDAR: az0,el0,az1,el1, az1 may exceed n_theta-1 = wrap) */
  uint32_t* count;   /* [n] tiles touched (0 = culled) */
  uint32_t* key;     /* [n] float32 squared distance bits */
  double* feat;      /* [3][n] evaluated colour / LiDAR features */
  double* margin;    /* [n] smallest distance of a discrete decision to its threshold */
  int n_culled_invalid;
  int n_culled_rays;
} orc_projected;

} /* extern "C" */

namespace {

const double kPi = 3.14159265358979323846;

/* ------------------------------------------------------------------------------------
 * Particle parameters.  Sec. 3.1: Sigma = R S S^T R^T.  READING: q = (w,x,y,z) is
 * normalised, S = diag(exp(log_scale)), opacity = sigmoid(logit).
 * ---------------------------------------------------------------------------------- */
struct Particle {
  bool ok;
  double qn[4];   /* normalised quaternion */
  double qnorm;
  double mu[3];
  double R[9];    /* row-major */
  double s[3];
  double sigma;
  double Sigma[9];
  double Binv[9]; /* Sigma^{-1} */
  bool filtered;  /* beam-divergence filter applied: Sigma holds Sigma_hat, L its Cholesky factor */
  double L[9];
};

void quat_to_rot(const double q[4], double R[9]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* derivative of R(q) with respect to each quaternion component (row-major 3x3 each) */
void quat_to_rot_jacobian(const double q[4], double J[4][9]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  const double dw[9] = {0, -2 * z, 2 * y, 2 * z, 0, -2 * x, -2 * y, 2 * x, 0};
  const double dx[9] = {0, 2 * y, 2 * z, 2 * y, -4 * x, -2 * w, 2 * z, 2 * w, -4 * x};
  const double dy[9] = {-4 * y, 2 * x, 2 * w, 2 * x, 0, 2 * z, -2 * w, 2 * z, -4 * y};
  const double dz[9] = {-4 * z, -2 * w, 2 * x, 2 * w, -4 * z, 2 * y, 2 * x, 2 * y, 0};
  std::memcpy(J[0], dw, sizeof dw);
  std::memcpy(J[1], dx, sizeof dx);
  std::memcpy(J[2], dy, sizeof dy);
  std::memcpy(J[3], dz, sizeof dz);
}

bool inverse3(const double A[9], double out[9]) {
  const double c00 = A[4] * A[8] - A[5] * A[7];
  const double c01 = A[5] * A[6] - A[3] * A[8];
  const double c02 = A[3] * A[7] - A[4] * A[6];
  const double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
  if (!(det > 0) || !std::isfinite(det)) return false;
  out[0] = c00 / det;
  out[1] = (A[2] * A[7] - A[1] * A[8]) / det;
  out[2] = (A[1] * A[5] - A[2] * A[4]) / det;
  out[3] = c01 / det;
  out[4] = (A[0] * A[8] - A[2] * A[6]) / det;
  out[5] = (A[2] * A[3] - A[0] * A[5]) / det;
  out[6] = c02 / det;
  out[7] = (A[1] * A[6] - A[0] * A[7]) / det;
  out[8] = (A[0] * A[4] - A[1] * A[3]) / det;
  return true;
}

Particle make_particle(const orc_gaussians* g, int i) {
  Particle p;
  std::memset(&p, 0, sizeof p);
  const int n = g->n;
  double q[4];
  bool finite = true;
  for (int a = 0; a < 3; ++a) {
    p.mu[a] = g->mean[a * n + i];
    finite = finite && std::isfinite(p.mu[a]) && std::isfinite(g->log_scale[a * n + i]);
  }
  for (int a = 0; a < 4; ++a) {
    q[a] = g->quat[a * n + i];
    finite = finite && std::isfinite(q[a]);
  }
  finite = finite && std::isfinite(g->opacity_logit[i]);
  p.qnorm = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  if (!finite || !(p.qnorm > 0)) { p.ok = false; return p; }
  for (int a = 0; a < 4; ++a) p.qn[a] = q[a] / p.qnorm;
  quat_to_rot(p.qn, p.R);
  for (int a = 0; a < 3; ++a) p.s[a] = std::exp(g->log_scale[a * n + i]);
  p.sigma = 1.0 / (1.0 + std::exp(-g->opacity_logit[i]));
  /* Sigma = R diag(s^2) R^T, written as the plain triple product */
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double acc = 0;
      for (int k = 0; k < 3; ++k) acc += p.R[r * 3 + k] * p.s[k] * p.s[k] * p.R[c * 3 + k];
      p.Sigma[r * 3 + c] = acc;
    }
  p.ok = inverse3(p.Sigma, p.Binv);
  return p;
}

/* ------------------------------------------------------------------------------------
 * Beam-divergence filter (appendix, Eq. 6).  READING: the paper names the smoothed
 * covariance Sigma_hat without defining it; following the 3D smoothing filter it cites, the
 * particle is widened in the plane orthogonal to d = (mu - o)/|mu - o| by the beam's variance
 * at that range, Sigma_hat = Sigma + (r tan(theta/2))^2 (I - d d^T), r = |mu - o|, theta the
 * full divergence angle; the response is exp(-(x-mu)^T Sigma_hat^{-1} (x-mu) / 2) with the
 * opacity left unscaled, as the paper prescribes.  The UT's sigma points then use the
 * Cholesky factor of Sigma_hat as the matrix square root.
 * ---------------------------------------------------------------------------------- */
bool cholesky3(const double A[9], double L[9]) {
  for (int i = 0; i < 9; ++i) L[i] = 0;
  for (int j = 0; j < 3; ++j) {
    double d = A[j * 3 + j];
    for (int k = 0; k < j; ++k) d -= L[j * 3 + k] * L[j * 3 + k];
    if (!(d > 0)) return false;
    L[j * 3 + j] = std::sqrt(d);
    for (int i = j + 1; i < 3; ++i) {
      double v = A[i * 3 + j];
      for (int k = 0; k < j; ++k) v -= L[i * 3 + k] * L[j * 3 + k];
      L[i * 3 + j] = v / L[j * 3 + j];
    }
  }
  return true;
}

void apply_beam_divergence(const orc_sensor* s, Particle& p) {
  if (!p.ok || s->kind != 2 || !(s->beam_divergence > 0)) return;
  double v[3] = {p.mu[0] - s->origin[0], p.mu[1] - s->origin[1], p.mu[2] - s->origin[2]};
  const double r = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  if (!(r > 0)) return;
  for (int a = 0; a < 3; ++a) v[a] /= r;
  const double w = r * std::tan(0.5 * s->beam_divergence);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) p.Sigma[i * 3 + j] += w * w * ((i == j ? 1.0 : 0.0) - v[i] * v[j]);
  p.filtered = true;
  p.ok = inverse3(p.Sigma, p.Binv) && cholesky3(p.Sigma, p.L);
}

/* ------------------------------------------------------------------------------------
 * Real spherical harmonics (Sec. 3.1: SH^c, SH^l up to degree 3; Eq. 1 "SH_i(d)").
 * Built from the general definition: Legendre polynomials P_l by Bonnet's recursion,
 * associated functions P_l^m = (-1)^m (1-z^2)^{m/2} d^m P_l/dz^m (Condon-Shortley phase),
 * normalisation K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!), and on the unit sphere
 * (1-z^2)^{m/2} cos(m phi) = Re (x+iy)^m, (1-z^2)^{m/2} sin(m phi) = Im (x+iy)^m.
 * Y_l0 = K P_l(z); Y_lm = sqrt2 K Pi_l^m(z) Re(x+iy)^m (m>0); sqrt2 K Pi_l^|m|(z) Im(x+iy)^|m| (m<0),
 * with Pi_l^m = (-1)^m d^m P_l/dz^m.  Index k = l^2 + l + m.
 * ---------------------------------------------------------------------------------- */
struct SHBasis {
  double pi[4][4][4]; /* pi[l][m][j]: coefficient of z^j in Pi_l^m(z) */
  double K[4][4];
  SHBasis() {
    double P[4][4] = {{0}};
    P[0][0] = 1;
    P[1][1] = 1;
    for (int l = 1; l < 3; ++l)
      for (int j = 0; j < 4; ++j)
        P[l + 1][j] = ((2 * l + 1) * (j > 0 ? P[l][j - 1] : 0.0) - l * P[l - 1][j]) / (l + 1);
    auto fact = [](int v) { double f = 1; for (int t = 2; t <= v; ++t) f *= t; return f; };
    for (int l = 0; l < 4; ++l)
      for (int m = 0; m <= l; ++m) {
        double c[4];
        for (int j = 0; j < 4; ++j) c[j] = P[l][j];
        for (int d = 0; d < m; ++d) {
          for (int j = 0; j < 3; ++j) c[j] = (j + 1) * c[j + 1];
          c[3] = 0;
        }
        const double sign = (m % 2) ? -1.0 : 1.0;
        for (int j = 0; j < 4; ++j) pi[l][m][j] = sign * c[j];
        K[l][m] = std::sqrt((2 * l + 1) / (4 * kPi) * fact(l - m) / fact(l + m));
      }
  }
  /* Y[k] and, if dY != nullptr, dY[k][0..2] = gradient of the polynomial form in (x,y,z) */
  void eval(int deg, const double d[3], double* Y, double (*dY)[3]) const {
    const double x = d[0], y = d[1], z = d[2];
    double A[4], B[4];
    A[0] = 1; B[0] = 0;
    for (int m = 1; m < 4; ++m) {
      A[m] = x * A[m - 1] - y * B[m - 1];
      B[m] = x * B[m - 1] + y * A[m - 1];
    }
    for (int l = 0; l <= deg; ++l)
      for (int m = -l; m <= l; ++m) {
        const int am = m < 0 ? -m : m;
        double pz = 0, dpz = 0, zp = 1;
        for (int j = 0; j < 4; ++j) {
          pz += pi[l][am][j] * zp;
          if (j + 1 < 4) dpz += (j + 1) * pi[l][am][j + 1] * zp;
          zp *= z;
        }
        const double norm = (m == 0) ? K[l][0] : std::sqrt(2.0) * K[l][am];
        double xyv, gx, gy;
        if (m == 0) { xyv = 1; gx = 0; gy = 0; }
        else if (m > 0) { xyv = A[am]; gx = am * A[am - 1]; gy = -am * B[am - 1]; }
        else { xyv = B[am]; gx = am * B[am - 1]; gy = am * A[am - 1]; }
        const int k = l * l + l + m;
        Y[k] = norm * pz * xyv;
        if (dY) {
          dY[k][0] = norm * pz * gx;
          dY[k][1] = norm * pz * gy;
          dY[k][2] = norm * dpz * xyv;
        }
      }
  }
};

const SHBasis& sh_basis() {
  static const SHBasis b;
  return b;
}

/* Per-Gaussian features (Eq. 1, Sec. 3.2).  READING: SH evaluated once per Gaussian at
 * the unit direction from the sensor origin to the mean (3DGS practice); camera colour =
 * max(0, f + 0.5), LiDAR features raw.  clamp[c] = 1 when the camera clamp is active. */
void sh_features_raw(const orc_gaussians* g, int i, const double mu[3], const double o[3],
                     double f[3]) {
  const int K = (g->sh_degree + 1) * (g->sh_degree + 1);
  double v[3] = {mu[0] - o[0], mu[1] - o[1], mu[2] - o[2]};
  const double len = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  double dir[3] = {0, 0, 1};
  if (len > 0) for (int a = 0; a < 3; ++a) dir[a] = v[a] / len;
  double Y[16];
  sh_basis().eval(g->sh_degree, dir, Y, nullptr);
  for (int c = 0; c < 3; ++c) {
    double acc = 0;
    for (int k = 0; k < K; ++k) acc += g->feat[(k * 3 + c) * g->n + i] * Y[k];
    f[c] = acc;
  }
}

void gaussian_features(const orc_gaussians* g, int i, const double mu[3], const double o[3],
                       double out[3], int clamp[3]) {
  double f[3];
  sh_features_raw(g, i, mu, o, f);
  for (int c = 0; c < 3; ++c) {
    if (g->feat_kind == 0) {
      clamp[c] = !(f[c] + 0.5 > 0);
      out[c] = clamp[c] ? 0.0 : f[c] + 0.5;
    } else {
      clamp[c] = 0;
      out[c] = f[c];
    }
  }
}

/* ------------------------------------------------------------------------------------
 * Sensor projection g(x) (Sec. 3.2 "arbitrary camera models"; Eq. 3 for LiDAR).
 * READING: pinhole valid iff z > near; equidistant fisheye theta = atan2(|xy|, z),
 * theta_d = theta (1 + k1 t^2 + k2 t^4 + k3 t^6 + k4 t^8), valid iff |x| > near and
 * theta <= theta_max; LiDAR (azimuth, elevation) = (atan2(y,x) in [0,2pi), asin(z/r)),
 * valid iff r > near; orthographic (fx x + cx, fy y + cy), valid iff z > near.
 * margin receives the distance of the validity decision to its threshold.
 * ---------------------------------------------------------------------------------- */
/* ------------------------------------------------------------------------------------
 * Sensor pose.  A static sensor has one pose.  A moving one (rolling shutter, spinning LiDAR)
 * interpolates between its poses at t = 0 and t = 1.  READING (the paper gives no formula):
 * the origin moves linearly, o(t) = (1 - t) o0 + t o1, and the rotation by spherical linear
 * interpolation of the two unit quaternions (shorter arc), i.e. constant angular velocity.
 * ---------------------------------------------------------------------------------- */
void rot_to_quat(const float Rf[9], double q[4]) {
  double R[9];
  for (int i = 0; i < 9; ++i) R[i] = Rf[i];
  /* largest of the four |q_i| first, for a well-conditioned extraction */
  const double t = R[0] + R[4] + R[8];
  if (t > 0) {
    const double r = std::sqrt(1 + t), f = 0.5 / r;
    q[0] = 0.5 * r; q[1] = (R[7] - R[5]) * f; q[2] = (R[2] - R[6]) * f; q[3] = (R[3] - R[1]) * f;
  } else if (R[0] >= R[4] && R[0] >= R[8]) {
    const double r = std::sqrt(1 + R[0] - R[4] - R[8]), f = 0.5 / r;
    q[0] = (R[7] - R[5]) * f; q[1] = 0.5 * r; q[2] = (R[1] + R[3]) * f; q[3] = (R[2] + R[6]) * f;
  } else if (R[4] >= R[8]) {
    const double r = std::sqrt(1 - R[0] + R[4] - R[8]), f = 0.5 / r;
    q[0] = (R[2] - R[6]) * f; q[1] = (R[1] + R[3]) * f; q[2] = 0.5 * r; q[3] = (R[5] + R[7]) * f;
  } else {
    const double r = std::sqrt(1 - R[0] - R[4] + R[8]), f = 0.5 / r;
    q[0] = (R[3] - R[1]) * f; q[1] = (R[2] + R[6]) * f; q[2] = (R[5] + R[7]) * f; q[3] = 0.5 * r;
  }
  const double nq = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int i = 0; i < 4; ++i) q[i] /= nq;
}

void pose_at(const orc_sensor* s, double t, double R[9], double o[3]) {
  if (!s->moving) {
    for (int i = 0; i < 9; ++i) R[i] = s->R_sw[i];
    for (int a = 0; a < 3; ++a) o[a] = s->origin[a];
    return;
  }
  double q0[4], q1[4];
  rot_to_quat(s->R_sw, q0);
  rot_to_quat(s->R_sw1, q1);
  double dot = q0[0] * q1[0] + q0[1] * q1[1] + q0[2] * q1[2] + q0[3] * q1[3];
  if (dot < 0) {
    for (int i = 0; i < 4; ++i) q1[i] = -q1[i];
    dot = -dot;
  }
  double w0 = 1 - t, w1 = t;
  if (dot < 1 - 1e-12) {
    const double th = std::acos(std::min(dot, 1.0));
    w0 = std::sin((1 - t) * th) / std::sin(th);
    w1 = std::sin(t * th) / std::sin(th);
  }
  double q[4];
  for (int i = 0; i < 4; ++i) q[i] = w0 * q0[i] + w1 * q1[i];
  const double nq = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int i = 0; i < 4; ++i) q[i] /= nq;
  quat_to_rot(q, R);
  for (int a = 0; a < 3; ++a) o[a] = (1 - t) * (double)s->origin[a] + t * (double)s->origin1[a];
}

void to_sensor_pose(const double R[9], const double o[3], const double xw[3], double xs[3]) {
  double d[3];
  for (int a = 0; a < 3; ++a) d[a] = xw[a] - o[a];
  for (int r = 0; r < 3; ++r) xs[r] = R[r * 3 + 0] * d[0] + R[r * 3 + 1] * d[1] + R[r * 3 + 2] * d[2];
}

bool project_point_pose(const orc_sensor* s, const double R[9], const double o[3], const double xw[3],
                        double uv[2], double* margin);

/* Time-dependent projection (the appendix on time-dependent effects: sensor motion inside
 * the projection function, sigma points projected independently).  READING: the frame time
 * of a camera row v is v / H (rows read out top to bottom, row r at (r + 0.5) / H) and of a
 * LiDAR azimuth phi in [0, 2 pi) is phi / (2 pi) (column a fired at a / n_az); a point is
 * projected with the pose at t = 1/2, then rs_iters - 1 more times with the pose at the time
 * of its previous projection (fixed point t = time(g(x; pose(t)))). */
bool project_point(const orc_sensor* s, const double xw[3], double uv[2], double* margin) {
  double R[9], o[3];
  if (!s->moving) {
    pose_at(s, 0.0, R, o);
    return project_point_pose(s, R, o, xw, uv, margin);
  }
  double t = 0.5;
  for (int it = 0; it < std::max(s->rs_iters, 1); ++it) {
    pose_at(s, t, R, o);
    if (!project_point_pose(s, R, o, xw, uv, margin)) return false;
    if (s->kind == 2) {
      t = uv[0] / (2 * kPi);
      *margin = std::min(*margin, std::min(uv[0], 2 * kPi - uv[0]));   /* the sweep's seam */
    } else {
      t = std::min(std::max(uv[1] / s->height, 0.0), 1.0);
    }
  }
  return true;
}

bool project_point_pose(const orc_sensor* s, const double R[9], const double o[3], const double xw[3],
                        double uv[2], double* margin) {
  double p[3];
  to_sensor_pose(R, o, xw, p);
  const double x = p[0], y = p[1], z = p[2];
  switch (s->kind) {
    case 0: {
      *margin = std::min(*margin, std::fabs(z - s->near_));
      if (!(z > s->near_)) return false;
      uv[0] = s->fx * x / z + s->cx;
      uv[1] = s->fy * y / z + s->cy;
      return true;
    }
    case 3: {
      *margin = std::min(*margin, std::fabs(z - s->near_));
      if (!(z > s->near_)) return false;
      uv[0] = s->fx * x + s->cx;
      uv[1] = s->fy * y + s->cy;
      return true;
    }
    case 1: {
      const double r = std::sqrt(x * x + y * y + z * z);
      const double rho = std::sqrt(x * x + y * y);
      const double theta = std::atan2(rho, z);
      *margin = std::min(*margin, std::min(std::fabs(r - s->near_), std::fabs(theta - s->theta_max)));
      if (!(r > s->near_) || !(theta <= s->theta_max)) return false;
      const double t2 = theta * theta;
      const double td = theta * (1 + s->k[0] * t2 + s->k[1] * t2 * t2 + s->k[2] * t2 * t2 * t2 +
                                 s->k[3] * t2 * t2 * t2 * t2);
      if (rho > 0) {
        uv[0] = s->cx + s->fx * td * x / rho;
        uv[1] = s->cy + s->fy * td * y / rho;
      } else {
        uv[0] = s->cx;
        uv[1] = s->cy;
      }
      return true;
    }
    case 2: {
      const double r = std::sqrt(x * x + y * y + z * z);
      *margin = std::min(*margin, std::fabs(r - s->near_));
      if (!(r > s->near_)) return false;
      double phi = std::atan2(y, x);
      if (phi < 0) phi += 2 * kPi;
      uv[0] = phi;
      uv[1] = std::asin(z / r);
      return true;
    }
  }
  return false;
}

/* ------------------------------------------------------------------------------------
 * Unscented transform (Sec. 3.2, "Particle Contributions and Response": 7 sigma points
 * project to a 2D conic).  READING: the scaled UT of Julier & Uhlmann / Wan & van der
 * Merwe with n = 3, lambda = a^2 (n + kappa) - n, sigma points mu +- sqrt(n + lambda)
 * s_j R[:,j] (columns of the square root R S), weights Wm0 = lambda/(n+lambda),
 * Wc0 = Wm0 + 1 - a^2 + b, Wi = 1/(2(n+lambda)).  Any invalid sigma point culls the particle.
 * For LiDAR the sigma azimuths are unwrapped into (phi0 - pi, phi0 + pi].
 * ---------------------------------------------------------------------------------- */
bool unscented_transform(const orc_sensor* s, const Particle& p, const orc_params* prm,
                         double m[2], double cov[3], double* margin) {
  const int n = 3;
  const double a = prm->ut_alpha, b = prm->ut_beta, kap = prm->ut_kappa;
  const double lambda = a * a * (n + kap) - n;
  const double c = n + lambda;
  if (!(c > 0)) return false;
  const double gamma = std::sqrt(c);
  double pts[7][3];
  for (int d = 0; d < 3; ++d) pts[0][d] = p.mu[d];
  for (int j = 0; j < 3; ++j)
    for (int d = 0; d < 3; ++d) {
      const double col = p.filtered ? p.L[d * 3 + j] : p.s[j] * p.R[d * 3 + j];   /* sqrt(Sigma) column j */
      pts[1 + j][d] = p.mu[d] + gamma * col;
      pts[4 + j][d] = p.mu[d] - gamma * col;
    }
  double g[7][2];
  for (int k = 0; k < 7; ++k)
    if (!project_point(s, pts[k], g[k], margin)) return false;
  if (s->kind == 2) {
    for (int k = 1; k < 7; ++k) {
      while (g[k][0] - g[0][0] > kPi) g[k][0] -= 2 * kPi;
      while (g[k][0] - g[0][0] <= -kPi) g[k][0] += 2 * kPi;
    }
  }
  const double wm0 = lambda / c, wc0 = lambda / c + 1 - a * a + b, wi = 1.0 / (2 * c);
  m[0] = m[1] = 0;
  for (int k = 0; k < 7; ++k) {
    const double w = k == 0 ? wm0 : wi;
    m[0] += w * g[k][0];
    m[1] += w * g[k][1];
  }
  cov[0] = cov[1] = cov[2] = 0;
  for (int k = 0; k < 7; ++k) {
    const double w = k == 0 ? wc0 : wi;
    const double du = g[k][0] - m[0], dv = g[k][1] - m[1];
    cov[0] += w * du * du;
    cov[1] += w * du * dv;
    cov[2] += w * dv * dv;
  }
  return std::isfinite(cov[0]) && std::isfinite(cov[2]) && cov[0] >= 0 && cov[2] >= 0;
}

double frac_dist(double v) { return std::fabs(v - std::nearbyint(v)); }

int sensor_tiles_x(const orc_sensor* s) {
  return s->kind == 2 ? s->n_theta : (s->width + s->tile - 1) / s->tile;
}
int sensor_tiles_y(const orc_sensor* s) {
  return s->kind == 2 ? s->n_phi : (s->height + s->tile - 1) / s->tile;
}

/* SAT query over culling cells [x0,x1] x [y0,y1] (Alg. 2: n = A - B - C + D). */
long sat_query(const orc_sensor* s, int x0, int x1, int y0, int y1) {
  const int W = s->cull_el + 1;
  auto S = [&](int i, int j) { return (long)s->sat[(long)i * W + j]; };
  return S(x1 + 1, y1 + 1) - S(x0, y1 + 1) - S(x1 + 1, y0) + S(x0, y0);
}

}  // namespace

extern "C" {

/* ------------------------------------------------------------------------------------
 * Alg. 1 (ElevationTiling), Sec. 3.3 "Tiling".  READING of the garbled listing: the loop
 * runs over the r histogram bins; a boundary is placed at the upper edge (i+1) of every
 * bin where the cumulative count crosses b/N_phi of the total (integer comparison
 * C_i * N_phi >= b * C_max, repeated while it holds); boundaries are offset by Phi_min;
 * N_theta = ceil(max rays per elevation tile / M).  Histogram of per-ray elevations =
 * per-beam elevations weighted by n_az.  Beam b is in tile k iff T_k <= e_b < T_{k+1}
 * (last tile closed).
 * ---------------------------------------------------------------------------------- */
int orc_lidar_tiling(const float* beam_elev, int n_beams, int n_az, int n_phi, int M, int r_bins,
                     double* bounds_out, int* beam_start_out, int* n_theta_out) {
  if (n_beams <= 0 || n_phi <= 0 || M <= 0 || r_bins <= 0 || n_az <= 0) return -1;
  double emin = beam_elev[0], emax = beam_elev[0];
  for (int b = 0; b < n_beams; ++b) {
    emin = std::min(emin, (double)beam_elev[b]);
    emax = std::max(emax, (double)beam_elev[b]);
  }
  if (!(emax > emin)) return -1;
  const double w = (emax - emin) / r_bins;
  std::vector<long> H(r_bins, 0), C(r_bins, 0);
  for (int b = 0; b < n_beams; ++b) {
    int bin = (int)std::floor(((double)beam_elev[b] - emin) / w);
    bin = std::min(std::max(bin, 0), r_bins - 1);
    H[bin] += n_az;
  }
  long run = 0;
  for (int i = 0; i < r_bins; ++i) { run += H[i]; C[i] = run; }
  const long Cmax = C[r_bins - 1];
  std::vector<int> T;
  T.push_back(0);
  int b = 1;
  for (int i = 0; i < r_bins; ++i)
    while (b <= n_phi && C[i] * (long)n_phi >= (long)b * Cmax) { T.push_back(i + 1); ++b; }
  for (int k = 0; k <= n_phi; ++k) bounds_out[k] = emin + T[k] * w;
  /* beams per tile, then re-histogram in rays */
  long hmax = 0;
  int beam = 0;
  for (int k = 0; k < n_phi; ++k) {
    beam_start_out[k] = beam;
    const bool last = (k == n_phi - 1);
    while (beam < n_beams && ((double)beam_elev[beam] < bounds_out[k + 1] || last)) ++beam;
    hmax = std::max(hmax, (long)(beam - beam_start_out[k]) * n_az);
  }
  beam_start_out[n_phi] = n_beams;
  *n_theta_out = (int)((hmax + M - 1) / M);
  return 0;
}

/* Ray mask over the culling grid and its summed-area table (Sec. 3.3 "Ray-based Culling",
 * Appendix B).  READING: cull_az uniform azimuth cells over [0, 2 pi); cull_el uniform
 * elevation cells over [T_0, T_{N_phi}]; ray (b, a) lies in azimuth cell floor(a cull_az / n_az)
 * and elevation cell min(floor((e_b - T_0) cull_el / (T_N - T_0)), cull_el - 1).
 * sat[i][j] = number of occupied cells with azimuth < i and elevation < j. */
int orc_ray_sat(const float* beam_elev, int n_beams, int n_az, double emin, double emax,
                int cull_az, int cull_el, int* mask_out, int* sat_out) {
  std::vector<int> mask((size_t)cull_az * cull_el, 0);
  for (int b = 0; b < n_beams; ++b) {
    int ce = (int)std::floor(((double)beam_elev[b] - emin) * cull_el / (emax - emin));
    ce = std::min(std::max(ce, 0), cull_el - 1);
    for (int a = 0; a < n_az; ++a) {
      const int ca = (int)((long)a * cull_az / n_az);
      mask[(size_t)ca * cull_el + ce] = 1;
    }
  }
  const int W = cull_el + 1;
  for (int i = 0; i <= cull_az; ++i)
    for (int j = 0; j <= cull_el; ++j) {
      long v = 0;
      if (i > 0 && j > 0)
        v = (long)sat_out[(size_t)(i - 1) * W + j] + sat_out[(size_t)i * W + (j - 1)] -
            sat_out[(size_t)(i - 1) * W + (j - 1)] + mask[(size_t)(i - 1) * cull_el + (j - 1)];
      sat_out[(size_t)i * W + j] = (int)v;
    }
  if (mask_out) std::memcpy(mask_out, mask.data(), mask.size() * sizeof(int));
  return 0;
}

/* ------------------------------------------------------------------------------------
 * Projection of every particle: UT moments, 3-sigma extent, tile rect (Sec. 3.2 "tiling
 * and culling as in 3DGS"), LiDAR ray-based culling (Alg. 2, Alg. 3), depth key, features.
 * READING: extent e = 3 sqrt(diag Sigma'); camera tiles floor((m -+ e)/tile) clamped to the
 * image; LiDAR azimuth tiles floor(phi N_theta / 2 pi) wrapping modulo N_theta, elevation
 * tiles by the tiling boundaries; depth key = float32 squared distance to the sensor
 * origin, computed ((dx*dx + dy*dy) + dz*dz) with dx = mu_x - o_x, all float32.
 * ---------------------------------------------------------------------------------- */
int orc_project(const orc_gaussians* g, const orc_sensor* s, const orc_params* prm,
                orc_projected* out) {
  const int n = g->n;
  const int TX = sensor_tiles_x(s), TY = sensor_tiles_y(s);
  int n_inv = 0, n_cull = 0;
  const double o[3] = {s->origin[0], s->origin[1], s->origin[2]};
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : n_inv, n_cull)
  for (int i = 0; i < n; ++i) {
    Particle p = make_particle(g, i);
    apply_beam_divergence(s, p);
    double margin = 1e300, m[2] = {0, 0}, cov[3] = {0, 0, 0};
    bool ok = p.ok && unscented_transform(s, p, prm, m, cov, &margin);
    int x0 = 0, y0 = 0, x1 = -1, y1 = -1;
    uint32_t count = 0;
    if (ok) {
      const double eu = 3 * std::sqrt(cov[0]), ev = 3 * std::sqrt(cov[2]);
      if (s->kind != 2) {
        const double a0 = (m[0] - eu) / s->tile, a1 = (m[0] + eu) / s->tile;
        const double b0 = (m[1] - ev) / s->tile, b1 = (m[1] + ev) / s->tile;
        margin = std::min({margin, frac_dist(a0), frac_dist(a1), frac_dist(b0), frac_dist(b1)});
        x0 = (int)std::max(std::floor(a0), -1.0); x1 = (int)std::min(std::floor(a1), (double)TX);
        y0 = (int)std::max(std::floor(b0), -1.0); y1 = (int)std::min(std::floor(b1), (double)TY);
        if (x1 < 0 || y1 < 0 || x0 > TX - 1 || y0 > TY - 1) {
          x0 = y0 = 0; x1 = y1 = -1;
        } else {
          x0 = std::max(x0, 0); y0 = std::max(y0, 0);
          x1 = std::min(x1, TX - 1); y1 = std::min(y1, TY - 1);
          count = (uint32_t)((x1 - x0 + 1) * (y1 - y0 + 1));
        }
      } else {
        const double lo = m[1] - ev, hi = m[1] + ev;
        const double* T = s->elev_bounds;
        const int NP = s->n_phi;
        for (int k = 0; k <= NP; ++k)
          margin = std::min({margin, std::fabs(lo - T[k]), std::fabs(hi - T[k])});
        if (!(hi < T[0] || lo > T[NP])) {
          int e0 = 0, e1 = 0;
          for (int k = 1; k < NP; ++k) { if (T[k] <= lo) e0 = k; if (T[k] <= hi) e1 = k; }
          const double f0 = (m[0] - eu) * s->n_theta / (2 * kPi);
          const double f1 = (m[0] + eu) * s->n_theta / (2 * kPi);
          margin = std::min({margin, frac_dist(f0), frac_dist(f1)});
          /* an extent of at least 2 pi covers every azimuth tile */
          const bool full_az = eu >= kPi;
          long a0 = full_az ? 0 : (long)std::floor(f0), a1 = full_az ? s->n_theta - 1 : (long)std::floor(f1);
          if (a1 - a0 + 1 >= s->n_theta) { a0 = 0; a1 = s->n_theta - 1; }
          else {
            long a0w = ((a0 % s->n_theta) + s->n_theta) % s->n_theta;
            a1 = a0w + (a1 - a0);
            a0 = a0w;
          }
          x0 = (int)a0; x1 = (int)a1; y0 = e0; y1 = e1;
          count = (uint32_t)((x1 - x0 + 1) * (y1 - y0 + 1));
          if (s->cull) {
            /* Alg. 2 / Alg. 3: occupancy of the extent in the denser culling grid */
            const double span = T[NP] - T[0];
            const double c0 = (m[0] - eu) * s->cull_az / (2 * kPi);
            const double c1 = (m[0] + eu) * s->cull_az / (2 * kPi);
            const double r0 = (lo - T[0]) * s->cull_el / span, r1 = (hi - T[0]) * s->cull_el / span;
            margin = std::min({margin, frac_dist(c0), frac_dist(c1), frac_dist(r0), frac_dist(r1)});
            long ca0 = full_az ? 0 : (long)std::floor(c0), ca1 = full_az ? s->cull_az - 1 : (long)std::floor(c1);
            int ce0 = (int)std::max(std::floor(r0), 0.0), ce1 = (int)std::min(std::floor(r1), (double)(s->cull_el - 1));
            long occ = 0;
            if (ce0 <= ce1) {
              if (ca1 - ca0 + 1 >= s->cull_az) occ = sat_query(s, 0, s->cull_az - 1, ce0, ce1);
              else {
                const long w0 = ((ca0 % s->cull_az) + s->cull_az) % s->cull_az;
                const long w1 = w0 + (ca1 - ca0);
                if (w1 < s->cull_az) occ = sat_query(s, (int)w0, (int)w1, ce0, ce1);
                else occ = sat_query(s, (int)w0, s->cull_az - 1, ce0, ce1) +
                           sat_query(s, 0, (int)(w1 - s->cull_az), ce0, ce1);
              }
            }
            if (occ == 0) { count = 0; ++n_cull; }
          }
        } else {
          x0 = y0 = 0; x1 = y1 = -1;
        }
      }
    } else {
      ++n_inv;
    }
    out->valid[i] = ok ? 1 : 0;
    out->mean2[i] = m[0]; out->mean2[n + i] = m[1];
    out->cov2[i] = cov[0]; out->cov2[n + i] = cov[1]; out->cov2[2 * n + i] = cov[2];
    out->rect[i] = x0; out->rect[n + i] = y0; out->rect[2 * n + i] = x1; out->rect[3 * n + i] = y1;
    out->count[i] = count;
    out->margin[i] = margin;
    /* depth key (float32 arithmetic by definition) */
    const float dx = (float)g->mean[i] - s->origin[0];
    const float dy = (float)g->mean[n + i] - s->origin[1];
    const float dz = (float)g->mean[2 * n + i] - s->origin[2];
    const float xx = dx * dx, yy = dy * dy, zz = dz * dz;
    const float key = (xx + yy) + zz;
    uint32_t bits;
    std::memcpy(&bits, &key, 4);
    out->key[i] = bits;
    double f[3] = {0, 0, 0};
    int cl[3];
    if (p.ok) gaussian_features(g, i, p.mu, o, f, cl);
    for (int c = 0; c < 3; ++c) out->feat[c * n + i] = f[c];
  }
  out->n_culled_invalid = n_inv;
  out->n_culled_rays = n_cull;
  return 0;
}

/* Tile lists: every (tile, particle) pair of a non-zero count, ordered by (tile, depth key,
 * particle index) -- std::stable_sort on (tile, key) over pairs emitted in index order.
 * ranges[2][n_tiles] = [start, end).  pairs_* must hold sum(count) entries. */
uint64_t orc_count_pairs(const uint32_t* count, int n) {
  uint64_t t = 0;
  for (int i = 0; i < n; ++i) t += count[i];
  return t;
}

int orc_bin(const orc_sensor* s, int n, const int* rect, const uint32_t* count, const uint32_t* key,
            uint32_t* pair_tile, uint32_t* pair_gauss, uint32_t* ranges) {
  const int TX = sensor_tiles_x(s), TY = sensor_tiles_y(s);
  struct Pair { uint32_t tile, key, g; };
  std::vector<Pair> pairs;
  for (int i = 0; i < n; ++i) {
    if (count[i] == 0) continue;
    const int x0 = rect[i], y0 = rect[n + i], x1 = rect[2 * n + i], y1 = rect[3 * n + i];
    for (int y = y0; y <= y1; ++y)
      for (int x = x0; x <= x1; ++x) {
        const int xt = (s->kind == 2) ? (x % TX) : x;
        pairs.push_back({(uint32_t)(y * TX + xt), key[i], (uint32_t)i});
      }
  }
  std::stable_sort(pairs.begin(), pairs.end(), [](const Pair& a, const Pair& b) {
    return a.tile != b.tile ? a.tile < b.tile : a.key < b.key;
  });
  const int NT = TX * TY;
  for (int t = 0; t < 2 * NT; ++t) ranges[t] = 0;
  for (size_t j = 0; j < pairs.size(); ++j) {
    pair_tile[j] = pairs[j].tile;
    pair_gauss[j] = pairs[j].g;
    if (j == 0 || pairs[j - 1].tile != pairs[j].tile) ranges[pairs[j].tile] = (uint32_t)j;
    ranges[NT + pairs[j].tile] = (uint32_t)(j + 1);
  }
  return 0;
}

}  /* extern "C" */

namespace {

/* ------------------------------------------------------------------------------------
 * Compositing (Eq. 1) with the 3D particle response evaluated at the distance of maximum
 * response along the ray (Sec. 3.2, following 3DGRT):
 *   v = mu - o;  tau* = d^T B v / d^T B d  (B = Sigma^{-1});  y = o + tau* d - mu;
 *   rho = exp(-y^T B y / 2);  alpha = min(sigma rho, alpha_max);  skipped if alpha < alpha_min
 *   or tau* < near;  w = alpha T;  C += w c;  depth += w tau*;  omega += w;  T *= 1 - alpha;
 *   stop after the particle that brings T below t_min.
 * READING: alpha_min = 1/255, alpha_max = 0.99, t_min = 1e-4 (3DGS practice), depth is the
 * unnormalised sum of w tau*, colour is premultiplied (background left to the caller).
 * ---------------------------------------------------------------------------------- */
struct Contrib {
  uint32_t g;
  int clamped;
};

struct PerGaussian {
  std::vector<Particle> P;
  std::vector<double> feat;   /* [3][n] */
  std::vector<int> clamp;     /* [3][n] */
};

PerGaussian per_gaussian(const orc_gaussians* g, const orc_sensor* s) {
  PerGaussian pg;
  const int n = g->n;
  pg.P.resize(n);
  pg.feat.assign(3 * (size_t)n, 0.0);
  pg.clamp.assign(3 * (size_t)n, 0);
  const double o[3] = {s->origin[0], s->origin[1], s->origin[2]};
#pragma omp parallel for schedule(static)
  for (int i = 0; i < n; ++i) {
    pg.P[i] = make_particle(g, i);
    apply_beam_divergence(s, pg.P[i]);
    double f[3] = {0, 0, 0};
    int cl[3] = {0, 0, 0};
    if (pg.P[i].ok) gaussian_features(g, i, pg.P[i].mu, o, f, cl);
    for (int c = 0; c < 3; ++c) { pg.feat[c * (size_t)n + i] = f[c]; pg.clamp[c * (size_t)n + i] = cl[c]; }
  }
  return pg;
}

struct Response {
  double tau, D2, rho;
  double y[3], Bd[3], dBd;
};

Response response(const Particle& p, const double o[3], const double d[3]) {
  Response r;
  double v[3] = {p.mu[0] - o[0], p.mu[1] - o[1], p.mu[2] - o[2]};
  for (int a = 0; a < 3; ++a) r.Bd[a] = p.Binv[a * 3] * d[0] + p.Binv[a * 3 + 1] * d[1] + p.Binv[a * 3 + 2] * d[2];
  r.dBd = d[0] * r.Bd[0] + d[1] * r.Bd[1] + d[2] * r.Bd[2];
  r.tau = (v[0] * r.Bd[0] + v[1] * r.Bd[1] + v[2] * r.Bd[2]) / r.dBd;
  for (int a = 0; a < 3; ++a) r.y[a] = o[a] + r.tau * d[a] - p.mu[a];
  double By[3];
  for (int a = 0; a < 3; ++a) By[a] = p.Binv[a * 3] * r.y[0] + p.Binv[a * 3 + 1] * r.y[1] + p.Binv[a * 3 + 2] * r.y[2];
  r.D2 = r.y[0] * By[0] + r.y[1] * By[1] + r.y[2] * By[2];
  r.rho = std::exp(-0.5 * r.D2);
  return r;
}

struct RayResult {
  double feat[3], depth, omega, T;
  uint32_t nproc;
  double margin; /* smallest relative distance of a skip / clamp / stop decision to its threshold */
};

void ray_geometry(const orc_sensor* s, int r, long R, double o[3], double d[3]) {
  for (int a = 0; a < 3; ++a) {
    o[a] = s->moving ? (double)s->ray_org[a * R + r] : (double)s->origin[a];
    d[a] = s->ray_dir[a * R + r];
  }
}

bool ray_valid(const double d[3]) { return d[0] != 0 || d[1] != 0 || d[2] != 0; }

RayResult composite_ray(const PerGaussian& pg, int n, const orc_params* prm, double near_,
                        const double o[3], const double d[3], const uint32_t* list, uint32_t len,
                        std::vector<Contrib>* rec) {
  RayResult rr;
  std::memset(&rr, 0, sizeof rr);
  rr.T = 1.0;
  rr.margin = 1e300;
  if (!ray_valid(d)) return rr;
  for (uint32_t j = 0; j < len; ++j) {
    const uint32_t gi = list[j];
    rr.nproc = j + 1;
    const Particle& p = pg.P[gi];
    const Response q = response(p, o, d);
    rr.margin = std::min(rr.margin, std::fabs(q.tau - near_) / std::max(std::fabs(near_), 1e-300));
    if (q.tau < near_) continue;
    const double a = p.sigma * q.rho;
    rr.margin = std::min({rr.margin, std::fabs(a - prm->alpha_min) / prm->alpha_min,
                          std::fabs(a - prm->alpha_max) / prm->alpha_max});
    const int clamped = a > prm->alpha_max;
    const double alpha = clamped ? prm->alpha_max : a;
    if (alpha < prm->alpha_min) continue;
    const double w = alpha * rr.T;
    for (int c = 0; c < 3; ++c) rr.feat[c] += w * pg.feat[c * (size_t)n + gi];
    rr.depth += w * q.tau;
    rr.omega += w;
    rr.T *= (1 - alpha);
    if (rec) rec->push_back({gi, clamped});
    if (prm->t_min > 0) rr.margin = std::min(rr.margin, std::fabs(rr.T - prm->t_min) / prm->t_min);
    if (rr.T < prm->t_min) break;
  }
  return rr;
}

/* rays of tile t: camera pixels of the 16x16 block; LiDAR beams of the elevation tile times
 * azimuth steps a with floor(a N_theta / n_az) equal to the azimuth tile. */
void tile_rays(const orc_sensor* s, int t, std::vector<int>& rays) {
  rays.clear();
  const int TX = sensor_tiles_x(s);
  const int tx = t % TX, ty = t / TX;
  if (s->kind != 2) {
    for (int y = ty * s->tile; y < std::min((ty + 1) * s->tile, s->height); ++y)
      for (int x = tx * s->tile; x < std::min((tx + 1) * s->tile, s->width); ++x)
        rays.push_back(y * s->width + x);
  } else {
    for (int b = s->beam_start[ty]; b < s->beam_start[ty + 1]; ++b)
      for (int a = 0; a < s->n_az; ++a)
        if ((long)a * s->n_theta / s->n_az == tx) rays.push_back(b * s->n_az + a);
  }
}

double softmax_drop(const double z[3]) {
  /* Sec. 3.2: ray-drop probability = softmax over (beta_hit, beta_drop) = channels 1, 2 */
  const double mx = std::max(z[1], z[2]);
  const double eh = std::exp(z[1] - mx), ed = std::exp(z[2] - mx);
  return ed / (eh + ed);
}

}  // namespace

extern "C" {

/* Composite every ray over its tile's list.  Outputs (R = number of rays):
 * feat[3][R] premultiplied colour (camera) or LiDAR features zeta, depth[R], omega[R],
 * t_final[R], nproc[R] (list entries visited), drop[R] (LiDAR ray-drop probability,
 * may be NULL).  mode 0: tiled lists; mode 1: brute force over all particles ordered by
 * (key, index) and gated by "the ray's tile lies in the particle's rect". */
int orc_composite(const orc_gaussians* g, const orc_sensor* s, const orc_params* prm,
                  const uint32_t* pair_gauss, const uint32_t* ranges, int mode,
                  const int* rect, const uint32_t* count, const uint32_t* key,
                  double* feat, double* depth, double* omega, double* t_final, uint32_t* nproc,
                  double* drop, double* margin) {
  const int n = g->n;
  const PerGaussian pg = per_gaussian(g, s);
  const int TX = sensor_tiles_x(s), TY = sensor_tiles_y(s), NT = TX * TY;
  const long R = (s->kind == 2) ? (long)s->n_beams * s->n_az : (long)s->width * s->height;
  std::vector<uint32_t> order;
  if (mode == 1) {
    for (int i = 0; i < n; ++i) if (count[i]) order.push_back(i);
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return key[a] < key[b]; });
  }
#pragma omp parallel for schedule(dynamic, 1)
  for (int t = 0; t < NT; ++t) {
    std::vector<int> rays;
    tile_rays(s, t, rays);
    std::vector<uint32_t> list;
    const uint32_t* lp;
    uint32_t len;
    if (mode == 0) { lp = pair_gauss + ranges[t]; len = ranges[NT + t] - ranges[t]; }
    else {
      const int tx = t % TX, ty = t / TX;
      for (uint32_t gi : order) {
        const int x0 = rect[gi], y0 = rect[n + gi], x1 = rect[2 * n + gi], y1 = rect[3 * n + gi];
        bool in_y = ty >= y0 && ty <= y1, in_x;
        if (s->kind == 2) in_x = ((tx - x0) % TX + TX) % TX <= x1 - x0;
        else in_x = tx >= x0 && tx <= x1;
        if (in_x && in_y) list.push_back(gi);
      }
      lp = list.data();
      len = (uint32_t)list.size();
    }
    for (int r : rays) {
      double o[3], d[3];
      ray_geometry(s, r, R, o, d);
      const RayResult rr = composite_ray(pg, n, prm, s->near_, o, d, lp, len, nullptr);
      for (int c = 0; c < 3; ++c) feat[c * R + r] = rr.feat[c];
      depth[r] = rr.depth;
      omega[r] = rr.omega;
      t_final[r] = rr.T;
      nproc[r] = rr.nproc;
      if (drop) drop[r] = softmax_drop(rr.feat);
      if (margin) margin[r] = rr.margin;
    }
  }
  return 0;
}

/* Composite only the listed rays (tiled lists); outputs are indexed like ray_ids. */
int orc_composite_rays(const orc_gaussians* g, const orc_sensor* s, const orc_params* prm,
                       const uint32_t* pair_gauss, const uint32_t* ranges, const long* ray_ids, int m,
                       double* feat, double* depth, double* omega, double* t_final, uint32_t* nproc,
                       double* drop, double* margin) {
  const int n = g->n;
  const PerGaussian pg = per_gaussian(g, s);
  const int TX = sensor_tiles_x(s), TY = sensor_tiles_y(s), NT = TX * TY;
  const long R = (s->kind == 2) ? (long)s->n_beams * s->n_az : (long)s->width * s->height;
#pragma omp parallel for schedule(dynamic, 16)
  for (int i = 0; i < m; ++i) {
    const long r = ray_ids[i];
    int t;
    if (s->kind != 2) {
      t = (int)((r / s->width) / s->tile) * TX + (int)((r % s->width) / s->tile);
    } else {
      const int b = (int)(r / s->n_az), a = (int)(r % s->n_az);
      int k = 0;
      while (k + 1 < s->n_phi && s->beam_start[k + 1] <= b) ++k;
      t = k * TX + (int)((long)a * s->n_theta / s->n_az);
    }
    double o[3], d[3];
    ray_geometry(s, (int)r, R, o, d);
    const RayResult rr = composite_ray(pg, n, prm, s->near_, o, d, pair_gauss + ranges[t],
                                       ranges[NT + t] - ranges[t], nullptr);
    for (int c = 0; c < 3; ++c) feat[c * (long)m + i] = rr.feat[c];
    depth[i] = rr.depth;
    omega[i] = rr.omega;
    t_final[i] = rr.T;
    nproc[i] = rr.nproc;
    if (drop) drop[i] = softmax_drop(rr.feat);
    if (margin) margin[i] = rr.margin;
  }
  (void)TY;
  return 0;
}

}  /* extern "C" */

namespace {

/* ------------------------------------------------------------------------------------
 * Adjoint.  Differentiated function = the forward above with its discrete structure held
 * fixed (tile lists, culls, the alpha_min skip, the alpha_max clamp, the colour clamp and
 * the termination index).  Upstream per ray: g_feat[3], g_depth, g_omega and (LiDAR)
 * g_drop.  Chain: features -> SH coefficients and (through the SH direction) the mean;
 * alpha -> opacity and D^2; D^2, tau* -> mean and B = Sigma^{-1}; B -> Sigma -> (R, s)
 * -> (normalised quaternion, log-scale) -> raw quaternion.
 * ---------------------------------------------------------------------------------- */
struct GradAcc {
  double dfeat[3], dsigma, dmu[3], dB[9];
};

struct Upstream {
  const double *g_feat, *g_depth, *g_omega, *g_drop; /* g_drop may be NULL */
};

/* per-ray adjoint given the forward's contributing sequence */
void ray_adjoint(const PerGaussian& pg, int n, const orc_params* prm, const double o[3],
                 const double d[3], const std::vector<Contrib>& seq, const double gf_in[3],
                 double g_depth, double g_omega, double g_drop, std::vector<GradAcc>& acc) {
  const size_t m = seq.size();
  if (m == 0) return;
  std::vector<Response> rs(m);
  std::vector<double> alpha(m), T(m);
  double t = 1.0, zeta[3] = {0, 0, 0};
  for (size_t i = 0; i < m; ++i) {
    const Particle& p = pg.P[seq[i].g];
    rs[i] = response(p, o, d);
    alpha[i] = seq[i].clamped ? prm->alpha_max : p.sigma * rs[i].rho;
    T[i] = t;
    for (int c = 0; c < 3; ++c) zeta[c] += alpha[i] * t * pg.feat[c * (size_t)n + seq[i].g];
    t *= 1 - alpha[i];
  }
  const double Tfinal = t;
  double gf[3] = {gf_in[0], gf_in[1], gf_in[2]};
  if (g_drop != 0) {
    const double pd = softmax_drop(zeta);
    gf[1] += -g_drop * pd * (1 - pd);
    gf[2] += g_drop * pd * (1 - pd);
  }
  double suffix = 0; /* sum over later contributions of w_j (g . c_j + g_depth tau_j) */
  for (size_t ii = m; ii-- > 0;) {
    const uint32_t gi = seq[ii].g;
    const Particle& p = pg.P[gi];
    const Response& q = rs[ii];
    const double w = alpha[ii] * T[ii];
    double a_i = g_depth * q.tau;
    for (int c = 0; c < 3; ++c) a_i += gf[c] * pg.feat[c * (size_t)n + gi];
    const double dalpha = T[ii] * a_i - suffix / (1 - alpha[ii]) + g_omega * Tfinal / (1 - alpha[ii]);
    suffix += w * a_i;
    GradAcc& A = acc[gi];
    for (int c = 0; c < 3; ++c) A.dfeat[c] += gf[c] * w;
    const double dtau = g_depth * w;
    double dD2 = 0;
    if (!seq[ii].clamped) {
      A.dsigma += dalpha * q.rho;
      dD2 = dalpha * p.sigma * q.rho * (-0.5);
    }
    /* D2 = min_t (t d - v)^T B (t d - v): dD2/dv = -2 B y, dD2/dB = y y^T (y = t* d - v) */
    double By[3];
    for (int a = 0; a < 3; ++a) By[a] = p.Binv[a * 3] * q.y[0] + p.Binv[a * 3 + 1] * q.y[1] + p.Binv[a * 3 + 2] * q.y[2];
    /* tau = d^T B v / d^T B d: dtau/dv = B d / dBd, dtau/dB = -sym(d y^T) / dBd */
    for (int a = 0; a < 3; ++a) A.dmu[a] += dD2 * (-2 * By[a]) + dtau * q.Bd[a] / q.dBd;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        A.dB[a * 3 + b] += dD2 * q.y[a] * q.y[b] - dtau * 0.5 * (d[a] * q.y[b] + q.y[a] * d[b]) / q.dBd;
  }
}

void chain_to_params(const orc_gaussians* g, const orc_sensor* s, const PerGaussian& pg,
                     const std::vector<GradAcc>& acc, double* d_mean, double* d_quat,
                     double* d_log_scale, double* d_logit, double* d_feat) {
  const int n = g->n;
  const int K = (g->sh_degree + 1) * (g->sh_degree + 1);
  const double o[3] = {s->origin[0], s->origin[1], s->origin[2]};
#pragma omp parallel for schedule(static)
  for (int i = 0; i < n; ++i) {
    const Particle& p = pg.P[i];
    const GradAcc& A = acc[i];
    for (int a = 0; a < 3; ++a) d_mean[a * n + i] = 0, d_log_scale[a * n + i] = 0;
    for (int a = 0; a < 4; ++a) d_quat[a * n + i] = 0;
    d_logit[i] = 0;
    for (int k = 0; k < K; ++k) for (int c = 0; c < 3; ++c) d_feat[(k * 3 + c) * n + i] = 0;
    if (!p.ok) continue;
    /* opacity */
    d_logit[i] = A.dsigma * p.sigma * (1 - p.sigma);
    /* dL/dR and dL/dlog_scale from G = dL/dB (Sec. 3.2: Sigma = R S S^T R^T) */
    double GS[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    double GR[9];
    if (!p.filtered) {
      /* B = R diag(1/s^2) R^T: dL/dR = (G + G^T) R diag(1/s^2), dL/dlog_scale_j =
       * -2 (R^T G R)_jj / s_j^2.  The same derivative as the route through Sigma below, taken
       * without forming -B G B, whose entries reach (1/s_min^2)^2 |G| and leave the rotation
       * gradient of a thin particle to cancellation. */
      for (int a = 0; a < 3; ++a)
        for (int j = 0; j < 3; ++j) {
          double v = 0;
          for (int k = 0; k < 3; ++k) v += (A.dB[a * 3 + k] + A.dB[k * 3 + a]) * p.R[k * 3 + j];
          GR[a * 3 + j] = v / (p.s[j] * p.s[j]);
        }
      for (int j = 0; j < 3; ++j) {
        double v = 0;
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) v += p.R[a * 3 + j] * A.dB[a * 3 + b] * p.R[b * 3 + j];
        d_log_scale[j * n + i] = -2 * v / (p.s[j] * p.s[j]);
      }
    } else {
      /* B = Sigma_hat^{-1}: dL/dSigma_hat = -B G B */
      double GB[9];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          double v = 0;
          for (int k = 0; k < 3; ++k) v += A.dB[a * 3 + k] * p.Binv[k * 3 + b];
          GB[a * 3 + b] = v;
        }
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          double v = 0;
          for (int k = 0; k < 3; ++k) v += p.Binv[a * 3 + k] * GB[k * 3 + b];
          GS[a * 3 + b] = -v;
        }
      /* Sigma_hat = R diag(s^2) R^T + (smoothing, free of R and s) with GS symmetric:
       * dL/dR = (GS + GS^T) R diag(s^2), dL/ds_j = 2 s_j (R^T GS R)_jj,
       * dL/dlog_scale_j = s_j dL/ds_j */
      for (int a = 0; a < 3; ++a)
        for (int j = 0; j < 3; ++j) {
          double v = 0;
          for (int k = 0; k < 3; ++k) v += (GS[a * 3 + k] + GS[k * 3 + a]) * p.R[k * 3 + j];
          GR[a * 3 + j] = v * p.s[j] * p.s[j];
        }
      for (int j = 0; j < 3; ++j) {
        double v = 0;
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) v += p.R[a * 3 + j] * GS[a * 3 + b] * p.R[b * 3 + j];
        d_log_scale[j * n + i] = 2 * p.s[j] * v * p.s[j];
      }
    }
    double J[4][9], dqn[4];
    quat_to_rot_jacobian(p.qn, J);
    for (int k = 0; k < 4; ++k) {
      double v = 0;
      for (int e = 0; e < 9; ++e) v += GR[e] * J[k][e];
      dqn[k] = v;
    }
    const double dot = dqn[0] * p.qn[0] + dqn[1] * p.qn[1] + dqn[2] * p.qn[2] + dqn[3] * p.qn[3];
    for (int k = 0; k < 4; ++k) d_quat[k * n + i] = (dqn[k] - p.qn[k] * dot) / p.qnorm;
    /* features: SH coefficients and the SH direction */
    double v[3] = {p.mu[0] - o[0], p.mu[1] - o[1], p.mu[2] - o[2]};
    const double len = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    double dir[3] = {0, 0, 1};
    if (len > 0) for (int a = 0; a < 3; ++a) dir[a] = v[a] / len;
    double Y[16], dY[16][3];
    sh_basis().eval(g->sh_degree, dir, Y, dY);
    double ddir[3] = {0, 0, 0};
    for (int c = 0; c < 3; ++c) {
      const double dc = pg.clamp[c * (size_t)n + i] ? 0.0 : A.dfeat[c];
      for (int k = 0; k < K; ++k) {
        d_feat[(k * 3 + c) * n + i] = dc * Y[k];
        const double coef = g->feat[(k * 3 + c) * n + i];
        for (int a = 0; a < 3; ++a) ddir[a] += dc * coef * dY[k][a];
      }
    }
    double dmu[3] = {A.dmu[0], A.dmu[1], A.dmu[2]};
    /* beam divergence: Sigma_hat = Sigma + t^2 (|v|^2 I - v v^T), t = tan(theta/2), so GS also
     * reaches the mean, d/dv [GS : t^2 (|v|^2 I - v v^T)] = t^2 (2 tr(GS) v - (GS + GS^T) v) */
    if (p.filtered) {
      const double t = std::tan(0.5 * s->beam_divergence), t2 = t * t;
      const double tr = GS[0] + GS[4] + GS[8];
      for (int a = 0; a < 3; ++a) {
        double sv = 0;
        for (int b = 0; b < 3; ++b) sv += (GS[a * 3 + b] + GS[b * 3 + a]) * v[b];
        dmu[a] += t2 * (2 * tr * v[a] - sv);
      }
    }
    if (len > 0) {
      const double dd = ddir[0] * dir[0] + ddir[1] * dir[1] + ddir[2] * dir[2];
      for (int a = 0; a < 3; ++a) dmu[a] += (ddir[a] - dir[a] * dd) / len;
    }
    for (int a = 0; a < 3; ++a) d_mean[a * n + i] = dmu[a];
  }
}

struct Frozen {
  std::vector<std::vector<Contrib>> seq; /* per ray */
};

Frozen forward_record(const orc_gaussians* g, const orc_sensor* s, const orc_params* prm,
                      const PerGaussian& pg, const uint32_t* pair_gauss, const uint32_t* ranges,
                      const std::vector<char>& active) {
  const int TX = sensor_tiles_x(s), TY = sensor_tiles_y(s), NT = TX * TY;
  const long R = (s->kind == 2) ? (long)s->n_beams * s->n_az : (long)s->width * s->height;
  Frozen fz;
  fz.seq.resize(R);
#pragma omp parallel for schedule(dynamic, 1)
  for (int t = 0; t < NT; ++t) {
    std::vector<int> rays;
    tile_rays(s, t, rays);
    for (int r : rays) {
      if (!active[r]) continue;   /* no upstream on this ray: it adds nothing to the gradient */
      double o[3], d[3];
      ray_geometry(s, r, R, o, d);
      composite_ray(pg, g->n, prm, s->near_, o, d, pair_gauss + ranges[t], ranges[NT + t] - ranges[t], &fz.seq[r]);
    }
  }
  return fz;
}

/* Rays with a non-zero upstream gradient.  The functional is a sum over rays of upstream
 * times outputs, so a ray whose upstream is all zero contributes exactly zero: the adjoint
 * and the finite differences skip its forward sequence. */
std::vector<char> upstream_active(long R, const double* g_feat, const double* g_depth, const double* g_omega,
                                  const double* g_drop) {
  std::vector<char> a(R);
  for (long r = 0; r < R; ++r)
    a[r] = g_feat[r] != 0 || g_feat[R + r] != 0 || g_feat[2 * R + r] != 0 || g_depth[r] != 0 ||
           g_omega[r] != 0 || (g_drop && g_drop[r] != 0);
  return a;
}

/* value of the linear-in-outputs functional (plus the LiDAR drop term) on one ray, with
 * the frozen structure; features use frozen colour clamps */
double frozen_ray_value(const PerGaussian& pg, int n, const orc_params* prm, const double o[3],
                        const double d[3], const std::vector<Contrib>& seq, const double gf[3],
                        double g_depth, double g_omega, double g_drop) {
  double T = 1, f[3] = {0, 0, 0}, dep = 0, om = 0;
  for (const Contrib& c : seq) {
    const Particle& p = pg.P[c.g];
    const Response q = response(p, o, d);
    const double alpha = c.clamped ? prm->alpha_max : p.sigma * q.rho;
    const double w = alpha * T;
    for (int k = 0; k < 3; ++k) f[k] += w * pg.feat[k * (size_t)n + c.g];
    dep += w * q.tau;
    om += w;
    T *= 1 - alpha;
  }
  double v = gf[0] * f[0] + gf[1] * f[1] + gf[2] * f[2] + g_depth * dep + g_omega * om;
  if (g_drop != 0) v += g_drop * softmax_drop(f);
  return v;
}

}  // namespace

extern "C" {

/* Analytic FP64 gradient of sum_r (g_feat.feat + g_depth depth + g_omega omega + g_drop drop)
 * with respect to every particle parameter (frozen structure, see above). */
int orc_backward(const orc_gaussians* g, const orc_sensor* s, const orc_params* prm,
                 const uint32_t* pair_gauss, const uint32_t* ranges,
                 const double* g_feat, const double* g_depth, const double* g_omega,
                 const double* g_drop, double* d_mean, double* d_quat, double* d_log_scale,
                 double* d_logit, double* d_feat) {
  const int n = g->n;
  const PerGaussian pg = per_gaussian(g, s);
  const long R = (s->kind == 2) ? (long)s->n_beams * s->n_az : (long)s->width * s->height;
  const Frozen fz = forward_record(g, s, prm, pg, pair_gauss, ranges,
                                   upstream_active(R, g_feat, g_depth, g_omega, g_drop));
  std::vector<GradAcc> acc(n);
  std::memset(acc.data(), 0, sizeof(GradAcc) * n);
  for (long r = 0; r < R; ++r) {   /* serial: accumulation order fixed */
    double o[3], d[3];
    ray_geometry(s, (int)r, R, o, d);
    const double gf[3] = {g_feat[r], g_feat[R + r], g_feat[2 * R + r]};
    ray_adjoint(pg, n, prm, o, d, fz.seq[r], gf, g_depth[r], g_omega[r], g_drop ? g_drop[r] : 0.0, acc);
  }
  chain_to_params(g, s, pg, acc, d_mean, d_quat, d_log_scale, d_logit, d_feat);
  return 0;
}

/* Central finite differences (step h) of the same frozen-structure functional, for the
 * particles listed in sel[n_sel].  Parameter order per particle: mean(3), quat(4),
 * log_scale(3), logit(1), feat(3K); out[n_sel][11 + 3K].  The const parameter arrays are
 * copied and perturbed internally. */
int orc_fd_grad(const orc_gaussians* g, const orc_sensor* s, const orc_params* prm,
                const uint32_t* pair_gauss, const uint32_t* ranges,
                const double* g_feat, const double* g_depth, const double* g_omega,
                const double* g_drop, const int* sel, int n_sel, double h, double* out) {
  const int n = g->n;
  const int K = (g->sh_degree + 1) * (g->sh_degree + 1);
  const int NPAR = 11 + 3 * K;
  const PerGaussian pg0 = per_gaussian(g, s);
  const long R = (s->kind == 2) ? (long)s->n_beams * s->n_az : (long)s->width * s->height;
  const Frozen fz = forward_record(g, s, prm, pg0, pair_gauss, ranges,
                                   upstream_active(R, g_feat, g_depth, g_omega, g_drop));
  std::vector<std::vector<int>> rays_of(n);
  for (long r = 0; r < R; ++r)
    for (const Contrib& c : fz.seq[r])
      if (rays_of[c.g].empty() || rays_of[c.g].back() != (int)r) rays_of[c.g].push_back((int)r);
  const double o[3] = {s->origin[0], s->origin[1], s->origin[2]};
#pragma omp parallel for schedule(dynamic, 1)
  for (int si = 0; si < n_sel; ++si) {
    const int gi = sel[si];
    /* private copies of this particle's parameters inside a one-particle view */
    std::vector<double> mean(g->mean, g->mean + 3 * (size_t)n);
    std::vector<double> quat(g->quat, g->quat + 4 * (size_t)n);
    std::vector<double> ls(g->log_scale, g->log_scale + 3 * (size_t)n);
    std::vector<double> lg(g->opacity_logit, g->opacity_logit + n);
    std::vector<double> ft(g->feat, g->feat + 3 * (size_t)K * n);
    orc_gaussians gv = *g;
    gv.mean = mean.data(); gv.quat = quat.data(); gv.log_scale = ls.data();
    gv.opacity_logit = lg.data(); gv.feat = ft.data();
    PerGaussian pg = pg0;
    for (int pidx = 0; pidx < NPAR; ++pidx) {
      double* slot;
      if (pidx < 3) slot = &mean[pidx * (size_t)n + gi];
      else if (pidx < 7) slot = &quat[(pidx - 3) * (size_t)n + gi];
      else if (pidx < 10) slot = &ls[(pidx - 7) * (size_t)n + gi];
      else if (pidx < 11) slot = &lg[gi];
      else slot = &ft[(pidx - 11) * (size_t)n + gi];
      const double keep = *slot;
      double val[2];
      for (int side = 0; side < 2; ++side) {
        *slot = keep + (side ? -h : h);
        pg.P[gi] = make_particle(&gv, gi);
        apply_beam_divergence(s, pg.P[gi]);
        double f[3];
        sh_features_raw(&gv, gi, pg.P[gi].mu, o, f);
        for (int c = 0; c < 3; ++c)   /* colour clamp held at its unperturbed state */
          pg.feat[c * (size_t)n + gi] = pg0.clamp[c * (size_t)n + gi] ? 0.0 :
              (g->feat_kind == 0 ? f[c] + 0.5 : f[c]);
        double tot = 0;
        for (int r : rays_of[gi]) {
          double ro[3], rd[3];
          ray_geometry(s, r, R, ro, rd);
          const double gf[3] = {g_feat[r], g_feat[R + r], g_feat[2 * R + r]};
          tot += frozen_ray_value(pg, n, prm, ro, rd, fz.seq[r], gf, g_depth[r], g_omega[r],
                                  g_drop ? g_drop[r] : 0.0);
        }
        val[side] = tot;
      }
      *slot = keep;
      pg.P[gi] = pg0.P[gi];
      for (int c = 0; c < 3; ++c) pg.feat[c * (size_t)n + gi] = pg0.feat[c * (size_t)n + gi];
      out[(size_t)si * NPAR + pidx] = (val[0] - val[1]) / (2 * h);
    }
  }
  return 0;
}

/* Sets the OpenMP threads of the following calls (timing of the CPU baseline on one core). */
void orc_set_num_threads(int t) { omp_set_num_threads(t > 0 ? t : 1); }

/* OpenMP threads the oracle runs with. */
int orc_num_threads(void) {
  int t = 1;
#pragma omp parallel
  {
#pragma omp single
    t = omp_get_num_threads();
  }
  return t;
}

/* Plain SH values (for pinning the basis against an independent library). */
int orc_sh_eval(int deg, const double* dirs, int m, double* Y) {
  const int K = (deg + 1) * (deg + 1);
  for (int i = 0; i < m; ++i) {
    double y[16];
    sh_basis().eval(deg, dirs + 3 * i, y, nullptr);
    for (int k = 0; k < K; ++k) Y[(size_t)i * K + k] = y[k];
  }
  return 0;
}

/* Single-point sensor projection (for pinning the projection functions). */
/* pose of a (moving) sensor at frame time t: R[9] world->sensor rows, o[3] */
int orc_pose_at(const orc_sensor* s, double t, double* R, double* o) {
  pose_at(s, t, R, o);
  return 0;
}

int orc_project_points(const orc_sensor* s, const double* xw, int m, double* uv, int* ok) {
  for (int i = 0; i < m; ++i) {
    double margin = 1e300;
    ok[i] = project_point(s, xw + 3 * i, uv + 2 * i, &margin) ? 1 : 0;
  }
  return 0;
}

}  /* extern "C" */
