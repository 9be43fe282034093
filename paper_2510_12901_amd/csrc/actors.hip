// actors.hip -- rigid actor transforms of the scene graph (Sec. 3.1, scene representation).
//
// A dynamic object's particles live in the object's frame; at render time its SE(3) pose
// for the timestamp moves their means and covariances to the world: mu_w = R_a mu + t_a and,
// with Sigma = R(q) S S^T R(q)^T, the world quaternion q_w = q_a * q (Hamilton product).
// Scale, opacity and features are untouched, so the world set shares those arrays.
//
// k_actor_fwd: one lane per particle, 60 bytes of HBM traffic (actor id, mean and quaternion
// in, mean and quaternion out); the pose table is small and stays in the caches.  The
// transform runs once per timestamp, so every sensor rendered at that time shares it.
// k_actor_bwd: one lane per particle, the adjoint to the object-frame parameters and the
// pose (7 values per actor, reduced per wavefront when the wavefront holds one actor, as
// it does for particles stored actor by actor, else added lane by lane).
#include "ut_internal.hpp"

namespace ut {
namespace {

struct PoseK {
  double q[4];   // normalised rotation (w, x, y, z)
  double qn;     // |q| before normalisation
  double t[3];
  double R[9];
};

__device__ __forceinline__ PoseK load_pose(const ut_actor_pose* poses, int a) {
  const float4 lo = reinterpret_cast<const float4*>(poses + a)[0];
  const float4 hi = reinterpret_cast<const float4*>(poses + a)[1];
  PoseK p;
  const double w = lo.x, x = lo.y, y = lo.z, z = lo.w;
  p.qn = sqrt(w * w + x * x + y * y + z * z);
  const double iq = 1.0 / p.qn;
  p.q[0] = w * iq; p.q[1] = x * iq; p.q[2] = y * iq; p.q[3] = z * iq;
  p.t[0] = hi.x; p.t[1] = hi.y; p.t[2] = hi.z;
  const double qw = p.q[0], qx = p.q[1], qy = p.q[2], qz = p.q[3];
  p.R[0] = 1 - 2 * (qy * qy + qz * qz); p.R[1] = 2 * (qx * qy - qw * qz);     p.R[2] = 2 * (qx * qz + qw * qy);
  p.R[3] = 2 * (qx * qy + qw * qz);     p.R[4] = 1 - 2 * (qx * qx + qz * qz); p.R[5] = 2 * (qy * qz - qw * qx);
  p.R[6] = 2 * (qx * qz - qw * qy);     p.R[7] = 2 * (qy * qz + qw * qx);     p.R[8] = 1 - 2 * (qx * qx + qy * qy);
  return p;
}

// Hamilton product a * b, (w, x, y, z)
__device__ __forceinline__ void qmul(const double a[4], const double b[4], double r[4]) {
  r[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
  r[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
  r[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
  r[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}

__global__ __launch_bounds__(256) void k_actor_fwd(const float* __restrict__ mean, const float* __restrict__ quat,
                                                    const int32_t* __restrict__ actor,
                                                    const ut_actor_pose* __restrict__ poses, int n_act,
                                                    float* mean_w, float* quat_w, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int a = actor[i];
  float m[3] = {mean[i], mean[n + i], mean[2 * n + i]};
  float q[4] = {quat[i], quat[n + i], quat[2 * n + i], quat[3 * n + i]};
  if (a >= 0 && a < n_act) {
    const PoseK p = load_pose(poses, a);
    const double mx = m[0], my = m[1], mz = m[2];
    m[0] = (float)__builtin_fma(p.R[0], mx, __builtin_fma(p.R[1], my, __builtin_fma(p.R[2], mz, p.t[0])));
    m[1] = (float)__builtin_fma(p.R[3], mx, __builtin_fma(p.R[4], my, __builtin_fma(p.R[5], mz, p.t[1])));
    m[2] = (float)__builtin_fma(p.R[6], mx, __builtin_fma(p.R[7], my, __builtin_fma(p.R[8], mz, p.t[2])));
    const double qo[4] = {q[0], q[1], q[2], q[3]};
    double r[4];
    qmul(p.q, qo, r);
    q[0] = (float)r[0]; q[1] = (float)r[1]; q[2] = (float)r[2]; q[3] = (float)r[3];
  }
  mean_w[i] = m[0]; mean_w[n + i] = m[1]; mean_w[2 * n + i] = m[2];
  quat_w[i] = q[0]; quat_w[n + i] = q[1]; quat_w[2 * n + i] = q[2]; quat_w[3 * n + i] = q[3];
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Every lane of a launched wavefront stays active through the reductions (the grid is a
// whole number of workgroups; lanes past n contribute zeros).
__global__ __launch_bounds__(256) void k_actor_bwd(const float* __restrict__ mean, const float* __restrict__ quat,
                                                    const int32_t* __restrict__ actor,
                                                    const ut_actor_pose* __restrict__ poses, int n_act,
                                                    const float* dmw, const float* dqw, float* dmean,
                                                    float* dquat, double* __restrict__ d_pose, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = i < n;
  const int a = in ? actor[i] : -1;
  const bool mine = in && a >= 0 && a < n_act;
  double pg[7] = {0, 0, 0, 0, 0, 0, 0};
  if (in) {
    const double gm[3] = {dmw[i], dmw[n + i], dmw[2 * n + i]};
    const double gq[4] = {dqw[i], dqw[n + i], dqw[2 * n + i], dqw[3 * n + i]};
    if (!mine) {
      dmean[i] = (float)gm[0]; dmean[n + i] = (float)gm[1]; dmean[2 * n + i] = (float)gm[2];
      dquat[i] = (float)gq[0]; dquat[n + i] = (float)gq[1]; dquat[2 * n + i] = (float)gq[2]; dquat[3 * n + i] = (float)gq[3];
    } else {
      const PoseK p = load_pose(poses, a);
      const double mu[3] = {mean[i], mean[n + i], mean[2 * n + i]};
      const double qo[4] = {quat[i], quat[n + i], quat[2 * n + i], quat[3 * n + i]};
      // mu_w = R mu + t: dL/dmu = R^T g, dL/dt = g, dL/dR = g mu^T
      dmean[i] = (float)(p.R[0] * gm[0] + p.R[3] * gm[1] + p.R[6] * gm[2]);
      dmean[n + i] = (float)(p.R[1] * gm[0] + p.R[4] * gm[1] + p.R[7] * gm[2]);
      dmean[2 * n + i] = (float)(p.R[2] * gm[0] + p.R[5] * gm[1] + p.R[8] * gm[2]);
      // q_w = q_a * q: the left factor's adjoint multiplies by conj(q_a) on the left, the
      // right factor's by conj(q) on the right
      const double cqa[4] = {p.q[0], -p.q[1], -p.q[2], -p.q[3]};
      const double cqo[4] = {qo[0], -qo[1], -qo[2], -qo[3]};
      double dq[4], dqa[4];
      qmul(cqa, gq, dq);
      qmul(gq, cqo, dqa);
      dquat[i] = (float)dq[0]; dquat[n + i] = (float)dq[1]; dquat[2 * n + i] = (float)dq[2]; dquat[3 * n + i] = (float)dq[3];
      double dR[9];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) dR[r * 3 + c] = gm[r] * mu[c];
      // R(q) -> q (partial derivatives of the rotation polynomial)
      const double w = p.q[0], x = p.q[1], y = p.q[2], z = p.q[3];
      dqa[0] += 2 * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
      dqa[1] += 2 * (y * dR[1] + z * dR[2] + y * dR[3] - 2 * x * dR[4] - w * dR[5] + z * dR[6] + w * dR[7] - 2 * x * dR[8]);
      dqa[2] += 2 * (-2 * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] + z * dR[7] - 2 * y * dR[8]);
      dqa[3] += 2 * (-2 * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2 * z * dR[4] + y * dR[5] + x * dR[6] + y * dR[7]);
      // through the normalisation q_hat = q / |q|
      const double dot = dqa[0] * w + dqa[1] * x + dqa[2] * y + dqa[3] * z;
      const double iq = 1.0 / p.qn;
      pg[0] = (dqa[0] - w * dot) * iq;
      pg[1] = (dqa[1] - x * dot) * iq;
      pg[2] = (dqa[2] - y * dot) * iq;
      pg[3] = (dqa[3] - z * dot) * iq;
      pg[4] = gm[0]; pg[5] = gm[1]; pg[6] = gm[2];
    }
  }
  if (!d_pose) return;   // uniform across the grid
  const int a0 = __shfl(a, 0);
  if (__all(a == a0)) {
    if (a0 < 0 || a0 >= n_act) return;
#pragma unroll
    for (int k = 0; k < 7; ++k) {
      const double v = wave_sum(pg[k]);
      if (__lane_id() == 0 && v != 0.0) unsafeAtomicAdd(d_pose + (size_t)a0 * 7 + k, v);
    }
  } else if (mine) {
#pragma unroll
    for (int k = 0; k < 7; ++k)
      if (pg[k] != 0.0) unsafeAtomicAdd(d_pose + (size_t)a * 7 + k, pg[k]);
  }
}

}  // namespace

hipError_t launch_actor_transform(const ut_gaussians& g, const int32_t* actor, const ut_actor_pose* poses,
                                  int n_act, float* mean_w, float* quat_w, hipStream_t st) {
  if (g.n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((g.n + 255) / 256);
  hipLaunchKernelGGL(k_actor_fwd, dim3(blocks), dim3(256), 0, st, g.mean, g.quat, actor, poses, n_act,
                     mean_w, quat_w, g.n);
  return hipGetLastError();
}

hipError_t launch_actor_backward(const ut_gaussians& g, const int32_t* actor, const ut_actor_pose* poses,
                                 int n_act, const float* dmw, const float* dqw, float* dmean, float* dquat,
                                 double* d_pose, hipStream_t st) {
  if (d_pose && n_act > 0) {
    const hipError_t e = fill_f64(d_pose, 0.0, (size_t)n_act * 7, st);
    if (e != hipSuccess) return e;
  }
  if (g.n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((g.n + 255) / 256);
  hipLaunchKernelGGL(k_actor_bwd, dim3(blocks), dim3(256), 0, st, g.mean, g.quat, actor, poses, n_act,
                     dmw, dqw, dmean, dquat, d_pose, g.n);
  return hipGetLastError();
}

}  // namespace ut
