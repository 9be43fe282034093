// ut_sh.hpp -- real spherical harmonics up to degree 3 (Condon-Shortley phase, ordered by
// l then m = -l..l) as Cartesian polynomials of a unit direction, and their gradients.
// Normalisations: 1/(2 sqrt pi), sqrt(3/(4 pi)), sqrt(15/pi)/2, sqrt(5/pi)/4, sqrt(15/pi)/4,
// sqrt(35/(2 pi))/4, sqrt(105/pi)/2, sqrt(21/(2 pi))/4, sqrt(7/pi)/4, sqrt(105/pi)/4.
#pragma once

#include <hip/hip_runtime.h>

namespace ut {

constexpr double kSh0 = 0.28209479177387814;
constexpr double kSh1 = 0.4886025119029199;
constexpr double kSh2a = 1.0925484305920792;
constexpr double kSh2b = 0.31539156525252005;
constexpr double kSh2c = 0.5462742152960396;
constexpr double kSh3a = 0.5900435899266435;
constexpr double kSh3b = 2.890611442640554;
constexpr double kSh3c = 0.4570457994644658;
constexpr double kSh3d = 0.3731763325901154;
constexpr double kSh3e = 1.445305721320277;

__device__ __forceinline__ int sh_count(int deg) { return (deg + 1) * (deg + 1); }

// Y[k] for k < (deg+1)^2 at unit direction (x, y, z)
__device__ __forceinline__ void sh_basis(int deg, double x, double y, double z, double Y[16]) {
  Y[0] = kSh0;
  if (deg < 1) return;
  Y[1] = -kSh1 * y;
  Y[2] = kSh1 * z;
  Y[3] = -kSh1 * x;
  if (deg < 2) return;
  const double xx = x * x, yy = y * y, zz = z * z;
  Y[4] = kSh2a * x * y;
  Y[5] = -kSh2a * y * z;
  Y[6] = kSh2b * (2 * zz - xx - yy);
  Y[7] = -kSh2a * x * z;
  Y[8] = kSh2c * (xx - yy);
  if (deg < 3) return;
  Y[9] = -kSh3a * y * (3 * xx - yy);
  Y[10] = kSh3b * x * y * z;
  Y[11] = -kSh3c * y * (4 * zz - xx - yy);
  Y[12] = kSh3d * z * (2 * zz - 3 * xx - 3 * yy);
  Y[13] = -kSh3c * x * (4 * zz - xx - yy);
  Y[14] = kSh3e * z * (xx - yy);
  Y[15] = -kSh3a * x * (xx - 3 * yy);
}

// gradient of the polynomial Y[k] with respect to (x, y, z): G[k][0..2]
__device__ __forceinline__ void sh_basis_grad(int deg, double x, double y, double z, double G[16][3]) {
  G[0][0] = G[0][1] = G[0][2] = 0;
  if (deg < 1) return;
  G[1][0] = 0;     G[1][1] = -kSh1; G[1][2] = 0;
  G[2][0] = 0;     G[2][1] = 0;     G[2][2] = kSh1;
  G[3][0] = -kSh1; G[3][1] = 0;     G[3][2] = 0;
  if (deg < 2) return;
  const double xx = x * x, yy = y * y, zz = z * z;
  G[4][0] = kSh2a * y;       G[4][1] = kSh2a * x;       G[4][2] = 0;
  G[5][0] = 0;               G[5][1] = -kSh2a * z;      G[5][2] = -kSh2a * y;
  G[6][0] = -2 * kSh2b * x;  G[6][1] = -2 * kSh2b * y;  G[6][2] = 4 * kSh2b * z;
  G[7][0] = -kSh2a * z;      G[7][1] = 0;               G[7][2] = -kSh2a * x;
  G[8][0] = 2 * kSh2c * x;   G[8][1] = -2 * kSh2c * y;  G[8][2] = 0;
  if (deg < 3) return;
  G[9][0] = -kSh3a * 6 * x * y;
  G[9][1] = -kSh3a * (3 * xx - 3 * yy);
  G[9][2] = 0;
  G[10][0] = kSh3b * y * z;
  G[10][1] = kSh3b * x * z;
  G[10][2] = kSh3b * x * y;
  G[11][0] = -kSh3c * (-2 * x * y);
  G[11][1] = -kSh3c * (4 * zz - xx - 3 * yy);
  G[11][2] = -kSh3c * 8 * y * z;
  G[12][0] = kSh3d * (-6 * x * z);
  G[12][1] = kSh3d * (-6 * y * z);
  G[12][2] = kSh3d * (6 * zz - 3 * xx - 3 * yy);
  G[13][0] = -kSh3c * (4 * zz - 3 * xx - yy);
  G[13][1] = -kSh3c * (-2 * x * y);
  G[13][2] = -kSh3c * 8 * x * z;
  G[14][0] = kSh3e * 2 * x * z;
  G[14][1] = -kSh3e * 2 * y * z;
  G[14][2] = kSh3e * (xx - yy);
  G[15][0] = -kSh3a * (3 * xx - 3 * yy);
  G[15][1] = -kSh3a * (-6 * x * y);
  G[15][2] = 0;
}

}  // namespace ut
