// Real spherical harmonics up to degree 3 (FP64 device code).
//
// View-dependent colour of the 3DGS formulation the paper builds on:
// rgb = max(0, sum_k sh_k Y_k(dir) + 0.5). Orthonormal real SH as Cartesian
// polynomials of the unit direction, m = -l..l within degree l (index
// l*l + l + m), with the sign (-1)^m. Normalisations:
//   k0 = 1/(2 sqrt(pi)), k1 = sqrt(3/(4 pi)), k2a = sqrt(15/pi)/2,
//   k2b = sqrt(5/pi)/4, k2c = sqrt(15/pi)/4, k3a = sqrt(35/(2 pi))/4,
//   k3b = sqrt(105/pi)/2, k3c = sqrt(21/(2 pi))/4, k3d = sqrt(7/pi)/4,
//   k3e = sqrt(105/pi)/4.
#pragma once

namespace gs {

constexpr double kSH0 = 0.28209479177387814;
constexpr double kSH1 = 0.48860251190291992;
constexpr double kSH2a = 1.0925484305920792;
constexpr double kSH2b = 0.31539156525252005;
constexpr double kSH2c = 0.54627421529603959;
constexpr double kSH3a = 0.59004358992664352;
constexpr double kSH3b = 2.8906114426405538;
constexpr double kSH3c = 0.45704579946446572;
constexpr double kSH3d = 0.3731763325901154;
constexpr double kSH3e = 1.4453057213202769;

// Y[k] for k < (deg+1)^2 at the unit vector (x, y, z).
__device__ __forceinline__ void sh_basis(int deg, double x, double y, double z, double* Y) {
  Y[0] = kSH0;
  if (deg < 1) return;
  Y[1] = -kSH1 * y;
  Y[2] = kSH1 * z;
  Y[3] = -kSH1 * x;
  if (deg < 2) return;
  const double xx = x * x, yy = y * y, zz = z * z;
  Y[4] = kSH2a * (x * y);
  Y[5] = -kSH2a * (y * z);
  Y[6] = kSH2b * (2.0 * zz - xx - yy);
  Y[7] = -kSH2a * (x * z);
  Y[8] = kSH2c * (xx - yy);
  if (deg < 3) return;
  Y[9] = -kSH3a * y * (3.0 * xx - yy);
  Y[10] = kSH3b * (x * y * z);
  Y[11] = -kSH3c * y * (4.0 * zz - xx - yy);
  Y[12] = kSH3d * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
  Y[13] = -kSH3c * x * (4.0 * zz - xx - yy);
  Y[14] = kSH3e * z * (xx - yy);
  Y[15] = -kSH3a * x * (xx - 3.0 * yy);
}

// Accumulates sum_k w[k] * grad Y_k into (gx, gy, gz).
__device__ __forceinline__ void sh_basis_grad_dot(int deg, double x, double y, double z,
                                                  const double* w, double& gx, double& gy,
                                                  double& gz) {
  gx = 0.0; gy = 0.0; gz = 0.0;
  if (deg < 1) return;
  gy += -kSH1 * w[1];
  gz += kSH1 * w[2];
  gx += -kSH1 * w[3];
  if (deg < 2) return;
  const double xx = x * x, yy = y * y, zz = z * z;
  // Y4 = k2a xy
  gx += kSH2a * y * w[4];  gy += kSH2a * x * w[4];
  // Y5 = -k2a yz
  gy += -kSH2a * z * w[5]; gz += -kSH2a * y * w[5];
  // Y6 = k2b (2zz - xx - yy)
  gx += -2.0 * kSH2b * x * w[6]; gy += -2.0 * kSH2b * y * w[6]; gz += 4.0 * kSH2b * z * w[6];
  // Y7 = -k2a xz
  gx += -kSH2a * z * w[7]; gz += -kSH2a * x * w[7];
  // Y8 = k2c (xx - yy)
  gx += 2.0 * kSH2c * x * w[8]; gy += -2.0 * kSH2c * y * w[8];
  if (deg < 3) return;
  // Y9 = -k3a (3xxy - yyy)
  gx += -kSH3a * 6.0 * x * y * w[9]; gy += -kSH3a * (3.0 * xx - 3.0 * yy) * w[9];
  // Y10 = k3b xyz
  gx += kSH3b * y * z * w[10]; gy += kSH3b * x * z * w[10]; gz += kSH3b * x * y * w[10];
  // Y11 = -k3c (4yzz - xxy - yyy)
  gx += -kSH3c * (-2.0 * x * y) * w[11];
  gy += -kSH3c * (4.0 * zz - xx - 3.0 * yy) * w[11];
  gz += -kSH3c * (8.0 * y * z) * w[11];
  // Y12 = k3d (2zzz - 3xxz - 3yyz)
  gx += kSH3d * (-6.0 * x * z) * w[12];
  gy += kSH3d * (-6.0 * y * z) * w[12];
  gz += kSH3d * (6.0 * zz - 3.0 * xx - 3.0 * yy) * w[12];
  // Y13 = -k3c (4xzz - xxx - xyy)
  gx += -kSH3c * (4.0 * zz - 3.0 * xx - yy) * w[13];
  gy += -kSH3c * (-2.0 * x * y) * w[13];
  gz += -kSH3c * (8.0 * x * z) * w[13];
  // Y14 = k3e (xxz - yyz)
  gx += kSH3e * 2.0 * x * z * w[14]; gy += -kSH3e * 2.0 * y * z * w[14];
  gz += kSH3e * (xx - yy) * w[14];
  // Y15 = -k3a (xxx - 3xyy)
  gx += -kSH3a * (3.0 * xx - 3.0 * yy) * w[15]; gy += -kSH3a * (-6.0 * x * y) * w[15];
}

}  // namespace gs
