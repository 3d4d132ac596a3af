// Cosine for the source EMF E cos(omega t + phase), host and device.
//
// Cody and Waite's argument reduction: k = rint(x * 2/pi) and
// r = ((x - k P1) - k P2) - k P3 with P1 + P2 + P3 = pi/2, where P1 and P2
// carry at most 30 significant bits so k P1 and k P2 are exact for
// |k| < 2^23 (|x| < 1.3e7). cos x is then +-cos r or +-sin r by k mod 4,
// with both evaluated by their Taylor series on |r| <= pi/4, truncated after
// the r^19 (sine) and r^20 (cosine) terms, where the remainder is below
// 1e-22. A compact replacement for the library cosine, whose
// large-argument path needs many more registers than the time loop can
// spare.
#pragma once

#include <hip/hip_runtime.h>

namespace emt {

__host__ __device__ inline double emf_cos(double x) {
  const double kP1 = 1.570796325802803;       // 0x1.921fb54p+0
  const double kP2 = 9.920935791635221e-10;   // 0x1.10b46118p-30
  const double kP3 = 5.170182981794105e-19;   // 0x1.313198a2e037p-61
  const double k = rint(x * 0.6366197723675814);
  const double r = ((x - k * kP1) - k * kP2) - k * kP3;
  const double z = r * r;
  // sin r = r (1 - z/3! + z^2/5! - ... - z^9/19!)
  double s = -8.22063524662433e-18;
  s = s * z + 2.8114572543455206e-15;
  s = s * z - 7.647163731819816e-13;
  s = s * z + 1.6059043836821613e-10;
  s = s * z - 2.505210838544172e-08;
  s = s * z + 2.7557319223985893e-06;
  s = s * z - 0.0001984126984126984;
  s = s * z + 0.008333333333333333;
  s = s * z - 0.16666666666666666;
  const double sin_r = r + r * (z * s);
  // cos r = 1 - z/2! + z^2/4! - ... + z^10/20!
  double c = 4.110317623312165e-19;
  c = c * z - 1.5619206968586225e-16;
  c = c * z + 4.779477332387385e-14;
  c = c * z - 1.1470745597729725e-11;
  c = c * z + 2.08767569878681e-09;
  c = c * z - 2.755731922398589e-07;
  c = c * z + 2.48015873015873e-05;
  c = c * z - 0.001388888888888889;
  c = c * z + 0.041666666666666664;
  c = c * z - 0.5;
  const double cos_r = 1.0 + z * c;
  const long long q = (long long)k & 3;
  return q == 0 ? cos_r : (q == 1 ? -sin_r : (q == 2 ? -cos_r : sin_r));
}

}  // namespace emt
