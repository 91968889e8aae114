// Element kinematics shared by the element kernels: F = I + H, J - 1 and
// ln J in double (cancellation-free for FP64 states), F^-T.
#pragma once

#include <hip/hip_runtime.h>

namespace nle {

// x / d in double from the hardware reciprocal estimate refined by two
// Newton-Raphson corrections (reciprocal, then quotient).
__device__ __forceinline__ double div_d(double x, double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(fma(-d, r, 1.0), r, r);
  double q = x * r;
  return fma(fma(-d, q, x), r, q);
}

// ln(1 + x) in double.  For |x| < 1/4 the series of 2 atanh(t), t = x/(2+x)
// (terms t^(2k+1)/(2k+1), truncated where t^2^k < 1e-17) is cheaper than the
// general routine; larger |x| falls back to log1p.
__device__ __forceinline__ double log1p_d(double x) {
  if (fabs(x) < 0.25) {
    const double t = div_d(x, 2.0 + x);
    const double t2 = t * t;
    double p = 1.0 / 21.0;
    p = fma(p, t2, 1.0 / 19.0);
    p = fma(p, t2, 1.0 / 17.0);
    p = fma(p, t2, 1.0 / 15.0);
    p = fma(p, t2, 1.0 / 13.0);
    p = fma(p, t2, 1.0 / 11.0);
    p = fma(p, t2, 1.0 / 9.0);
    p = fma(p, t2, 1.0 / 7.0);
    p = fma(p, t2, 1.0 / 5.0);
    p = fma(p, t2, 1.0 / 3.0);
    p = fma(p, t2, 1.0);
    return 2.0 * t * p;
  }
  return log1p(x);
}

// Element kinematics: F = I + H, J - 1, ln J (double), F^-T.
template <typename T>
struct Kin {
  T F[3][3];
  T FiT[3][3];
  double jm1, J, lnJ;
  bool bad;
};

template <typename T>
__device__ __forceinline__ void kinematics(const T H[3][3], Kin<T> &k) {
  double jm1;
  if (sizeof(T) == 8) {
    // det(I + H) - 1 = tr H + ((tr H)^2 - tr(H^2)) / 2 + det H: no cancellation
    // when J is near one, which keeps the FP64 residual's volumetric term exact
    double h[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) h[i][j] = double(H[i][j]);
    const double tr = h[0][0] + h[1][1] + h[2][2];
    const double tr2 = h[0][0] * h[0][0] + h[1][1] * h[1][1] + h[2][2] * h[2][2] +
                       2.0 * (h[0][1] * h[1][0] + h[0][2] * h[2][0] + h[1][2] * h[2][1]);
    const double deth = h[0][0] * (h[1][1] * h[2][2] - h[1][2] * h[2][1]) -
                        h[0][1] * (h[1][0] * h[2][2] - h[1][2] * h[2][0]) +
                        h[0][2] * (h[1][0] * h[2][1] - h[1][1] * h[2][0]);
    jm1 = tr + 0.5 * (tr * tr - tr2) + deth;
  } else {
    // FP32 state: I + H is exact in double, and det(I + H) - 1 in double keeps
    // ~12 significant digits of J - 1 (more than the FP32 inputs carry)
    double f[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) f[i][j] = double(H[i][j]) + (i == j ? 1.0 : 0.0);
    jm1 = f[0][0] * (f[1][1] * f[2][2] - f[1][2] * f[2][1]) -
          f[0][1] * (f[1][0] * f[2][2] - f[1][2] * f[2][0]) +
          f[0][2] * (f[1][0] * f[2][1] - f[1][1] * f[2][0]) - 1.0;
  }
  k.bad = !(jm1 > -1.0);
  if (k.bad) jm1 = 0.0;
  k.jm1 = jm1;
  k.J = 1.0 + jm1;
  k.lnJ = log1p_d(jm1);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) k.F[i][j] = H[i][j] + (i == j ? T(1) : T(0));
  const T(&F)[3][3] = k.F;
  T ij;
  if (sizeof(T) == 8)
    ij = T(1.0 / k.J);
  else
    ij = T(__builtin_amdgcn_rcpf(float(k.J)));
  // cof F / J
  k.FiT[0][0] = (F[1][1] * F[2][2] - F[1][2] * F[2][1]) * ij;
  k.FiT[0][1] = (F[1][2] * F[2][0] - F[1][0] * F[2][2]) * ij;
  k.FiT[0][2] = (F[1][0] * F[2][1] - F[1][1] * F[2][0]) * ij;
  k.FiT[1][0] = (F[0][2] * F[2][1] - F[0][1] * F[2][2]) * ij;
  k.FiT[1][1] = (F[0][0] * F[2][2] - F[0][2] * F[2][0]) * ij;
  k.FiT[1][2] = (F[0][1] * F[2][0] - F[0][0] * F[2][1]) * ij;
  k.FiT[2][0] = (F[0][1] * F[1][2] - F[0][2] * F[1][1]) * ij;
  k.FiT[2][1] = (F[0][2] * F[1][0] - F[0][0] * F[1][2]) * ij;
  k.FiT[2][2] = (F[0][0] * F[1][1] - F[0][1] * F[1][0]) * ij;
}

}  // namespace nle
