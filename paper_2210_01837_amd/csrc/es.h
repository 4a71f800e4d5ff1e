// Exponential-of-semicircle envelope (Sec. 3.5, eq. es-scalar) and the
// periodic cell arithmetic shared by the particle kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace fcmdp {

// phi(t) = exp(beta (sqrt(1 - (t/alpha)^2) - 1)) / I  for |t| <= alpha, else 0.
// The support test is done in double on the double argument; the envelope is
// evaluated in precision T (float in the mixed path).
template <typename T>
__device__ inline T es_eval(double t, double alpha, double beta,
                            double inv_norm);

template <>
__device__ inline double es_eval<double>(double t, double alpha, double beta,
                                         double inv_norm) {
  if (fabs(t) > alpha) return 0.0;
  const double r = t / alpha;
  return exp(beta * (sqrt((1.0 - r) * (1.0 + r)) - 1.0)) * inv_norm;
}

template <>
__device__ inline float es_eval<float>(double t, double alpha, double beta,
                                       double inv_norm) {
  if (fabs(t) > alpha) return 0.0f;
  const float r = (float)(t / alpha);
  return expf((float)beta * (sqrtf((1.0f - r) * (1.0f + r)) - 1.0f)) *
         (float)inv_norm;
}

// phi'(t), the derivative of the envelope, set to zero for |t| > tstar: the
// point beyond its maximum where |phi'| is smallest before it grows without
// bound at the edge of the support (torques through the kernel derivative,
// Sec. 3.4).  tstar < alpha.
template <typename T>
__device__ inline T es_deval(double t, double alpha, double beta,
                             double inv_norm, double tstar);

template <>
__device__ inline double es_deval<double>(double t, double alpha, double beta,
                                          double inv_norm, double tstar) {
  if (fabs(t) > tstar) return 0.0;
  const double r = t / alpha;
  const double s = sqrt((1.0 - r) * (1.0 + r));
  return exp(beta * (s - 1.0)) * inv_norm * beta * (-r / alpha) / s;
}

template <>
__device__ inline float es_deval<float>(double t, double alpha, double beta,
                                        double inv_norm, double tstar) {
  if (fabs(t) > tstar) return 0.0f;
  const float r = (float)(t / alpha);
  const float s = sqrtf((1.0f - r) * (1.0f + r));
  return expf((float)beta * (s - 1.0f)) * (float)inv_norm * (float)beta *
         (-r / (float)alpha) / s;
}

// x wrapped into [0, L)
__device__ inline double wrap_coord(double x, double L) {
  double r = x - L * floor(x / L);
  if (r >= L) r -= L;
  if (r < 0.0) r += L;
  return r;
}

// cell index i = floor(x/h) in [0, N) and fractional offset f in [0, 1)
__device__ inline void cell_of(double x, double h, int N, int* i, double* f) {
  const double t = x / h;
  double fl = floor(t);
  int k = (int)fl;
  *f = t - fl;
  if (k >= N) k -= N;
  if (k < 0) k += N;
  *i = k;
}

}  // namespace fcmdp
