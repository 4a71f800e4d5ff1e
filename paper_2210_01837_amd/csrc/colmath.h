// Complex float64 helpers and small dense solves shared by the column
// kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "fcmdp_internal.h"

namespace fcmdp {

struct Z2 {
  double x, y;
};
__device__ inline Z2 zmk(double a, double b) { Z2 r; r.x = a; r.y = b; return r; }
__device__ inline Z2 operator+(Z2 a, Z2 b) { return zmk(a.x + b.x, a.y + b.y); }
__device__ inline Z2 operator-(Z2 a, Z2 b) { return zmk(a.x - b.x, a.y - b.y); }
__device__ inline Z2 operator*(double s, Z2 a) { return zmk(s * a.x, s * a.y); }
__device__ inline Z2 operator*(Z2 a, Z2 b) {
  return zmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline Z2 zdiv(Z2 a, double d) { return zmk(a.x / d, a.y / d); }
// i * s * a for real s
__device__ inline Z2 imul(double s, Z2 a) { return zmk(-s * a.y, s * a.x); }

struct ColParams {
  DevParams dp;
  double scale;       // 1 / (Nx Ny)
  double kxs, kys;    // 2 pi / Lx, 2 pi / Ly
  const double* dctf; // forward Chebyshev transform [c][n] in FP64
};

// Column (kxi, nyi) of the exact low-wavenumber square |nx|, |ny| <= ns
// (index into lowk_coef), or -1.
__device__ inline int lowk_col(const DevParams& dp, int kxi, int nyi) {
  const int ns = dp.lowk_ns;
  if (ns < 0 || kxi > ns || nyi > ns || nyi < -ns) return -1;
  return kxi * (2 * ns + 1) + nyi + ns;
}

// 6x6 real Gaussian elimination with partial pivoting, complex RHS.
__device__ inline void solve6(double A[6][6], Z2 b[6]) {
  for (int c = 0; c < 6; ++c) {
    int piv = c;
    double best = fabs(A[c][c]);
    for (int r = c + 1; r < 6; ++r)
      if (fabs(A[r][c]) > best) { best = fabs(A[r][c]); piv = r; }
    if (piv != c) {
      for (int k = 0; k < 6; ++k) { double t = A[c][k]; A[c][k] = A[piv][k]; A[piv][k] = t; }
      Z2 t = b[c]; b[c] = b[piv]; b[piv] = t;
    }
    const double inv = 1.0 / A[c][c];
    for (int r = c + 1; r < 6; ++r) {
      const double f = A[r][c] * inv;
      if (f == 0.0) continue;
      for (int k = c; k < 6; ++k) A[r][k] -= f * A[c][k];
      b[r] = b[r] - f * b[c];
    }
  }
  for (int c = 5; c >= 0; --c) {
    Z2 v = b[c];
    for (int k = c + 1; k < 6; ++k) v = v - A[c][k] * b[k];
    b[c] = zdiv(v, A[c][c]);
  }
}

}  // namespace fcmdp
