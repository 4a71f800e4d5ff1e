// Column solve with eight lanes per (kx, ky) column (Nz <= 32).
//
// Same mathematics as columns.hip (steps 2-6 of Sec. 3.4 plus the spectral
// vorticity), laid out for registers instead of per-thread scratch: lane l of
// a column's 8-lane group holds Chebyshev coefficients n = 4l .. 4l+3 of every
// vector, in float64.  The sequential parts become segmented scans over the
// 8 lanes (each lane first combines its own two unknowns per parity, then
// the partial results are combined across lanes with shuffles):
//   * Chebyshev derivative  b_m = 2 sum_{n > m, n - m odd} n a_n  -- a suffix
//     sum per parity;
//   * the BVP of each parity (tridiagonal rows m >= 2 plus one dense boundary
//     row): the elimination multipliers alpha_i = -L_i / (D_i + U_i
//     alpha_{i+1}) are a Moebius recurrence (suffix product of 2x2 matrices),
//     beta_i an affine suffix recurrence, and y_i = P_i y_0 + Q_i with prefix
//     products / affine prefixes, y_0 from the dense row by a lane reduction.
// The Chebyshev transforms are done per lane as small dot products; the
// inverse transform goes through an LDS coefficient buffer so each lane can
// evaluate whole band nodes.
#include "fcmdp_internal.h"
#include "colmath.h"

namespace fcmdp {

constexpr int kSeg = 8;     // lanes per column
constexpr int kNpl = 4;     // coefficients per lane
// columns per workgroup: the LDS coefficient buffer holds 5 vectors x 32
// coefficients per column (40 KiB either way)
template <typename T> struct ColsPerBlock;
template <> struct ColsPerBlock<float> { static constexpr int value = 32; };
template <> struct ColsPerBlock<double> { static constexpr int value = 16; };

struct Vec {
  Z2 v[kNpl];
};

__device__ inline double shd(double a, int src) { return __shfl(a, src, kSeg); }
__device__ inline Z2 shz(Z2 a, int src) {
  return zmk(__shfl(a.x, src, kSeg), __shfl(a.y, src, kSeg));
}
__device__ inline double red(double a) {
#pragma unroll
  for (int m = 1; m < kSeg; m <<= 1) a += __shfl_xor(a, m, kSeg);
  return a;
}
__device__ inline Z2 red(Z2 a) { return zmk(red(a.x), red(a.y)); }
__device__ inline Vec vzero() {
  Vec r;
#pragma unroll
  for (int j = 0; j < kNpl; ++j) r.v[j] = zmk(0, 0);
  return r;
}

// d/dz of a Chebyshev series (times 2/H).
__device__ inline Vec seg_deriv(const Vec& a, int l, double s2H) {
  Z2 q[kNpl];
#pragma unroll
  for (int j = 0; j < kNpl; ++j) q[j] = (double)(4 * l + j) * a.v[j];
  const Z2 E = q[0] + q[2];     // even-n terms of this lane
  const Z2 O = q[1] + q[3];     // odd-n terms
  Z2 sE = E, sO = O;            // inclusive suffix sums over lanes
#pragma unroll
  for (int k = 1; k < kSeg; k <<= 1) {
    const int src = l + k < kSeg ? l + k : kSeg - 1;
    const Z2 tE = shz(sE, src), tO = shz(sO, src);
    if (l + k < kSeg) {
      sE = sE + tE;
      sO = sO + tO;
    }
  }
  Z2 SE = shz(sE, l + 1 < kSeg ? l + 1 : kSeg - 1);
  Z2 SO = shz(sO, l + 1 < kSeg ? l + 1 : kSeg - 1);
  if (l == kSeg - 1) {
    SE = zmk(0, 0);
    SO = zmk(0, 0);
  }
  Vec b;
  b.v[3] = (2.0 * s2H) * SE;
  b.v[2] = (2.0 * s2H) * (q[3] + SO);
  b.v[1] = (2.0 * s2H) * (q[2] + SE);
  const double c0 = (l == 0) ? 1.0 : 2.0;
  b.v[0] = (c0 * s2H) * (q[1] + q[3] + SO);
  return b;
}

// Operator data of one parity for the Robin BVP (depends on kappa only).
// Slot s = 0, 1 of lane l is unknown i = 2l + s, coefficient m = 2i + p.
struct Par {
  double alpha[2];
  double P[2];
  double invD[2];
  double a[2];
  double e[2];
  double lo[2], di[2], up[2];
  double eP;
};

__device__ inline void m2mul(const double* A, const double* B, double* C) {
  C[0] = A[0] * B[0] + A[1] * B[2];
  C[1] = A[0] * B[1] + A[1] * B[3];
  C[2] = A[2] * B[0] + A[3] * B[2];
  C[3] = A[2] * B[1] + A[3] * B[3];
}

__device__ Par seg_prepare(double kappa, int N, int l, int p) {
  Par q;
  const double k2 = kappa * kappa;
  double T[2][4];
  double Dd[2], Uu[2];
  bool act[2], row[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int i = 2 * l + s;
    const int m = 2 * i + p;
    act[s] = m < N;
    row[s] = act[s] && i >= 1;
    q.e[s] = act[s] ? (double)m * m + kappa : 0.0;
    if (row[s]) {
      q.lo[s] = (m - 2 == 0 ? 2.0 : 1.0) / (4.0 * m * (m - 1));
      q.di[s] = 1.0 / (2.0 * ((double)m * m - 1.0));
      q.up[s] = (m + 2 < N) ? 1.0 / (4.0 * m * (m + 1)) : 0.0;
      const double L = -k2 * q.lo[s];
      Dd[s] = 1.0 + k2 * q.di[s];
      Uu[s] = -k2 * q.up[s];
      T[s][0] = 0.0; T[s][1] = -L; T[s][2] = Uu[s]; T[s][3] = Dd[s];
    } else {
      q.lo[s] = q.di[s] = q.up[s] = 0.0;
      Dd[s] = 1.0;
      Uu[s] = 0.0;
      T[s][0] = 1.0; T[s][1] = 0.0; T[s][2] = 0.0; T[s][3] = 1.0;
    }
  }
  // suffix products of the 2x2 Moebius matrices, normalised (only ratios matter)
  double Y[4];
  m2mul(T[0], T[1], Y);
#pragma unroll
  for (int k = 1; k < kSeg; k <<= 1) {
    const int src = l + k < kSeg ? l + k : kSeg - 1;
    double Yk[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) Yk[e] = shd(Y[e], src);
    if (l + k < kSeg) {
      double Z[4];
      m2mul(Y, Yk, Z);
      const double sc = fmax(fmax(fabs(Z[0]), fabs(Z[1])), fmax(fabs(Z[2]), fabs(Z[3])));
      const double inv = sc > 0.0 ? 1.0 / sc : 1.0;
#pragma unroll
      for (int e = 0; e < 4; ++e) Y[e] = Z[e] * inv;
    }
  }
  double X[4];
  {
    const int src = l + 1 < kSeg ? l + 1 : kSeg - 1;
#pragma unroll
    for (int e = 0; e < 4; ++e) X[e] = shd(Y[e], src);
    if (l == kSeg - 1) { X[0] = 1.0; X[1] = 0.0; X[2] = 0.0; X[3] = 1.0; }
  }
  double S1[4], S0[4];
  m2mul(T[1], X, S1);
  m2mul(T[0], S1, S0);
  q.alpha[1] = S1[1] / S1[3];
  q.alpha[0] = S0[1] / S0[3];
  if (l == 0) q.alpha[0] = 1.0;              // i = 0: P_0 = 1
  if (!act[0]) q.alpha[0] = 0.0;
  if (!act[1]) q.alpha[1] = 0.0;
  // Delta_i = D_i + U_i alpha_{i+1}
  double anext[2];
  anext[0] = q.alpha[1];
  {
    const double t = shd(q.alpha[0], l + 1 < kSeg ? l + 1 : kSeg - 1);
    anext[1] = (l + 1 < kSeg) ? t : 0.0;
  }
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    if (row[s]) {
      const double delta = Dd[s] + Uu[s] * anext[s];
      q.invD[s] = 1.0 / delta;
      q.a[s] = -Uu[s] * q.invD[s];
    } else {
      q.invD[s] = 0.0;
      q.a[s] = 0.0;
    }
  }
  // prefix products P_i = alpha_i P_{i-1}
  double Yp = q.alpha[0] * q.alpha[1];
#pragma unroll
  for (int k = 1; k < kSeg; k <<= 1) {
    const double t = shd(Yp, l >= k ? l - k : 0);
    if (l >= k) Yp *= t;
  }
  double Pin = shd(Yp, l >= 1 ? l - 1 : 0);
  if (l == 0) Pin = 1.0;
  q.P[0] = q.alpha[0] * Pin;
  q.P[1] = q.alpha[1] * q.P[0];
  q.eP = red(q.e[0] * q.P[0] + q.e[1] * q.P[1]);
  return q;
}

// Robin BVP y'' - k^2 y = r, (d/dz + k) y(H) = gH, (d/dz - k) y(0) = g0.
__device__ Vec seg_solve(const Par* q, const Vec& r, Z2 gH, Z2 g0, double H,
                         int l) {
  const double h2 = 0.25 * H * H;
  Vec y;
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const Par& Q = q[p];
    const Z2 r0 = r.v[p], r1 = r.v[2 + p];
    const Z2 rm2 = shz(r1, l >= 1 ? l - 1 : 0);          // r_{m-2} of slot 0
    const Z2 rp2 = shz(r0, l + 1 < kSeg ? l + 1 : kSeg - 1);  // r_{m+2} of slot 1
    const Z2 R0 = h2 * (Q.lo[0] * rm2 - Q.di[0] * r0 + Q.up[0] * r1);
    const Z2 R1 = h2 * (Q.lo[1] * r0 - Q.di[1] * r1 + Q.up[1] * rp2);
    const Z2 b0 = Q.invD[0] * R0, b1 = Q.invD[1] * R1;
    // beta: suffix affine recurrence beta_i = a_i beta_{i+1} + b_i
    double A = Q.a[0] * Q.a[1];
    Z2 B = Q.a[0] * b1 + b0;
#pragma unroll
    for (int k = 1; k < kSeg; k <<= 1) {
      const int src = l + k < kSeg ? l + k : kSeg - 1;
      const double Ak = shd(A, src);
      const Z2 Bk = shz(B, src);
      if (l + k < kSeg) {
        B = A * Bk + B;
        A = A * Ak;
      }
    }
    Z2 bin = shz(B, l + 1 < kSeg ? l + 1 : kSeg - 1);
    if (l == kSeg - 1) bin = zmk(0, 0);
    const Z2 be1 = Q.a[1] * bin + b1;
    Z2 be0 = Q.a[0] * be1 + b0;
    if (l == 0) be0 = zmk(0, 0);
    // Q_i = alpha_i Q_{i-1} + beta_i (prefix), Q_0 = 0
    double Aq = Q.alpha[1] * Q.alpha[0];
    Z2 Bq = Q.alpha[1] * be0 + be1;
#pragma unroll
    for (int k = 1; k < kSeg; k <<= 1) {
      const int src = l >= k ? l - k : 0;
      const double Ak = shd(Aq, src);
      const Z2 Bk = shz(Bq, src);
      if (l >= k) {
        Bq = Aq * Bk + Bq;
        Aq = Aq * Ak;
      }
    }
    Z2 qin = shz(Bq, l >= 1 ? l - 1 : 0);
    if (l == 0) qin = zmk(0, 0);
    const Z2 Q0 = Q.alpha[0] * qin + be0;
    const Z2 Q1 = Q.alpha[1] * Q0 + be1;
    const Z2 eQ = red(Q.e[0] * Q0 + Q.e[1] * Q1);
    const Z2 g = p == 0 ? (0.25 * H) * (gH - g0) : (0.25 * H) * (gH + g0);
    const Z2 y0 = zdiv(g - eQ, Q.eP);
    y.v[p] = Q.P[0] * y0 + Q0;
    y.v[2 + p] = Q.P[1] * y0 + Q1;
  }
  return y;
}

// k = 0: y'' = r with y(0) = 0 and y'(H) = 0 (bottom wall) or y(H) = 0.
__device__ Vec seg_zero_mode(const Vec& r, double H, int N, int geometry,
                             int l) {
  const double h2 = 0.25 * H * H;
  Vec y = vzero();
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const Z2 r0 = r.v[p], r1 = r.v[2 + p];
    const Z2 rm2 = shz(r1, l >= 1 ? l - 1 : 0);
    const Z2 rp2 = shz(r0, l + 1 < kSeg ? l + 1 : kSeg - 1);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int m = 4 * l + 2 * s + p;
      if (m >= 2 && m < N) {
        const double lo = (m - 2 == 0 ? 2.0 : 1.0) / (4.0 * m * (m - 1));
        const double di = 1.0 / (2.0 * ((double)m * m - 1.0));
        const double up = (m + 2 < N) ? 1.0 / (4.0 * m * (m + 1)) : 0.0;
        const Z2 rm = s == 0 ? rm2 : r0;
        const Z2 rc = s == 0 ? r0 : r1;
        const Z2 rp = s == 0 ? r1 : rp2;
        y.v[2 * s + p] = h2 * (lo * rm - di * rc + up * rp);
      }
    }
  }
  Z2 sp = zmk(0, 0), sm = zmk(0, 0), sn2 = zmk(0, 0);
#pragma unroll
  for (int j = 0; j < kNpl; ++j) {
    const double n = 4.0 * l + j;
    sp = sp + y.v[j];
    sm = sm + ((j & 1) ? -1.0 : 1.0) * y.v[j];
    sn2 = sn2 + (n * n) * y.v[j];
  }
  sp = red(sp);
  sm = red(sm);
  sn2 = red(sn2);
  if (l == 0) {
    if (geometry == 0) {
      y.v[1] = -1.0 * sn2;
      y.v[0] = y.v[1] - sm;
    } else {
      y.v[0] = -0.5 * (sp + sm);
      y.v[1] = -0.5 * (sp - sm);
    }
  }
  return y;
}

__device__ inline Z2 bsum_bottom(const Vec& a) {   // sum (-1)^n a_n
  return red(a.v[0] - a.v[1] + a.v[2] - a.v[3]);
}
__device__ inline Z2 bsum_top(const Vec& a) {      // sum a_n
  return red(a.v[0] + a.v[1] + a.v[2] + a.v[3]);
}

// Chebyshev coefficients (this lane's four) of f(z_c) and z_c f(z_c) for a
// real node function given distributed four nodes per lane.
__device__ inline void seg_basis(const double fb[kNpl], const double* __restrict__ zc,
                                 const double* __restrict__ Mf, int N, int l,
                                 double E[kNpl], double ZE[kNpl]) {
#pragma unroll
  for (int j = 0; j < kNpl; ++j) { E[j] = 0.0; ZE[j] = 0.0; }
#pragma unroll
  for (int c = 0; c < 4 * kSeg; ++c) {
    const double fc = shd(fb[c & 3], c >> 2);
    if (c < N) {
      const double zf = zc[c] * fc;
      const double* row = Mf + c * N + 4 * l;
#pragma unroll
      for (int j = 0; j < kNpl; ++j) {
        if (4 * l + j < N) {
          const double m = row[j];
          E[j] += m * fc;
          ZE[j] += m * zf;
        }
      }
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256)
k_columns_seg(ColParams cp, const int* __restrict__ band,
              const cplx_t<T>* __restrict__ in, cplx_t<T>* __restrict__ out,
              const double* __restrict__ zc, const double* __restrict__ Mf,
              const double* __restrict__ Pi) {
  using C = cplx_t<T>;
  constexpr int kCols = ColsPerBlock<T>::value;
  extern __shared__ unsigned char lds_raw[];
  C* buf = reinterpret_cast<C*>(lds_raw);   // [kCols][5][32]
  const DevParams& dp = cp.dp;
  const int lo = band[0], hi = band[1];
  if (lo > hi) return;
  const int K = dp.Nkx * dp.Ny;
  const int N = dp.Nz;
  const int P = hi - lo + 1;
  const size_t PS = (size_t)K;
  const int cl = threadIdx.x / kSeg;
  const int l = threadIdx.x % kSeg;
  const int idx = blockIdx.x * kCols + cl;
  const bool valid = idx < K;
  const int kxi = valid ? idx / dp.Ny : 0;
  const int kyi = valid ? idx - kxi * dp.Ny : 0;
  const bool nyq = !valid || kxi == dp.Nx / 2 || kyi == dp.Ny / 2;
  const double kx = 2.0 * M_PI * kxi / dp.Lx;
  const int nyi = kyi <= dp.Ny / 2 ? kyi : kyi - dp.Ny;
  const double ky = 2.0 * M_PI * nyi / dp.Ly;
  const double k = sqrt(kx * kx + ky * ky);
  const double H = dp.H, eta = dp.eta, s2H = 2.0 / H;

  Vec U = vzero(), V = vzero(), W = vzero(), DU, DV;
  if (!nyq) {
    // Chebyshev transform of f + (1/2)(ik_y g_z, -ik_x g_z, ik_x g_y - ik_y g_x)
    // and of g_x, g_y (their z-derivatives enter the curl below)
    Vec A[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) A[v] = vzero();
    for (int c = 0; c < P; ++c) {
      const int ca = lo + c;
      Z2 val[6];
#pragma unroll
      for (int ch = 0; ch < 6; ++ch) {
        const C t = in[(ch * N + ca) * PS + idx];
        val[ch] = zmk((double)t.x, (double)t.y);
      }
      Z2 comb[5];
      comb[0] = val[0] + imul(0.5 * ky, val[5]);
      comb[1] = val[1] - imul(0.5 * kx, val[5]);
      comb[2] = val[2] + imul(0.5 * kx, val[4]) - imul(0.5 * ky, val[3]);
      comb[3] = val[3];
      comb[4] = val[4];
      const double* row = Mf + ca * N + 4 * l;
#pragma unroll
      for (int j = 0; j < kNpl; ++j) {
        const double m = (4 * l + j < N) ? row[j] : 0.0;
#pragma unroll
        for (int v = 0; v < 5; ++v) A[v].v[j] = A[v].v[j] + m * comb[v];
      }
    }
    const Vec dgy = seg_deriv(A[4], l, s2H);
    const Vec dgx = seg_deriv(A[3], l, s2H);
    Vec fx, fy, fz;
#pragma unroll
    for (int j = 0; j < kNpl; ++j) {
      fx.v[j] = A[0].v[j] - 0.5 * dgy.v[j];
      fy.v[j] = A[1].v[j] + 0.5 * dgx.v[j];
      fz.v[j] = A[2].v[j];
    }
    if (k == 0.0) {
      Vec r;
#pragma unroll
      for (int j = 0; j < kNpl; ++j) r.v[j] = (-1.0 / eta) * fx.v[j];
      U = seg_zero_mode(r, H, N, dp.geometry, l);
#pragma unroll
      for (int j = 0; j < kNpl; ++j) r.v[j] = (-1.0 / eta) * fy.v[j];
      V = seg_zero_mode(r, H, N, dp.geometry, l);
    } else {
      const double kappa = 0.5 * k * H;
      Par q[2];
      q[0] = seg_prepare(kappa, N, l, 0);
      q[1] = seg_prepare(kappa, N, l, 1);
      const Vec dfz = seg_deriv(fz, l, s2H);
      Vec r;
#pragma unroll
      for (int j = 0; j < kNpl; ++j)
        r.v[j] = imul(kx, fx.v[j]) + imul(ky, fy.v[j]) + dfz.v[j];
      const Vec p = seg_solve(q, r, zmk(0, 0), zmk(0, 0), H, l);
      const Z2 pH = bsum_top(p), p0 = bsum_bottom(p);
      const double ie = 1.0 / eta;
#pragma unroll
      for (int j = 0; j < kNpl; ++j) r.v[j] = ie * (imul(kx, p.v[j]) - fx.v[j]);
      U = seg_solve(q, r, imul(-kx / (2.0 * k * eta), pH),
                    imul(kx / (2.0 * k * eta), p0), H, l);
#pragma unroll
      for (int j = 0; j < kNpl; ++j) r.v[j] = ie * (imul(ky, p.v[j]) - fy.v[j]);
      V = seg_solve(q, r, imul(-ky / (2.0 * k * eta), pH),
                    imul(ky / (2.0 * k * eta), p0), H, l);
      const Vec dp_ = seg_deriv(p, l, s2H);
#pragma unroll
      for (int j = 0; j < kNpl; ++j) r.v[j] = ie * (dp_.v[j] - fz.v[j]);
      W = seg_solve(q, r, (0.5 / eta) * pH, (0.5 / eta) * p0, H, l);

      // wall correction, evaluated on all nodes and transformed
      const Z2 u0 = -1.0 * bsum_bottom(U), v0 = -1.0 * bsum_bottom(V),
               w0 = -1.0 * bsum_bottom(W);
      double fb[kNpl], E[kNpl], ZE[kNpl];
#pragma unroll
      for (int j = 0; j < kNpl; ++j) {
        const int c = 4 * l + j;
        fb[j] = c < N ? exp(-k * zc[c]) : 0.0;
      }
      seg_basis(fb, zc, Mf, N, l, E, ZE);
      if (dp.geometry == 0) {
        const Z2 Ac = imul(k, w0) + kx * u0 + ky * v0;
        const Z2 Bc = k * w0 - imul(kx, u0) - imul(ky, v0);
        const double rx = kx / k, ry = ky / k;
#pragma unroll
        for (int j = 0; j < kNpl; ++j) {
          U.v[j] = U.v[j] + (-rx * ZE[j]) * Ac + E[j] * u0;
          V.v[j] = V.v[j] + (-ry * ZE[j]) * Ac + E[j] * v0;
          W.v[j] = W.v[j] + ZE[j] * Bc + E[j] * w0;
        }
      } else {
        const Z2 uH = -1.0 * bsum_top(U), vH = -1.0 * bsum_top(V),
                 wH = -1.0 * bsum_top(W);
        const double Ex = exp(-k * H);
        const double hh = H / (2.0 * eta), e2 = 1.0 / (2.0 * eta);
        const Z2 uL0 = (1.0 / k) * (kx * u0 + ky * v0);
        const Z2 uT0 = (1.0 / k) * (kx * v0 - ky * u0);
        const Z2 uLH = (1.0 / k) * (kx * uH + ky * vH);
        const Z2 uTH = (1.0 / k) * (kx * vH - ky * uH);
        double M6[6][6] = {{0, 0, 1, Ex, 0, 0},
                           {0, 0, 0, 0, 1, Ex},
                           {hh * Ex, -hh, Ex, 1, 0, 0},
                           {hh * Ex, hh, 0, 0, Ex, 1},
                           {e2, e2 * Ex, k, k * Ex, -k, k * Ex},
                           {e2 * Ex, e2, k * Ex, k, -k * Ex, k}};
        Z2 X[6] = {imul(1.0, uL0), w0, imul(1.0, uLH), wH, zmk(0, 0), zmk(0, 0)};
        solve6(M6, X);
        const Z2 C0 = X[0], D0 = X[1];
        const Z2 CL = imul(-1.0, X[2]), DL = imul(-1.0, X[3]);
        const Z2 Cz = X[4], Dz = X[5];
        const double det = 1.0 - Ex * Ex;
        const Z2 CT = zdiv(uT0 - Ex * uTH, det);
        const Z2 DT = zdiv(uTH - Ex * uT0, det);
        const double rx = kx / k, ry = ky / k;
        const Z2 Cx = rx * CL - ry * CT, Cy = ry * CL + rx * CT;
        const Z2 Dx = rx * DL - ry * DT, Dy = ry * DL + rx * DT;
        double Ep[kNpl], ZEp[kNpl];
#pragma unroll
        for (int j = 0; j < kNpl; ++j) {
          const int c = 4 * l + j;
          fb[j] = c < N ? exp(k * (zc[c] - H)) : 0.0;
        }
        seg_basis(fb, zc, Mf, N, l, Ep, ZEp);
        const double ax = kx / (2.0 * eta * k), ay = ky / (2.0 * eta * k);
        const Z2 pu0 = imul(-ax, C0), pu1 = imul(ax, D0);
        const Z2 pv0 = imul(-ay, C0), pv1 = imul(ay, D0);
#pragma unroll
        for (int j = 0; j < kNpl; ++j) {
          U.v[j] = U.v[j] + ZE[j] * pu0 + ZEp[j] * pu1 + E[j] * Cx + Ep[j] * Dx;
          V.v[j] = V.v[j] + ZE[j] * pv0 + ZEp[j] * pv1 + E[j] * Cy + Ep[j] * Dy;
          W.v[j] = W.v[j] + (e2 * ZE[j]) * C0 + (e2 * ZEp[j]) * D0 + E[j] * Cz +
                   Ep[j] * Dz;
        }
      }
    }
  }
  DU = seg_deriv(U, l, s2H);
  DV = seg_deriv(V, l, s2H);

  // coefficients to LDS, then each lane evaluates whole band nodes
  {
    const Vec* vs[5] = {&U, &V, &W, &DU, &DV};
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
      for (int j = 0; j < kNpl; ++j) {
        C t;
        t.x = (T)vs[v]->v[j].x;
        t.y = (T)vs[v]->v[j].y;
        buf[(cl * 5 + v) * 32 + 4 * l + j] = t;
      }
  }
  __syncthreads();
  if (!valid) return;
  const C* cb = buf + cl * 5 * 32;
  const double sc = cp.scale;
  for (int c = l; c < P; c += kSeg) {
    const int ca = lo + c;
    const double* prow = Pi + ca * N;
    Z2 s[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) s[v] = zmk(0, 0);
    for (int n = 0; n < N; ++n) {
      const double pc = prow[n];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const C t = cb[v * 32 + n];
        s[v] = s[v] + pc * zmk((double)t.x, (double)t.y);
      }
    }
    Z2 o[6];
    o[0] = s[0];
    o[1] = s[1];
    o[2] = s[2];
    o[3] = 0.5 * (imul(ky, s[2]) - s[4]);
    o[4] = 0.5 * (s[3] - imul(kx, s[2]));
    o[5] = 0.5 * (imul(kx, s[1]) - imul(ky, s[0]));
#pragma unroll
    for (int ch = 0; ch < 6; ++ch) {
      C t;
      t.x = (T)(sc * o[ch].x);
      t.y = (T)(sc * o[ch].y);
      out[(ch * N + ca) * PS + idx] = t;
    }
  }
}

hipError_t launch_columns_seg(const fcmdp_solver* s, const void* spec_in,
                              void* spec_out, hipStream_t st) {
  ColParams cp;
  cp.dp = s->dp;
  cp.scale = 1.0 / ((double)s->dp.Nx * (double)s->dp.Ny);
  const int K = s->dp.Nkx * s->dp.Ny;
  if (s->mixed) {
    constexpr int cols = ColsPerBlock<float>::value;
    hipLaunchKernelGGL(k_columns_seg<float>, dim3((K + cols - 1) / cols),
                       dim3(cols * kSeg), cols * 5 * 32 * sizeof(float2), st,
                       cp, s->band, (const float2*)spec_in, (float2*)spec_out,
                       s->zc, s->dct_f, s->dct_i);
  } else {
    constexpr int cols = ColsPerBlock<double>::value;
    hipLaunchKernelGGL(k_columns_seg<double>, dim3((K + cols - 1) / cols),
                       dim3(cols * kSeg), cols * 5 * 32 * sizeof(double2), st,
                       cp, s->band, (const double2*)spec_in, (double2*)spec_out,
                       s->zc, s->dct_f, s->dct_i);
  }
  return hipGetLastError();
}

}  // namespace fcmdp
