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
// DPP moves inside 16-lane rows (an 8-lane group is half a row; values that
// cross a group edge are discarded by the callers' lane guards).
//   from_up<K>(v):   value of lane l + K    (row_shl:K)
//   from_down<K>(v): value of lane l - K    (row_shr:K)
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(dpp_i<CTRL>(hi), dpp_i<CTRL>(lo));
}
template <int K> __device__ __forceinline__ double from_up(double v) {
  return dpp_d<0x100 + K>(v);
}
template <int K> __device__ __forceinline__ double from_down(double v) {
  return dpp_d<0x110 + K>(v);
}
template <int K> __device__ __forceinline__ Z2 from_up(Z2 a) {
  return zmk(from_up<K>(a.x), from_up<K>(a.y));
}
template <int K> __device__ __forceinline__ Z2 from_down(Z2 a) {
  return zmk(from_down<K>(a.x), from_down<K>(a.y));
}

// sum over the 8 lanes of a group: quad_perm xor 1, xor 2, then the
// half-row mirror pairs each quad with the other quad of the group
__device__ __forceinline__ double red(double a) {
  a += dpp_d<0xB1>(a);
  a += dpp_d<0x4E>(a);
  a += dpp_d<0x141>(a);
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
  {
    Z2 tE = from_up<1>(sE), tO = from_up<1>(sO);
    if (l + 1 < kSeg) { sE = sE + tE; sO = sO + tO; }
    tE = from_up<2>(sE); tO = from_up<2>(sO);
    if (l + 2 < kSeg) { sE = sE + tE; sO = sO + tO; }
    tE = from_up<4>(sE); tO = from_up<4>(sO);
    if (l + 4 < kSeg) { sE = sE + tE; sO = sO + tO; }
  }
  Z2 SE = from_up<1>(sE);
  Z2 SO = from_up<1>(sO);
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

// 1/x from the hardware estimate and two Newton steps (within an ulp or two
// of the rounded quotient; x is a normal, finite number here).
__device__ __forceinline__ double frcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// Operator data of one parity for the Robin BVP (depends on kappa only).
// Slot s = 0, 1 of lane l is unknown i = 2l + s, coefficient m = 2i + p.
// Only what the scans produce is kept; the row coefficients are recomputed.
struct Par {
  double alpha[2];
  double P[2];
  double invD[2];
  double invEP;        // 1 / sum_i e_i P_i (dense boundary row)
};

struct Row {
  double lo, di, up;   // B^2 row m: c_{m-2}/(4m(m-1)), 1/(2(m^2-1)), 1/(4m(m+1))
  bool row;            // an interior row (m >= 2, m < N)
};

// B^2 row coefficients by m, computed at compile time (no divisions in the
// kernels): lo = c_{m-2}/(4m(m-1)), di = 1/(2(m^2-1)), up = 1/(4m(m+1)).
struct RowTable {
  double lo[kMaxNz], di[kMaxNz], up[kMaxNz];
  constexpr RowTable() : lo(), di(), up() {
    for (int m = 2; m < kMaxNz; ++m) {
      lo[m] = (m == 2 ? 2.0 : 1.0) / (4.0 * m * (m - 1));
      di[m] = 1.0 / (2.0 * ((double)m * m - 1.0));
      up[m] = 1.0 / (4.0 * m * (m + 1));
    }
  }
};
__constant__ RowTable kRowTable = RowTable();

__device__ inline Row row_of(int m, int N) {
  Row r;
  r.row = m >= 2 && m < N;
  const int mm = r.row ? m : 2;
  r.lo = r.row ? kRowTable.lo[mm] : 0.0;
  r.di = r.row ? kRowTable.di[mm] : 0.0;
  r.up = (r.row && m + 2 < N) ? kRowTable.up[mm] : 0.0;
  return r;
}

__device__ inline void m2mul(const double* A, const double* B, double* C) {
  C[0] = A[0] * B[0] + A[1] * B[2];
  C[1] = A[0] * B[1] + A[1] * B[3];
  C[2] = A[2] * B[0] + A[3] * B[2];
  C[3] = A[2] * B[1] + A[3] * B[3];
}

__device__ __forceinline__ Par seg_prepare(double kappa, int N, int l, int p) {
  Par q;
  const double k2 = kappa * kappa;
  double T[2][4];
  double Dd[2], Uu[2], e[2];
  bool act[2], row[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int m = 4 * l + 2 * s + p;
    act[s] = m < N;
    const Row rw = row_of(m, N);
    row[s] = rw.row;
    e[s] = act[s] ? (double)m * m + kappa : 0.0;
    if (row[s]) {
      Dd[s] = 1.0 + k2 * rw.di;
      Uu[s] = -k2 * rw.up;
      T[s][0] = 0.0; T[s][1] = k2 * rw.lo; T[s][2] = Uu[s]; T[s][3] = Dd[s];
    } else {
      Dd[s] = 1.0;
      Uu[s] = 0.0;
      T[s][0] = 1.0; T[s][1] = 0.0; T[s][2] = 0.0; T[s][3] = 1.0;
    }
  }
  // suffix products of the 2x2 Moebius matrices; only ratios matter, so each
  // partial product is rescaled by a power of two (exact) to keep it near 1
  double Y[4];
  m2mul(T[0], T[1], Y);
  auto mstep = [&](double* Yk, bool take) {
    if (take) {
      double Z[4];
      m2mul(Y, Yk, Z);
      const double sc = fmax(fmax(fabs(Z[0]), fabs(Z[1])), fmax(fabs(Z[2]), fabs(Z[3])));
      const int e = sc > 0.0 ? -ilogb(sc) : 0;
#pragma unroll
      for (int c = 0; c < 4; ++c) Y[c] = ldexp(Z[c], e);
    }
  };
  {
    double Yk[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) Yk[c] = from_up<1>(Y[c]);
    mstep(Yk, l + 1 < kSeg);
#pragma unroll
    for (int c = 0; c < 4; ++c) Yk[c] = from_up<2>(Y[c]);
    mstep(Yk, l + 2 < kSeg);
#pragma unroll
    for (int c = 0; c < 4; ++c) Yk[c] = from_up<4>(Y[c]);
    mstep(Yk, l + 4 < kSeg);
  }
  double X[4];
  {
#pragma unroll
    for (int c = 0; c < 4; ++c) X[c] = from_up<1>(Y[c]);
    if (l == kSeg - 1) { X[0] = 1.0; X[1] = 0.0; X[2] = 0.0; X[3] = 1.0; }
  }
  double S1[4], S0[4];
  m2mul(T[1], X, S1);
  m2mul(T[0], S1, S0);
  q.alpha[1] = S1[1] * frcp(S1[3]);
  q.alpha[0] = S0[1] * frcp(S0[3]);
  if (l == 0) q.alpha[0] = 1.0;              // i = 0: P_0 = 1
  if (!act[0]) q.alpha[0] = 0.0;
  if (!act[1]) q.alpha[1] = 0.0;
  // Delta_i = D_i + U_i alpha_{i+1}
  double anext[2];
  anext[0] = q.alpha[1];
  {
    const double t = from_up<1>(q.alpha[0]);
    anext[1] = (l + 1 < kSeg) ? t : 0.0;
  }
#pragma unroll
  for (int s = 0; s < 2; ++s)
    q.invD[s] = row[s] ? frcp(Dd[s] + Uu[s] * anext[s]) : 0.0;
  // prefix products P_i = alpha_i P_{i-1}
  double Yp = q.alpha[0] * q.alpha[1];
  {
    double t = from_down<1>(Yp);
    if (l >= 1) Yp *= t;
    t = from_down<2>(Yp);
    if (l >= 2) Yp *= t;
    t = from_down<4>(Yp);
    if (l >= 4) Yp *= t;
  }
  double Pin = from_down<1>(Yp);
  if (l == 0) Pin = 1.0;
  q.P[0] = q.alpha[0] * Pin;
  q.P[1] = q.alpha[1] * q.P[0];
  q.invEP = frcp(red(e[0] * q.P[0] + e[1] * q.P[1]));
  return q;
}

// Robin BVP y'' - k^2 y = r, (d/dz + k) y(H) = gH, (d/dz - k) y(0) = g0.
__device__ __forceinline__ Vec seg_solve(const Par* q, const Vec& r, Z2 gH, Z2 g0, double H,
                         double kappa, int N, int l) {
  const double h2 = 0.25 * H * H;
  const double k2 = kappa * kappa;
  Vec y;
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const Par& Q = q[p];
    const int m0 = 4 * l + p, m1 = 4 * l + 2 + p;
    const Row w0 = row_of(m0, N), w1 = row_of(m1, N);
    const Z2 r0 = r.v[p], r1 = r.v[2 + p];
    const Z2 rm2 = from_down<1>(r1);                     // r_{m-2} of slot 0
    const Z2 rp2 = from_up<1>(r0);                       // r_{m+2} of slot 1
    const Z2 R0 = h2 * (w0.lo * rm2 - w0.di * r0 + w0.up * r1);
    const Z2 R1 = h2 * (w1.lo * r0 - w1.di * r1 + w1.up * rp2);
    const Z2 b0 = Q.invD[0] * R0, b1 = Q.invD[1] * R1;
    const double a0 = k2 * w0.up * Q.invD[0];   // -U_i / Delta_i
    const double a1 = k2 * w1.up * Q.invD[1];
    // beta: suffix affine recurrence beta_i = a_i beta_{i+1} + b_i
    double A = a0 * a1;
    Z2 B = a0 * b1 + b0;
    {
      double Ak = from_up<1>(A);
      Z2 Bk = from_up<1>(B);
      if (l + 1 < kSeg) { B = A * Bk + B; A = A * Ak; }
      Ak = from_up<2>(A);
      Bk = from_up<2>(B);
      if (l + 2 < kSeg) { B = A * Bk + B; A = A * Ak; }
      Ak = from_up<4>(A);
      Bk = from_up<4>(B);
      if (l + 4 < kSeg) { B = A * Bk + B; A = A * Ak; }
    }
    Z2 bin = from_up<1>(B);
    if (l == kSeg - 1) bin = zmk(0, 0);
    const Z2 be1 = a1 * bin + b1;
    Z2 be0 = a0 * be1 + b0;
    if (l == 0) be0 = zmk(0, 0);
    // Q_i = alpha_i Q_{i-1} + beta_i (prefix), Q_0 = 0
    double Aq = Q.alpha[1] * Q.alpha[0];
    Z2 Bq = Q.alpha[1] * be0 + be1;
    {
      double Ak = from_down<1>(Aq);
      Z2 Bk = from_down<1>(Bq);
      if (l >= 1) { Bq = Aq * Bk + Bq; Aq = Aq * Ak; }
      Ak = from_down<2>(Aq);
      Bk = from_down<2>(Bq);
      if (l >= 2) { Bq = Aq * Bk + Bq; Aq = Aq * Ak; }
      Ak = from_down<4>(Aq);
      Bk = from_down<4>(Bq);
      if (l >= 4) { Bq = Aq * Bk + Bq; Aq = Aq * Ak; }
    }
    Z2 qin = from_down<1>(Bq);
    if (l == 0) qin = zmk(0, 0);
    const Z2 Q0 = Q.alpha[0] * qin + be0;
    const Z2 Q1 = Q.alpha[1] * Q0 + be1;
    const double e0 = m0 < N ? (double)m0 * m0 + kappa : 0.0;
    const double e1 = m1 < N ? (double)m1 * m1 + kappa : 0.0;
    const Z2 eQ = red(e0 * Q0 + e1 * Q1);
    const Z2 g = p == 0 ? (0.25 * H) * (gH - g0) : (0.25 * H) * (gH + g0);
    const Z2 y0 = Q.invEP * (g - eQ);
    y.v[p] = Q.P[0] * y0 + Q0;
    y.v[2 + p] = Q.P[1] * y0 + Q1;
  }
  return y;
}

// 6x6 real system with complex right-hand side, one row per lane of the
// 8-lane group (lanes 6, 7 idle): Gaussian elimination with partial pivoting.
// A lane passes its row (a[0..5], b); on return lanes 0..5 hold x[lane].
__device__ __forceinline__ Z2 seg_solve6(double a[6], Z2 b, int l) {
  const bool active = l < 6;
  for (int c = 0; c < 6; ++c) {
    // pivot: largest |a[c]| among rows c..5 (lowest lane wins ties)
    double v = (active && l >= c) ? fabs(a[c]) : -1.0;
    int who = l;
#pragma unroll
    for (int m = 1; m < kSeg; m <<= 1) {
      const double ov = __shfl_xor(v, m, kSeg);
      const int ow = __shfl_xor(who, m, kSeg);
      if (ov > v || (ov == v && ow < who)) { v = ov; who = ow; }
    }
    // swap rows c and who
    double pr[6];
    Z2 pb;
#pragma unroll
    for (int k = 0; k < 6; ++k) pr[k] = shd(a[k], who);
    pb = shz(b, who);
    double cr[6];
    Z2 cb;
#pragma unroll
    for (int k = 0; k < 6; ++k) cr[k] = shd(a[k], c);
    cb = shz(b, c);
    if (l == who && who != c) {
#pragma unroll
      for (int k = 0; k < 6; ++k) a[k] = cr[k];
      b = cb;
    }
    if (l == c) {
#pragma unroll
      for (int k = 0; k < 6; ++k) a[k] = pr[k];
      b = pb;
    }
    // eliminate below the pivot (pivot row = pr, pb)
    if (active && l > c) {
      const double f = a[c] / pr[c];
#pragma unroll
      for (int k = 0; k < 6; ++k) a[k] -= f * pr[k];
      b = b - f * pb;
    }
  }
  // back substitution: x_c = (b_c - sum_{k>c} a_ck x_k) / a_cc
  Z2 x = zmk(0, 0);
  for (int c = 5; c >= 0; --c) {
    Z2 s = b;
#pragma unroll
    for (int k = 0; k < 6; ++k)
      if (k > c) s = s - a[k] * shz(x, k);
    const Z2 xc = zdiv(s, a[c]);
    const Z2 xb = shz(xc, c);
    if (l == c) x = xb;
  }
  return x;
}

// k = 0: y'' = r with y(0) = 0 and y'(H) = 0 (bottom wall) or y(H) = 0.
__device__ __forceinline__ Vec seg_zero_mode(const Vec& r, double H, int N, int geometry,
                             int l, double a0 = 0.0, double aH = 0.0,
                             double g0 = 0.0, double gH = 0.0) {
  const double h2 = 0.25 * H * H;
  Vec y = vzero();
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const Z2 r0 = r.v[p], r1 = r.v[2 + p];
    const Z2 rm2 = from_down<1>(r1);
    const Z2 rp2 = from_up<1>(r0);
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
  const bool slip = geometry == 1 && (a0 != 0.0 || aH != 0.0 || g0 != 0.0 || gH != 0.0);
  Z2 y0s = zmk(0, 0), y1s = zmk(0, 0), sdm = zmk(0, 0);
  if (slip || a0 != 0.0) {       // Robin conditions, as in ps_zero_mode
#pragma unroll
    for (int j = 0; j < kNpl; ++j) {
      const double n = 4.0 * l + j;
      sdm = sdm + (((j & 1) ? 1.0 : -1.0) * n * n) * y.v[j];
    }
    sdm = red(sdm);
  }
  if (slip) {
    y1s = frcp(2.0 + a0 + aH) * (zmk(gH - g0, 0) + sm - sp - a0 * sdm - aH * sn2);
    y0s = zmk(gH, 0) - sp - aH * sn2 - (1.0 + aH) * y1s;
  }
  if (l == 0) {
    if (geometry == 0) {
      // y'(H) = 0: y1 = -sn2; y(0) - l_0 y'(0) = g0 (a0 = 2 l_0 / H):
      // y0 = g0 + y1 - sm + a0 (y1 + sdm)
      y.v[1] = -1.0 * sn2;
      y.v[0] = y.v[1] - sm;
      if (g0 != 0.0) y.v[0] = y.v[0] + zmk(g0, 0);
      if (a0 != 0.0) y.v[0] = y.v[0] + a0 * (sdm - sn2);
    } else if (slip) {
      y.v[0] = y0s;
      y.v[1] = y1s;
    } else {
      y.v[0] = -0.5 * (sp + sm);
      y.v[1] = -0.5 * (sp - sm);
    }
  }
  return y;
}

// z-derivative sums at the walls, in units of 2/H: top = sum n^2 a_n
// (T_n'(1) = n^2), bot = sum (-1)^(n+1) n^2 a_n (T_n'(-1)); four consecutive
// coefficients per lane (n = 4 l + j)
__device__ inline void seg_dsums(const Vec& a, int l, Z2& top, Z2& bot) {
  Z2 t = zmk(0, 0), b = zmk(0, 0);
#pragma unroll
  for (int j = 0; j < kNpl; ++j) {
    const double n = 4.0 * l + j;
    t = t + (n * n) * a.v[j];
    b = b + (((j & 1) ? 1.0 : -1.0) * n * n) * a.v[j];
  }
  top = red(t);
  bot = red(b);
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
#pragma unroll 4
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

// ---- parity-split layout ----------------------------------------------------
// The even and odd coefficient systems are independent except through the
// derivative, so the eight lanes of a column split by parity: lane l has
// parity p = l / 4 and position q = l % 4 in its group, and slot s (0..3)
// holds unknown i = 4 q + s of that parity, coefficient m = 2 i + p = 8 q +
// 2 s + p.  Every scan then runs over four lanes (two steps) for one parity
// instead of over eight lanes (three steps) for both.
__device__ __forceinline__ int ps_m(int l, int s) { return 8 * (l & 3) + 2 * s + (l >> 2); }

// sum over the four lanes of a parity group (one quad)
__device__ __forceinline__ double red4(double a) {
  a += dpp_d<0xB1>(a);
  a += dpp_d<0x4E>(a);
  return a;
}
__device__ inline Z2 red4(Z2 a) { return zmk(red4(a.x), red4(a.y)); }
// value of the same slot in the other parity group (lane l xor 4)
// (ds_swizzle bit mode: and-mask 31, or-mask 0, xor-mask 4)
__device__ __forceinline__ double swz_xor4(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_ds_swizzle(hi, 0x101F),
                          __builtin_amdgcn_ds_swizzle(lo, 0x101F));
}
__device__ __forceinline__ Z2 other_group(Z2 a) {
  return zmk(swz_xor4(a.x), swz_xor4(a.y));
}

struct Par4 {
  double alpha[kNpl];
  double P[kNpl];
  double invD[kNpl];
  double invEP;        // 1 / sum_i e_i P_i (dense boundary row)
};

// Operator data of this lane's parity for the Robin BVP (kappa only); see
// seg_prepare for the two-slot form of the same recurrences.
__device__ __forceinline__ Par4 ps_prepare(double kappa, int N, int l) {
  Par4 q;
  const int g = l & 3;
  const double k2 = kappa * kappa;
  double T[kNpl][4];
  double Dd[kNpl], Uu[kNpl], e[kNpl];
  bool act[kNpl], row[kNpl];
#pragma unroll
  for (int s = 0; s < kNpl; ++s) {
    const int m = ps_m(l, s);
    act[s] = m < N;
    const Row rw = row_of(m, N);
    row[s] = rw.row;
    e[s] = act[s] ? (double)m * m + kappa : 0.0;
    if (row[s]) {
      Dd[s] = 1.0 + k2 * rw.di;
      Uu[s] = -k2 * rw.up;
      T[s][0] = 0.0; T[s][1] = k2 * rw.lo; T[s][2] = Uu[s]; T[s][3] = Dd[s];
    } else {
      Dd[s] = 1.0;
      Uu[s] = 0.0;
      T[s][0] = 1.0; T[s][1] = 0.0; T[s][2] = 0.0; T[s][3] = 1.0;
    }
  }
  auto norm = [](double* Z) {
    const double sc = fmax(fmax(fabs(Z[0]), fabs(Z[1])), fmax(fabs(Z[2]), fabs(Z[3])));
    const int ex = sc > 0.0 ? -ilogb(sc) : 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) Z[c] = ldexp(Z[c], ex);
  };
  // product of this lane's four Moebius matrices, then suffix products over
  // the lanes of the group (rescaled by powers of two; only ratios matter)
  double Y[4], Z[4];
  m2mul(T[2], T[3], Z);
  m2mul(T[1], Z, Y);
  m2mul(T[0], Y, Z);
  norm(Z);
#pragma unroll
  for (int c = 0; c < 4; ++c) Y[c] = Z[c];
  {
    double Yk[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) Yk[c] = from_up<1>(Y[c]);
    if (g + 1 < 4) { m2mul(Y, Yk, Z); norm(Z); for (int c = 0; c < 4; ++c) Y[c] = Z[c]; }
#pragma unroll
    for (int c = 0; c < 4; ++c) Yk[c] = from_up<2>(Y[c]);
    if (g + 2 < 4) { m2mul(Y, Yk, Z); norm(Z); for (int c = 0; c < 4; ++c) Y[c] = Z[c]; }
  }
  double X[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) X[c] = from_up<1>(Y[c]);
  if (g == 3) { X[0] = 1.0; X[1] = 0.0; X[2] = 0.0; X[3] = 1.0; }
  double Sx[4];
#pragma unroll
  for (int s = kNpl - 1; s >= 0; --s) {
    m2mul(T[s], X, Sx);
    q.alpha[s] = Sx[1] * frcp(Sx[3]);
    norm(Sx);
#pragma unroll
    for (int c = 0; c < 4; ++c) X[c] = Sx[c];
  }
  if (g == 0) q.alpha[0] = 1.0;                // i = 0: P_0 = 1
#pragma unroll
  for (int s = 0; s < kNpl; ++s)
    if (!act[s]) q.alpha[s] = 0.0;
  // Delta_i = D_i + U_i alpha_{i+1}
  double anext[kNpl];
#pragma unroll
  for (int s = 0; s + 1 < kNpl; ++s) anext[s] = q.alpha[s + 1];
  {
    const double t = from_up<1>(q.alpha[0]);
    anext[kNpl - 1] = (g + 1 < 4) ? t : 0.0;
  }
#pragma unroll
  for (int s = 0; s < kNpl; ++s)
    q.invD[s] = row[s] ? frcp(Dd[s] + Uu[s] * anext[s]) : 0.0;
  // prefix products P_i = alpha_i P_{i-1}
  double Yp = q.alpha[0] * q.alpha[1] * q.alpha[2] * q.alpha[3];
  {
    double t = from_down<1>(Yp);
    if (g >= 1) Yp *= t;
    t = from_down<2>(Yp);
    if (g >= 2) Yp *= t;
  }
  double Pin = from_down<1>(Yp);
  if (g == 0) Pin = 1.0;
  q.P[0] = q.alpha[0] * Pin;
#pragma unroll
  for (int s = 1; s < kNpl; ++s) q.P[s] = q.alpha[s] * q.P[s - 1];
  double ep = 0.0;
#pragma unroll
  for (int s = 0; s < kNpl; ++s) ep += e[s] * q.P[s];
  q.invEP = frcp(red4(ep));
  return q;
}

// Robin BVP y'' - k^2 y = r, (d/dz + k) y(H) = gH, (d/dz - k) y(0) = g0, for
// this lane's parity (same recurrences as seg_solve, four slots per lane).
__device__ __forceinline__ Vec ps_solve(const Par4& Q, const Vec& r, Z2 gH, Z2 g0,
                                        double H, double kappa, int N, int l) {
  const int g = l & 3, p = l >> 2;
  const double h2 = 0.25 * H * H;
  const double k2 = kappa * kappa;
  const Z2 rm2 = from_down<1>(r.v[kNpl - 1]);        // r_{m-2} of slot 0
  const Z2 rp2 = from_up<1>(r.v[0]);                 // r_{m+2} of slot 3
  Z2 b[kNpl];
  double a[kNpl];
#pragma unroll
  for (int s = 0; s < kNpl; ++s) {
    const Row w = row_of(ps_m(l, s), N);
    const Z2 rm = s == 0 ? rm2 : r.v[s - 1];
    const Z2 rp = s == kNpl - 1 ? rp2 : r.v[s + 1];
    const Z2 R = h2 * (w.lo * rm - w.di * r.v[s] + w.up * rp);
    b[s] = Q.invD[s] * R;
    a[s] = k2 * w.up * Q.invD[s];                    // -U_i / Delta_i
  }
  // beta: suffix affine recurrence beta_i = a_i beta_{i+1} + b_i
  double A = a[kNpl - 1];
  Z2 B = b[kNpl - 1];
#pragma unroll
  for (int s = kNpl - 2; s >= 0; --s) {
    B = a[s] * B + b[s];
    A = a[s] * A;
  }
  {
    double Ak = from_up<1>(A);
    Z2 Bk = from_up<1>(B);
    if (g + 1 < 4) { B = A * Bk + B; A = A * Ak; }
    Ak = from_up<2>(A);
    Bk = from_up<2>(B);
    if (g + 2 < 4) { B = A * Bk + B; A = A * Ak; }
  }
  Z2 bin = from_up<1>(B);
  if (g == 3) bin = zmk(0, 0);
  Z2 be[kNpl];
  be[kNpl - 1] = a[kNpl - 1] * bin + b[kNpl - 1];
#pragma unroll
  for (int s = kNpl - 2; s >= 0; --s) be[s] = a[s] * be[s + 1] + b[s];
  if (g == 0) be[0] = zmk(0, 0);
  // Q_i = alpha_i Q_{i-1} + beta_i (prefix), Q_0 = 0
  double Aq = Q.alpha[0];
  Z2 Bq = be[0];
#pragma unroll
  for (int s = 1; s < kNpl; ++s) {
    Bq = Q.alpha[s] * Bq + be[s];
    Aq = Q.alpha[s] * Aq;
  }
  {
    double Ak = from_down<1>(Aq);
    Z2 Bk = from_down<1>(Bq);
    if (g >= 1) { Bq = Aq * Bk + Bq; Aq = Aq * Ak; }
    Ak = from_down<2>(Aq);
    Bk = from_down<2>(Bq);
    if (g >= 2) { Bq = Aq * Bk + Bq; Aq = Aq * Ak; }
  }
  Z2 qin = from_down<1>(Bq);
  if (g == 0) qin = zmk(0, 0);
  Z2 Qv[kNpl];
  Qv[0] = Q.alpha[0] * qin + be[0];
#pragma unroll
  for (int s = 1; s < kNpl; ++s) Qv[s] = Q.alpha[s] * Qv[s - 1] + be[s];
  Z2 eq = zmk(0, 0);
#pragma unroll
  for (int s = 0; s < kNpl; ++s) {
    const int m = ps_m(l, s);
    const double e = m < N ? (double)m * m + kappa : 0.0;
    eq = eq + e * Qv[s];
  }
  const Z2 eQ = red4(eq);
  const Z2 gg = p == 0 ? (0.25 * H) * (gH - g0) : (0.25 * H) * (gH + g0);
  const Z2 y0 = Q.invEP * (gg - eQ);
  Vec y;
#pragma unroll
  for (int s = 0; s < kNpl; ++s) y.v[s] = Q.P[s] * y0 + Qv[s];
  return y;
}

// d/dz of a Chebyshev series (times 2/H): b_m = c_m (2/H) sum over n > m of
// opposite parity of 2 n a_n (c_0 = 1/2, else 1).  Each group sums its own
// weighted coefficients from the top; the even outputs take the odd group's
// inclusive sums, the odd outputs the even group's sums from the next
// unknown on.
__device__ inline Vec ps_deriv(const Vec& a, int l, double s2H) {
  const int g = l & 3, p = l >> 2;
  Z2 w[kNpl];
#pragma unroll
  for (int s = 0; s < kNpl; ++s) w[s] = (double)ps_m(l, s) * a.v[s];
  // inclusive suffix sums over this group's unknowns
  Z2 tot = w[0] + w[1] + w[2] + w[3];
  Z2 suf = tot;                                      // sum over lanes >= g
  {
    Z2 t = from_up<1>(suf);
    if (g + 1 < 4) suf = suf + t;
    t = from_up<2>(suf);
    if (g + 2 < 4) suf = suf + t;
  }
  Z2 after = from_up<1>(suf);                        // sum over lanes > g
  if (g == 3) after = zmk(0, 0);
  Z2 S[kNpl];                                        // inclusive, per slot
  S[kNpl - 1] = w[kNpl - 1] + after;
#pragma unroll
  for (int s = kNpl - 2; s >= 0; --s) S[s] = w[s] + S[s + 1];
  // even group: sums from the next unknown on (for the odd outputs)
  Z2 X[kNpl];
#pragma unroll
  for (int s = 0; s < kNpl; ++s) X[s] = p == 1 ? S[s] : (s + 1 < kNpl ? S[s + 1] : after);
  Vec b;
#pragma unroll
  for (int s = 0; s < kNpl; ++s) {
    const Z2 v = other_group(X[s]);
    const double c = (p == 0 && g == 0 && s == 0) ? 1.0 : 2.0;
    b.v[s] = (c * s2H) * v;
  }
  return b;
}

__device__ inline Z2 ps_bsum_bottom(const Vec& a, int l) {   // sum (-1)^n a_n
  const Z2 t = a.v[0] + a.v[1] + a.v[2] + a.v[3];
  return red((l >> 2) ? -1.0 * t : t);
}
__device__ inline Z2 ps_bsum_top(const Vec& a) {             // sum a_n
  return red(a.v[0] + a.v[1] + a.v[2] + a.v[3]);
}
// the derivative sums of seg_dsums in the parity-split layout
__device__ inline void ps_dsums(const Vec& a, int l, Z2& top, Z2& bot) {
  Z2 t = zmk(0, 0);
#pragma unroll
  for (int s = 0; s < kNpl; ++s) {
    const double n = ps_m(l, s);
    t = t + (n * n) * a.v[s];
  }
  top = red(t);
  bot = red((l >> 2) ? t : -1.0 * t);                 // (-1)^(n+1)
}

// k = 0: y'' = r with y(0) = 0 and y'(H) = 0 (bottom wall) or y(H) = 0.
__device__ __forceinline__ Vec ps_zero_mode(const Vec& r, double H, int N, int geometry,
                                            int l, double a0 = 0.0, double aH = 0.0,
                                            double g0 = 0.0, double gH = 0.0) {
  const double h2 = 0.25 * H * H;
  const Z2 rm2 = from_down<1>(r.v[kNpl - 1]);
  const Z2 rp2 = from_up<1>(r.v[0]);
  Vec y = vzero();
#pragma unroll
  for (int s = 0; s < kNpl; ++s) {
    const Row w = row_of(ps_m(l, s), N);
    const Z2 rm = s == 0 ? rm2 : r.v[s - 1];
    const Z2 rp = s == kNpl - 1 ? rp2 : r.v[s + 1];
    if (w.row) y.v[s] = h2 * (w.lo * rm - w.di * r.v[s] + w.up * rp);
  }
  Z2 sp = zmk(0, 0), sm = zmk(0, 0), sn2 = zmk(0, 0);
  const double sgn = (l >> 2) ? -1.0 : 1.0;
#pragma unroll
  for (int s = 0; s < kNpl; ++s) {
    const double n = ps_m(l, s);
    sp = sp + y.v[s];
    sm = sm + sgn * y.v[s];
    sn2 = sn2 + (n * n) * y.v[s];
  }
  sp = red(sp);
  sm = red(sm);
  sn2 = red(sn2);
  // slip lengths or wall velocities: the general Robin rows
  const bool slip = geometry == 1 && (a0 != 0.0 || aH != 0.0 || g0 != 0.0 || gH != 0.0);
  Z2 y0s = zmk(0, 0), y1s = zmk(0, 0), sdm = zmk(0, 0);
  if (slip || a0 != 0.0) {
    // sdm = sum_{n >= 2} (-1)^{n+1} n^2 y_n
#pragma unroll
    for (int s = 0; s < kNpl; ++s) {
      const double n = ps_m(l, s);
      sdm = sdm + (-sgn * n * n) * y.v[s];
    }
    sdm = red(sdm);
  }
  if (slip) {
    // y(0) - l_0 y'(0) = g0, y(H) + l_H y'(H) = gH with a = 2 l / H:
    // y0 - (1 + a0) y1 = g0 - sm + a0 sdm, y0 + (1 + aH) y1 = gH - sp - aH sn2
    y1s = frcp(2.0 + a0 + aH) * (zmk(gH - g0, 0) + sm - sp - a0 * sdm - aH * sn2);
    y0s = zmk(gH, 0) - sp - aH * sn2 - (1.0 + aH) * y1s;
  }
  if ((l & 3) == 0) {                                // slot 0 holds m = 0 or 1
    const bool odd = l >> 2;
    if (geometry == 0) {
      // y'(H) = 0: y1 = -sn2; y(0) - l_0 y'(0) = g0 (wall velocity; a0 =
      // 2 l_0 / H): y0 = g0 + y1 - sm + a0 (y1 + sdm)
      y.v[0] = odd ? -1.0 * sn2 : -1.0 * sn2 - sm;
      if (!odd && g0 != 0.0) y.v[0] = y.v[0] + zmk(g0, 0);
      if (!odd && a0 != 0.0) y.v[0] = y.v[0] + a0 * (sdm - sn2);
    } else if (slip) {
      y.v[0] = odd ? y1s : y0s;
    } else {
      y.v[0] = odd ? -0.5 * (sp - sm) : -0.5 * (sp + sm);
    }
  }
  return y;
}

// Steps 2 (derivative part) to 6 for one column, from the Chebyshev
// coefficients A[0..2] of f + (1/2)(ik_y g_z, -ik_x g_z, ik_x g_y - ik_y g_x)
// and A[3], A[4] of g_x, g_y: body force, DP solve, wall correction, k = 0.
// The input vectors are fetched through `load(v)` whenever needed (v = 0..4:
// the three body-force combinations above and g_x, g_y), so that a caller
// holding them in LDS keeps few of them live in registers; the body force
// f = (A0 - 1/2 D g_y, A1 + 1/2 D g_x, A2) is rebuilt where it is used.
// `basis(which, out)` returns this lane's four Chebyshev coefficients of the
// correction's node functions: which = 0: e^{-k z}, 1: z e^{-k z},
// 2: e^{k (z - H)}, 3: z e^{k (z - H)} (the last two for the slit channel).
// SPLIT selects the parity-split coefficient layout (ps_*) instead of four
// consecutive coefficients per lane.  FO (forces only): there is no dipole
// density, `load` provides v = 0..2 only and f is A0, A1, A2 itself.
// Wall velocities of one column (unnormalised xy DFT; zero without a
// non-uniform field): (i) = u^W, v^W at z = 0, then at z = H, loaded where
// they are used (no registers held across the solve).
template <typename T>
struct WallRef {
  const cplx_t<T>* p;
  size_t K;
  int idx;
  __device__ WallRef(const DevParams& dp, int idx_)
      : p(static_cast<const cplx_t<T>*>(dp.wallspec)),
        K((size_t)dp.Nkx * dp.Ny), idx(idx_) {}
  __device__ Z2 operator()(int i) const {
    if (!p) return zmk(0, 0);
    const cplx_t<T> v = p[i * K + idx];
    return zmk((double)v.x, (double)v.y);
  }
};

template <int GEOM, bool SPLIT = false, bool FO = false, bool BS = false,
          typename Load, typename Basis, typename Wall>
__device__ __forceinline__ void seg_column_solve(const Load& load, const Basis& basis,
                                 const DevParams& dp, int N, int l,
                                 double kx, double ky, double k,
                                 const Wall& wall, Vec& U,
                                 Vec& V, Vec& W) {
  const double H = dp.H, eta = dp.eta, s2H = 2.0 / H;
  U = vzero();
  V = vzero();
  W = vzero();
  auto deriv = [&](const Vec& a) {
    if constexpr (SPLIT) return ps_deriv(a, l, s2H);
    else return seg_deriv(a, l, s2H);
  };
  auto bot = [&](const Vec& a) {
    if constexpr (SPLIT) return ps_bsum_bottom(a, l);
    else return bsum_bottom(a);
  };
  // slip lengths (App. A; a bottom wall has l_0 only) as a = 2 l / H; zero
  // for no slip
  const double a0s = 2.0 * dp.slip0 / H;
  const double aHs = GEOM == 1 ? 2.0 * dp.slipH / H : 0.0;
  // uniform wall velocities: the k = 0 wall data in the unnormalised xy DFT
  // (a constant c transforms to c Nx Ny); a non-uniform field adds its own
  // k = 0 coefficient (its mean times Nx Ny)
  const double nxy = (double)dp.Nx * (double)dp.Ny;
  auto body_x = [&]() {
    Vec f = load(0);
    if constexpr (!FO) {
      const Vec dgy = deriv(load(4));
#pragma unroll
      for (int j = 0; j < kNpl; ++j) f.v[j] = f.v[j] - 0.5 * dgy.v[j];
    }
    return f;
  };
  auto body_y = [&]() {
    Vec f = load(1);
    if constexpr (!FO) {
      const Vec dgx = deriv(load(3));
#pragma unroll
      for (int j = 0; j < kNpl; ++j) f.v[j] = f.v[j] + 0.5 * dgx.v[j];
    }
    return f;
  };
  if (k == 0.0) {
    const double g0x = nxy * dp.wall0[0] + wall(0).x;
    const double g0y = nxy * dp.wall0[1] + wall(1).x;
    const double gHx = GEOM == 1 ? nxy * dp.wallH[0] + wall(2).x : 0.0;
    const double gHy = GEOM == 1 ? nxy * dp.wallH[1] + wall(3).x : 0.0;
    Vec r = body_x();
#pragma unroll
    for (int j = 0; j < kNpl; ++j) r.v[j] = (-1.0 / eta) * r.v[j];
    if constexpr (SPLIT) U = ps_zero_mode(r, H, N, GEOM, l, a0s, aHs, g0x, gHx);
    else U = seg_zero_mode(r, H, N, GEOM, l, a0s, aHs, g0x, gHx);
    r = body_y();
#pragma unroll
    for (int j = 0; j < kNpl; ++j) r.v[j] = (-1.0 / eta) * r.v[j];
    if constexpr (SPLIT) V = ps_zero_mode(r, H, N, GEOM, l, a0s, aHs, g0y, gHy);
    else V = seg_zero_mode(r, H, N, GEOM, l, a0s, aHs, g0y, gHy);
  } else {
    const double kappa = 0.5 * k * H;
    Par q[2];
    Par4 q4;
    if constexpr (SPLIT) {
      q4 = ps_prepare(kappa, N, l);
    } else {
      q[0] = seg_prepare(kappa, N, l, 0);
      q[1] = seg_prepare(kappa, N, l, 1);
    }
    auto solve = [&](const Vec& rr, Z2 gH, Z2 g0) {
      if constexpr (SPLIT) return ps_solve(q4, rr, gH, g0, H, kappa, N, l);
      else return seg_solve(q, rr, gH, g0, H, kappa, N, l);
    };
    Vec r = deriv(load(2));
    {
      const Vec fx = body_x();
#pragma unroll
      for (int j = 0; j < kNpl; ++j) r.v[j] = r.v[j] + imul(kx, fx.v[j]);
    }
    {
      const Vec fy = body_y();
#pragma unroll
      for (int j = 0; j < kNpl; ++j) r.v[j] = r.v[j] + imul(ky, fy.v[j]);
    }
    const Vec p = solve(r, zmk(0, 0), zmk(0, 0));
    const Z2 pH = bsum_top(p), p0 = bot(p);
    const double ie = frcp(eta), ik = frcp(k);
    {
      const Vec dp_ = deriv(p);
      const Vec fz = load(2);
#pragma unroll
      for (int j = 0; j < kNpl; ++j) r.v[j] = ie * (dp_.v[j] - fz.v[j]);
    }
    W = solve(r, (0.5 * ie) * pH, (0.5 * ie) * p0);
    {
      const Vec fx = body_x();
#pragma unroll
      for (int j = 0; j < kNpl; ++j) r.v[j] = ie * (imul(kx, p.v[j]) - fx.v[j]);
    }
    const double ax = 0.5 * kx * ik * ie, ay = 0.5 * ky * ik * ie;
    U = solve(r, imul(-ax, pH), imul(ax, p0));
    {
      const Vec fy = body_y();
#pragma unroll
      for (int j = 0; j < kNpl; ++j) r.v[j] = ie * (imul(ky, p.v[j]) - fy.v[j]);
    }
    V = solve(r, imul(-ay, pH), imul(ay, p0));

    // wall correction, evaluated on all nodes and transformed; boundary
    // data u^W - u_DP at the walls (eq. bcnoslip0; App. A, eq. u0uHformula)
    const Z2 u0 = wall(0) - bot(U), v0 = wall(1) - bot(V), w0 = -1.0 * bot(W);
    double E[kNpl], ZE[kNpl];
    basis(0, E);
    basis(1, ZE);
    if constexpr (GEOM == 0) {
      const double l0 = dp.slip0;
      if constexpr (!BS) {
        const Z2 Ac = imul(k, w0) + kx * u0 + ky * v0;
        const Z2 Bc = k * w0 - imul(kx, u0) - imul(ky, v0);
        const double rx = kx * ik, ry = ky * ik;
#pragma unroll
        for (int j = 0; j < kNpl; ++j) {
          U.v[j] = U.v[j] + (-rx * ZE[j]) * Ac + E[j] * u0;
          V.v[j] = V.v[j] + (-ry * ZE[j]) * Ac + E[j] * v0;
          W.v[j] = W.v[j] + ZE[j] * Bc + E[j] * w0;
        }
      } else {
        // slip length l_0 at the bottom wall: boundary data u_0 + l_0
        // u_DP'(0), then B = (k w_0 (1 + k l_0) - i (k_x u_0 + k_y v_0)) /
        // (1 + 2 k l_0), C_x = (u_0 - l_0 (i k_x / k) B) / (1 + k l_0);
        // u += -(i k_x / k) B z e^{-kz} + C_x e^{-kz}, w += B z e^{-kz} +
        // w_0 e^{-kz}
        Z2 tu, bu, tv, bv;
        if constexpr (SPLIT) { ps_dsums(U, l, tu, bu); ps_dsums(V, l, tv, bv); }
        else { seg_dsums(U, l, tu, bu); seg_dsums(V, l, tv, bv); }
        const Z2 us0 = u0 + (l0 * s2H) * bu, vs0 = v0 + (l0 * s2H) * bv;
        const double kl0 = k * l0;
        const Z2 Bs = frcp(1.0 + 2.0 * kl0) *
                      ((k * (1.0 + kl0)) * w0 - imul(kx, us0) - imul(ky, vs0));
        const double i1 = frcp(1.0 + kl0);
        const Z2 Cx = i1 * (us0 - imul(l0 * kx * ik, Bs));
        const Z2 Cy = i1 * (vs0 - imul(l0 * ky * ik, Bs));
        const Z2 Px = imul(-kx * ik, Bs), Py = imul(-ky * ik, Bs);
#pragma unroll
        for (int j = 0; j < kNpl; ++j) {
          U.v[j] = U.v[j] + ZE[j] * Px + E[j] * Cx;
          V.v[j] = V.v[j] + ZE[j] * Py + E[j] * Cy;
          W.v[j] = W.v[j] + ZE[j] * Bs + E[j] * w0;
        }
      }
    } else {
      Z2 uH = wall(2) - bsum_top(U), vH = wall(3) - bsum_top(V);
      const Z2 wH = -1.0 * bsum_top(W);
      const double Ex = exp(-k * H);
      const double hh = 0.5 * H * ie, e2 = 0.5 * ie;
      // partial slip (App. A): boundary data u_0 = -u_DP(0) + l_0 u_DP'(0),
      // u_H = -u_DP(H) - l_H u_DP'(H) (v likewise), Robin rows below
      const double l0 = dp.slip0, lH = dp.slipH;
      const bool slip = l0 != 0.0 || lH != 0.0;
      Z2 us0 = u0, vs0 = v0;
      if (slip) {
        Z2 tu, bu, tv, bv;
        if constexpr (SPLIT) { ps_dsums(U, l, tu, bu); ps_dsums(V, l, tv, bv); }
        else { seg_dsums(U, l, tu, bu); seg_dsums(V, l, tv, bv); }
        us0 = us0 + (l0 * s2H) * bu;
        vs0 = vs0 + (l0 * s2H) * bv;
        uH = uH - (lH * s2H) * tu;
        vH = vH - (lH * s2H) * tv;
      }
      const double kl0 = k * l0, klH = k * lH;
      const Z2 uL0 = ik * (kx * us0 + ky * vs0);
      const Z2 uT0 = ik * (kx * vs0 - ky * us0);
      const Z2 uLH = ik * (kx * uH + ky * vH);
      const Z2 uTH = ik * (kx * vH - ky * uH);
      // longitudinal 6x6 system, one row per lane (unknowns C0, D0~,
      // i C_L, i D_L~, C_z, D_z~; D~ = D e^{kH})
      double row6[6] = {0, 0, 0, 0, 0, 0};
      Z2 rhs6 = zmk(0, 0);
      switch (l) {
        case 0: row6[2] = 1; row6[3] = Ex; rhs6 = imul(1.0, uL0);
                if (slip) {
                  row6[0] = -l0 * e2; row6[1] = l0 * e2 * Ex;
                  row6[2] = 1.0 + kl0; row6[3] = (1.0 - kl0) * Ex;
                }
                break;
        case 1: row6[4] = 1; row6[5] = Ex; rhs6 = w0; break;
        case 2: row6[0] = hh * Ex; row6[1] = -hh; row6[2] = Ex; row6[3] = 1;
                rhs6 = imul(1.0, uLH);
                if (slip) {
                  row6[0] = hh * Ex * (1.0 + lH / H - klH);
                  row6[1] = -hh * (1.0 + lH / H + klH);
                  row6[2] = Ex * (1.0 - klH); row6[3] = 1.0 + klH;
                }
                break;
        case 3: row6[0] = hh * Ex; row6[1] = hh; row6[4] = Ex; row6[5] = 1;
                rhs6 = wH; break;
        case 4: row6[0] = e2; row6[1] = e2 * Ex; row6[2] = k; row6[3] = k * Ex;
                row6[4] = -k; row6[5] = k * Ex; break;
        case 5: row6[0] = e2 * Ex; row6[1] = e2; row6[2] = k * Ex; row6[3] = k;
                row6[4] = -k * Ex; row6[5] = k; break;
        default: break;
      }
      const Z2 x6 = seg_solve6(row6, rhs6, l);
      const Z2 C0 = shz(x6, 0), D0 = shz(x6, 1);
      const Z2 CL = imul(-1.0, shz(x6, 2)), DL = imul(-1.0, shz(x6, 3));
      const Z2 Cz = shz(x6, 4), Dz = shz(x6, 5);
      Z2 CT, DT;
      if (!slip) {
        const double idet = frcp(1.0 - Ex * Ex);
        CT = idet * (uT0 - Ex * uTH);
        DT = idet * (uTH - Ex * uT0);
      } else {
        // (1 + k l0) C_T + (1 - k l0) e^{-kH} D~_T = u_T0,
        // e^{-kH} (1 - k lH) C_T + (1 + k lH) D~_T = u_TH
        const double idet = frcp((1.0 + kl0) * (1.0 + klH) -
                                 (1.0 - kl0) * (1.0 - klH) * Ex * Ex);
        CT = idet * ((1.0 + klH) * uT0 - ((1.0 - kl0) * Ex) * uTH);
        DT = idet * ((1.0 + kl0) * uTH - (Ex * (1.0 - klH)) * uT0);
      }
      const double rx = kx * ik, ry = ky * ik;
      const Z2 Cx = rx * CL - ry * CT, Cy = ry * CL + rx * CT;
      const Z2 Dx = rx * DL - ry * DT, Dy = ry * DL + rx * DT;
      double Ep[kNpl], ZEp[kNpl];
      basis(2, Ep);
      basis(3, ZEp);
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

template <typename T, int GEOM, bool BS>
__global__ void __launch_bounds__(256)
k_columns_seg(ColParams cp, const int* __restrict__ band,
              const cplx_t<T>* in, cplx_t<T>* out,
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
  // exact low-wavenumber vertical force (mixed slit channel): f_z's
  // coefficients come from the FP64 route, only the torque part of the third
  // combination is transformed here
  const int lcol = nyq ? -1 : lowk_col(dp, kxi, nyi);
  if (!nyq) {
    // Chebyshev transform of f + (1/2)(ik_y g_z, -ik_x g_z, ik_x g_y - ik_y g_x)
    // and of g_x, g_y (their z-derivatives enter the curl below)
    Vec A[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) A[v] = vzero();
#pragma unroll 1
    for (int c = 0; c < P; ++c) {
      const int ca = lo + c;
      Z2 val[6];
#pragma unroll
      for (int ch = 0; ch < 6; ++ch) {
        // without torques the dipole channels are zero and not read
        const C t = (ch < 3 || dp.nch_in == 6) ? in[(ch * N + ca) * PS + idx] : C{};
        val[ch] = zmk((double)t.x, (double)t.y);
      }
      Z2 comb[5];
      comb[0] = val[0] + imul(0.5 * ky, val[5]);
      comb[1] = val[1] - imul(0.5 * kx, val[5]);
      comb[2] = (lcol >= 0 && dp.lowk_coef ? zmk(0, 0) : val[2]) +
                imul(0.5 * kx, val[4]) - imul(0.5 * ky, val[3]);
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
    if (lcol >= 0 && dp.lowk_coef) {
#pragma unroll
      for (int j = 0; j < kNpl; ++j) {
        const int n = 4 * l + j;
        if (n < N) {
          const double2 e = dp.lowk_coef[(size_t)lcol * N + n];
          A[2].v[j] = A[2].v[j] + zmk(e.x, e.y);
        }
      }
    }
    auto basis = [&](int which, double out[kNpl]) {
      double fb[kNpl], E[kNpl], ZE[kNpl];
#pragma unroll
      for (int j = 0; j < kNpl; ++j) {
        const int c = 4 * l + j;
        fb[j] = c >= N ? 0.0 : (which < 2 ? exp(-k * zc[c]) : exp(k * (zc[c] - H)));
      }
      seg_basis(fb, zc, Mf, N, l, E, ZE);
#pragma unroll
      for (int j = 0; j < kNpl; ++j) out[j] = (which & 1) ? ZE[j] : E[j];
    };
    seg_column_solve<GEOM, false, false, BS>([&](int v) { return A[v]; }, basis, dp, N, l, kx,
                           ky, k, WallRef<T>(dp, idx), U, V, W);
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
#pragma unroll 1
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
      if (ch >= dp.nch_out) break;               // vorticity only when wanted
      C t;
      t.x = (T)(sc * o[ch].x);
      t.y = (T)(sc * o[ch].y);
      out[(ch * N + ca) * PS + idx] = t;
    }
  }
}

// ---------------------------------------------------------------------------
// Mixed-precision variant: the Chebyshev transforms as FP32 MFMA products at
// workgroup level (the 32 node rows of all node vectors of 16 columns, and
// back), the per-column solve in FP64 on eight lanes as above.  Per column
// the node vectors are the five body-force combinations (10 reals) and the
// wall correction's node functions e^{-k z}, z e^{-k z} (and, between two
// walls, e^{k(z-H)}, z e^{k(z-H)}), so their coefficients come out of the
// same product.
//   X[c][v]  = node values (layout in MfmaLayout)                    (LDS, fp32)
//   Cf[n][v] = sum_c Mt[n][c] X[c][v]          (v_mfma_f32_16x16x4f32)
//   solve: Cf -> coefficients of u, v, w, du/dz, dv/dz (in place)
//   D[c][v]  = sum_n T_n(s_c) Cf[n][v]         (MFMA again), then omega and
//              the 1/(Nx Ny) scale at the band nodes.
// Operand layout of v_mfma_f32_16x16x4f32 (wave64): A[i][k] comes from lane
// i + 16k, B[k][j] from lane j + 16k, and D[4(l/16) + r][l%16] is returned in
// register r of lane l.
typedef float f4v __attribute__((ext_vector_type(4)));
constexpr int kMCols = 16;                 // columns per workgroup
constexpr int kMThreads = kMCols * kSeg;   // 128
// XC columns: [0, 16 VR) the complex node vectors of the 16 columns
// (col * VR + component; rows = band nodes c - lo; VR = 10 reals for the five
// vectors, 6 for the three force components of a forces-only apply), then
// [16 VR, 16 VR + 16 NB) the NB correction node functions (col * NB + b; rows
// = all nodes c).
template <int GEOM, bool FO> struct MfmaLayout {
  static constexpr int kBasis = GEOM == 0 ? 2 : 4;     // correction node functions
  static constexpr int kVR = FO ? 6 : 10;              // reals per column
  static constexpr int kSpec = kMCols * kVR;           // spectral reals per row
  // reals per row; the odd pad spreads the eight lanes of a column (rows
  // 8 (l % 4) + 2 j + l / 4) over different LDS banks
  static constexpr int kMV = kSpec + kMCols * kBasis + 1;
  static constexpr int kSpecTiles = 2 * (kSpec / 16);  // forward, band rows
  static constexpr int kBasisTiles = 2 * kBasis;       // forward, all nodes
  static constexpr int kInvPerWave = 2 * (kSpec / 16) / (kMThreads / 64);
};

// (kx, ky) indices of column col of a group whose first column has indices
// (kx0, ky0): columns run over ky fastest.
__device__ __forceinline__ void col_index(int kx0, int ky0, int col, int Ny,
                                          int& kxi, int& kyi) {
  kxi = kx0;
  kyi = ky0 + col;
  while (kyi >= Ny) { kyi -= Ny; ++kxi; }
}

// FO: forces only (no torques in, no vorticity out): three node vectors per
// column instead of five and three output channels.
template <int GEOM, bool FO, bool BS>
__global__ void __launch_bounds__(kMThreads) __attribute__((amdgpu_waves_per_eu(2, 8)))
k_columns_mfma(ColParams cp, const int* __restrict__ band,
               const float2* in, float2* out,
               const double* __restrict__ zc, const float* __restrict__ Mf32,
               const float* __restrict__ Pi32) {
  using Lay = MfmaLayout<GEOM, FO>;
  constexpr int kMV = Lay::kMV, kSpec = Lay::kSpec, NB = Lay::kBasis;
  constexpr int VR = Lay::kVR;
  // one buffer: node values (A), then coefficients (B, C), then band node
  // values (D, E); each transform keeps its output tiles in registers until
  // every wave has finished reading its input
  __shared__ float XC[32 * kMV];
  const DevParams& dp = cp.dp;
  const int lo = band[0], hi = band[1];
  if (lo > hi) return;
  const int K = dp.Nkx * dp.Ny;
  const int N = dp.Nz;
  const int P = hi - lo + 1;
  const int Pp = (P + 3) & ~3;             // band rows padded for k-steps of 4
  const int Np = (N + 3) & ~3;             // node count padded likewise
  const size_t PS = (size_t)K;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const float H = (float)dp.H;
  const int idx0 = blockIdx.x * kMCols;
  // (kx, ky) index of the group's first column; the others follow in ky
  const int kx0 = idx0 / dp.Ny, ky0 = idx0 - kx0 * dp.Ny;
  const float kxs = (float)cp.kxs, kys = (float)cp.kys;
  const int i16 = lane & 15, k4 = lane >> 4;

  // Matrix operands of the transforms, loaded once per wavefront (before the
  // node values, so that their latency overlaps).  Wavefront w computes the
  // output rows 16 w .. 16 w + 15 of every forward tile, and the band rows
  // c0w .. c0w + 15 of every inverse tile.
  static_assert(kMThreads == 128, "two wavefronts per workgroup");
  const int ctiles = (P + 15) / 16;          // 1 or 2 (P <= N <= 32)
  const int c0w = ctiles == 2 ? wave * 16 : 0;
  float aS[8], aB[8], aI[8];
  {
    const int n = wave * 16 + i16;
    const int cI = c0w + i16;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int c = 4 * j + k4;
      aS[j] = (c < P && n < N) ? Mf32[(lo + c) * N + n] : 0.f;
      aB[j] = (c < N && n < N) ? Mf32[c * N + n] : 0.f;
      aI[j] = (cI < P && c < N) ? Pi32[(lo + cI) * N + c] : 0.f;
    }
  }

  // --- A: band node values of the body-force combinations, and the
  //     correction's node functions at all nodes --------------------------
  // each thread takes a pair of adjacent columns (one 16-byte access per
  // channel; K and the group start are even, so a pair is either inside
  // the spectrum or past its end)
  static_assert(kMCols % 2 == 0, "column pairs");
#pragma unroll
  for (int i = 0; i < 32 * (kMCols / 2) / kMThreads; ++i) {
    const int it = tid + i * kMThreads;
    const int c = it / (kMCols / 2), col = 2 * (it % (kMCols / 2));  // band-relative row
    const int idx = idx0 + col;
    float kxv[2], kyv[2];
    bool lkv[2];   // column of the exact low-wavenumber square (f_z via FP64)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      int kxi, kyi;
      col_index(kx0, ky0, col + h, dp.Ny, kxi, kyi);
      kxv[h] = kxs * (float)kxi;
      const int nyi = kyi <= dp.Ny / 2 ? kyi : kyi - dp.Ny;
      kyv[h] = kys * (float)nyi;
      lkv[h] = lowk_col(dp, kxi, nyi) >= 0;
    }
    if (c < P && idx < K) {
      // without torques the dipole channels are zero and not read
      const bool dip = !FO && dp.nch_in == 6;
      float4 v[6];
#pragma unroll
      for (int ch = 0; ch < 6; ++ch)
        v[ch] = (ch < 3 || dip)
                    ? *reinterpret_cast<const float4*>(in + (ch * N + lo + c) * PS + idx)
                    : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        float2 w[6];
#pragma unroll
        for (int ch = 0; ch < 6; ++ch)
          w[ch] = h == 0 ? make_float2(v[ch].x, v[ch].y) : make_float2(v[ch].z, v[ch].w);
        const float kx = kxv[h], ky = kyv[h];
        float* xr = XC + c * kMV + (col + h) * VR;
        // in the low-wavenumber square f_z is added after the transform
        const float2 fz = lkv[h] ? make_float2(0.f, 0.f) : w[2];
        if constexpr (FO) {
          xr[0] = w[0].x; xr[1] = w[0].y;
          xr[2] = w[1].x; xr[3] = w[1].y;
          xr[4] = fz.x; xr[5] = fz.y;
          continue;
        }
        // f~x = Fx + (1/2) i ky Gz ; f~y = Fy - (1/2) i kx Gz ;
        // f~z = Fz + (1/2)(i kx Gy - i ky Gx)
        xr[0] = w[0].x - 0.5f * ky * w[5].y;
        xr[1] = w[0].y + 0.5f * ky * w[5].x;
        xr[2] = w[1].x + 0.5f * kx * w[5].y;
        xr[3] = w[1].y - 0.5f * kx * w[5].x;
        xr[4] = fz.x - 0.5f * kx * w[4].y + 0.5f * ky * w[3].y;
        xr[5] = fz.y + 0.5f * kx * w[4].x - 0.5f * ky * w[3].x;
        xr[6] = w[3].x; xr[7] = w[3].y;
        xr[8] = w[4].x; xr[9] = w[4].y;
      }
    } else {
#pragma unroll
      for (int e = 0; e < 2 * VR; ++e) XC[c * kMV + col * VR + e] = 0.f;
    }
    // c is also the absolute node of the correction functions
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      float* br = XC + c * kMV + kSpec + (col + h) * NB;
      float eb = 0.f, ezb = 0.f, et = 0.f, ezt = 0.f;
      if (c < N && idx < K) {
        const float kx = kxv[h], ky = kyv[h];
        const float k = sqrtf(kx * kx + ky * ky);
        const float z = (float)zc[c];
        eb = expf(-k * z);
        ezb = z * eb;
        if constexpr (GEOM == 1) {
          et = expf(k * (z - H));
          ezt = z * et;
        }
      }
      br[0] = eb;
      br[1] = ezb;
      if constexpr (GEOM == 1) {
        br[2] = et;
        br[3] = ezt;
      }
    }
  }
  __syncthreads();

  // --- B: forward Chebyshev transform, Cf = Mt X ----------------------------
  //     spectral tiles sum over the band nodes, correction tiles over all;
  //     wavefront w owns the tiles (w, v0) for every column block v0
  {
    constexpr int kST = Lay::kSpecTiles / 2, kBT = Lay::kBasisTiles / 2;
    f4v acc[kST + kBT];
#pragma unroll
    for (int t = 0; t < kST + kBT; ++t) acc[t] = f4v{0.f, 0.f, 0.f, 0.f};
    // k-steps outermost: the independent tiles keep the matrix pipe busy
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float* row = XC + (4 * j + k4) * kMV + i16;
      if (4 * j < Pp) {
        float b[kST];
#pragma unroll
        for (int t = 0; t < kST; ++t) b[t] = row[t * 16];
#pragma unroll
        for (int t = 0; t < kST; ++t)
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(aS[j], b[t], acc[t], 0, 0, 0);
      }
      if (4 * j < Np) {
        float b[kBT];
#pragma unroll
        for (int t = 0; t < kBT; ++t) b[t] = row[kSpec + t * 16];
#pragma unroll
        for (int t = 0; t < kBT; ++t)
          acc[kST + t] = __builtin_amdgcn_mfma_f32_16x16x4f32(aB[j], b[t], acc[kST + t],
                                                              0, 0, 0);
      }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kST + kBT; ++t) {
      const int v0 = t < kST ? t * 16 : kSpec + (t - kST) * 16;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        XC[(wave * 16 + 4 * k4 + r) * kMV + v0 + i16] = acc[t][r];
    }
  }
  __syncthreads();

  // --- C: per-column FP64 solve on eight lanes ------------------------------
  {
    const int cl = tid / kSeg, l = tid % kSeg;
    const int idx = idx0 + cl;
    const bool valid = idx < K;
    int kxi, kyi;
    col_index(kx0, ky0, cl, dp.Ny, kxi, kyi);
    const bool nyq = !valid || kxi == dp.Nx / 2 || kyi == dp.Ny / 2;
    const double kx = cp.kxs * kxi;
    const int nyi = kyi <= dp.Ny / 2 ? kyi : kyi - dp.Ny;
    const double ky = cp.kys * nyi;
    const double k = sqrt(kx * kx + ky * ky);
    const double s2H = 2.0 / dp.H;
    // parity-split layout: slot j of lane l is coefficient 8 (l % 4) + 2 j
    // + l / 4
    const int m0 = ps_m(l, 0);
    float* cbase = XC + m0 * kMV + cl * VR;
    float* bbase = XC + m0 * kMV + kSpec + cl * NB;
    Vec U = vzero(), V = vzero(), W = vzero();
    const int lcol = nyq ? -1 : lowk_col(dp, kxi, nyi);
    if (!nyq) {
      auto load = [&](int v) {
        Vec a;
#pragma unroll
        for (int j = 0; j < kNpl; ++j) {
          float* cr = cbase + 2 * j * kMV + 2 * v;
          a.v[j] = zmk((double)cr[0], (double)cr[1]);
        }
        // low-wavenumber square: f_z's coefficients in FP64, from the FP64
        // route of the apply, or (stage entry point, no such route) from an
        // FP64 transform of the input's f_z band values
        if (v == 2 && lcol >= 0) {
          if (dp.lowk_coef) {
#pragma unroll
            for (int j = 0; j < kNpl; ++j) {
              const int m = m0 + 2 * j;
              if (m < N) {
                const double2 e = dp.lowk_coef[(size_t)lcol * N + m];
                a.v[j] = a.v[j] + zmk(e.x, e.y);
              }
            }
          } else {
            for (int c = 0; c < P; ++c) {
              const float2 t = in[(2 * N + lo + c) * PS + idx];
              const Z2 fz = zmk((double)t.x, (double)t.y);
#pragma unroll
              for (int j = 0; j < kNpl; ++j) {
                const int m = m0 + 2 * j;
                if (m < N) a.v[j] = a.v[j] + cp.dctf[(lo + c) * N + m] * fz;
              }
            }
          }
        }
        return a;
      };
      auto basis = [&](int which, double o[kNpl]) {
        if (lcol >= 0) {
          // low-wavenumber square: node functions and transform in FP64
          // (their combination cancels strongly as kH -> 0)
#pragma unroll
          for (int j = 0; j < kNpl; ++j) o[j] = 0.0;
          for (int c = 0; c < N; ++c) {
            const double z = zc[c];
            const double e = which < 2 ? exp(-k * z) : exp(k * (z - dp.H));
            const double f = (which & 1) ? z * e : e;
#pragma unroll
            for (int j = 0; j < kNpl; ++j) {
              const int m = m0 + 2 * j;
              if (m < N) o[j] = fma(cp.dctf[c * N + m], f, o[j]);
            }
          }
          return;
        }
#pragma unroll
        for (int j = 0; j < kNpl; ++j) o[j] = (double)bbase[2 * j * kMV + which];
      };
      seg_column_solve<GEOM, true, FO, BS>(load, basis, dp, N, l, kx, ky, k,
                                       WallRef<float>(dp, kxi * dp.Ny + kyi),
                                       U, V, W);
    }
    // the column's coefficients are read only by its own eight lanes (one
    // wavefront, in lockstep): overwrite them in place
    auto store = [&](int v, const Vec& a) {
#pragma unroll
      for (int j = 0; j < kNpl; ++j) {
        float* cr = cbase + 2 * j * kMV + 2 * v;
        cr[0] = (float)a.v[j].x;
        cr[1] = (float)a.v[j].y;
      }
    };
    store(0, U);
    store(1, V);
    store(2, W);
    if constexpr (!FO) {
      store(3, ps_deriv(U, l, s2H));
      store(4, ps_deriv(V, l, s2H));
    }
  }
  __syncthreads();

  // --- D: inverse transform to the band nodes, D = T Cf -----------------------
  //     wavefront w owns the tiles (c0w, v0); with one band tile the two
  //     wavefronts split the column blocks
  {
    constexpr int kIT = Lay::kInvPerWave;
    // tiles of this wavefront: with two band tiles, every column block;
    // with one, the column blocks w, w + 2, ...
    const int nt = ctiles == 2 ? kIT : kIT / 2;
    auto col0 = [&](int t) { return ctiles == 2 ? t * 16 : (wave + 2 * t) * 16; };
    f4v acc[kIT];
#pragma unroll
    for (int t = 0; t < kIT; ++t) acc[t] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (4 * j < Np) {
        const float* row = XC + (4 * j + k4) * kMV + i16;
        float b[kIT];
#pragma unroll
        for (int t = 0; t < kIT; ++t) b[t] = t < nt ? row[col0(t)] : 0.f;
#pragma unroll
        for (int t = 0; t < kIT; ++t)
          if (t < nt)
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(aI[j], b[t], acc[t], 0, 0, 0);
      }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kIT; ++t) {
      if (t < nt) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          XC[(c0w + 4 * k4 + r) * kMV + col0(t) + i16] = acc[t][r];
      }
    }
  }
  __syncthreads();

  // --- E: omega = (1/2) curl u at the nodes, scale, store ----------------------
  const float sc = (float)cp.scale;
  for (int it = tid; it < P * (kMCols / 2); it += kMThreads) {
    const int c = it / (kMCols / 2), col = 2 * (it % (kMCols / 2));
    const int idx = idx0 + col;
    if (idx >= K) continue;
    float2 o[2][6];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      int kxi, kyi;
      col_index(kx0, ky0, col + h, dp.Ny, kxi, kyi);
      const float kx = kxs * (float)kxi;
      const int nyi = kyi <= dp.Ny / 2 ? kyi : kyi - dp.Ny;
      const float ky = kys * (float)nyi;
      float* d = XC + c * kMV + (col + h) * VR;
      const float ur = d[0], ui = d[1], vr = d[2], vi = d[3], wr = d[4], wi = d[5];
      o[h][0] = make_float2(sc * ur, sc * ui);
      o[h][1] = make_float2(sc * vr, sc * vi);
      o[h][2] = make_float2(sc * wr, sc * wi);
      if constexpr (FO) continue;
      const float dur = d[6], dui = d[7], dvr = d[8], dvi = d[9];
      // ox = (i ky w - dv/dz)/2, oy = (du/dz - i kx w)/2, oz = (i kx v - i ky u)/2
      o[h][3] = make_float2(0.5f * sc * (-ky * wi - dvr), 0.5f * sc * (ky * wr - dvi));
      o[h][4] = make_float2(0.5f * sc * (dur + kx * wi), 0.5f * sc * (dui - kx * wr));
      o[h][5] = make_float2(0.5f * sc * (-kx * vi + ky * ui),
                            0.5f * sc * (kx * vr - ky * ur));
    }
    // the vorticity channels only when angular velocities are wanted
    const int nch = FO ? 3 : dp.nch_out;
#pragma unroll
    for (int ch = 0; ch < 6; ++ch)
      if (ch < nch)
        *reinterpret_cast<float4*>(out + (ch * N + lo + c) * PS + idx) =
            make_float4(o[0][ch].x, o[0][ch].y, o[1][ch].x, o[1][ch].y);
  }
}

// BS: slip length at a bottom wall (the correction's slip branch is a
// separate instance, so that the no-slip kernels keep their registers)
template <int GEOM, bool BS>
static void launch_seg_kernels(const fcmdp_solver* s, const ColParams& cp,
                               const void* spec_in, void* spec_out, hipStream_t st) {
  const int K = s->dp.Nkx * s->dp.Ny;
  if (s->mixed && s->dct_f32 && !s->force_vector_dct) {
    const dim3 g((K + kMCols - 1) / kMCols);
    if (s->dp.nch_in == 3 && s->dp.nch_out == 3)
      hipLaunchKernelGGL((k_columns_mfma<GEOM, true, BS>), g, dim3(kMThreads), 0, st,
                         cp, s->band, (const float2*)spec_in, (float2*)spec_out,
                         s->zc, s->dct_f32, s->dct_i32);
    else
      hipLaunchKernelGGL((k_columns_mfma<GEOM, false, BS>), g, dim3(kMThreads), 0, st,
                         cp, s->band, (const float2*)spec_in, (float2*)spec_out,
                         s->zc, s->dct_f32, s->dct_i32);
  } else if (s->mixed) {
    constexpr int cols = ColsPerBlock<float>::value;
    hipLaunchKernelGGL((k_columns_seg<float, GEOM, BS>), dim3((K + cols - 1) / cols),
                       dim3(cols * kSeg), cols * 5 * 32 * sizeof(float2), st,
                       cp, s->band, (const float2*)spec_in, (float2*)spec_out,
                       s->zc, s->dct_f, s->dct_i);
  } else {
    constexpr int cols = ColsPerBlock<double>::value;
    hipLaunchKernelGGL((k_columns_seg<double, GEOM, BS>), dim3((K + cols - 1) / cols),
                       dim3(cols * kSeg), cols * 5 * 32 * sizeof(double2), st,
                       cp, s->band, (const double2*)spec_in, (double2*)spec_out,
                       s->zc, s->dct_f, s->dct_i);
  }
}

hipError_t launch_columns_seg(const fcmdp_solver* s, const void* spec_in,
                              void* spec_out, hipStream_t st) {
  ColParams cp;
  cp.dp = s->dp;
  cp.scale = 1.0 / ((double)s->dp.Nx * (double)s->dp.Ny);
  cp.kxs = 2.0 * M_PI / s->dp.Lx;
  cp.kys = 2.0 * M_PI / s->dp.Ly;
  cp.dctf = s->dct_f;
  if (s->dp.geometry == 1)
    launch_seg_kernels<1, false>(s, cp, spec_in, spec_out, st);
  else if (s->dp.slip0 != 0.0)
    launch_seg_kernels<0, true>(s, cp, spec_in, spec_out, st);
  else
    launch_seg_kernels<0, false>(s, cp, spec_in, spec_out, st);
  return hipGetLastError();
}

}  // namespace fcmdp
