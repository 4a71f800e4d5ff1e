// Per-wavenumber column solve: steps 2 (Chebyshev part) to 6 of Sec. 3.4 plus
// the spectral vorticity, for every (kx, ky) column of the xy spectrum.
//
// One thread owns one column and works in float64 throughout (the mixed
// path's FP64 island).  Per column:
//   1. Chebyshev coefficients of the six node vectors (f, g) on the band of
//      planes that the particles touch (zero elsewhere), by the type-I DCT.
//   2. body force  f + (1/2) curl g  with d/dz by the Chebyshev recurrence.
//   3. k != 0: pressure BVP (eq. poissonfs, DtN eq. DtoNmapp), boundary
//      values by direct summation, three velocity BVPs (eq. momentumfs,
//      DtN eqs. DtoNmapuv, DtoNmapw) -- Sec. 3.1.
//   4. wall correction: bottom wall closed form (Sec. 3.2), slit channel
//      (App. A, no slip) from the longitudinal 6x6 + transverse 2x2 real
//      systems; evaluated on the Chebyshev nodes, transformed and added.
//   5. k = 0: w = 0 and u'' = -f/eta with the wall conditions (Sec. 3.3,
//      App. A.2).
//   6. omega = (1/2) curl u, inverse DCT to the band nodes, times 1/(Nx Ny).
//
// BVP discretisation (shared reading with the CPU oracle, stated in its own
// words there): rows m >= 2 of  y - kappa^2 B^2 y = (H^2/4) B^2 r  in the
// Chebyshev variable, plus the two Robin rows.  The system splits into even
// and odd coefficients; each half is tridiagonal plus one dense boundary row
// and is solved here in O(Nz) by elimination from the top coefficient down,
// folding the dense row along the way.
#include "fcmdp_internal.h"
#include "colmath.h"

namespace fcmdp {

// Chebyshev derivative d/dz (coefficients), b[N-1] = 0,
// c_{n-1} b_{n-1} = b_{n+1} + 2 n a_n, times 2/H.
__device__ void cheb_deriv(const Z2* a, Z2* b, int N, double H) {
  Z2 bn1 = zmk(0, 0);   // b_{n+1}
  Z2 bn = zmk(0, 0);    // b_n
  b[N - 1] = zmk(0, 0);
  for (int n = N - 1; n >= 1; --n) {
    Z2 v = bn1 + (2.0 * n) * a[n];
    if (n - 1 == 0) v = 0.5 * v;
    bn1 = bn;
    bn = v;
    b[n - 1] = v;
  }
  const double s = 2.0 / H;
  for (int n = 0; n < N; ++n) b[n] = s * b[n];
}

// Robin BVP  y'' - k^2 y = r,  (d/dz + k) y(H) = gH,  (d/dz - k) y(0) = g0
// in the integrated Chebyshev form; r, y: Chebyshev coefficients.
__device__ void bvp_robin(const Z2* r, Z2 gH, Z2 g0, double kappa, double H,
                          int N, Z2* y, double* al, Z2* be) {
  const double k2 = kappa * kappa;
  const double h2 = 0.25 * H * H;
  for (int par = 0; par < 2; ++par) {
    const int Mp = (N - par + 1) / 2;
    const Z2 g = par == 0 ? (0.25 * H) * (gH - g0) : (0.25 * H) * (gH + g0);
    double ecur;
    {
      const double n = par + 2.0 * (Mp - 1);
      ecur = n * n + kappa;
    }
    Z2 gcur = g;
    double al_up = 0.0;
    Z2 be_up = zmk(0, 0);
    for (int i = Mp - 1; i >= 1; --i) {
      const int m = par + 2 * i;
      const double cm2 = (m - 2 == 0) ? 2.0 : 1.0;
      const double lo = cm2 / (4.0 * m * (m - 1));
      const double di = 1.0 / (2.0 * (m * m - 1.0));
      const double up = (m + 2 < N) ? 1.0 / (4.0 * m * (m + 1)) : 0.0;
      Z2 Rm = lo * r[m - 2] - di * r[m];
      if (m + 2 < N) Rm = Rm + up * r[m + 2];
      Rm = h2 * Rm;
      const double L = -k2 * lo;
      const double D = 1.0 + k2 * di;
      const double U = -k2 * up;
      const double delta = D + U * al_up;
      const double a = -L / delta;
      const Z2 b = zdiv(Rm - U * be_up, delta);
      al[i] = a;
      be[i] = b;
      gcur = gcur - ecur * b;
      const double nm1 = par + 2.0 * (i - 1);
      ecur = (nm1 * nm1 + kappa) + ecur * a;
      al_up = a;
      be_up = b;
    }
    Z2 yprev = zdiv(gcur, ecur);
    y[par] = yprev;
    for (int i = 1; i < Mp; ++i) {
      yprev = al[i] * yprev + be[i];
      y[par + 2 * i] = yprev;
    }
  }
}

// k = 0: y'' = r with y(0) = 0 and y'(H) = 0 (bottom wall) or y(H) = 0
// (slit channel).  Interior rows are explicit because kappa = 0.
__device__ void bvp_zero_mode(const Z2* r, double H, int N, int geometry,
                              Z2* y) {
  const double h2 = 0.25 * H * H;
  Z2 Sp = zmk(0, 0), Sm = zmk(0, 0), Sn2 = zmk(0, 0);
  for (int m = 2; m < N; ++m) {
    const double cm2 = (m - 2 == 0) ? 2.0 : 1.0;
    Z2 v = (cm2 / (4.0 * m * (m - 1))) * r[m - 2] -
           (1.0 / (2.0 * (m * m - 1.0))) * r[m];
    if (m + 2 < N) v = v + (1.0 / (4.0 * m * (m + 1))) * r[m + 2];
    v = h2 * v;
    y[m] = v;
    Sp = Sp + v;
    Sm = Sm + ((m & 1) ? -1.0 : 1.0) * v;
    Sn2 = Sn2 + (double)(m * m) * v;
  }
  if (geometry == 0) {
    y[1] = -1.0 * Sn2;
    y[0] = y[1] - Sm;
  } else {
    y[0] = -0.5 * (Sp + Sm);
    y[1] = -0.5 * (Sp - Sm);
  }
}

// Chebyshev coefficients of a real node vector (all N nodes).
__device__ void dct_real(const double* v, const double* __restrict__ Mf,
                         int N, double* out) {
  for (int n = 0; n < N; ++n) out[n] = 0.0;
  for (int c = 0; c < N; ++c) {
    const double vc = v[c];
    const double* row = Mf + c * N;
    for (int n = 0; n < N; ++n) out[n] += row[n] * vc;
  }
}

template <typename T, int NZ>
__global__ void __launch_bounds__(64)
k_columns(ColParams cp, const int* __restrict__ band,
          const cplx_t<T>* in, cplx_t<T>* out,
          const double* __restrict__ zc, const double* __restrict__ Mf,
          const double* __restrict__ Pi) {
  const DevParams& dp = cp.dp;
  const int K = dp.Nkx * dp.Ny;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= K) return;
  const int lo = band[0], hi = band[1];
  if (lo > hi) return;
  const int N = dp.Nz;
  const size_t PS = (size_t)K;
  const int kxi = idx / dp.Ny;
  const int kyi = idx - kxi * dp.Ny;
  using C = cplx_t<T>;
  if (kxi == dp.Nx / 2 || kyi == dp.Ny / 2) {
    C zero; zero.x = T(0); zero.y = T(0);
    for (int ch = 0; ch < dp.nch_out; ++ch)
      for (int c = lo; c <= hi; ++c) out[(ch * N + c) * PS + idx] = zero;
    return;
  }
  const double kx = 2.0 * M_PI * kxi / dp.Lx;
  const int nyi = kyi <= dp.Ny / 2 ? kyi : kyi - dp.Ny;
  const double ky = 2.0 * M_PI * nyi / dp.Ly;
  const double k = sqrt(kx * kx + ky * ky);
  const double H = dp.H, eta = dp.eta;

  Z2 A[6][NZ];      // coefficient vectors
  Z2 tmp[NZ], tmp2[NZ];
  double al[NZ];
  Z2 be[NZ];

  // 1. Chebyshev transform of the band node values
  for (int ch = 0; ch < 6; ++ch) {
    for (int n = 0; n < N; ++n) A[ch][n] = zmk(0, 0);
    if (ch >= dp.nch_in) continue;                // no torques: g = 0
    for (int c = lo; c <= hi; ++c) {
      const C v = in[(ch * N + c) * PS + idx];
      const Z2 z = zmk((double)v.x, (double)v.y);
      const double* row = Mf + c * N;
      for (int n = 0; n < N; ++n) A[ch][n] = A[ch][n] + row[n] * z;
    }
  }
  // 2. body force f + (1/2) curl g  -> A[0..2]
  cheb_deriv(A[4], tmp, N, H);                      // d/dz g_y
  for (int n = 0; n < N; ++n)
    A[0][n] = A[0][n] + 0.5 * (imul(ky, A[5][n]) - tmp[n]);
  cheb_deriv(A[3], tmp, N, H);                      // d/dz g_x
  for (int n = 0; n < N; ++n)
    A[1][n] = A[1][n] + 0.5 * (tmp[n] - imul(kx, A[5][n]));
  for (int n = 0; n < N; ++n)
    A[2][n] = A[2][n] + 0.5 * (imul(kx, A[4][n]) - imul(ky, A[3][n]));

  if (k == 0.0) {
    // 5. zero mode: u'' = -f/eta, w = 0
    for (int n = 0; n < N; ++n) tmp[n] = (-1.0 / eta) * A[0][n];
    bvp_zero_mode(tmp, H, N, dp.geometry, A[3]);
    for (int n = 0; n < N; ++n) tmp[n] = (-1.0 / eta) * A[1][n];
    bvp_zero_mode(tmp, H, N, dp.geometry, A[4]);
    for (int n = 0; n < N; ++n) {
      A[0][n] = A[3][n];
      A[1][n] = A[4][n];
      A[2][n] = zmk(0, 0);
    }
  } else {
    const double kappa = 0.5 * k * H;
    // 3. pressure
    cheb_deriv(A[2], tmp, N, H);
    for (int n = 0; n < N; ++n)
      A[3][n] = imul(kx, A[0][n]) + imul(ky, A[1][n]) + tmp[n];
    bvp_robin(A[3], zmk(0, 0), zmk(0, 0), kappa, H, N, A[4], al, be);
    Z2 pH = zmk(0, 0), p0 = zmk(0, 0);
    for (int n = 0; n < N; ++n) {
      pH = pH + A[4][n];
      p0 = p0 + ((n & 1) ? -1.0 : 1.0) * A[4][n];
    }
    // velocities
    const double ie = 1.0 / eta;
    for (int n = 0; n < N; ++n) A[3][n] = ie * (imul(kx, A[4][n]) - A[0][n]);
    bvp_robin(A[3], imul(-kx / (2.0 * k * eta), pH), imul(kx / (2.0 * k * eta), p0),
              kappa, H, N, A[0], al, be);
    for (int n = 0; n < N; ++n) A[3][n] = ie * (imul(ky, A[4][n]) - A[1][n]);
    bvp_robin(A[3], imul(-ky / (2.0 * k * eta), pH), imul(ky / (2.0 * k * eta), p0),
              kappa, H, N, A[1], al, be);
    cheb_deriv(A[4], tmp, N, H);
    for (int n = 0; n < N; ++n) A[3][n] = ie * (tmp[n] - A[2][n]);
    bvp_robin(A[3], (0.5 / eta) * pH, (0.5 / eta) * p0, kappa, H, N, A[2], al,
              be);
    // 4. wall correction
    Z2 u0 = zmk(0, 0), v0 = zmk(0, 0), w0 = zmk(0, 0);
    Z2 uH = zmk(0, 0), vH = zmk(0, 0), wH = zmk(0, 0);
    for (int n = 0; n < N; ++n) {
      const double sg = (n & 1) ? -1.0 : 1.0;
      u0 = u0 - sg * A[0][n]; v0 = v0 - sg * A[1][n]; w0 = w0 - sg * A[2][n];
      uH = uH - A[0][n]; vH = vH - A[1][n]; wH = wH - A[2][n];
    }
    double bas[NZ], Em[NZ], ZEm[NZ];
    for (int c = 0; c < N; ++c) bas[c] = exp(-k * zc[c]);
    dct_real(bas, Mf, N, Em);
    for (int c = 0; c < N; ++c) bas[c] = zc[c] * exp(-k * zc[c]);
    dct_real(bas, Mf, N, ZEm);
    if (dp.geometry == 0) {
      const Z2 Acoef = imul(k, w0) + kx * u0 + ky * v0;
      const Z2 Bcoef = k * w0 - imul(kx, u0) - imul(ky, v0);
      const double rx = kx / k, ry = ky / k;
      for (int n = 0; n < N; ++n) {
        A[0][n] = A[0][n] + (-rx * ZEm[n]) * Acoef + Em[n] * u0;
        A[1][n] = A[1][n] + (-ry * ZEm[n]) * Acoef + Em[n] * v0;
        A[2][n] = A[2][n] + ZEm[n] * Bcoef + Em[n] * w0;
      }
    } else {
      const double E = exp(-k * H);
      const double hh = H / (2.0 * eta), e2 = 1.0 / (2.0 * eta);
      const Z2 uL0 = (1.0 / k) * (kx * u0 + ky * v0);
      const Z2 uT0 = (1.0 / k) * (kx * v0 - ky * u0);
      const Z2 uLH = (1.0 / k) * (kx * uH + ky * vH);
      const Z2 uTH = (1.0 / k) * (kx * vH - ky * uH);
      double M6[6][6] = {
          {0, 0, 1, E, 0, 0},
          {0, 0, 0, 0, 1, E},
          {hh * E, -hh, E, 1, 0, 0},
          {hh * E, hh, 0, 0, E, 1},
          {e2, e2 * E, k, k * E, -k, k * E},
          {e2 * E, e2, k * E, k, -k * E, k}};
      Z2 X[6] = {imul(1.0, uL0), w0, imul(1.0, uLH), wH, zmk(0, 0), zmk(0, 0)};
      solve6(M6, X);
      const Z2 C0 = X[0], D0 = X[1];
      const Z2 CL = imul(-1.0, X[2]), DL = imul(-1.0, X[3]);
      const Z2 Cz = X[4], Dz = X[5];
      const double det = 1.0 - E * E;
      const Z2 CT = zdiv(uT0 - E * uTH, det);
      const Z2 DT = zdiv(uTH - E * uT0, det);
      const double rx = kx / k, ry = ky / k;
      const Z2 Cx = rx * CL - ry * CT, Cy = ry * CL + rx * CT;
      const Z2 Dx = rx * DL - ry * DT, Dy = ry * DL + rx * DT;
      double Ep[NZ], ZEp[NZ];
      for (int c = 0; c < N; ++c) bas[c] = exp(k * (zc[c] - H));
      dct_real(bas, Mf, N, Ep);
      for (int c = 0; c < N; ++c) bas[c] = zc[c] * exp(k * (zc[c] - H));
      dct_real(bas, Mf, N, ZEp);
      const double ax = kx / (2.0 * eta * k), ay = ky / (2.0 * eta * k);
      const Z2 pu0 = imul(-ax, C0), pu1 = imul(ax, D0);   // -C0 i ax, D0 i ax
      const Z2 pv0 = imul(-ay, C0), pv1 = imul(ay, D0);
      for (int n = 0; n < N; ++n) {
        A[0][n] = A[0][n] + ZEm[n] * pu0 + ZEp[n] * pu1 + Em[n] * Cx + Ep[n] * Dx;
        A[1][n] = A[1][n] + ZEm[n] * pv0 + ZEp[n] * pv1 + Em[n] * Cy + Ep[n] * Dy;
        A[2][n] = A[2][n] + (e2 * ZEm[n]) * C0 + (e2 * ZEp[n]) * D0 + Em[n] * Cz +
                  Ep[n] * Dz;
      }
    }
  }
  // 6. vorticity omega = (1/2) curl u
  cheb_deriv(A[1], tmp, N, H);    // d/dz v
  cheb_deriv(A[0], tmp2, N, H);   // d/dz u
  for (int n = 0; n < N; ++n) {
    A[3][n] = 0.5 * (imul(ky, A[2][n]) - tmp[n]);
    A[4][n] = 0.5 * (tmp2[n] - imul(kx, A[2][n]));
    A[5][n] = 0.5 * (imul(kx, A[1][n]) - imul(ky, A[0][n]));
  }
  // inverse transform to the band nodes (vorticity only when wanted)
  for (int ch = 0; ch < dp.nch_out; ++ch) {
    for (int c = lo; c <= hi; ++c) {
      const double* row = Pi + c * N;
      Z2 s = zmk(0, 0);
      for (int n = 0; n < N; ++n) s = s + row[n] * A[ch][n];
      C o;
      o.x = (T)(cp.scale * s.x);
      o.y = (T)(cp.scale * s.y);
      out[(ch * N + c) * PS + idx] = o;
    }
  }
}

hipError_t launch_columns(const fcmdp_solver* s, const void* spec_in,
                          void* spec_out, hipStream_t st) {
  // (partial slip and wall velocities are solved by the eight-lane kernels
  // only)
  const bool slip = s->dp.slip0 != 0.0 || s->dp.slipH != 0.0 ||
                    s->dp.wall0[0] != 0.0 || s->dp.wall0[1] != 0.0 ||
                    s->dp.wallH[0] != 0.0 || s->dp.wallH[1] != 0.0 ||
                    s->dp.wallspec != nullptr;
  if (s->dp.Nz <= 32 && (!s->force_generic_columns || slip))
    return launch_columns_seg(s, spec_in, spec_out, st);
  ColParams cp;
  cp.dp = s->dp;
  cp.scale = 1.0 / ((double)s->dp.Nx * (double)s->dp.Ny);
  cp.kxs = 2.0 * M_PI / s->dp.Lx;
  cp.kys = 2.0 * M_PI / s->dp.Ly;
  cp.dctf = s->dct_f;
  const int K = s->dp.Nkx * s->dp.Ny;
  dim3 g((K + 63) / 64);
  const bool small = s->dp.Nz <= 32;
  if (s->mixed) {
    if (small)
      hipLaunchKernelGGL((k_columns<float, 32>), g, dim3(64), 0, st, cp,
                         s->band, (const float2*)spec_in, (float2*)spec_out,
                         s->zc, s->dct_f, s->dct_i);
    else
      hipLaunchKernelGGL((k_columns<float, 64>), g, dim3(64), 0, st, cp,
                         s->band, (const float2*)spec_in, (float2*)spec_out,
                         s->zc, s->dct_f, s->dct_i);
  } else {
    if (small)
      hipLaunchKernelGGL((k_columns<double, 32>), g, dim3(64), 0, st, cp,
                         s->band, (const double2*)spec_in, (double2*)spec_out,
                         s->zc, s->dct_f, s->dct_i);
    else
      hipLaunchKernelGGL((k_columns<double, 64>), g, dim3(64), 0, st, cp,
                         s->band, (const double2*)spec_in, (double2*)spec_out,
                         s->zc, s->dct_f, s->dct_i);
  }
  return hipGetLastError();
}

}  // namespace fcmdp
