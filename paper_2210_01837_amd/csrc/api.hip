// Host side of libfcmdp: parameter validation, derived quantities and tables,
// device workspace, and the exported C ABI (include/fcmdp.h).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <utility>
#include <vector>

#include "fcmdp_internal.h"

using fcmdp::FFTPlan;

namespace {

const double kPi = 3.14159265358979323846264338327950288;

// Gauss-Legendre nodes and weights on [-1, 1] (Newton on P_n).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
    double pp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = 0.0;
      for (int j = 1; j <= n; ++j) {
        const double p2 = p1;
        p1 = p0;
        p0 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p2) / j;
      }
      pp = n * (z * p0 - p1) / (z * z - 1.0);
      const double dz = p0 / pp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * pp * pp);
  }
}

// Normalisation of the ES envelope: integral over [-alpha, alpha] of
// exp(beta (sqrt(1 - (t/alpha)^2) - 1)), with t = alpha sin(theta).
double es_norm(double alpha, double beta) {
  std::vector<double> x, w;
  gauss_legendre(160, x, w);
  double s = 0.0;
  for (size_t i = 0; i < x.size(); ++i) {
    const double th = 0.5 * kPi * x[i];
    s += w[i] * std::exp(beta * (std::cos(th) - 1.0)) * std::cos(th);
  }
  return alpha * 0.5 * kPi * s;
}

// cos(pi * num / den) with exact argument reduction of num modulo 2*den.
double cospi_frac(long num, long den) {
  long r = num % (2 * den);
  if (r < 0) r += 2 * den;
  return (double)std::cos((long double)kPi * (long double)r / (long double)den);
}
double sinpi_frac(long num, long den) {
  long r = num % (2 * den);
  if (r < 0) r += 2 * den;
  return (double)std::sin((long double)kPi * (long double)r / (long double)den);
}
// e^{-2 pi i j / n} for j < n (interleaved re, im)
std::vector<double> roots_of_unity(int n) {
  std::vector<double> r(2 * (size_t)n);
  for (int j = 0; j < n; ++j) {
    r[2 * (size_t)j] = cospi_frac(2L * j, n);
    r[2 * (size_t)j + 1] = -sinpi_frac(2L * j, n);
  }
  return r;
}

// Clenshaw-Curtis weights on the N extrema points of [-1, 1] (the classical
// explicit cosine-sum formula).
std::vector<double> clenshaw_curtis(int N) {
  const int n = N - 1;
  std::vector<double> w(N, 0.0);
  std::vector<double> v(N, 1.0);
  if (n % 2 == 0) {
    w[0] = w[n] = 1.0 / (n * (double)n - 1.0);
    for (int c = 1; c < n; ++c) {
      double s = 1.0;
      for (int k = 1; k < n / 2; ++k)
        s -= 2.0 * cospi_frac(2L * k * c, n) / (4.0 * k * k - 1.0);
      s -= cospi_frac((long)n * c, n) / (n * (double)n - 1.0);
      w[c] = 2.0 * s / n;
    }
  } else {
    w[0] = w[n] = 1.0 / (n * (double)n);
    for (int c = 1; c < n; ++c) {
      double s = 1.0;
      for (int k = 1; k <= (n - 1) / 2; ++k)
        s -= 2.0 * cospi_frac(2L * k * c, n) / (4.0 * k * k - 1.0);
      w[c] = 2.0 * s / n;
    }
  }
  return w;
}

bool make_plan(int n, FFTPlan* plan) {
  plan->n = n;
  plan->nstages = 0;
  int m = n;
  while (m % 8 == 0) { plan->radix[plan->nstages++] = 8; m /= 8; }
  while (m % 4 == 0) { plan->radix[plan->nstages++] = 4; m /= 4; }
  while (m % 2 == 0) { plan->radix[plan->nstages++] = 2; m /= 2; }
  const int primes[] = {3, 5, 7, 11, 13, 17};
  for (int p : primes)
    while (m % p == 0) {
      if (plan->nstages >= fcmdp::kMaxStages) return false;
      plan->radix[plan->nstages++] = p;
      m /= p;
    }
  return m == 1 && plan->nstages < fcmdp::kMaxStages;
}

// Plan for the row-owned transforms: radix 8 for the power-of-two part (one
// 16, 4 or 2 for the remainder), then the odd primes.  Picks the fewest
// threads per row (64, 128 or 256) for which every stage leaves at most
// wave_nbi_cap(R) butterflies per thread; false if none does.
bool make_wave_plan(int n, bool fp32, FFTPlan* plan, int* tpr) {
  plan->n = n;
  plan->nstages = 0;
  int m = n, a = 0;
  while (m % 2 == 0) { m /= 2; ++a; }
  std::vector<int> r;
  if (a % 3 == 1) {
    if (a >= 4) { r.push_back(16); a -= 4; } else { r.push_back(2); a -= 1; }
  } else if (a % 3 == 2) {
    r.push_back(4);
    a -= 2;
  }
  while (a >= 3) { r.push_back(8); a -= 3; }
  const int primes[] = {3, 5, 7, 11, 13, 17};
  for (int q : primes)
    while (m % q == 0) { r.push_back(q); m /= q; }
  if (m != 1 || (int)r.size() >= fcmdp::kMaxStages) return false;
  for (int t = 64; t <= 256; t *= 2) {
    bool ok = true;
    for (int R : r)
      if ((n / R + t - 1) / t > fcmdp::wave_nbi_cap(fp32, R)) ok = false;
    if (ok) {
      for (int R : r) plan->radix[plan->nstages++] = R;
      *tpr = t;
      return true;
    }
  }
  return false;
}

// largest power of two <= maxrows with rows * row_bytes within the LDS budget
int rows_fitting(size_t row_bytes, int maxrows) {
  int r = maxrows;
  while (r > 1 && (size_t)r * row_bytes > fcmdp::kLdsBudget) r /= 2;
  return (size_t)r * row_bytes <= fcmdp::kLdsBudget ? r : 0;
}

// rows per workgroup of the x passes: the most (up to 16) that fit, and
// twelve when sixteen do not fit but twelve do (1350-point rows): more
// wavefronts and longer transposed runs than eight
int default_rows_x(size_t row_bytes) {
  const int r = rows_fitting(row_bytes, 16);
  return r == 8 && 12 * row_bytes <= fcmdp::kLdsBudget ? 12 : r;
}

int validate(const fcmdp_params* p) {
  if (!p) return FCMDP_EINVAL;
  if (p->geometry != FCMDP_BOTTOM_WALL && p->geometry != FCMDP_SLIT_CHANNEL)
    return FCMDP_EINVAL;
  if (p->precision != FCMDP_FP64 && p->precision != FCMDP_MIXED)
    return FCMDP_EINVAL;
  if (!(p->Lx > 0) || !(p->Ly > 0) || !(p->H > 0) || !(p->eta > 0))
    return FCMDP_EINVAL;
  if (!(p->beta_m > 0) || !(p->beta_d > 0)) return FCMDP_EINVAL;
  if (p->Nx < 8 || p->Ny < 8 || (p->Nx & 1) || (p->Ny & 1)) return FCMDP_EINVAL;
  if (p->Nz < 8 || p->Nz > fcmdp::kMaxNz) return FCMDP_EINVAL;
  // the kernels hold a 7-point window (|offset| <= 3 cells)
  if (p->w != 4 && p->w != 6) return FCMDP_EINVAL;
  if (p->max_particles < 0 || p->max_particles > (int64_t)1 << 30)
    return FCMDP_EINVAL;
  // partial slip, solved by the eight-lane column kernels; a bottom wall
  // has a slip length at z = 0 only
  if (!(p->slip0 >= 0) || !(p->slipH >= 0) || !std::isfinite(p->slip0) ||
      !std::isfinite(p->slipH))
    return FCMDP_EINVAL;
  if (p->geometry == FCMDP_BOTTOM_WALL && p->slipH != 0) return FCMDP_EINVAL;
  if ((p->slip0 != 0 || p->slipH != 0) && p->Nz > 32) return FCMDP_EINVAL;
  // uniform wall velocities: finite; a bottom wall has no wall at z = H
  for (int c = 0; c < 2; ++c) {
    if (!std::isfinite(p->wall0[c]) || !std::isfinite(p->wallH[c]))
      return FCMDP_EINVAL;
    if (p->geometry == FCMDP_BOTTOM_WALL && p->wallH[c] != 0) return FCMDP_EINVAL;
    if ((p->wall0[c] != 0 || p->wallH[c] != 0) && p->Nz > 32) return FCMDP_EINVAL;
  }
  // torques through the kernel derivative: the three-channel kernels
  if (p->torque_route != FCMDP_TORQUE_CURL && p->torque_route != FCMDP_TORQUE_DERIVATIVE)
    return FCMDP_EINVAL;
  if (p->torque_route == FCMDP_TORQUE_DERIVATIVE && p->Nz > 32) return FCMDP_EINVAL;
  const double hx = p->Lx / p->Nx, hy = p->Ly / p->Ny;
  if (std::fabs(hx - hy) > 1e-12 * hx) return FCMDP_EINVAL;
  const double alpha = 0.5 * p->w * hx;
  if (p->geometry == FCMDP_BOTTOM_WALL && !(p->H > alpha)) return FCMDP_EINVAL;
  if (p->geometry == FCMDP_SLIT_CHANNEL && !(p->H >= 2.0 * alpha))
    return FCMDP_EINVAL;
  FFTPlan a, b;
  if (!make_plan(p->Nx / 2, &a) || !make_plan(p->Ny, &b)) return FCMDP_EINVAL;
  if ((long long)p->Nx * p->Ny >= (1LL << 31) - 1) return FCMDP_EINVAL;
  // LDS of the workgroup-per-row transforms (one row, two buffers), which
  // every size must support; the wave-per-row transforms need less
  const size_t csz = p->precision == FCMDP_MIXED ? 8 : 16;
  if (2 * (size_t)p->Ny * csz > fcmdp::kLdsBudget) return FCMDP_EINVAL;
  if ((size_t)(p->Nx + 1) * csz > fcmdp::kLdsBudget) return FCMDP_EINVAL;
  return FCMDP_OK;
}

// number of z-window slots: most Chebyshev nodes in a closed interval of
// length 2 alpha, plus the one-node padding on each side and one spare.
int z_window_slots(int Nz, double H, double alpha) {
  std::vector<double> z(Nz);
  for (int c = 0; c < Nz; ++c) z[c] = 0.5 * H * (1.0 + cospi_frac(c, Nz - 1));
  int best = 0;
  for (int c0 = 0; c0 < Nz; ++c0) {
    int cnt = 0;
    for (int c = c0; c < Nz; ++c)
      if (z[c0] - z[c] <= 2.0 * alpha * (1.0 + 1e-12)) ++cnt;
    if (cnt > best) best = cnt;
  }
  int zw = best + 3;
  return zw > Nz ? Nz : zw;
}

struct Sizes {
  size_t grid, spec, keys, vals, hist, cells, pinfo, pw, pf, psi;
  // exact low-wavenumber vertical force (mixed slit channel), 0 when off
  size_t psi64, fzlo, lowk_part, lowk_coef, lowk_ex, lowk_ey;
  // torques through the kernel derivative, 0 when off
  size_t pdw, dpsi;
};

// Truncation point t* of the dipole kernel's derivative: with r = t/alpha
// and s = sqrt(1 - r^2), |phi'| is proportional to r e^{beta (s - 1)} / s,
// whose stationary points solve beta s^3 - beta s + 1 = 0; the smaller root
// in (0, 1) is the minimum before |phi'| grows without bound at the edge of
// the support (the larger one is its maximum).  Bisection on the
// decreasing branch (the cubic falls on (0, 1/sqrt(3))); alpha when there
// is no interior minimum.
double derivative_cutoff(double alpha, double beta) {
  auto f = [&](double x) { return beta * x * x * x - beta * x + 1.0; };
  double a = 0.0, b = 1.0 / std::sqrt(3.0);
  if (f(b) > 0.0) return alpha;
  for (int it = 0; it < 200; ++it) {
    const double m = 0.5 * (a + b);
    (f(m) > 0.0 ? a : b) = m;
  }
  const double sv = 0.5 * (a + b);
  return alpha * std::sqrt(1.0 - sv * sv);
}

// Half-width ns of the square |nx|, |ny| <= ns of wavenumbers whose vertical
// force takes the FP64 route (mixed slit channel; 0 = none): every column
// with kH < 1 (ns = ceil(L / (2 pi H)) for the longer period L), capped so
// that the square stays clear of the Nyquist modes.
int lowk_half_width(const fcmdp_params* p) {
  if (p->precision != FCMDP_MIXED || p->geometry != FCMDP_SLIT_CHANNEL ||
      p->Nz > 32)
    return 0;
  const double L = p->Lx > p->Ly ? p->Lx : p->Ly;
  int ns = (int)std::ceil(L / (2.0 * kPi * p->H) - 1e-12);
  const int nmax = (p->Nx < p->Ny ? p->Nx : p->Ny) / 2 - 1;
  if (ns > nmax) ns = nmax;
  if (ns > fcmdp::kLowkMaxNs) ns = fcmdp::kLowkMaxNs;
  return ns < 1 ? 0 : ns;
}

Sizes sizes_for(const fcmdp_params* p, int64_t cap, int ZW) {
  const size_t T = p->precision == FCMDP_MIXED ? 4 : 8;
  Sizes s;
  const size_t nkx = (size_t)p->Nx / 2 + 1;
  s.grid = 6 * (size_t)p->Nz * p->Ny * p->Nx * T;
  s.spec = 6 * (size_t)p->Nz * nkx * p->Ny * 2 * T;
  const size_t c = cap > 0 ? (size_t)cap : 1;
  s.keys = c * 4;
  s.vals = c * 4;
  const size_t nblk = (c + 2047) / 2048;
  s.hist = (256 * nblk + 256) * 4;   // block histograms + digit totals
  s.cells = ((size_t)p->Nx * p->Ny + 1) * 4;
  s.pinfo = c * 16;
  s.pw = c * 32 * T;
  s.pf = c * 8 * T;
  // dense folded z weights [cap][2][Nz], padded for chunked readers that may
  // run past the last node
  s.psi = (c * 2 * (size_t)p->Nz + 64) * T;
  const int ns = lowk_half_width(p);
  const bool deriv = p->torque_route == FCMDP_TORQUE_DERIVATIVE;
  s.psi64 = s.fzlo = s.lowk_part = s.lowk_coef = s.lowk_ex = s.lowk_ey = 0;
  s.pdw = deriv ? c * 16 * T : 0;
  s.dpsi = deriv ? (c * (size_t)p->Nz + 64) * T : 0;
  if (ns > 0) {
    const size_t ncols = (size_t)(ns + 1) * (2 * ns + 1);
    s.psi64 = (c * (size_t)p->Nz * (deriv ? 2 : 1) + 64) * 8;
    s.fzlo = (size_t)p->Nz * p->Ny * p->Nx * 4;
    s.lowk_part = ((size_t)p->Nz * p->Ny * (ns + 1) + ncols * p->Nz) * 16;
    s.lowk_coef = ncols * p->Nz * 16;
    s.lowk_ex = (size_t)p->Nx * (ns + 1) * 16;
    s.lowk_ey = (size_t)p->Ny * 16;
  }
  (void)ZW;
  return s;
}

// Device tables are staged host-side into one buffer and uploaded with one
// allocation and one copy in stream order on the creation stream (finish());
// the host copy stays alive until that stream has been synchronised.  Each
// table starts on a 256-byte boundary.
struct Uploader {
  hipStream_t st;
  std::vector<unsigned char> host;
  std::vector<std::pair<void**, size_t>> slots;   // destination, offset
  void* base = nullptr;
  template <typename P, typename T>
  void to(P** dst, const std::vector<T>& v) {
    const size_t off = (host.size() + 255) & ~(size_t)255;
    const size_t bytes = sizeof(T) * v.size();
    host.resize(off + (bytes ? bytes : 16), 0);
    if (bytes) std::memcpy(host.data() + off, v.data(), bytes);
    slots.emplace_back(reinterpret_cast<void**>(dst), off);
  }
  // e^{-2 pi i m s / n} for m < count, from root[] = e^{-2 pi i j / N}
  // (N = n s, j < N; each root evaluated once)
  template <typename T, typename P>
  void twiddles(P** dst, const std::vector<double>& root, int s, int count) {
    std::vector<T> v(2 * (size_t)count);
    const size_t N = root.size() / 2;
    for (int m = 0; m < count; ++m) {
      const size_t j = ((size_t)m * s) % N;
      v[2 * m] = (T)root[2 * j];
      v[2 * m + 1] = (T)root[2 * j + 1];
    }
    to(dst, v);
  }
  int finish() {
    if (host.empty()) return FCMDP_OK;
    if (hipMallocAsync(&base, host.size(), st) != hipSuccess) {
      base = nullptr;
      return FCMDP_ENOMEM;
    }
    for (auto& sl : slots) *sl.first = static_cast<unsigned char*>(base) + sl.second;
    if (hipMemcpyAsync(base, host.data(), host.size(), hipMemcpyHostToDevice, st) !=
        hipSuccess)
      return FCMDP_EHIP;
    return FCMDP_OK;
  }
};

// The workspace buffers of a solver, carved from one stream-ordered
// allocation (one hipMallocAsync and one hipFreeAsync per solver; a serving
// pool creates and releases solvers while requests run).  256-byte aligned.
struct Arena {
  std::vector<std::pair<void**, size_t>> slots;   // destination, offset
  size_t total = 0;
  void* base = nullptr;
  template <typename P>
  void add(P** dst, size_t bytes) {
    const size_t off = (total + 255) & ~(size_t)255;
    total = off + (bytes ? bytes : 16);
    slots.emplace_back(reinterpret_cast<void**>(dst), off);
  }
  int finish(hipStream_t st) {
    if (hipMallocAsync(&base, total ? total : 16, st) != hipSuccess) {
      base = nullptr;
      return FCMDP_ENOMEM;
    }
    for (auto& sl : slots) *sl.first = static_cast<unsigned char*>(base) + sl.second;
    return FCMDP_OK;
  }
};

void free_all(fcmdp_solver* s, hipStream_t st) {
  // the workspace and table arenas hold every buffer of creation; the wall
  // spectrum and the Lanczos buffers are allocated on their own
  void* ptrs[] = {s->arena, s->tables, s->lz_basis, s->lz_red, s->wallspec};
  // stream-ordered frees: no device-wide synchronisation
  for (void* q : ptrs)
    if (q) (void)hipFreeAsync(q, st);
}

}  // namespace

extern "C" {

const char* fcmdp_strerror(int code) {
  switch (code) {
    case FCMDP_OK: return "ok";
    case FCMDP_EINVAL: return "invalid argument or unsupported size";
    case FCMDP_EDOMAIN: return "particles outside the fluid domain";
    case FCMDP_ENOMEM: return "device allocation failed";
    case FCMDP_EHIP: return "HIP runtime error";
    case FCMDP_ECAPACITY: return "more particles than the solver capacity";
    default: return "unknown error";
  }
}

int fcmdp_workspace_bytes(const fcmdp_params* p, int64_t n, size_t* bytes) {
  const int v = validate(p);
  if (v != FCMDP_OK) return v;
  if (!bytes || n < 0) return FCMDP_EINVAL;
  const double alpha = 0.5 * p->w * (p->Lx / p->Nx);
  const Sizes s = sizes_for(p, n, z_window_slots(p->Nz, p->H, alpha));
  *bytes = s.grid + s.spec + 2 * s.keys + 2 * s.vals + s.hist + s.cells +
           s.pinfo + s.pw + s.pf + s.psi + s.psi64 + s.fzlo + s.lowk_part +
           s.lowk_coef + s.lowk_ex + s.lowk_ey + s.pdw + s.dpsi +
           (size_t)p->Nz * p->Nz * 16 + 65536;
  return FCMDP_OK;
}

int fcmdp_create_solver(const fcmdp_params* p, void* hip_stream,
                        fcmdp_solver** out) {
  if (!out) return FCMDP_EINVAL;
  hipStream_t st = (hipStream_t)hip_stream;
  *out = nullptr;
  int v = validate(p);
  if (v != FCMDP_OK) return v;
  fcmdp_solver* s = new (std::nothrow) fcmdp_solver();
  if (!s) return FCMDP_ENOMEM;
  s->p = *p;
  s->mixed = p->precision == FCMDP_MIXED;
  if (hipGetDevice(&s->device) != hipSuccess ||
      hipDeviceGetAttribute(&s->num_cu, hipDeviceAttributeMultiprocessorCount,
                            s->device) != hipSuccess) {
    delete s;
    return FCMDP_EHIP;
  }
  const int Nz = p->Nz;
  fcmdp::DevParams& dp = s->dp;
  dp.geometry = p->geometry;
  dp.Nx = p->Nx;
  dp.Ny = p->Ny;
  dp.Nz = Nz;
  dp.Nkx = p->Nx / 2 + 1;
  dp.ncells = p->Nx * p->Ny;
  dp.half_w = p->w / 2;
  dp.nch_in = 6;
  dp.nch_out = 6;
  dp.slip0 = p->slip0;
  dp.slipH = p->slipH;
  for (int c = 0; c < 2; ++c) {
    dp.wall0[c] = p->wall0[c];
    dp.wallH[c] = p->wallH[c];
  }
  dp.wallspec = nullptr;
  dp.Lx = p->Lx;
  dp.Ly = p->Ly;
  dp.H = p->H;
  dp.h = p->Lx / p->Nx;
  dp.alpha = 0.5 * p->w * dp.h;
  dp.eta = p->eta;
  dp.beta_m = p->beta_m;
  dp.beta_d = p->beta_d;
  s->norm_m = es_norm(dp.alpha, p->beta_m);
  s->norm_d = es_norm(dp.alpha, p->beta_d);
  dp.inv_norm_m = 1.0 / s->norm_m;
  dp.inv_norm_d = 1.0 / s->norm_d;
  dp.ZW = z_window_slots(Nz, p->H, dp.alpha);
  dp.lowk_ns = -1;
  dp.lowk_coef = nullptr;
  dp.torque_deriv = p->torque_route == FCMDP_TORQUE_DERIVATIVE;
  dp.dt_torque = dp.dt_omega = 0;
  dp.tstar_d = derivative_cutoff(dp.alpha, p->beta_d);
  s->lowk_ns = lowk_half_width(p);
  s->cap = p->max_particles;
  s->nblk_cap = (int)((s->cap > 0 ? s->cap : 1) + 2047) / 2048;
  {
    int bits = 0;
    while (((int64_t)1 << bits) <= (int64_t)dp.ncells) ++bits;
    s->key_passes = (bits + 7) / 8;
  }
  make_plan(p->Nx / 2, &s->plan_x);
  make_plan(p->Ny, &s->plan_y);
  {
    const bool fp32 = s->mixed;
    const size_t csz = fp32 ? 8 : 16;
    // row-owned transforms in single precision only (the double-precision
    // stages do not fit the register budget of a 1024-thread workgroup)
    s->wave_x = fp32 && make_wave_plan(p->Nx / 2, fp32, &s->wplan_x, &s->tpr_x);
    s->wave_y = fp32 && make_wave_plan(p->Ny, fp32, &s->wplan_y, &s->tpr_y);
    s->codelet_x = fcmdp::fft_codelet(p->Nx / 2, fp32, &s->wplan_x, &s->tpr_x);
    s->codelet_y = fcmdp::fft_codelet(p->Ny, fp32, &s->wplan_y, &s->tpr_y);
    if (s->codelet_x >= 0) s->wave_x = true;
    if (s->codelet_y >= 0) s->wave_y = true;
    const size_t row_x = (size_t)fcmdp::fft_lds_row(s->codelet_x, p->Nx / 2, true) * csz;
    const size_t row_y = (size_t)fcmdp::fft_lds_row(s->codelet_y, p->Ny, false) * csz;
    s->rows_x = default_rows_x(row_x);
    // rows of the y pass are independent; one per workgroup packs LDS best
    s->rows_y = s->codelet_y >= 0 ? 1 : rows_fitting(row_y, 8);
    if (s->rows_x == 0) s->wave_x = false;
    if (s->rows_y == 0) s->wave_y = false;
  }

  // Workspace comes from the device's default memory pool in stream order.
  // Keep freed blocks in the pool (no release threshold), so that a solver
  // created after another was released reuses its memory instead of mapping
  // new pages (a serving pool creates and releases solvers continuously).
  {
    hipMemPool_t pool = nullptr;
    if (hipDeviceGetDefaultMemPool(&pool, s->device) == hipSuccess && pool) {
      uint64_t keep = UINT64_MAX;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
  }
  int err = FCMDP_OK;
  const Sizes z = sizes_for(p, s->cap, dp.ZW);
  // stream-ordered allocations on the creation stream (no device-wide
  // synchronisation, so applies in flight on other streams keep running)
  Arena arena;
  auto alloc = [&](auto** ptr, size_t bytes) { arena.add(ptr, bytes); };
  Uploader upload{st, {}, {}, nullptr};
  alloc(&s->grid, z.grid);
  alloc(&s->spec, z.spec);
  alloc(&s->keyA, z.keys);
  alloc(&s->keyB, z.keys);
  alloc(&s->valA, z.vals);
  alloc(&s->valB, z.vals);
  alloc(&s->hist, z.hist);
  alloc(&s->cell_start, z.cells);
  alloc(&s->pinfo, z.pinfo);
  alloc(&s->pw, z.pw);
  alloc(&s->pf, z.pf);
  alloc(&s->psi, z.psi);
  if (dp.torque_deriv) {
    alloc(&s->pdw, z.pdw);
    alloc(&s->dpsi, z.dpsi);
  }
  if (s->lowk_ns > 0) {
    alloc(&s->psi64, z.psi64);
    alloc(&s->fzlo, z.fzlo);
    alloc(&s->lowk_part, z.lowk_part);
    alloc(&s->lowk_coef, z.lowk_coef);
  }
  alloc(&s->band, 2 * sizeof(int));
  alloc(&s->nbad, sizeof(unsigned int));
  err = arena.finish(st);
  s->arena = arena.base;

  // Chebyshev tables
  if (err == FCMDP_OK) {
    const int N1 = Nz - 1;
    std::vector<double> zc(Nz), Mf((size_t)Nz * Nz), Pi((size_t)Nz * Nz);
    for (int c = 0; c < Nz; ++c) zc[c] = 0.5 * p->H * (1.0 + cospi_frac(c, N1));
    for (int c = 0; c < Nz; ++c)
      for (int n = 0; n < Nz; ++n) {
        const double cs = cospi_frac((long)n * c, N1);
        Pi[(size_t)c * Nz + n] = cs;
        double m = 2.0 / N1 * cs;
        if (c == 0 || c == N1) m *= 0.5;
        if (n == 0 || n == N1) m *= 0.5;
        Mf[(size_t)c * Nz + n] = m;
      }
    const std::vector<double> w = clenshaw_curtis(Nz);
    const double h2 = dp.h * dp.h;
    upload.to(&s->zc, zc);
    upload.to(&s->dct_f, Mf);
    upload.to(&s->dct_i, Pi);
    if (s->mixed) {
      std::vector<float> mf(Mf.begin(), Mf.end()), pf(Pi.begin(), Pi.end());
      upload.to(&s->dct_f32, mf);
      upload.to(&s->dct_i32, pf);
    }
    if (s->mixed) {
      std::vector<float> q(Nz);
      for (int c = 0; c < Nz; ++c) q[c] = (float)(h2 * 0.5 * p->H * w[c]);
      upload.to(&s->quad, q);
    } else {
      std::vector<double> q(Nz);
      for (int c = 0; c < Nz; ++c) q[c] = h2 * 0.5 * p->H * w[c];
      upload.to(&s->quad, q);
    }
    // small prime DFT constants
    std::vector<double> cs;
    const int primes[] = {3, 5, 7, 11, 13, 17};
    cs.assign(8, 0.0);       // slot 0 for radices without constants
    for (int P : primes) {
      s->dft_off[P] = (int)cs.size();
      for (int m = 0; m < P; ++m) {
        cs.push_back(cospi_frac(2L * m, P));
        cs.push_back(sinpi_frac(2L * m, P));
      }
    }
    upload.to(&s->dftc, cs);
    if (s->mixed) {
      std::vector<float> c32(cs.begin(), cs.end());
      upload.to(&s->dftc_t, c32);
    } else {
      upload.to(&s->dftc_t, cs);
    }
    if (s->lowk_ns > 0) {
      // e^{-2 pi i nx a / Nx} for nx = 0..ns ([a][nx]) and e^{-2 pi i m / Ny}
      const int nk = s->lowk_ns + 1;
      std::vector<double> ex(2 * (size_t)p->Nx * nk), ey(2 * (size_t)p->Ny);
      const std::vector<double> root = roots_of_unity(p->Nx);
      for (int a = 0; a < p->Nx; ++a)
        for (int n = 0; n < nk; ++n) {
          const long m = ((long)n * a) % p->Nx;
          ex[2 * ((size_t)a * nk + n)] = root[2 * (size_t)m];
          ex[2 * ((size_t)a * nk + n) + 1] = root[2 * (size_t)m + 1];
        }
      for (int m = 0; m < p->Ny; ++m) {
        ey[2 * (size_t)m] = cospi_frac(2L * m, p->Ny);
        ey[2 * (size_t)m + 1] = -sinpi_frac(2L * m, p->Ny);
      }
      upload.to(&s->lowk_ex, ex);
      upload.to(&s->lowk_ey, ey);
    }
    const int M = p->Nx / 2;
    const std::vector<double> rx = roots_of_unity(p->Nx);
    const std::vector<double> ry = p->Ny == p->Nx ? rx : roots_of_unity(p->Ny);
    if (s->mixed) {
      upload.twiddles<float>(&s->tw_x, rx, 2, M);       // roots of Nx / 2
      upload.twiddles<float>(&s->tw_y, ry, 1, p->Ny);
      upload.twiddles<float>(&s->tw_r, rx, 1, M + 1);
    } else {
      upload.twiddles<double>(&s->tw_x, rx, 2, M);
      upload.twiddles<double>(&s->tw_y, ry, 1, p->Ny);
      upload.twiddles<double>(&s->tw_r, rx, 1, M + 1);
    }
  }
  if (err == FCMDP_OK) {
    err = upload.finish();
    s->tables = upload.base;
  }
  if (err == FCMDP_OK) {
    if (fcmdp::launch_set_band(s, Nz, -1, st) != hipSuccess ||
        fcmdp::launch_fill(s->nbad, sizeof(unsigned int), st) != hipSuccess)
      err = FCMDP_EHIP;
  }
  // the creation stream only: the uploads are complete (and the host copies
  // may go) and the buffers are usable from any stream afterwards
  if (hipStreamSynchronize(st) != hipSuccess && err == FCMDP_OK) err = FCMDP_EHIP;
  if (err != FCMDP_OK) {
    free_all(s, st);
    (void)hipStreamSynchronize(st);
    delete s;
    return err;
  }
  *out = s;
  return FCMDP_OK;
}

void fcmdp_destroy_solver(fcmdp_solver* s, void* hip_stream) {
  if (!s) return;
  (void)hipSetDevice(s->device);
  for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
  s->events.clear();
  free_all(s, (hipStream_t)hip_stream);
  delete s;
}

int fcmdp_set_wall_velocity(fcmdp_solver* s, const void* wall,
                            void* hip_stream) {
  if (!s) return FCMDP_EINVAL;
  if (hipSetDevice(s->device) != hipSuccess) return FCMDP_EHIP;
  if (!wall) {
    s->dp.wallspec = nullptr;
    return FCMDP_OK;
  }
  // the wall data enter the eight-lane column kernels only
  if (s->dp.Nz > 32) return FCMDP_EINVAL;
  hipStream_t st = (hipStream_t)hip_stream;
  const size_t csz = s->mixed ? 8 : 16;
  if (!s->wallspec &&
      hipMallocAsync(&s->wallspec, 4 * (size_t)s->dp.Nkx * s->dp.Ny * csz, st) !=
          hipSuccess) {
    s->wallspec = nullptr;
    return FCMDP_EHIP;
  }
  const fcmdp::DevParams saved = s->dp;
  s->dp.nch_in = 3;
  s->dp.lowk_ns = -1;
  s->dp.lowk_coef = nullptr;
  s->dp.wallspec = nullptr;
  const hipError_t e = fcmdp::launch_wall_spectrum(s, wall, st);
  s->dp = saved;
  if (e != hipSuccess) return FCMDP_EHIP;
  s->dp.wallspec = s->wallspec;
  return FCMDP_OK;
}

int fcmdp_solver_info(const fcmdp_solver* s, double out[4]) {
  if (!s || !out) return FCMDP_EINVAL;
  out[0] = s->dp.h;
  out[1] = s->dp.alpha;
  out[2] = s->norm_m;
  out[3] = s->norm_d;
  return FCMDP_OK;
}

int fcmdp_status(fcmdp_solver* s, int64_t* n_bad) {
  if (!s) return FCMDP_EINVAL;
  if (hipSetDevice(s->device) != hipSuccess) return FCMDP_EHIP;
  unsigned int bad = 0;
  if (hipMemcpy(&bad, s->nbad, sizeof(bad), hipMemcpyDeviceToHost) !=
      hipSuccess)
    return FCMDP_EHIP;
  if (n_bad) *n_bad = bad;
  return bad ? FCMDP_EDOMAIN : FCMDP_OK;
}

static int check_particles(fcmdp_solver* s, int64_t n) {
  if (!s || n < 0) return FCMDP_EINVAL;
  if (n > s->cap) return FCMDP_ECAPACITY;
  if (hipSetDevice(s->device) != hipSuccess) return FCMDP_EHIP;
  return FCMDP_OK;
}

static int particle_front(fcmdp_solver* s, int n, const void* pos,
                          const void* F, const void* T, hipStream_t st) {
  if (fcmdp::launch_prep(s, n, pos, st) != hipSuccess) return FCMDP_EHIP;
  if (fcmdp::launch_sort(s, n, st) != hipSuccess) return FCMDP_EHIP;
  if (fcmdp::launch_records(s, n, pos, F, T, st) != hipSuccess)
    return FCMDP_EHIP;
  return FCMDP_OK;
}

int fcmdp_apply_mobility(fcmdp_solver* s, int64_t n, const void* pos,
                         const void* F, const void* T, void* U, void* Omega,
                         void* hip_stream) {
  int v = check_particles(s, n);
  if (v != FCMDP_OK) return v;
  hipStream_t st = (hipStream_t)hip_stream;
  if (n > 0 && (!pos || !F || !U)) return FCMDP_EINVAL;
  if (n == 0) {
    return fcmdp::launch_prep(s, 0, nullptr, st) == hipSuccess ? FCMDP_OK
                                                               : FCMDP_EHIP;
  }
  const int ni = (int)n;
  // without torques the grid and spectrum carry the three force channels;
  // without angular velocities the solve returns the three velocity channels.
  // Torques through the kernel derivative: three channels throughout, the
  // torques enter the spread and Omega the interpolation.
  const bool deriv = s->dp.torque_deriv != 0;
  s->dp.nch_in = (T && !deriv) ? 6 : 3;
  s->dp.nch_out = (Omega && !deriv) ? 6 : 3;
  s->dp.dt_torque = deriv && T;
  s->dp.dt_omega = deriv && Omega;
  const bool lowk = fcmdp::lowk_active(s);
  s->dp.lowk_ns = lowk ? s->lowk_ns : -1;
  s->dp.lowk_coef = lowk ? s->lowk_coef : nullptr;
  hipEvent_t ev[7] = {};
  const bool prof = s->profiling;
  if (prof) {
    for (auto& e : ev)
      if (hipEventCreate(&e) != hipSuccess) return FCMDP_EHIP;
  }
  auto mark = [&](int i) {
    if (prof) (void)hipEventRecord(ev[i], st);
  };
  mark(0);
  v = particle_front(s, ni, pos, F, T, st);
  if (v != FCMDP_OK) return v;
  mark(1);
  if (fcmdp::launch_spread(s, (int)n, s->grid, st) != hipSuccess) return FCMDP_EHIP;
  mark(2);
  if (fcmdp::launch_fft_forward(s, s->grid, s->spec, st) != hipSuccess)
    return FCMDP_EHIP;
  if (lowk && fcmdp::launch_lowk(s, s->grid, st) != hipSuccess)
    return FCMDP_EHIP;
  mark(3);
  if (fcmdp::launch_columns(s, s->spec, s->spec, st) != hipSuccess)
    return FCMDP_EHIP;
  mark(4);
  if (fcmdp::launch_fft_inverse(s, s->spec, s->grid, st) != hipSuccess)
    return FCMDP_EHIP;
  mark(5);
  if (fcmdp::launch_interp(s, ni, s->grid, U, Omega, st) != hipSuccess)
    return FCMDP_EHIP;
  mark(6);
  if (prof) s->events.insert(s->events.end(), ev, ev + 7);
  return FCMDP_OK;
}

int fcmdp_set_profiling(fcmdp_solver* s, int enable) {
  if (!s) return FCMDP_EINVAL;
  s->profiling = enable != 0;
  return FCMDP_OK;
}

int fcmdp_set_variant(fcmdp_solver* s, int key, int value) {
  if (!s) return FCMDP_EINVAL;
  const bool on = value != 0;
  const size_t csz = s->mixed ? 8 : 16;
  switch (key) {
    case FCMDP_VARIANT_GENERIC_FFT:
      s->force_generic_fft = on;
      return FCMDP_OK;
    case FCMDP_VARIANT_FFT_ROWS_X:
    case FCMDP_VARIANT_FFT_ROWS_Y: {
      const bool x = key == FCMDP_VARIANT_FFT_ROWS_X;
      // rows of the fixed plan (the larger) when there is one
      const size_t row =
          (size_t)fcmdp::fft_lds_row(x ? s->codelet_x : s->codelet_y,
                                     x ? s->p.Nx / 2 : s->p.Ny, x) * csz;
      const int maxr = x ? 16 : 8;   // capped at 1024 threads per workgroup
      int r = value;
      if (r == 0) r = x ? default_rows_x(row) : rows_fitting(row, maxr);
      if (r < 1 || r > maxr || ((r & (r - 1)) && r != 12) ||
          (size_t)r * row > fcmdp::kLdsBudget)
        return FCMDP_EINVAL;
      (x ? s->rows_x : s->rows_y) = r;
      return FCMDP_OK;
    }
    case FCMDP_VARIANT_SIMPLE_SPREAD:
      s->force_simple_spread = on;
      return FCMDP_OK;
    case FCMDP_VARIANT_SIMPLE_INTERP:
      s->force_simple_interp = on;
      return FCMDP_OK;
    case FCMDP_VARIANT_GENERIC_COLUMNS:
      s->force_generic_columns = on;
      return FCMDP_OK;
    case FCMDP_VARIANT_VECTOR_DCT:
      s->force_vector_dct = on;
      return FCMDP_OK;
    case FCMDP_VARIANT_NO_CODELET: {
      const bool fp32 = s->mixed;
      if (on) {
        s->codelet_x = s->codelet_y = -1;
        s->wave_x = fp32 && make_wave_plan(s->p.Nx / 2, fp32, &s->wplan_x, &s->tpr_x);
        s->wave_y = fp32 && make_wave_plan(s->p.Ny, fp32, &s->wplan_y, &s->tpr_y);
      } else {
        s->codelet_x = fcmdp::fft_codelet(s->p.Nx / 2, fp32, &s->wplan_x, &s->tpr_x);
        s->codelet_y = fcmdp::fft_codelet(s->p.Ny, fp32, &s->wplan_y, &s->tpr_y);
        if (s->codelet_x >= 0) s->wave_x = true;
        if (s->codelet_y >= 0) s->wave_y = true;
      }
      return FCMDP_OK;
    }
    case FCMDP_VARIANT_NO_PIPELINE:
      s->force_no_pipeline = on;
      return FCMDP_OK;
    case FCMDP_VARIANT_NO_LOWK:
      s->no_lowk = on;
      return FCMDP_OK;
    case FCMDP_VARIANT_WAVE_SPREAD:
      s->force_wave_spread = on;
      return FCMDP_OK;
    case FCMDP_VARIANT_SPREAD_WORKGROUPS:
      if (value < 0 || value > 65535) return FCMDP_EINVAL;
      s->spread_workgroups = value;
      return FCMDP_OK;
    case FCMDP_VARIANT_SPREAD_BLOCK_ROWS:
      if (value != 0 && value != 8 && value != 16) return FCMDP_EINVAL;
      s->spread_block_rows = value;
      return FCMDP_OK;
    case FCMDP_VARIANT_HALO_INTERP:
      s->force_halo_interp = on;
      return FCMDP_OK;
    case FCMDP_VARIANT_SPREAD_ORDER:
      if (value < 0 || value > 2) return FCMDP_EINVAL;
      s->spread_order = value;
      return FCMDP_OK;
    default:
      return FCMDP_EINVAL;
  }
}

int fcmdp_stage_times(fcmdp_solver* s, double ms[8], int64_t* napplies) {
  if (!s || !ms) return FCMDP_EINVAL;
  if (hipSetDevice(s->device) != hipSuccess) return FCMDP_EHIP;
  for (int i = 0; i < 8; ++i) ms[i] = 0.0;
  const size_t na = s->events.size() / 7;
  int rc = FCMDP_OK;
  if (na && hipEventSynchronize(s->events.back()) != hipSuccess) rc = FCMDP_EHIP;
  for (size_t a = 0; a < na && rc == FCMDP_OK; ++a)
    for (int i = 0; i < 6; ++i) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, s->events[7 * a + i],
                              s->events[7 * a + i + 1]) != hipSuccess) {
        rc = FCMDP_EHIP;
        break;
      }
      ms[i] += t;
    }
  for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
  s->events.clear();
  int band[2] = {0, -1};
  if (rc == FCMDP_OK &&
      hipMemcpy(band, s->band, sizeof(band), hipMemcpyDeviceToHost) != hipSuccess)
    rc = FCMDP_EHIP;
  ms[6] = band[0];
  ms[7] = band[1];
  if (napplies) *napplies = (int64_t)na;
  return rc;
}

static size_t grid_bytes(const fcmdp_solver* s) {
  return 6 * (size_t)s->dp.Nz * s->dp.Ny * s->dp.Nx * (s->mixed ? 4 : 8);
}
static size_t spec_bytes(const fcmdp_solver* s) {
  return 6 * (size_t)s->dp.Nz * s->dp.Nkx * s->dp.Ny * (s->mixed ? 8 : 16);
}
static bool band_ok(const fcmdp_solver* s, int lo, int hi) {
  return lo >= 0 && hi < s->dp.Nz && lo <= hi;
}

// the stage entry points work on the full six-channel layouts
// (and without the exact low-wavenumber vertical force, which needs the
// spread's FP64 residual plane)
static void all_channels(fcmdp_solver* s) {
  s->dp.nch_in = 6;
  s->dp.nch_out = 6;
  s->dp.lowk_ns = -1;
  s->dp.lowk_coef = nullptr;
  s->dp.dt_torque = s->dp.dt_omega = 0;
}

int fcmdp_stage_spread(fcmdp_solver* s, int64_t n, const void* pos,
                       const void* F, const void* T, void* grid,
                       void* hip_stream) {
  int v = check_particles(s, n);
  if (v != FCMDP_OK) return v;
  if (s->dp.torque_deriv) return FCMDP_EINVAL;   // six-channel layouts only
  if (!grid || (n > 0 && (!pos || !F))) return FCMDP_EINVAL;
  all_channels(s);
  hipStream_t st = (hipStream_t)hip_stream;
  if (fcmdp::launch_fill(grid, grid_bytes(s), st) != hipSuccess)
    return FCMDP_EHIP;
  if (n == 0) return FCMDP_OK;
  v = particle_front(s, (int)n, pos, F, T, st);
  if (v != FCMDP_OK) return v;
  return fcmdp::launch_spread(s, (int)n, grid, st) == hipSuccess ? FCMDP_OK
                                                         : FCMDP_EHIP;
}

int fcmdp_stage_fft_forward(fcmdp_solver* s, const void* grid, void* spectrum,
                            int c_lo, int c_hi, void* hip_stream) {
  if (!s || !grid || !spectrum || !band_ok(s, c_lo, c_hi)) return FCMDP_EINVAL;
  if (hipSetDevice(s->device) != hipSuccess) return FCMDP_EHIP;
  all_channels(s);
  hipStream_t st = (hipStream_t)hip_stream;
  if (fcmdp::launch_set_band(s, c_lo, c_hi, st) != hipSuccess) return FCMDP_EHIP;
  return fcmdp::launch_fft_forward(s, grid, spectrum, st) == hipSuccess
             ? FCMDP_OK
             : FCMDP_EHIP;
}

int fcmdp_stage_solve(fcmdp_solver* s, const void* spectrum_in,
                      void* spectrum_out, int c_lo, int c_hi,
                      void* hip_stream) {
  if (!s || !spectrum_in || !spectrum_out || !band_ok(s, c_lo, c_hi))
    return FCMDP_EINVAL;
  if (hipSetDevice(s->device) != hipSuccess) return FCMDP_EHIP;
  all_channels(s);
  // the mixed slit channel's kH < 1 columns transform f_z and the
  // correction's node functions in FP64 (from the FP32 input spectrum: the
  // spread's FP64 route is not part of this stage)
  if (fcmdp::lowk_active(s)) s->dp.lowk_ns = s->lowk_ns;
  hipStream_t st = (hipStream_t)hip_stream;
  if (fcmdp::launch_set_band(s, c_lo, c_hi, st) != hipSuccess) return FCMDP_EHIP;
  return fcmdp::launch_columns(s, spectrum_in, spectrum_out, st) == hipSuccess
             ? FCMDP_OK
             : FCMDP_EHIP;
}

int fcmdp_stage_fft_inverse(fcmdp_solver* s, const void* spectrum, void* grid,
                            int c_lo, int c_hi, void* hip_stream) {
  if (!s || !grid || !spectrum || !band_ok(s, c_lo, c_hi)) return FCMDP_EINVAL;
  if (hipSetDevice(s->device) != hipSuccess) return FCMDP_EHIP;
  all_channels(s);
  hipStream_t st = (hipStream_t)hip_stream;
  if (fcmdp::launch_set_band(s, c_lo, c_hi, st) != hipSuccess) return FCMDP_EHIP;
  // the y-pass works in place: run it on the solver's own spectrum buffer
  if (hipMemcpyAsync(s->spec, spectrum, spec_bytes(s), hipMemcpyDeviceToDevice,
                     st) != hipSuccess)
    return FCMDP_EHIP;
  return fcmdp::launch_fft_inverse(s, s->spec, grid, st) == hipSuccess
             ? FCMDP_OK
             : FCMDP_EHIP;
}

int fcmdp_stage_interp(fcmdp_solver* s, int64_t n, const void* pos,
                       const void* grid, void* U, void* Omega,
                       void* hip_stream) {
  int v = check_particles(s, n);
  if (v != FCMDP_OK) return v;
  if (s->dp.torque_deriv) return FCMDP_EINVAL;   // six-channel layouts only
  if (!grid || (n > 0 && (!pos || !U))) return FCMDP_EINVAL;
  if (n == 0) return FCMDP_OK;
  all_channels(s);
  hipStream_t st = (hipStream_t)hip_stream;
  v = particle_front(s, (int)n, pos, nullptr, nullptr, st);
  if (v != FCMDP_OK) return v;
  return fcmdp::launch_interp(s, (int)n, grid, U, Omega, st) == hipSuccess
             ? FCMDP_OK
             : FCMDP_EHIP;
}

}  // extern "C"
