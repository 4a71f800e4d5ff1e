// Brownian displacements g = M^{1/2} W by the Lanczos process (Sec. 5.2):
// the Krylov space of the translational mobility M (the forces-only apply,
// F -> U) built from W, and g_k = |W| V_k T_k^{1/2} e_1 with T_k the
// tridiagonal matrix of the recurrence (Chow and Saad's Krylov square root,
// the method the paper uses).  The iteration stops when the relative change
// |g_k - g_{k-1}| / |g_{k-1}| (the paper's convergence measure) falls below
// the tolerance.
//
// Each step: w = M v_j - beta_{j-1} v_{j-1}; the coefficients of w on every
// basis vector are removed twice (classical Gram-Schmidt, the first pass
// giving alpha_j), beta_j = |w|, v_{j+1} = w / beta_j.  Exact arithmetic
// gives the plain three-term recurrence; the full reorthogonalisation keeps
// the FP32 basis of the mixed path orthonormal.  Vectors stay on the device;
// reductions accumulate in FP64 in a fixed order (deterministic), and the
// small tridiagonal eigenproblem is solved on the host.
#include "fcmdp_internal.h"

#include <cmath>
#include <mutex>
#include <vector>

namespace fcmdp {

constexpr int kLzMax = 64;          // most Lanczos iterations per call
constexpr int kLzBlocks = 512;      // partial sums per reduction
constexpr int kLzThreads = 256;

struct LzCoef { double c[kLzMax + 1]; };

// partial[v][b] = sum over block b's share of i of a_v[i] * w[i]
template <typename T>
__global__ void __launch_bounds__(kLzThreads)
k_lz_dots(const T* __restrict__ basis, size_t stride, const T* __restrict__ w,
          size_t m, double* __restrict__ partial) {
  __shared__ double red[kLzThreads];
  const int v = blockIdx.y;
  const T* a = basis + (size_t)v * stride;
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * kLzThreads + threadIdx.x; i < m;
       i += (size_t)gridDim.x * kLzThreads)
    acc += (double)a[i] * (double)w[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = kLzThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(size_t)v * gridDim.x + blockIdx.x] = red[0];
}

// out[v] = sum_b partial[v][b]
__global__ void __launch_bounds__(kLzThreads)
k_lz_sum(const double* __restrict__ partial, int nb, double* __restrict__ out) {
  __shared__ double red[kLzThreads];
  const int v = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += kLzThreads) acc += partial[(size_t)v * nb + b];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = kLzThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[v] = red[0];
}

// w[i] = s * w[i] - sum_{v < nvec} c[v] basis_v[i]  (out of place when
// dst != w: dst = s * w - ...)
template <typename T>
__global__ void __launch_bounds__(kLzThreads)
k_lz_update(const T* __restrict__ basis, size_t stride, int nvec, LzCoef c,
            double s, const T* w, T* dst, size_t m) {
  for (size_t i = (size_t)blockIdx.x * kLzThreads + threadIdx.x; i < m;
       i += (size_t)gridDim.x * kLzThreads) {
    double x = s * (double)w[i];
    for (int v = 0; v < nvec; ++v) x -= c.c[v] * (double)basis[(size_t)v * stride + i];
    dst[i] = (T)x;
  }
}

// Eigen-decomposition of a symmetric k x k matrix (row-major, overwritten)
// by cyclic Jacobi rotations: A = Q diag(lam) Q^T, Q row-major.
static void jacobi_eigen(int k, std::vector<double>& A, std::vector<double>& lam,
                         std::vector<double>& Q) {
  Q.assign((size_t)k * k, 0.0);
  for (int i = 0; i < k; ++i) Q[(size_t)i * k + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) {
        const double a = A[(size_t)i * k + j];
        tot += a * a;
        if (i != j) off += a * a;
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < k; ++p)
      for (int q = p + 1; q < k; ++q) {
        const double apq = A[(size_t)p * k + q];
        if (apq == 0.0) continue;
        const double app = A[(size_t)p * k + p], aqq = A[(size_t)q * k + q];
        // rotation angle that zeroes A[p][q]: tan(2 theta) = 2 apq / (aqq - app)
        const double theta = 0.5 * std::atan2(2.0 * apq, aqq - app);
        const double c = std::cos(theta), s = std::sin(theta);
        for (int r = 0; r < k; ++r) {        // columns p, q: A <- A J
          const double arp = A[(size_t)r * k + p], arq = A[(size_t)r * k + q];
          A[(size_t)r * k + p] = c * arp - s * arq;
          A[(size_t)r * k + q] = s * arp + c * arq;
        }
        for (int r = 0; r < k; ++r) {        // rows p, q: A <- J^T A
          const double apr = A[(size_t)p * k + r], aqr = A[(size_t)q * k + r];
          A[(size_t)p * k + r] = c * apr - s * aqr;
          A[(size_t)q * k + r] = s * apr + c * aqr;
        }
        for (int r = 0; r < k; ++r) {        // Q <- Q J
          const double qrp = Q[(size_t)r * k + p], qrq = Q[(size_t)r * k + q];
          Q[(size_t)r * k + p] = c * qrp - s * qrq;
          Q[(size_t)r * k + q] = s * qrp + c * qrq;
        }
      }
  }
  lam.resize(k);
  for (int i = 0; i < k; ++i) lam[i] = A[(size_t)i * k + i];
}

// y = |W| T^{1/2} e_1 for the k x k tridiagonal T (alpha on the diagonal,
// beta beside it); eigenvalues below zero (rounding) are taken as zero.
static void sqrt_e1(int k, const double* alpha, const double* beta, double nrm,
                    std::vector<double>& y) {
  std::vector<double> A((size_t)k * k, 0.0), lam, Q;
  for (int i = 0; i < k; ++i) {
    A[(size_t)i * k + i] = alpha[i];
    if (i + 1 < k) A[(size_t)i * k + i + 1] = A[(size_t)(i + 1) * k + i] = beta[i];
  }
  jacobi_eigen(k, A, lam, Q);
  y.assign(k, 0.0);
  for (int e = 0; e < k; ++e) {
    const double w = std::sqrt(std::max(lam[e], 0.0)) * Q[e];   // Q[0][e]
    for (int i = 0; i < k; ++i) y[i] += Q[(size_t)i * k + e] * w;
  }
  for (int i = 0; i < k; ++i) y[i] *= nrm;
}

// Krylov basis and reduction scratch of one call
constexpr size_t kLzRedBytes = sizeof(double) * (kLzMax + 1) * (kLzBlocks + 1);
inline size_t lz_stride(int64_t n) { return (3 * (size_t)n + 63) & ~(size_t)63; }
template <typename T>
size_t lz_basis_bytes(int64_t n, int max_iter) {
  return (size_t)(max_iter + 1) * lz_stride(n) * sizeof(T);
}

// The Lanczos steps on caller-provided scratch: V the basis
// ((max_iter + 1) x stride words), red the reduction partial sums.  Every
// word of both is written before it is read.
template <typename T>
static int lanczos_core(fcmdp_solver* s, int64_t n, const void* pos,
                        const void* W, void* g, int max_iter, double tol,
                        int* iters_out, double* change_out, hipStream_t st,
                        T* V, double* red) {
  const size_t m = 3 * (size_t)n;
  const size_t stride = lz_stride(n);
  double* part = red;
  double* sums = red + (size_t)(kLzMax + 1) * kLzBlocks;
  const int gb = (int)std::min<size_t>(kLzBlocks, (m + kLzThreads - 1) / kLzThreads);

  // <basis_v, w> for v < nvec, returned on the host
  auto dots = [&](const T* basis, int nvec, const T* w, double* out) -> bool {
    hipLaunchKernelGGL(k_lz_dots<T>, dim3(gb, nvec), dim3(kLzThreads), 0, st,
                       basis, stride, w, m, part);
    hipLaunchKernelGGL(k_lz_sum, dim3(nvec), dim3(kLzThreads), 0, st, part, gb, sums);
    if (hipMemcpyAsync(out, sums, sizeof(double) * nvec, hipMemcpyDeviceToHost, st) !=
        hipSuccess)
      return false;
    return hipStreamSynchronize(st) == hipSuccess;
  };
  auto update = [&](int nvec, const double* c, double sc, const T* w, T* dst) {
    LzCoef cc = {};
    for (int v = 0; v < nvec; ++v) cc.c[v] = c[v];
    hipLaunchKernelGGL(k_lz_update<T>, dim3(gb), dim3(kLzThreads), 0, st,
                       (const T*)V, stride, nvec, cc, sc, w, dst, m);
  };

  double nrm2 = 0.0;
  if (!dots((const T*)W, 1, (const T*)W, &nrm2)) return FCMDP_EHIP;
  const double nrm = std::sqrt(nrm2);
  std::vector<double> alpha, beta, y, yprev;
  double change = 0.0;
  int k = 0;
  if (nrm > 0.0) {
    update(0, nullptr, 1.0 / nrm, (const T*)W, V);                // v_0
    for (int j = 0; j < max_iter; ++j) {
      T* vj = V + (size_t)j * stride;
      T* w = V + (size_t)(j + 1) * stride;
      int rc = fcmdp_apply_mobility(s, n, pos, vj, nullptr, w, nullptr, st);
      if (rc != FCMDP_OK) return rc;
      if (j > 0) {                                               // - beta v_{j-1}
        LzCoef cc = {};
        cc.c[0] = beta[j - 1];
        hipLaunchKernelGGL(k_lz_update<T>, dim3(gb), dim3(kLzThreads), 0, st,
                           (const T*)(V + (size_t)(j - 1) * stride), stride, 1, cc,
                           1.0, (const T*)w, w, m);
      }
      double c[kLzMax + 1];
      if (!dots(V, j + 1, w, c)) return FCMDP_EHIP;                // first pass
      alpha.push_back(c[j]);
      update(j + 1, c, 1.0, w, w);
      if (!dots(V, j + 1, w, c)) return FCMDP_EHIP;                // second pass
      update(j + 1, c, 1.0, w, w);
      double bb = 0.0;
      if (!dots(w, 1, w, &bb)) return FCMDP_EHIP;
      beta.push_back(std::sqrt(bb));
      k = j + 1;
      sqrt_e1(k, alpha.data(), beta.data(), nrm, y);
      if (k > 1) {
        double d = 0.0, p = 0.0;
        for (int i = 0; i < k; ++i) {
          const double yp = i < k - 1 ? yprev[i] : 0.0;
          d += (y[i] - yp) * (y[i] - yp);
          p += yp * yp;
        }
        change = p > 0.0 ? std::sqrt(d / p) : 0.0;
        if (change < tol) break;
      }
      yprev = y;
      // invariant subspace: the Krylov space is exhausted
      if (beta.back() <= 1e-13 * std::fabs(alpha[0])) break;
      if (j + 1 < max_iter) update(0, nullptr, 1.0 / beta.back(), w, w);
    }
  }
  // g = V_k y (zero when W = 0)
  if (k == 0) {
    if (hipMemsetAsync(g, 0, m * sizeof(T), st) != hipSuccess) return FCMDP_EHIP;
  } else {
    std::vector<double> cy(kLzMax + 1, 0.0);
    for (int i = 0; i < k; ++i) cy[i] = -y[i];
    update(k, cy.data(), 0.0, (const T*)V, (T*)g);
  }
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
    return FCMDP_EHIP;
  if (iters_out) *iters_out = k;
  if (change_out) *change_out = change;
  return FCMDP_OK;
}

template <typename T>
static int lanczos_impl(fcmdp_solver* s, int64_t n, const void* pos,
                        const void* W, void* g, int max_iter, double tol,
                        int* iters_out, double* change_out, hipStream_t st) {
  const size_t need = lz_basis_bytes<T>(n, max_iter);
  // stream-ordered (like the rest of the solver's workspace)
  if (need > s->lz_bytes) {
    if (s->lz_basis) (void)hipFreeAsync(s->lz_basis, st);
    s->lz_basis = nullptr;
    s->lz_bytes = 0;
    if (hipMallocAsync(&s->lz_basis, need, st) != hipSuccess) return FCMDP_ENOMEM;
    s->lz_bytes = need;
  }
  if (!s->lz_red && hipMallocAsync((void**)&s->lz_red, kLzRedBytes, st) != hipSuccess)
    return FCMDP_ENOMEM;
  return lanczos_core<T>(s, n, pos, W, g, max_iter, tol, iters_out, change_out,
                         st, (T*)s->lz_basis, s->lz_red);
}

// ---------------------------------------------------------------------------
// Allocation-free variant: the Krylov basis and the reduction partial sums
// live in one file-scope device array per GPU (kept until the process ends).
// Its host-side name is not a device address; the address each device gives
// it is looked up once per device (hipGetSymbolAddress, with that device
// current) and only that pointer is handed to kernels.
constexpr size_t kLzScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kLzScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch[kMaxDevices] = {};

// this device's address of `scratch` (the device must be current), or null
static void* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
      return nullptr;
    g_scratch[device] = p;
  }
  return g_scratch[device];
}

template <typename T>
static int lanczos_noalloc_impl(fcmdp_solver* s, int64_t n, const void* pos,
                                const void* W, void* g, int max_iter, double tol,
                                int* iters_out, double* change_out,
                                hipStream_t st) {
  unsigned char* base = (unsigned char*)scratch_ptr(s->device);
  if (!base) return FCMDP_EHIP;
  // partial sums first (256-byte aligned), then the basis
  const size_t red_bytes = (kLzRedBytes + 255) & ~(size_t)255;
  return lanczos_core<T>(s, n, pos, W, g, max_iter, tol, iters_out, change_out,
                         st, (T*)(base + red_bytes), (double*)base);
}

static bool lanczos_noalloc_fits(const fcmdp_solver* s, int64_t n, int max_iter) {
  const size_t red_bytes = (kLzRedBytes + 255) & ~(size_t)255;
  const size_t basis = s->mixed ? lz_basis_bytes<float>(n, max_iter)
                                : lz_basis_bytes<double>(n, max_iter);
  return red_bytes + basis <= kLzScratchBytes;
}

}  // namespace fcmdp

extern "C" int fcmdp_lanczos_sqrt_noalloc(fcmdp_solver* s, int64_t n,
                                          const void* pos, const void* W,
                                          void* g, int max_iter, double tol,
                                          int* iters, double* rel_change,
                                          void* hip_stream) {
  if (!s || n < 0 || max_iter < 1 || max_iter > fcmdp::kLzMax || !(tol >= 0))
    return FCMDP_EINVAL;
  if (n > s->cap) return FCMDP_ECAPACITY;
  if (n > 0 && (!pos || !W || !g)) return FCMDP_EINVAL;
  if (!fcmdp::lanczos_noalloc_fits(s, n, max_iter)) return FCMDP_ECAPACITY;
  if (hipSetDevice(s->device) != hipSuccess) return FCMDP_EHIP;
  if (iters) *iters = 0;
  if (rel_change) *rel_change = 0.0;
  if (n == 0) return FCMDP_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  return s->mixed
             ? fcmdp::lanczos_noalloc_impl<float>(s, n, pos, W, g, max_iter, tol,
                                                  iters, rel_change, st)
             : fcmdp::lanczos_noalloc_impl<double>(s, n, pos, W, g, max_iter, tol,
                                                   iters, rel_change, st);
}

extern "C" int fcmdp_lanczos_sqrt(fcmdp_solver* s, int64_t n, const void* pos,
                                  const void* W, void* g, int max_iter,
                                  double tol, int* iters, double* rel_change,
                                  void* hip_stream) {
  if (!s || n < 0 || max_iter < 1 || max_iter > fcmdp::kLzMax || !(tol >= 0))
    return FCMDP_EINVAL;
  if (n > s->cap) return FCMDP_ECAPACITY;
  if (n > 0 && (!pos || !W || !g)) return FCMDP_EINVAL;
  if (hipSetDevice(s->device) != hipSuccess) return FCMDP_EHIP;
  if (iters) *iters = 0;
  if (rel_change) *rel_change = 0.0;
  if (n == 0) return FCMDP_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  return s->mixed ? fcmdp::lanczos_impl<float>(s, n, pos, W, g, max_iter, tol,
                                               iters, rel_change, st)
                  : fcmdp::lanczos_impl<double>(s, n, pos, W, g, max_iter, tol,
                                                iters, rel_change, st);
}
