// Exact low-wavenumber vertical force density for the mixed-precision slit
// channel.
//
// In the slit channel the per-wavenumber solve (Sec. 3.1 DP problem plus the
// App. A correction) responds to node-to-node (rough in z) perturbations of
// the vertical force f_z increasingly strongly as kH -> 0, while the FP32
// grid, FFT and Chebyshev transform add exactly such perturbations (rounding
// of every grid value, of every z weight, of every butterfly).  Over a wide
// box (kH down to ~0.05 at 1448 x 1448 x 12) the rounding noise of the few
// columns with kH < 1 then dominates the error of the whole apply, and it
// grows with the box area.  The columns with |nx|, |ny| <= ns therefore take
// their f_z Chebyshev coefficients from this FP64 path instead:
//
//   spread  f_z accumulated in FP64 with FP64 z weights, stored as the FP32
//           grid value hi = (float) f_z plus the residual lo = (float)(f_z - hi)
//   x       T[c][b][nx]   = sum_a (hi + lo)[c][b][a] e^{-2 pi i nx a / Nx}
//           for nx = 0..ns (direct partial DFT, FP64)
//   y       Y[nx][ny][c]  = sum_b T[c][b][nx] e^{-2 pi i ny b / Ny}
//           for ny = -ns..ns
//   z       coef[n]       = sum_{c in band} Mf[c][n] Y[c]  (DCT-I, Sec. 3.4
//                            step 2, restricted to the band like the FP32 path)
//
// i.e. the same unnormalised xy DFT and Chebyshev transform as the FP32 path,
// evaluated without rounding noise above FP64's.  The column kernels add
// coef to the torque part of the third body-force combination (which stays
// on the FP32 path, weighted by k) and use FP64 correction node functions in
// those columns.
#include "fcmdp_internal.h"

namespace fcmdp {

namespace {

constexpr int kNB = 24;          // nx values per pass (complex accumulators)
constexpr int kChunk = 32;       // a values staged per step
constexpr int kLowkThreads = 256;

// x transform of the band planes of f_z: one workgroup per (row group g,
// band plane c); wave w sums the quarter w of the x range for 64 rows (lane
// = row), the quarters are added in a fixed order.
__global__ void __launch_bounds__(kLowkThreads)
k_lowk_x(DevParams dp, const int* __restrict__ band,
         const float* __restrict__ fz, const float* __restrict__ fzlo,
         const double2* __restrict__ ex, double2* __restrict__ T, int ns) {
  const int lo = band[0], hi = band[1];
  const int c = lo + blockIdx.y;
  if (lo > hi || c > hi) return;
  const int Nx = dp.Nx, Ny = dp.Ny;
  const int nk = ns + 1;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int b0 = blockIdx.x * kLowkRows;
  const int b = b0 + lane;
  const size_t plane = (size_t)c * Ny * Nx;
  // staging: [wave][a][row] (row stride 65 doubles: conflict-free writes of
  // the transposed loads); reused for the quarter sums
  constexpr int kStage = 4 * kChunk * 65, kRed = 3 * kNB * 64 * 2;
  __shared__ double lds[kStage > kRed ? kStage : kRed];
  double* X = lds + wave * kChunk * 65;
  const int a_beg = (wave * Nx) / 4, a_end = ((wave + 1) * Nx) / 4;
  for (int n0 = 0; n0 < nk; n0 += kNB) {
    double ar[kNB], ai[kNB];
#pragma unroll
    for (int j = 0; j < kNB; ++j) { ar[j] = 0.0; ai[j] = 0.0; }
    for (int a0 = a_beg; a0 < a_end; a0 += kChunk) {
      // stage rows b0..b0+63, columns a0..a0+31 as doubles (hi + lo);
      // lane l loads column a0 + l % 32 of rows l / 32, l / 32 + 2, ...
      __builtin_amdgcn_wave_barrier();
#pragma unroll 4
      for (int k = 0; k < 32; ++k) {
        const int r = lane / 32 + 2 * k, aa = a0 + (lane & 31);
        double v = 0.0;
        if (b0 + r < Ny && aa < a_end) {
          const size_t o = plane + (size_t)(b0 + r) * Nx + aa;
          v = (double)fz[o] + (double)fzlo[o];
        }
        X[(lane & 31) * 65 + r] = v;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const int na = min(kChunk, a_end - a0);
      for (int t = 0; t < na; ++t) {
        const double v = X[t * 65 + lane];
        const double2* e = ex + (size_t)(a0 + t) * nk + n0;
#pragma unroll
        for (int j = 0; j < kNB; ++j) {
          if (n0 + j < nk) {
            const double2 w = e[j];
            ar[j] = fma(v, w.x, ar[j]);
            ai[j] = fma(v, w.y, ai[j]);
          }
        }
      }
    }
    // quarters 1..3 to LDS, quarter 0 adds them in order and stores
    __syncthreads();
    if (wave > 0) {
      double* R = lds + (wave - 1) * kNB * 64 * 2;
#pragma unroll
      for (int j = 0; j < kNB; ++j) {
        R[(2 * j) * 64 + lane] = ar[j];
        R[(2 * j + 1) * 64 + lane] = ai[j];
      }
    }
    __syncthreads();
    if (wave == 0 && b < Ny) {
#pragma unroll
      for (int j = 0; j < kNB; ++j) {
        if (n0 + j < nk) {
          double sr = ar[j], si = ai[j];
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            const double* R = lds + q * kNB * 64 * 2;
            sr += R[(2 * j) * 64 + lane];
            si += R[(2 * j + 1) * 64 + lane];
          }
          T[((size_t)(c - lo) * Ny + b) * nk + n0 + j] = make_double2(sr, si);
        }
      }
    }
    __syncthreads();
  }
}

// y transform: one workgroup per (nx, band plane c); the 2 ns + 1 outputs
// ny = -ns..ns each split into 6 partial sums over b, added in order.
constexpr int kYParts = 6;
__global__ void __launch_bounds__(kLowkThreads)
k_lowk_y(DevParams dp, const int* __restrict__ band,
         const double2* __restrict__ T, const double2* __restrict__ ey,
         double2* __restrict__ Y, int ns) {
  const int lo = band[0], hi = band[1];
  const int c = lo + blockIdx.y;
  if (lo > hi || c > hi) return;
  const int nx = blockIdx.x;
  const int Ny = dp.Ny, nk = ns + 1, ny_n = 2 * ns + 1;
  extern __shared__ double2 ylds[];    // [Ny] column, then partial sums
  double2* col = ylds;
  double2* part = ylds + Ny;
  for (int b = threadIdx.x; b < Ny; b += blockDim.x)
    col[b] = T[((size_t)(c - lo) * Ny + b) * nk + nx];
  __syncthreads();
  for (int o = threadIdx.x; o < ny_n * kYParts; o += blockDim.x) {
    const int iy = o / kYParts, pr = o % kYParts;
    const int ny = iy - ns;
    const int bb = (pr * Ny) / kYParts, be = ((pr + 1) * Ny) / kYParts;
    // e^{-2 pi i ny b / Ny} from the table by exact index arithmetic
    const int step = ny < 0 ? ny + Ny : ny;
    int m = (int)(((long long)step * bb) % Ny);
    double sr = 0.0, si = 0.0;
    for (int b = bb; b < be; ++b) {
      const double2 v = col[b], w = ey[m];
      sr = fma(v.x, w.x, fma(-v.y, w.y, sr));
      si = fma(v.x, w.y, fma(v.y, w.x, si));
      m += step;
      if (m >= Ny) m -= Ny;
    }
    part[o] = make_double2(sr, si);
  }
  __syncthreads();
  for (int iy = threadIdx.x; iy < ny_n; iy += blockDim.x) {
    double sr = 0.0, si = 0.0;
    for (int pr = 0; pr < kYParts; ++pr) {
      sr += part[iy * kYParts + pr].x;
      si += part[iy * kYParts + pr].y;
    }
    Y[((size_t)(nx * ny_n + iy)) * dp.Nz + c] = make_double2(sr, si);
  }
}

// Chebyshev transform over the band nodes: one thread per (column, n).
__global__ void k_lowk_dct(DevParams dp, const int* __restrict__ band,
                           const double2* __restrict__ Y,
                           const double* __restrict__ Mf,
                           double2* __restrict__ coef, int ncols) {
  const int lo = band[0], hi = band[1];
  const int N = dp.Nz;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ncols * N) return;
  const int col = i / N, n = i % N;
  double sr = 0.0, si = 0.0;
  for (int c = lo; c <= hi; ++c) {
    const double m = Mf[c * N + n];
    const double2 v = Y[(size_t)col * N + c];
    sr = fma(m, v.x, sr);
    si = fma(m, v.y, si);
  }
  coef[(size_t)col * N + n] = make_double2(sr, si);
}

}  // namespace

bool lowk_active(const fcmdp_solver* s) {
  return s->lowk_ns > 0 && !s->no_lowk && s->mixed && s->dp.Nz <= 32 &&
         !s->force_generic_columns && !s->force_simple_spread;
}

hipError_t launch_lowk(const fcmdp_solver* s, const void* grid, hipStream_t st) {
  const DevParams& dp = s->dp;
  const int ns = s->lowk_ns;
  const int ny_n = 2 * ns + 1, ncols = (ns + 1) * ny_n;
  const size_t plane = (size_t)dp.Nx * dp.Ny;
  const float* fz = (const float*)grid + 2 * plane * dp.Nz;
  // lowk_part holds T (band planes first) and then Y
  double2* T = s->lowk_part;
  double2* Y = s->lowk_part + (size_t)dp.Nz * dp.Ny * (ns + 1);
  hipLaunchKernelGGL(k_lowk_x, dim3((dp.Ny + kLowkRows - 1) / kLowkRows, dp.Nz),
                     dim3(kLowkThreads), 0, st, dp, s->band, fz, s->fzlo,
                     s->lowk_ex, T, ns);
  const size_t ylds = ((size_t)dp.Ny + (size_t)ny_n * kYParts) * sizeof(double2);
  hipLaunchKernelGGL(k_lowk_y, dim3(ns + 1, dp.Nz), dim3(kLowkThreads), ylds, st,
                     dp, s->band, T, s->lowk_ey, Y, ns);
  const int nthr = ncols * dp.Nz;
  hipLaunchKernelGGL(k_lowk_dct, dim3((nthr + 255) / 256), dim3(256), 0, st, dp,
                     s->band, Y, s->dct_f, s->lowk_coef, ncols);
  return hipGetLastError();
}

}  // namespace fcmdp
