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
//           for nx = 0..ns (direct partial DFT as an FP64 MFMA product)
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

constexpr int kLowkThreads = 256;
constexpr int kAChunk = 32;      // x values staged per step
static_assert((2 * (kLowkMaxNs + 1) + 15) / 16 <= 4, "at most four column tiles");
typedef double d4v __attribute__((ext_vector_type(4)));

// x transform of the band planes of f_z as an FP64 matrix product,
//   T[row][j] = sum_a G[row][a] E[a][j],   row = (c, b), j = (nx, re|im),
// G = hi + lo of the spread, E[a][2 nx] = cos(2 pi nx a / Nx) and
// E[a][2 nx + 1] = -sin(...) (the table lowk_ex, NT column tiles of 16).
// One workgroup per 64 rows of one band plane; wave w owns rows
// 16 w .. 16 w + 15 and every column tile.  The x range is walked 32 values
// at a time: the next chunk's G and E are loaded into registers while the
// current chunk, staged in LDS, goes through v_mfma_f64_16x16x4f64 in
// k-steps of four.  Operand layout (wave64): A[i][k] from lane i + 16 k,
// B[k][j] from lane j + 16 k, and (unlike the FP32 16x16x4 product, whose
// register r holds row 4 (l / 16) + r) D[l / 16 + 4 r][l % 16] in register
// r of lane l.
template <int NT>
__global__ void __launch_bounds__(kLowkThreads)
k_lowk_x(DevParams dp, const int* __restrict__ band,
         const float* __restrict__ fz, const float* __restrict__ fzlo,
         const double* __restrict__ ex, double* __restrict__ T, int ns) {
  constexpr int kCols = 16 * NT;
  constexpr int kES = kCols + 1;                        // LDS row stride of E
  constexpr int kRowsPer = kLowkRows * kAChunk / kLowkThreads;   // G per thread
  constexpr int kEPer = (kAChunk * kCols + kLowkThreads - 1) / kLowkThreads;
  static_assert(kAChunk % 4 == 0 && kLowkThreads % kAChunk == 0, "staging");
  __shared__ double G[kLowkRows * (kAChunk + 1)];
  __shared__ double E[kAChunk * kES];
  const int lo = band[0], hi = band[1];
  const int c = lo + blockIdx.y;
  if (lo > hi || c > hi) return;
  const int Nx = dp.Nx, Ny = dp.Ny;
  const int ncol = 2 * (ns + 1);                        // real columns of T
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int b0 = blockIdx.x * kLowkRows;
  const size_t plane = (size_t)c * Ny * Nx;
  const int i16 = lane & 15, k4 = lane >> 4;
  // this thread's staging slots: column tid % 32 of rows tid / 32 + 8 i
  const int ga = tid % kAChunk, gr = tid / kAChunk;
  float ph[kRowsPer], pl[kRowsPer];
  double pe[kEPer];
  auto fetch = [&](int a0) {
    const int aa = a0 + ga;
#pragma unroll
    for (int i = 0; i < kRowsPer; ++i) {
      const int r = gr + (kLowkThreads / kAChunk) * i;
      ph[i] = pl[i] = 0.f;
      if (aa < Nx && b0 + r < Ny) {
        const size_t o = plane + (size_t)(b0 + r) * Nx + aa;
        ph[i] = fz[o];
        pl[i] = fzlo[o];
      }
    }
#pragma unroll
    for (int k = 0; k < kEPer; ++k) {
      const int e = tid + kLowkThreads * k;
      const int ar = e / kCols, j = e % kCols;
      pe[k] = (e < kAChunk * kCols && a0 + ar < Nx && j < ncol)
                  ? ex[(size_t)(a0 + ar) * ncol + j] : 0.0;
    }
  };
  d4v acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = d4v{0.0, 0.0, 0.0, 0.0};
  fetch(0);
  for (int a0 = 0; a0 < Nx; a0 += kAChunk) {
#pragma unroll
    for (int i = 0; i < kRowsPer; ++i)
      G[(gr + (kLowkThreads / kAChunk) * i) * (kAChunk + 1) + ga] =
          (double)ph[i] + (double)pl[i];
#pragma unroll
    for (int k = 0; k < kEPer; ++k) {
      const int e = tid + kLowkThreads * k;
      if (e < kAChunk * kCols) E[(e / kCols) * kES + e % kCols] = pe[k];
    }
    __syncthreads();
    if (a0 + kAChunk < Nx) fetch(a0 + kAChunk);    // in flight during the products
#pragma unroll
    for (int s4 = 0; s4 < kAChunk / 4; ++s4) {
      const double av = G[(16 * wave + i16) * (kAChunk + 1) + 4 * s4 + k4];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const double bv = E[(4 * s4 + k4) * kES + 16 * t + i16];
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[t], 0, 0, 0);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int j = 16 * t + i16;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int b = b0 + 16 * wave + k4 + 4 * r;
      if (b < Ny && j < ncol)
        T[((size_t)(c - lo) * Ny + b) * ncol + j] = acc[t][r];
    }
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
  const int nt = (2 * (ns + 1) + 15) / 16;         // 1..4 (ns <= kLowkMaxNs)
  const dim3 gx((dp.Ny + kLowkRows - 1) / kLowkRows, dp.Nz);
  const double* exd = (const double*)s->lowk_ex;
  double* Td = (double*)T;
  switch (nt) {
    case 1: hipLaunchKernelGGL(k_lowk_x<1>, gx, dim3(kLowkThreads), 0, st, dp,
                               s->band, fz, s->fzlo, exd, Td, ns); break;
    case 2: hipLaunchKernelGGL(k_lowk_x<2>, gx, dim3(kLowkThreads), 0, st, dp,
                               s->band, fz, s->fzlo, exd, Td, ns); break;
    case 3: hipLaunchKernelGGL(k_lowk_x<3>, gx, dim3(kLowkThreads), 0, st, dp,
                               s->band, fz, s->fzlo, exd, Td, ns); break;
    default: hipLaunchKernelGGL(k_lowk_x<4>, gx, dim3(kLowkThreads), 0, st, dp,
                                s->band, fz, s->fzlo, exd, Td, ns); break;
  }
  const size_t ylds = ((size_t)dp.Ny + (size_t)ny_n * kYParts) * sizeof(double2);
  hipLaunchKernelGGL(k_lowk_y, dim3(ns + 1, dp.Nz), dim3(kLowkThreads), ylds, st,
                     dp, s->band, T, s->lowk_ey, Y, ns);
  const int nthr = ncols * dp.Nz;
  hipLaunchKernelGGL(k_lowk_dct, dim3((nthr + 255) / 256), dim3(256), 0, st, dp,
                     s->band, Y, s->dct_f, s->lowk_coef, ncols);
  return hipGetLastError();
}

}  // namespace fcmdp
