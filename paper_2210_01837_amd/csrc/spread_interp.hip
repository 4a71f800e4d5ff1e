// ES spreading (step 1 of Sec. 3.4; eq. fcm with the wall images of eq.
// kernelnearwall) and interpolation (step 8; eqs. getpartvel, getpartvort).
//
// Spreading is a gather: one thread owns one grid column (x_a, y_b) and sums
// over the particles of the 7 x 7 cells whose kernels can reach it, read in
// cell-sorted order, so the result is deterministic and needs no atomics.
// The thread keeps a chunk of ZC z-planes x 6 channels in registers and
// writes each chunk once (coalesced across the block along x).
//
// Interpolation: one thread per particle (sorted order for locality) sums
// h^2 w_c u(x_a, y_b, z_c) times its separable weights over its 7 x 7 x
// window stencil.
#include "fcmdp_internal.h"
#include "es.h"

namespace fcmdp {

constexpr int kZC = 8;   // z-planes per register chunk

template <typename T>
__global__ void __launch_bounds__(128)
k_spread(DevParams dp, const int* __restrict__ band,
         const int* __restrict__ cell_start, const int4* __restrict__ pinfo,
         const T* __restrict__ pw, const T* __restrict__ pf,
         const T* __restrict__ psi, T* __restrict__ grid) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (a >= dp.Nx) return;
  const int lo = band[0], hi = band[1];
  const size_t plane = (size_t)dp.Nx * dp.Ny;
  const size_t chstride = plane * dp.Nz;
  const int ZW = dp.ZW;
  for (int c0 = lo; c0 <= hi; c0 += kZC) {
    T acc[kZC][6];
#pragma unroll
    for (int s = 0; s < kZC; ++s)
#pragma unroll
      for (int ch = 0; ch < 6; ++ch) acc[s][ch] = T(0);
    for (int dyi = 0; dyi < kWin; ++dyi) {
      // cells iy = b - (dyi - 3) reach row b with weight index dyi
      const int iy = wrap_index(b - (dyi - 3), dp.Ny);
      const int row = iy * dp.Nx;
      // x-cells a-3 .. a+3, split at the periodic seam
      int segs[2][2];
      int nseg = 0;
      const int x0 = a - 3, x1 = a + 3;
      if (x0 < 0) {
        segs[nseg][0] = x0 + dp.Nx; segs[nseg][1] = dp.Nx - 1; ++nseg;
        segs[nseg][0] = 0; segs[nseg][1] = x1; ++nseg;
      } else if (x1 >= dp.Nx) {
        segs[nseg][0] = x0; segs[nseg][1] = dp.Nx - 1; ++nseg;
        segs[nseg][0] = 0; segs[nseg][1] = x1 - dp.Nx; ++nseg;
      } else {
        segs[nseg][0] = x0; segs[nseg][1] = x1; ++nseg;
      }
      for (int sgi = 0; sgi < nseg; ++sgi) {
        const int p0 = cell_start[row + segs[sgi][0]];
        const int p1 = cell_start[row + segs[sgi][1] + 1];
        for (int p = p0; p < p1; ++p) {
          const int4 inf = pinfo[p];
          if (inf.w < c0 || inf.z >= c0 + kZC) continue;   // no overlap in z
          int dx = a - inf.x;
          if (dx > 3) dx -= dp.Nx;
          if (dx < -3) dx += dp.Nx;
          const T* w = pw + (size_t)p * 32;
          const T wm = w[dx + 3] * w[8 + dyi];
          const T wd = w[16 + dx + 3] * w[24 + dyi];
          if (wm == T(0) && wd == T(0)) continue;
          const T* f = pf + (size_t)p * 8;
          const T f0 = f[0] * wm, f1 = f[1] * wm, f2 = f[2] * wm;
          const T t0 = f[4] * wd, t1 = f[5] * wd, t2 = f[6] * wd;
          const T* ps = psi + (size_t)p * 2 * ZW;
#pragma unroll
          for (int s = 0; s < kZC; ++s) {
            const int zi = c0 + s - inf.z;
            if (zi >= 0 && zi < ZW) {
              const T pm = ps[zi];
              const T pd = ps[ZW + zi];
              acc[s][0] += f0 * pm;
              acc[s][1] += f1 * pm;
              acc[s][2] += f2 * pm;
              acc[s][3] += t0 * pd;
              acc[s][4] += t1 * pd;
              acc[s][5] += t2 * pd;
            }
          }
        }
      }
    }
#pragma unroll
    for (int s = 0; s < kZC; ++s) {
      const int c = c0 + s;
      if (c <= hi) {
#pragma unroll
        for (int ch = 0; ch < 6; ++ch)
          grid[ch * chstride + c * plane + (size_t)b * dp.Nx + a] = acc[s][ch];
      }
    }
  }
}

hipError_t launch_spread(const fcmdp_solver* s, void* grid, hipStream_t st) {
  dim3 block(128);
  dim3 g((s->dp.Nx + 127) / 128, s->dp.Ny);
  if (s->mixed)
    hipLaunchKernelGGL(k_spread<float>, g, block, 0, st, s->dp, s->band,
                       s->cell_start, s->pinfo, (const float*)s->pw,
                       (const float*)s->pf, (const float*)s->psi,
                       (float*)grid);
  else
    hipLaunchKernelGGL(k_spread<double>, g, block, 0, st, s->dp, s->band,
                       s->cell_start, s->pinfo, (const double*)s->pw,
                       (const double*)s->pf, (const double*)s->psi,
                       (double*)grid);
  return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(256)
k_interp(DevParams dp, int n, const uint32_t* __restrict__ skeys,
         const int* __restrict__ perm, const int4* __restrict__ pinfo,
         const T* __restrict__ pw, const T* __restrict__ psi,
         const T* __restrict__ quad, const T* __restrict__ grid,
         T* __restrict__ U, T* __restrict__ Om) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int j = perm[i];
  if (skeys[i] >= (uint32_t)dp.ncells) {
    const T nan = T(NAN);
    U[3 * (size_t)j + 0] = U[3 * (size_t)j + 1] = U[3 * (size_t)j + 2] = nan;
    if (Om)
      Om[3 * (size_t)j + 0] = Om[3 * (size_t)j + 1] =
          Om[3 * (size_t)j + 2] = nan;
    return;
  }
  const int4 inf = pinfo[i];
  const T* w = pw + (size_t)i * 32;
  const T* ps = psi + (size_t)i * 2 * dp.ZW;
  const size_t plane = (size_t)dp.Nx * dp.Ny;
  const size_t chstride = plane * dp.Nz;
  T u0 = 0, u1 = 0, u2 = 0, o0 = 0, o1 = 0, o2 = 0;
  for (int dyi = 0; dyi < kWin; ++dyi) {
    const T wym = w[8 + dyi], wyd = w[24 + dyi];
    if (wym == T(0) && wyd == T(0)) continue;
    const int bb = wrap_index(inf.y + dyi - 3, dp.Ny);
    for (int dxi = 0; dxi < kWin; ++dxi) {
      const T wm = w[dxi] * wym;
      const T wd = w[16 + dxi] * wyd;
      if (wm == T(0) && wd == T(0)) continue;
      const int aa = wrap_index(inf.x + dxi - 3, dp.Nx);
      const size_t col = (size_t)bb * dp.Nx + aa;
      for (int c = inf.z; c <= inf.w; ++c) {
        const int zi = c - inf.z;
        const T q = quad[c];
        const T qm = q * ps[zi] * wm;
        const T qd = q * ps[dp.ZW + zi] * wd;
        const size_t off = (size_t)c * plane + col;
        u0 += qm * grid[off];
        u1 += qm * grid[chstride + off];
        u2 += qm * grid[2 * chstride + off];
        o0 += qd * grid[3 * chstride + off];
        o1 += qd * grid[4 * chstride + off];
        o2 += qd * grid[5 * chstride + off];
      }
    }
  }
  U[3 * (size_t)j + 0] = u0;
  U[3 * (size_t)j + 1] = u1;
  U[3 * (size_t)j + 2] = u2;
  if (Om) {
    Om[3 * (size_t)j + 0] = o0;
    Om[3 * (size_t)j + 1] = o1;
    Om[3 * (size_t)j + 2] = o2;
  }
}

hipError_t launch_interp(const fcmdp_solver* s, int n, const void* grid,
                         void* U, void* Omega, hipStream_t st) {
  if (n == 0) return hipSuccess;
  dim3 g((n + 255) / 256);
  if (s->mixed)
    hipLaunchKernelGGL(k_interp<float>, g, dim3(256), 0, st, s->dp, n,
                       s->keyA, s->valA, s->pinfo, (const float*)s->pw,
                       (const float*)s->psi, (const float*)s->quad,
                       (const float*)grid, (float*)U, (float*)Omega);
  else
    hipLaunchKernelGGL(k_interp<double>, g, dim3(256), 0, st, s->dp, n,
                       s->keyA, s->valA, s->pinfo, (const double*)s->pw,
                       (const double*)s->psi, (const double*)s->quad,
                       (const double*)grid, (double*)U, (double*)Omega);
  return hipGetLastError();
}

}  // namespace fcmdp
