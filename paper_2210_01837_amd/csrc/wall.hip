// Non-uniform tangential wall velocities u^W(x, y) (eq. bcnoslip0; App. A,
// eqs. bcslip and u0uHformula): the nodal wall fields are taken through the
// solver's own forward xy transform (as planes of the grid) and their
// unnormalised spectra kept per column, [4][Nkx][Ny] = u^W, v^W at z = 0,
// then at z = H.  The column solve adds them to the correction's boundary
// data (k != 0) and to the k = 0 wall conditions.
#include "fcmdp_internal.h"

namespace fcmdp {
namespace {

// wall [nw][2][Ny][Nx] -> grid channels 0, 1 of planes 0 .. nw-1, channel 2
// of those planes zero (the transform runs three channels)
template <typename T>
__global__ void k_wall_stage(DevParams dp, int nw, const T* __restrict__ wall,
                             T* __restrict__ grid) {
  const size_t plane = (size_t)dp.Nx * dp.Ny;
  const size_t total = 3 * (size_t)nw * plane;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int ch = (int)(i / ((size_t)nw * plane));
  const size_t r = i - (size_t)ch * nw * plane;
  const int w = (int)(r / plane);
  const size_t e = r - (size_t)w * plane;
  const T v = ch < 2 ? wall[((size_t)w * 2 + ch) * plane + e] : T(0);
  grid[((size_t)ch * dp.Nz + w) * plane + e] = v;
}

// spectrum planes (ch, w) -> wallspec[2 w + ch]; Nyquist columns and the
// top wall of a bottom-wall geometry zero
template <typename T>
__global__ void k_wall_collect(DevParams dp, int nw,
                               const cplx_t<T>* __restrict__ spec,
                               cplx_t<T>* __restrict__ out) {
  const size_t K = (size_t)dp.Nkx * dp.Ny;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 4 * K) return;
  const int q = (int)(i / K);
  const size_t idx = i - (size_t)q * K;
  const int kxi = (int)(idx / dp.Ny), kyi = (int)(idx - (size_t)kxi * dp.Ny);
  const int w = q / 2, ch = q % 2;
  cplx_t<T> v;
  v.x = T(0);
  v.y = T(0);
  if (w < nw && kxi != dp.Nx / 2 && kyi != dp.Ny / 2)
    v = spec[((size_t)ch * dp.Nz + w) * K + idx];
  out[i] = v;
}

template <typename T>
hipError_t wall_impl(const fcmdp_solver* s, int nw, const void* wall,
                     hipStream_t st) {
  const DevParams& dp = s->dp;
  const size_t plane = (size_t)dp.Nx * dp.Ny;
  const size_t n1 = 3 * (size_t)nw * plane;
  hipLaunchKernelGGL(k_wall_stage<T>, dim3((unsigned)((n1 + 255) / 256)),
                     dim3(256), 0, st, dp, nw, (const T*)wall, (T*)s->grid);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_set_band(s, 0, nw - 1, st);
  if (e != hipSuccess) return e;
  e = launch_fft_forward(s, s->grid, s->spec, st);
  if (e != hipSuccess) return e;
  const size_t n2 = 4 * (size_t)dp.Nkx * dp.Ny;
  hipLaunchKernelGGL(k_wall_collect<T>, dim3((unsigned)((n2 + 255) / 256)),
                     dim3(256), 0, st, dp, nw, (const cplx_t<T>*)s->spec,
                     (cplx_t<T>*)s->wallspec);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_wall_spectrum(const fcmdp_solver* s, const void* wall,
                                hipStream_t st) {
  const int nw = s->dp.geometry == 1 ? 2 : 1;
  return s->mixed ? wall_impl<float>(s, nw, wall, st)
                  : wall_impl<double>(s, nw, wall, st);
}

}  // namespace fcmdp
