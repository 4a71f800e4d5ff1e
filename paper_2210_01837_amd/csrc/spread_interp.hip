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
          const T* ps = psi + (size_t)p * 2 * dp.Nz;
#pragma unroll
          for (int s = 0; s < kZC; ++s) {
            const int c = c0 + s;
            if (c >= inf.z && c <= inf.w) {
              const T pm = ps[c];
              const T pd = ps[dp.Nz + c];
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

// Wave-uniform spread: a wavefront owns an 8 x 8 patch of grid columns and
// walks, in cell-sorted order, every particle of the 14 x 14 cells whose
// kernels can reach the patch.  The particle is the same on all lanes; each
// lane adds its contribution to its own column when that column lies in the
// particle's 7 x 7 footprint.  Loop trip counts are uniform (no divergence
// between lanes of different cell occupancy) and every column sums its
// particles in a fixed order (deterministic).
//
// Staged path (at most kStage particles in the region, the usual case): lane
// j loads the record of the j-th region particle in parallel with the others
// (x/y weights, and per z-chunk its folded z weights, into a per-wavefront
// LDS block; position and strengths into registers), and the uniform loop
// reads particle v's values with LDS broadcasts and readlanes, so it waits on
// no global memory.  Denser regions take the same loop with scalar loads
// from global memory.  A first pass finds the z-nodes the region's particles
// touch; band planes outside them are written as zeros, the rest are split
// into equal chunks of at most ZC planes accumulated in registers.
constexpr int kPW = 8;   // patch edge per wavefront; 4 wavefronts side by side in x
constexpr int kSpreadZC = 10;                        // at most 14
template <typename T> struct SpreadStage;            // staged particles per region
template <> struct SpreadStage<float> { static constexpr int n = 64; };
template <> struct SpreadStage<double> { static constexpr int n = 32; };
constexpr int kStage = 64;                           // (upper bound of both)

template <typename T>
__device__ __forceinline__ T rdlane(T x, int v) {
  if constexpr (sizeof(T) == 4) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), v));
  } else {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), v);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), v);
    return __hiloint2double(hi, lo);
  }
}
__device__ __forceinline__ int rdlane_i(int x, int v) {
  return __builtin_amdgcn_readlane(x, v);
}

// LDS record of a staged particle: x/y weights of the M and D kernels
// (4 x 7; with DT also the D kernel's derivative along x and y, 2 x 7), then
// the folded z weights of the current chunk (ZC of each of M, D and, with
// DT, the z derivative of D).
template <int ZC, bool DT> struct SpreadRec {
  static constexpr int kW = DT ? 42 : 28;
  static constexpr int kPM = kW, kPD = kW + ZC, kPQ = kW + 2 * ZC;
  static constexpr int kLen = kW + (DT ? 3 : 2) * ZC + 1;     // odd stride
};

// One z-chunk of K planes (K <= ZC) over the staged particles; NCH = 3
// spreads the forces only (no torques), NCH = 6 forces and torques (the
// dipole density g).  DT (with NCH = 3): torques through the derivative of
// the dipole kernel, f += (1/2) grad Delta_D x tau, with grad Delta_D =
// (phi_D' phi_D psi_D, phi_D phi_D' psi_D, phi_D phi_D psi_D').
template <typename T, int ZC, int K, int NCH, bool FZ, bool DT>
__device__ __forceinline__ void spread_chunk(const T* __restrict__ recw,
                                             const double* __restrict__ rec64w,
                                             int total, int c0, int a, int b,
                                             bool inside, const DevParams& dp,
                                             const int4& inf, T F0, T F1, T F2,
                                             T G0, T G1, T G2, T (&acc)[ZC][NCH],
                                             double (&acc64)[ZC]) {
  using Rec = SpreadRec<ZC, DT>;
  constexpr int R64 = DT ? 2 : 1;      // FP64 z weights per node (M, D)
  for (int v = 0; v < total; ++v) {
    const int iz = rdlane_i(inf.z, v), iw = rdlane_i(inf.w, v);
    if (iw < c0 || iz >= c0 + K) continue;         // no overlap in z
    int dx = a - rdlane_i(inf.x, v) + 3;
    if (dx < 0) dx += dp.Nx; else if (dx >= dp.Nx) dx -= dp.Nx;
    int dy = b - rdlane_i(inf.y, v) + 3;
    if (dy < 0) dy += dp.Ny; else if (dy >= dp.Ny) dy -= dp.Ny;
    const T f0v = rdlane(F0, v), f1v = rdlane(F1, v), f2v = rdlane(F2, v);
    T g0v = T(0), g1v = T(0), g2v = T(0);
    if constexpr (NCH == 6 || DT) {
      g0v = rdlane(G0, v); g1v = rdlane(G1, v); g2v = rdlane(G2, v);
    }
    if (inside && dx >= 0 && dx <= 6 && dy >= 0 && dy <= 6) {
      const T* r = recw + v * Rec::kLen;
      const T wm = r[dx] * r[7 + dy];
      const T f0 = f0v * wm, f1 = f1v * wm, f2 = f2v * wm;
      if constexpr (DT) {
        // grad Delta_D = (a psi_D, b psi_D, c psi_D') per node
        const T ga = r[28 + dx] * r[21 + dy];      // phi_D'(x) phi_D(y)
        const T gb = r[14 + dx] * r[35 + dy];      // phi_D(x) phi_D'(y)
        const T gc = r[14 + dx] * r[21 + dy];      // phi_D(x) phi_D(y)
        // (1/2) grad Delta_D x tau = (px pd + qx pq, py pd + qy pq, pz pd)
        const T px = T(0.5) * g2v * gb, qx = T(-0.5) * g1v * gc;
        const T py = T(-0.5) * g2v * ga, qy = T(0.5) * g0v * gc;
        const T pz = T(0.5) * (g1v * ga - g0v * gb);
        if constexpr (FZ) {
          const double f2d = (double)f2v * ((double)r[dx] * (double)r[7 + dy]);
          const double pzd = 0.5 * ((double)g1v * ((double)r[28 + dx] * (double)r[21 + dy]) -
                                    (double)g0v * ((double)r[14 + dx] * (double)r[35 + dy]));
          const double* r64 = rec64w + v * R64 * ZC;
#pragma unroll
          for (int s = 0; s < K; ++s) {
            const T pm = r[Rec::kPM + s], pd = r[Rec::kPD + s], pq = r[Rec::kPQ + s];
            acc[s][0] += f0 * pm + px * pd + qx * pq;
            acc[s][1] += f1 * pm + py * pd + qy * pq;
            acc64[s] = fma(f2d, r64[s], fma(pzd, r64[ZC + s], acc64[s]));
          }
        } else {
#pragma unroll
          for (int s = 0; s < K; ++s) {
            const T pm = r[Rec::kPM + s], pd = r[Rec::kPD + s], pq = r[Rec::kPQ + s];
            acc[s][0] += f0 * pm + px * pd + qx * pq;
            acc[s][1] += f1 * pm + py * pd + qy * pq;
            acc[s][2] += f2 * pm + pz * pd;
          }
        }
        continue;
      }
      if constexpr (FZ) {
        // vertical force in FP64 with the FP64 z weights
        const double f2d = (double)f2v * ((double)r[dx] * (double)r[7 + dy]);
        const double* r64 = rec64w + v * ZC;
#pragma unroll
        for (int s = 0; s < K; ++s) {
          const T pm = r[Rec::kPM + s];
          acc[s][0] += f0 * pm; acc[s][1] += f1 * pm;
          acc64[s] = fma(f2d, r64[s], acc64[s]);
        }
      } else {
#pragma unroll
        for (int s = 0; s < K; ++s) {
          const T pm = r[Rec::kPM + s];
          acc[s][0] += f0 * pm; acc[s][1] += f1 * pm; acc[s][2] += f2 * pm;
        }
      }
      if constexpr (NCH == 6) {
        const T wd = r[14 + dx] * r[21 + dy];
        const T t0 = g0v * wd, t1 = g1v * wd, t2 = g2v * wd;
#pragma unroll
        for (int s = 0; s < K; ++s) {
          const T pd = r[Rec::kPD + s];
          acc[s][3] += t0 * pd; acc[s][4] += t1 * pd; acc[s][5] += t2 * pd;
        }
      }
    }
  }
}

// FZ (mixed slit channel): the vertical force f_z is accumulated in FP64
// with the FP64 z weights psi64 and stored as the FP32 grid value plus its
// residual in fzlo (the exact low-wavenumber route of lowk.hip).  DT: torques
// through the derivative of the dipole kernel (three grid channels).
template <typename T, int ZC, int NCH, bool FZ, bool DT>
__global__ void __launch_bounds__(256)
k_spread_wave(DevParams dp, const int* __restrict__ band,
              const int* __restrict__ cell_start, const int4* __restrict__ pinfo,
              const T* __restrict__ pw, const T* __restrict__ pf,
              const T* __restrict__ psi, const double* __restrict__ psi64,
              const T* __restrict__ pdw, const T* __restrict__ dpsi,
              T* __restrict__ grid, float* __restrict__ fzlo) {
  static_assert(!DT || NCH == 3, "derivative torques spread three channels");
  using Rec = SpreadRec<ZC, DT>;
  constexpr int R64 = DT ? 2 : 1;
  constexpr int kS = SpreadStage<T>::n;
  __shared__ T rec[4][kS][Rec::kLen];       // staged particle records per wavefront
  // their FP64 z weights (M, and with DT also D)
  __shared__ double rec64[FZ ? 4 : 1][FZ ? kS : 1][R64 * ZC];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int gx = (dp.Nx + 4 * kPW - 1) / (4 * kPW);
  const int gy = (dp.Ny + kPW - 1) / kPW;
  const int tile = xcd_tile(blockIdx.x, gx * gy);
  const int xw = ((tile % gx) * 4 + wv) * kPW;
  const int yw = (tile / gx) * kPW;
  if (xw >= dp.Nx) return;                 // whole wavefront; no barriers below
  const int lo = band[0], hi = band[1];
  const int a = xw + (lane & 7), b = yw + (lane >> 3);
  const bool inside = a < dp.Nx && b < dp.Ny;
  const int Nz = dp.Nz;
  const size_t plane = (size_t)dp.Nx * dp.Ny;
  const size_t chstride = plane * dp.Nz;
  const size_t col = (size_t)b * dp.Nx + a;
  // the 14 cell rows / columns that reach the patch (fewer on a tiny grid,
  // so that no cell is visited twice); columns split at the periodic seam
  const int nrows = dp.Ny < 2 * kPW - 2 ? dp.Ny : 2 * kPW - 2;
  const int ncols = dp.Nx < 2 * kPW - 2 ? dp.Nx : 2 * kPW - 2;
  const int xs = wrap_index(xw - 3, dp.Nx);
  const int xe0 = xs + ncols <= dp.Nx ? xs + ncols : dp.Nx;
  const int xe1 = xs + ncols - xe0;        // cells [0, xe1) after the seam
  // the region's particle ranges: lane 2r + s holds part s of cell row r
  int sstart = 0, scnt = 0;
  if (lane < 2 * nrows) {
    const int r = lane >> 1, sg = lane & 1;
    const int row = wrap_index(yw - 3 + r, dp.Ny) * dp.Nx;
    const int ca = sg ? 0 : xs, cb = sg ? xe1 : xe0;
    if (ca < cb) {
      sstart = cell_start[row + ca];
      scnt = cell_start[row + cb] - sstart;
    }
  }
  int incl = scnt;                         // inclusive prefix over lanes
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int t = __shfl_up(incl, d);
    if (lane >= d) incl += t;
  }
  const int soff = incl - scnt;
  const int total = rdlane_i(incl, 63);

  auto zero_outside = [&](int zmin, int zmax) {
    if (!inside) return;
    for (int c = lo; c <= hi; ++c) {
      if (c >= zmin && c <= zmax) continue;
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) grid[ch * chstride + c * plane + col] = T(0);
      if constexpr (FZ) fzlo[c * plane + col] = 0.f;
    }
  };
  auto store_chunk = [&](int c0, int zmax, T (&acc)[ZC][NCH], double (&acc64)[ZC]) {
    if (!inside) return;
#pragma unroll
    for (int s = 0; s < ZC; ++s) {
      const int c = c0 + s;
      if (c <= zmax) {
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
          if (FZ && ch == 2) {
            const float h = (float)acc64[s];
            grid[ch * chstride + c * plane + col] = h;
            fzlo[c * plane + col] = (float)(acc64[s] - (double)h);
          } else {
            grid[ch * chstride + c * plane + col] = acc[s][ch];
          }
        }
      }
    }
  };

  if (total <= kS) {
    // lane j holds the j-th region particle (rows in order, then x)
    int p = -1;
    for (int r = 0; r < 2 * nrows; ++r) {
      const int o = rdlane_i(soff, r), c = rdlane_i(scnt, r), st = rdlane_i(sstart, r);
      if (lane >= o && lane < o + c) p = st + (lane - o);
    }
    const bool has = lane < total;
    int4 inf = make_int4(0, 0, Nz, -1);
    T F0 = 0, F1 = 0, F2 = 0, G0 = 0, G1 = 0, G2 = 0;
    T* recw = &rec[wv][0][0];
    T* mine = &rec[wv][has ? lane : 0][0];
    if (has) {
      inf = pinfo[p];
      const T* f = pf + (size_t)p * 8;
      F0 = f[0]; F1 = f[1]; F2 = f[2];
      if constexpr (NCH == 6 || DT) { G0 = f[4]; G1 = f[5]; G2 = f[6]; }
      const T* w = pw + (size_t)p * 32;
#pragma unroll
      for (int d = 0; d < 7; ++d) {
        mine[d] = w[d];
        mine[7 + d] = w[8 + d];
        if constexpr (NCH == 6 || DT) {
          mine[14 + d] = w[16 + d];
          mine[21 + d] = w[24 + d];
        }
        if constexpr (DT) {
          mine[28 + d] = pdw[(size_t)p * 16 + d];
          mine[35 + d] = pdw[(size_t)p * 16 + 8 + d];
        }
      }
    }
    int zmin = inf.z, zmax = inf.w;
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
      zmin = min(zmin, __shfl_xor(zmin, m));
      zmax = max(zmax, __shfl_xor(zmax, m));
    }
    zmin = rdlane_i(zmin, 0);
    zmax = rdlane_i(zmax, 0);
    zero_outside(zmin, zmax);
    // equal chunks of at most ZC planes
    const int range = zmax - zmin + 1;
    const int npass = (range + ZC - 1) / ZC;
    const int zc = npass > 0 ? (range + npass - 1) / npass : ZC;
    // this lane's particle's folded z weights of a chunk (dense, zero outside
    // its window; nodes past Nz read padding and are never stored), loaded
    // one chunk ahead into registers so that their latency overlaps the
    // current chunk's sums
    T zm[ZC], zd[ZC], zq[ZC];
    double z64[FZ ? R64 * ZC : 1];
    auto zload = [&](int c0) {
      if (!has) return;
      const T* ps = psi + (size_t)p * 2 * Nz;
#pragma unroll
      for (int s = 0; s < ZC; ++s) {
        if (s < zc) {
          zm[s] = ps[c0 + s];
          if constexpr (NCH == 6 || DT) zd[s] = ps[Nz + c0 + s];
          if constexpr (DT) zq[s] = dpsi[(size_t)p * Nz + c0 + s];
          if constexpr (FZ) {
            const double* p64 = psi64 + (size_t)p * R64 * Nz;
            z64[s] = p64[c0 + s];
            if constexpr (DT) z64[ZC + s] = p64[Nz + c0 + s];
          }
        }
      }
    };
    if (zmin <= zmax) zload(zmin);
    for (int c0 = zmin; c0 <= zmax; c0 += zc) {
      if (has) {
#pragma unroll
        for (int s = 0; s < ZC; ++s) {
          if (s < zc) {
            mine[Rec::kPM + s] = zm[s];
            if constexpr (NCH == 6 || DT) mine[Rec::kPD + s] = zd[s];
            if constexpr (DT) mine[Rec::kPQ + s] = zq[s];
            if constexpr (FZ) {
              rec64[wv][lane][s] = z64[s];
              if constexpr (DT) rec64[wv][lane][ZC + s] = z64[ZC + s];
            }
          }
        }
      }
      if (c0 + zc <= zmax) zload(c0 + zc);
      // the records are read by every lane of this wavefront only
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      T acc[ZC][NCH];
      double acc64[ZC];
#pragma unroll
      for (int s = 0; s < ZC; ++s) {
        acc64[s] = 0.0;
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) acc[s][ch] = T(0);
      }
#define FCMDP_CHUNK(K)                                                         \
  case K:                                                                      \
    if constexpr (K <= ZC)                                                     \
      spread_chunk<T, ZC, K, NCH, FZ, DT>(recw, &rec64[FZ ? wv : 0][0][0],    \
                                          total,                               \
                                      c0, a, b, inside, dp, inf, F0, F1, F2,   \
                                      G0, G1, G2, acc, acc64);                 \
    break;
      switch (zc) {
        FCMDP_CHUNK(1) FCMDP_CHUNK(2) FCMDP_CHUNK(3) FCMDP_CHUNK(4) FCMDP_CHUNK(5)
        FCMDP_CHUNK(6) FCMDP_CHUNK(7) FCMDP_CHUNK(8) FCMDP_CHUNK(9) FCMDP_CHUNK(10)
        FCMDP_CHUNK(11) FCMDP_CHUNK(12) FCMDP_CHUNK(13) FCMDP_CHUNK(14)
        default: break;
      }
#undef FCMDP_CHUNK
      store_chunk(c0, min(zmax, c0 + zc - 1), acc, acc64);
      __builtin_amdgcn_wave_barrier();
    }
    return;
  }

  // dense region: the same loop with scalar loads from global memory
  int zmin = dp.Nz, zmax = -1;
  for (int r = 0; r < 2 * nrows; ++r) {
    const int st = rdlane_i(sstart, r), c = rdlane_i(scnt, r);
    for (int q = st; q < st + c; ++q) {
      const int4 inf = pinfo[q];
      zmin = min(zmin, inf.z);
      zmax = max(zmax, inf.w);
    }
  }
  zero_outside(zmin, zmax);
  for (int c0 = zmin; c0 <= zmax; c0 += ZC) {
    T acc[ZC][NCH];
    double acc64[ZC];
#pragma unroll
    for (int s = 0; s < ZC; ++s) {
      acc64[s] = 0.0;
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) acc[s][ch] = T(0);
    }
    for (int r = 0; r < 2 * nrows; ++r) {
      const int p0 = rdlane_i(sstart, r), p1 = p0 + rdlane_i(scnt, r);
      for (int q = p0; q < p1; ++q) {
        const int4 inf = pinfo[q];
        if (inf.w < c0 || inf.z >= c0 + ZC) continue;   // no overlap in z
        const T* ps = psi + (size_t)q * 2 * Nz;
        T pm[ZC], pd[ZC], pq[ZC];
#pragma unroll
        for (int s = 0; s < ZC; ++s) {
          pm[s] = ps[c0 + s];
          pd[s] = (NCH == 6 || DT) ? ps[Nz + c0 + s] : T(0);
          pq[s] = DT ? dpsi[(size_t)q * Nz + c0 + s] : T(0);
        }
        int dx = a - inf.x + 3;
        if (dx < 0) dx += dp.Nx; else if (dx >= dp.Nx) dx -= dp.Nx;
        int dy = b - inf.y + 3;
        if (dy < 0) dy += dp.Ny; else if (dy >= dp.Ny) dy -= dp.Ny;
        const T* f = pf + (size_t)q * 8;
        const T F0 = f[0], F1 = f[1], F2 = f[2];
        const T G0 = f[4], G1 = f[5], G2 = f[6];
        if (inside && dx >= 0 && dx <= 6 && dy >= 0 && dy <= 6) {
          const T* w = pw + (size_t)q * 32;
          const T wm = w[dx] * w[8 + dy];
          const T wd = w[16 + dx] * w[24 + dy];
          const T f0 = F0 * wm, f1 = F1 * wm, f2 = F2 * wm;
          const T t0 = G0 * wd, t1 = G1 * wd, t2 = G2 * wd;
          if constexpr (DT) {
            const T* dw = pdw + (size_t)q * 16;
            const T ga = dw[dx] * w[24 + dy];
            const T gb = w[16 + dx] * dw[8 + dy];
            const T gc = w[16 + dx] * w[24 + dy];
            const T px = T(0.5) * G2 * gb, qx = T(-0.5) * G1 * gc;
            const T py = T(-0.5) * G2 * ga, qy = T(0.5) * G0 * gc;
            const T pz = T(0.5) * (G1 * ga - G0 * gb);
            double f2d = 0.0, pzd = 0.0;
            const double* p64 = nullptr;
            if constexpr (FZ) {
              f2d = (double)F2 * ((double)w[dx] * (double)w[8 + dy]);
              pzd = 0.5 * ((double)G1 * ((double)dw[dx] * (double)w[24 + dy]) -
                           (double)G0 * ((double)w[16 + dx] * (double)dw[8 + dy]));
              p64 = psi64 + (size_t)q * R64 * Nz;
            }
#pragma unroll
            for (int s = 0; s < ZC; ++s) {
              acc[s][0] += f0 * pm[s] + px * pd[s] + qx * pq[s];
              acc[s][1] += f1 * pm[s] + py * pd[s] + qy * pq[s];
              if constexpr (FZ)
                acc64[s] = fma(f2d, p64[c0 + s], fma(pzd, p64[Nz + c0 + s], acc64[s]));
              else
                acc[s][2] += f2 * pm[s] + pz * pd[s];
            }
            continue;
          }
          double f2d = 0.0;
          if constexpr (FZ) f2d = (double)F2 * ((double)w[dx] * (double)w[8 + dy]);
#pragma unroll
          for (int s = 0; s < ZC; ++s) {
            acc[s][0] += f0 * pm[s]; acc[s][1] += f1 * pm[s];
            if constexpr (FZ)
              acc64[s] = fma(f2d, psi64[(size_t)q * R64 * Nz + c0 + s], acc64[s]);
            else
              acc[s][2] += f2 * pm[s];
            if constexpr (NCH == 6) {
              acc[s][3] += t0 * pd[s]; acc[s][4] += t1 * pd[s]; acc[s][5] += t2 * pd[s];
            }
          }
        }
      }
    }
    store_chunk(c0, zmax, acc, acc64);
  }
}

template <typename T, int NCH, bool FZ = false, bool DT = false>
static void spread_wave(const fcmdp_solver* s, void* grid, hipStream_t st) {
  dim3 g(((s->dp.Nx + 4 * kPW - 1) / (4 * kPW)) * ((s->dp.Ny + kPW - 1) / kPW));
  hipLaunchKernelGGL((k_spread_wave<T, kSpreadZC, NCH, FZ, DT>), g, dim3(256), 0,
                     st, s->dp, s->band, s->cell_start, s->pinfo, (const T*)s->pw,
                     (const T*)s->pf, (const T*)s->psi,
                     FZ ? (const double*)s->psi64 : nullptr,
                     DT ? (const T*)s->pdw : nullptr, DT ? (const T*)s->dpsi : nullptr,
                     (T*)grid, FZ ? s->fzlo : nullptr);
}

hipError_t launch_spread(const fcmdp_solver* s, int n, void* grid, hipStream_t st) {
  if (s->dp.dt_torque) {
    // torques through the derivative of the dipole kernel: three channels
    if (s->mixed && s->dp.lowk_ns >= 0)
      spread_wave<float, 3, true, true>(s, grid, st);
    else if (s->mixed && !s->force_wave_spread && !s->force_simple_spread &&
             spread_mfma_fits(s))
      return launch_spread_mfma(s, n, grid, st);
    else if (s->mixed)
      spread_wave<float, 3, false, true>(s, grid, st);
    else
      spread_wave<double, 3, false, true>(s, grid, st);
    return hipGetLastError();
  }
  if (!s->force_simple_spread) {
    // without torques only the three force channels are spread
    const bool dip = s->dp.nch_in == 6;
    if (s->mixed && s->dp.lowk_ns < 0 && !s->force_wave_spread && spread_mfma_fits(s))
      return launch_spread_mfma(s, n, grid, st);
    if (s->mixed && s->dp.lowk_ns >= 0)
      dip ? spread_wave<float, 6, true>(s, grid, st)
          : spread_wave<float, 3, true>(s, grid, st);
    else if (s->mixed)
      dip ? spread_wave<float, 6>(s, grid, st) : spread_wave<float, 3>(s, grid, st);
    else
      dip ? spread_wave<double, 6>(s, grid, st) : spread_wave<double, 3>(s, grid, st);
    return hipGetLastError();
  }
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
  const T* ps = psi + (size_t)i * 2 * dp.Nz;
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
        const T q = quad[c];
        const T qm = q * ps[c] * wm;
        const T qd = q * ps[dp.Nz + c] * wd;
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

// Tiled interpolation: a workgroup owns a 26 x 26 block of xy cells and
// interpolates the particles whose cell lies in it ("home" particles, at most
// `cap` per pass).  Their weights are cached in LDS; the z-nodes they touch
// give the tile's z range, and only those planes of the block plus its 3-cell
// halo are staged in LDS, ZC planes at a time.  An 8-lane group handles one
// particle (lane = x offset of the 7-point window) and reduces its partial
// sums with shuffles in a fixed order, so results are deterministic.  The LDS
// footprint is kept small enough for several workgroups per CU.
constexpr int kTile = 26;
constexpr int kRX = kTile + 6;
constexpr int kIThreads = 512;   // threads per interpolation workgroup
// per particle: wxM[7] wyM[7] wxD[7] wyD[7] (and with DT wxD'[7] wyD'[7])
template <bool DT> struct IRec { static constexpr int n = DT ? 42 : 28; };

// NCH = 6 interpolates velocities and angular velocities (Omega from the
// grid's vorticity channels), NCH = 3 the velocities only (the vorticity
// channels are then not read).  DT (with NCH = 3): Omega = (1/2) sum
// u x grad Delta_D with the derivative of the dipole kernel.
template <typename T, int ZC, int NCH, bool DT = false>
__global__ void __launch_bounds__(kIThreads)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 2, 8)))
k_interp_tiled(DevParams dp, const int* __restrict__ band,
               const int* __restrict__ cell_start,
               const int4* __restrict__ pinfo, const T* __restrict__ pw,
               const T* __restrict__ psi, const T* __restrict__ quad,
               const T* __restrict__ grid, const int* __restrict__ perm,
               const T* __restrict__ pdw, const T* __restrict__ dpsi,
               T* __restrict__ U, T* __restrict__ Om, int cap) {
  static_assert(!DT || NCH == 3, "derivative route reads the velocity channels");
  constexpr int kRec = IRec<DT>::n;
  constexpr int NOUT = (NCH == 6 || DT) ? 6 : 3;         // U (and Omega)
  extern __shared__ unsigned char lds_raw[];
  T* G = reinterpret_cast<T*>(lds_raw);                 // [ZC][NCH][kRX][kRX]
  T* pcw = G + ZC * NCH * kRX * kRX;                    // [cap][kRec]
  T* acc = pcw + cap * kRec;                            // [cap][NOUT]
  int4* pci = reinterpret_cast<int4*>(acc + cap * NOUT); // [cap]
  int* pcj = reinterpret_cast<int*>(pci + cap);         // [cap] output index
  int* pcp = pcj + cap;                                 // [cap] sorted index
  // folded z weights of the current chunk per home particle (M, D and with
  // DT the z derivative of D), staged with the grid planes
  constexpr int NZS = (DT ? 3 : 2) * ZC;
  T* pz = reinterpret_cast<T*>(pcp + cap);              // [cap][NZS]
  __shared__ int rowoff[kTile + 1];
  __shared__ int rowstart[kTile];
  __shared__ int ytab[kRX];
  __shared__ int zr[2];

  const int lo = band[0], hi = band[1];
  if (lo > hi) return;
  const int tid = threadIdx.x;
  const int gxt = (dp.Nx + kTile - 1) / kTile, gyt = (dp.Ny + kTile - 1) / kTile;
  const int tile = xcd_tile(blockIdx.x, gxt * gyt);
  const int tx0 = (tile % gxt) * kTile, ty0 = (tile / gxt) * kTile;
  if (tid < kRX) ytab[tid] = wrap_index(ty0 - 3 + tid, dp.Ny);
  if (tid < kTile) {
    const int iy = ty0 + tid;
    int s0 = 0, e0 = 0;
    if (iy < dp.Ny) {
      s0 = cell_start[iy * dp.Nx + tx0];
      e0 = cell_start[iy * dp.Nx + min(tx0 + kTile, dp.Nx)];
    }
    rowstart[tid] = s0;
    rowoff[tid + 1] = e0 - s0;
  }
  __syncthreads();
  if (tid == 0) {
    rowoff[0] = 0;
    for (int r = 0; r < kTile; ++r) rowoff[r + 1] += rowoff[r];
  }
  __syncthreads();
  const int nhome = rowoff[kTile];
  if (nhome == 0) return;
  const size_t plane = (size_t)dp.Nx * dp.Ny;
  const size_t chstride = plane * dp.Nz;
  const int g = tid / 8, l = tid % 8;
  constexpr int NG = kIThreads / 8;
  constexpr int kRG = kIThreads / kRX;        // row groups in the staging loop
  const int rx = tid % kRX, rg = tid / kRX;
  const int xa = wrap_index(tx0 - 3 + rx, dp.Nx);

  for (int base = 0; base < nhome; base += cap) {
    const int np = min(cap, nhome - base);
    if (tid == 0) { zr[0] = dp.Nz; zr[1] = -1; }
    __syncthreads();
    int zlo = dp.Nz, zhi = -1;
    for (int h = tid; h < np; h += kIThreads) {
      const int hp = base + h;
      int r = 0;
      while (r + 1 < kTile && rowoff[r + 1] <= hp) ++r;
      const int p = rowstart[r] + (hp - rowoff[r]);
      const int4 inf = pinfo[p];
      pci[h] = inf;
      pcj[h] = perm[p];
      pcp[h] = p;
      zlo = min(zlo, inf.z);
      zhi = max(zhi, inf.w);
      const T* w = pw + (size_t)p * 32;
      T* d = pcw + h * kRec;
#pragma unroll
      for (int e = 0; e < 7; ++e) {
        d[e] = w[e];
        d[7 + e] = w[8 + e];
        d[14 + e] = w[16 + e];
        d[21 + e] = w[24 + e];
        if constexpr (DT) {
          d[28 + e] = pdw[(size_t)p * 16 + e];
          d[35 + e] = pdw[(size_t)p * 16 + 8 + e];
        }
      }
#pragma unroll
      for (int e = 0; e < NOUT; ++e) acc[h * NOUT + e] = T(0);
    }
    if (zhi >= 0) {
      atomicMin(&zr[0], zlo);
      atomicMax(&zr[1], zhi);
    }
    __syncthreads();
    const int c_first = zr[0], c_last = zr[1];
    // staging is software pipelined: the rows of the next chunk are loaded
    // into registers while the current chunk is interpolated from LDS.
    // Thread (rg, rx) owns rows rg + kRG e (e = 0, 1, ...) of kRX values;
    // with kRX = 2 kRG, row rg + kRG e is halo row rg + kRG (e & 1) of
    // plane-channel e / 2, so every address is a compile-time offset from
    // two per-thread row bases.
    static_assert(kRX == 2 * kRG, "staging layout");
    constexpr int kPer = 2 * NCH * ZC;
    T pre[kPer];
    T prez[NZS];              // home particle tid's z weights of the chunk
    const bool stager = tid < kRG * kRX;
    const size_t yrow0 = stager ? (size_t)ytab[rg] * dp.Nx + xa : 0;
    const size_t yrow1 = stager ? (size_t)ytab[rg + kRG] * dp.Nx + xa : 0;
    const bool zstager = tid < np;
    const T* zsrc = psi + (size_t)(zstager ? pcp[tid] : 0) * 2 * dp.Nz;
    const T* dsrc = DT ? dpsi + (size_t)(zstager ? pcp[tid] : 0) * dp.Nz : nullptr;
    auto fetch = [&](int c0) {
      const int nz = min(ZC, c_last - c0 + 1);
      const T* gb = grid + (size_t)c0 * plane;
#pragma unroll
      for (int e = 0; e < kPer; ++e) {
        const int t = e >> 1, ch = t % NCH, sidx = t / NCH;
        if (stager && sidx < nz)
          pre[e] = gb[ch * chstride + (size_t)sidx * plane + ((e & 1) ? yrow1 : yrow0)];
      }
#pragma unroll
      for (int sidx = 0; sidx < ZC; ++sidx) {
        if (zstager && sidx < nz) {
          prez[sidx] = zsrc[c0 + sidx];
          prez[ZC + sidx] = zsrc[dp.Nz + c0 + sidx];
          if constexpr (DT) prez[2 * ZC + sidx] = dsrc[c0 + sidx];
        }
      }
    };
    if (c_first <= c_last) fetch(c_first);
    for (int c0 = c_first; c0 <= c_last; c0 += ZC) {
      const int nz = min(ZC, c_last - c0 + 1);
#pragma unroll
      for (int e = 0; e < kPer; ++e) {
        const int sidx = (e >> 1) / NCH;
        if (stager && sidx < nz) G[(rg + kRG * e) * kRX + rx] = pre[e];
      }
      if (zstager) {
#pragma unroll
        for (int e = 0; e < NZS; ++e)
          if (e % ZC < nz) pz[tid * NZS + e] = prez[e];
      }
      T q[ZC];
#pragma unroll
      for (int sidx = 0; sidx < ZC; ++sidx) q[sidx] = sidx < nz ? quad[c0 + sidx] : T(0);
      __syncthreads();
      if (c0 + ZC <= c_last) fetch(c0 + ZC);
      for (int h = g; h < np; h += NG) {
        const int4 inf = pci[h];
        if (inf.w < c0 || inf.z > c0 + nz - 1) continue;   // no z overlap
        T a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0, a5 = 0;
        if (DT && l < 7) {
          const T* w = pcw + h * kRec;
          const T* zs = pz + h * NZS;
          const T wxm = w[l], wxd = w[14 + l], wxq = w[28 + l];
          const int px = inf.x - tx0 + l;
          const int ry0 = inf.y - ty0;
          T pm[ZC], pd[ZC], pq[ZC];
#pragma unroll
          for (int sidx = 0; sidx < ZC; ++sidx) {
            const bool ok = sidx < nz;
            pm[sidx] = ok ? q[sidx] * zs[sidx] : T(0);
            pd[sidx] = ok ? q[sidx] * zs[ZC + sidx] : T(0);
            pq[sidx] = ok ? q[sidx] * zs[2 * ZC + sidx] : T(0);
          }
          for (int dy = 0; dy < 7; ++dy) {
            const T wm = wxm * w[7 + dy];
            const T ga = wxq * w[21 + dy];          // phi_D'(x) phi_D(y)
            const T gb = wxd * w[35 + dy];          // phi_D(x) phi_D'(y)
            const T gc = wxd * w[21 + dy];          // phi_D(x) phi_D(y)
            const int ry = ry0 + dy;
#pragma unroll
            for (int sidx = 0; sidx < ZC; ++sidx) {
              if (sidx < nz) {
                const T qm = pm[sidx] * wm;
                const T gx = pd[sidx] * ga, gy = pd[sidx] * gb, gz = pq[sidx] * gc;
                const T* gp = G + (sidx * NCH * kRX + ry) * kRX + px;
                constexpr int CS = kRX * kRX;
                const T u = gp[0], v = gp[CS], ww = gp[2 * CS];
                a0 += qm * u;
                a1 += qm * v;
                a2 += qm * ww;
                // u x grad Delta_D (the 1/2 is applied at the end)
                a3 += v * gz - ww * gy;
                a4 += ww * gx - u * gz;
                a5 += u * gy - v * gx;
              }
            }
          }
        } else if (!DT && l < 7) {
          const T* w = pcw + h * kRec;
          // dense folded z weights of this particle (zero outside its
          // window), staged for the chunk
          const T* zs = pz + h * NZS;
          const T wxm = w[l], wxd = w[14 + l];
          const int px = inf.x - tx0 + l;
          const int ry0 = inf.y - ty0;
          T pm[ZC], pd[ZC];
#pragma unroll
          for (int sidx = 0; sidx < ZC; ++sidx) {
            const bool ok = sidx < nz;
            pm[sidx] = ok ? q[sidx] * zs[sidx] : T(0);
            pd[sidx] = ok ? q[sidx] * zs[ZC + sidx] : T(0);
          }
          for (int dy = 0; dy < 7; ++dy) {
            const T wm = wxm * w[7 + dy];
            const T wd = wxd * w[21 + dy];
            const int ry = ry0 + dy;
#pragma unroll
            for (int sidx = 0; sidx < ZC; ++sidx) {
              if (sidx < nz) {
                const T qm = pm[sidx] * wm;
                const T qd = pd[sidx] * wd;
                const T* gp = G + (sidx * NCH * kRX + ry) * kRX + px;
                constexpr int CS = kRX * kRX;
                a0 += qm * gp[0];
                a1 += qm * gp[CS];
                a2 += qm * gp[2 * CS];
                if constexpr (NCH == 6) {
                  a3 += qd * gp[3 * CS];
                  a4 += qd * gp[4 * CS];
                  a5 += qd * gp[5 * CS];
                }
              }
            }
          }
        }
#pragma unroll
        for (int m = 1; m < 8; m <<= 1) {
          a0 += __shfl_xor(a0, m, 8);
          a1 += __shfl_xor(a1, m, 8);
          a2 += __shfl_xor(a2, m, 8);
          a3 += __shfl_xor(a3, m, 8);
          a4 += __shfl_xor(a4, m, 8);
          a5 += __shfl_xor(a5, m, 8);
        }
        if (l == 0) {
          T* ac = acc + h * NOUT;
          ac[0] += a0; ac[1] += a1; ac[2] += a2;
          if constexpr (NOUT == 6) { ac[3] += a3; ac[4] += a4; ac[5] += a5; }
        }
      }
      __syncthreads();
    }
    for (int h = tid; h < np; h += kIThreads) {
      const int j = pcj[h];
      const T* ac = acc + h * NOUT;
      U[3 * (size_t)j + 0] = ac[0];
      U[3 * (size_t)j + 1] = ac[1];
      U[3 * (size_t)j + 2] = ac[2];
      if constexpr (NOUT == 6) {
        const T half = DT ? T(0.5) : T(1);
        Om[3 * (size_t)j + 0] = half * ac[3];
        Om[3 * (size_t)j + 1] = half * ac[4];
        Om[3 * (size_t)j + 2] = half * ac[5];
      }
    }
    __syncthreads();
  }
}

// NaN outputs for particles outside the domain (sorted to the end)
template <typename T>
__global__ void k_interp_invalid(int n, int ncells, const uint32_t* __restrict__ skeys,
                                 const int* __restrict__ perm, T* __restrict__ U,
                                 T* __restrict__ Om) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || skeys[i] < (uint32_t)ncells) return;
  const int j = perm[i];
  const T nan = T(NAN);
  U[3 * (size_t)j + 0] = U[3 * (size_t)j + 1] = U[3 * (size_t)j + 2] = nan;
  if (Om) Om[3 * (size_t)j + 0] = Om[3 * (size_t)j + 1] = Om[3 * (size_t)j + 2] = nan;
}

template <typename T, int ZC, int NCH, bool DT = false>
static size_t interp_lds(int cap) {
  constexpr int NOUT = (NCH == 6 || DT) ? 6 : 3;
  constexpr int NZS = (DT ? 3 : 2) * ZC;
  return (size_t)ZC * NCH * kRX * kRX * sizeof(T) +
         (size_t)cap * (IRec<DT>::n + NOUT) * sizeof(T) + (size_t)cap * (16 + 4 + 4) +
         (size_t)cap * NZS * sizeof(T);
}

template <typename T>
static hipError_t interp_tiled(const fcmdp_solver* s, int n, const T* grid,
                               T* U, T* Om, hipStream_t st) {
  const DevParams& dp = s->dp;
  hipLaunchKernelGGL(k_interp_invalid<T>, dim3((n + 255) / 256), dim3(256), 0,
                     st, n, dp.ncells, s->keyA, s->valA, U, Om);
  dim3 g(((dp.Nx + kTile - 1) / kTile) * ((dp.Ny + kTile - 1) / kTile));
  // home particles cached per pass: a monolayer at area fraction 0.5 with
  // R_h = 1.731 h has ~0.22 particles per xy cell, ~150 per 26 x 26 tile;
  // denser tiles take several passes.  176 keeps two workgroups per CU.
  const int cap = sizeof(T) == 4 ? 176 : 96;
  // planes staged per chunk: as many for three channels as for six, so that
  // the velocities are the same bits whether or not Omega is wanted
  constexpr int ZC = sizeof(T) == 4 ? 2 : 1;
  if (Om && dp.dt_omega) {
    // angular velocities through the derivative of the dipole kernel
    const size_t lds = interp_lds<T, ZC, 3, true>(cap);
    hipLaunchKernelGGL((k_interp_tiled<T, ZC, 3, true>), g, dim3(kIThreads), lds,
                       st, dp, s->band, s->cell_start, s->pinfo, (const T*)s->pw,
                       (const T*)s->psi, (const T*)s->quad, grid, s->valA,
                       (const T*)s->pdw, (const T*)s->dpsi, U, Om, cap);
  } else if (Om && dp.nch_out == 6) {
    const size_t lds = interp_lds<T, ZC, 6>(cap);
    hipLaunchKernelGGL((k_interp_tiled<T, ZC, 6>), g, dim3(kIThreads), lds, st,
                       dp, s->band, s->cell_start, s->pinfo, (const T*)s->pw,
                       (const T*)s->psi, (const T*)s->quad, grid, s->valA,
                       nullptr, nullptr, U, Om, cap);
  } else {
    const size_t lds = interp_lds<T, ZC, 3>(cap);
    hipLaunchKernelGGL((k_interp_tiled<T, ZC, 3>), g, dim3(kIThreads), lds, st,
                       dp, s->band, s->cell_start, s->pinfo, (const T*)s->pw,
                       (const T*)s->psi, (const T*)s->quad, grid, s->valA,
                       nullptr, nullptr, U, nullptr, cap);
  }
  return hipGetLastError();
}

hipError_t launch_interp(const fcmdp_solver* s, int n, const void* grid,
                         void* U, void* Omega, hipStream_t st) {
  if (n == 0) return hipSuccess;
  if ((!s->force_simple_interp || s->dp.dt_omega) && !s->force_halo_interp &&
      interp_part_fits(s, n))
    return launch_interp_part(s, n, grid, U, Omega, st);
  if (!s->force_simple_interp || s->dp.dt_omega) {
    if (s->mixed)
      return interp_tiled<float>(s, n, (const float*)grid, (float*)U,
                                 (float*)Omega, st);
    return interp_tiled<double>(s, n, (const double*)grid, (double*)U,
                                (double*)Omega, st);
  }
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
