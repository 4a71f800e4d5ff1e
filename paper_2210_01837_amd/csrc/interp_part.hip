// Interpolation over aligned grid tiles with partial sums (step 8 of Sec.
// 3.4: U_j = int u Delta_M^W, Omega_j = (1/2) int (curl u) Delta_D^W, eqs.
// getpartvel / getpartvort, trapezoid rule in x and y and Clenshaw-Curtis
// weights in z).
//
// The grid is cut into tiles of 32 columns x 16 rows.  A workgroup stages
// only its own tile's planes (no halo), so every grid value is read from
// HBM once, in whole 128-byte rows.  It takes every particle whose 7 x 7
// window meets the tile (the particles of the tile's cells widened by three
// cells on each side), sums the window nodes that lie inside the tile, and
// writes that partial sum to the particle's slot for this tile.  A window
// meets at most nqx tiles along x (2, or 3 when the last tile column is
// narrower than 6 nodes) and nqy along y; slot (qx, qy) holds the part from
// the qx-th and qy-th tile counted from the one holding the window's first
// node.  A second kernel adds a particle's slots in that fixed order, so the
// result is the same on every run.  Particles with the same slots never
// share a tile, so no two workgroups write the same slot.
#include "fcmdp_internal.h"

namespace fcmdp {

namespace {

constexpr int kPX = 32;               // tile columns (128-byte rows in FP32)
constexpr int kPY = 16;               // tile rows
constexpr int kKP = 2;                // particles per four-lane group and pass
constexpr int kPRW = kPX + 6;         // cell columns whose windows meet a tile
constexpr int kPRH = kPY + 6;         // cell rows
constexpr int kPSeg = 2 * kPRH;       // cell-row segments (split at the seam)
constexpr int kPThreads = 512;
constexpr int kSegW = (kPSeg + 63) / 64;  // wavefronts of the segment scan

template <typename T> struct V16;
template <> struct V16<float> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct V16<double> { typedef double type __attribute__((ext_vector_type(2))); };

template <typename T> struct V8;
template <> struct V8<float> { typedef float type __attribute__((ext_vector_type(2))); };
template <> struct V8<double> { typedef double type __attribute__((ext_vector_type(2))); };

// per particle in LDS: the y weights wyM[7] wyD[7] (and with DT wyD'[7]);
// the x weights are read from the records once, at the end of a pass
template <bool DT> struct PRec { static constexpr int n = DT ? 21 : 14; };

__device__ __forceinline__ int wrap_near(int v, int n) {
  // v in [-n, 2n)
  return v < 0 ? v + n : (v >= n ? v - n : v);
}

// NCH = 6: velocities and angular velocities (Omega from the vorticity
// channels); 3: velocities only, or (DT) Omega = (1/2) sum u x grad Delta_D
// through the derivative of the dipole kernel.
template <typename T, int ZC, int NCH, bool DT>
__global__ void __launch_bounds__(kPThreads)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 2, 8)))
k_interp_part(DevParams dp, const int* __restrict__ band,
              const int* __restrict__ cell_start, const int4* __restrict__ pinfo,
              const T* __restrict__ pw, const T* __restrict__ psi,
              const T* __restrict__ quad, const T* __restrict__ grid,
              const T* __restrict__ pdw, const T* __restrict__ dpsi,
              T* __restrict__ part, int cap, int nqx, int nqy) {
  static_assert(!DT || NCH == 3, "derivative route reads the velocity channels");
  constexpr int kRec = PRec<DT>::n;
  constexpr int NOUT = (NCH == 6 || DT) ? 6 : 3;
  constexpr int NZS = (DT ? 3 : 2) * ZC;
  using vec = typename V16<T>::type;
  constexpr int VW = 16 / sizeof(T);          // elements per 16-byte load
  constexpr int TPR = kPX / VW;               // threads per staged row
  constexpr int RPP = kPThreads / TPR;        // rows per staging pass
  constexpr int NROW = ZC * NCH * kPY;        // staged rows per chunk
  constexpr int NLD = (NROW + RPP - 1) / RPP; // loads per thread per chunk
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* G = reinterpret_cast<T*>(lds_raw);                 // [ZC][NCH][kPY][kPX]
  T* pcw = G + NROW * kPX;                              // [cap][kRec]
  T* pz = pcw + cap * kRec;                             // [cap][NZS]
  int4* pci = reinterpret_cast<int4*>(pz + cap * NZS);  // [cap] window
  int* pcp = reinterpret_cast<int*>(pci + cap);         // [cap] sorted index
  int* pcs = pcp + cap;                                 // [cap] slot
  __shared__ int segoff[kPSeg + 1];
  __shared__ int segst[kPSeg];
  __shared__ int wsum[kSegW];
  __shared__ int zr[2];

  const int lo = band[0], hi = band[1];
  if (lo > hi) return;
  const int tid = threadIdx.x;
  const int Nx = dp.Nx, Ny = dp.Ny;
  const int gxt = (Nx + kPX - 1) / kPX, gyt = (Ny + kPY - 1) / kPY;
  const int tile = xcd_tile(blockIdx.x, gxt * gyt);
  const int tcx = tile % gxt, tcy = tile / gxt;
  const int tx0 = tcx * kPX, ty0 = tcy * kPY;
  const int tw = min(kPX, Nx - tx0), th = min(kPY, Ny - ty0);

  // cell-row segments of the particles' region: row r, part k (k = 1 is the
  // part past the periodic seam in x); a prefix sum over the segments, one
  // wavefront per 64 of them
  int sg_cnt = 0, sg_st = 0, sg_incl = 0;
  if (tid < 64 * kSegW) {
    if (tid < 2 * (th + 6)) {
      const int r = tid >> 1, k = tid & 1;
      const int row = wrap_near(ty0 - 3 + r, Ny) * Nx;
      const int xs = wrap_near(tx0 - 3, Nx), len = tw + 6;
      const int xe0 = xs + len <= Nx ? xs + len : Nx;
      const int ca = k ? 0 : xs, cb = k ? xs + len - xe0 : xe0;
      if (ca < cb) {
        sg_st = cell_start[row + ca];
        sg_cnt = cell_start[row + cb] - sg_st;
      }
    }
    const int lane = tid & 63;
    sg_incl = sg_cnt;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int t = __shfl_up(sg_incl, d);
      if (lane >= d) sg_incl += t;
    }
    if (lane == 63) wsum[tid >> 6] = sg_incl;
  }
  __syncthreads();
  if (tid < 64 * kSegW) {
    for (int w = 0; w < (tid >> 6); ++w) sg_incl += wsum[w];
    if (tid < kPSeg) {
      segst[tid] = sg_st;
      segoff[tid + 1] = sg_incl;
    }
    if (tid == 0) segoff[0] = 0;
  }
  __syncthreads();
  const int nreg = segoff[kPSeg];
  if (nreg == 0) return;
  const size_t plane = (size_t)Nx * Ny;
  const size_t chstride = plane * dp.Nz;
  // four lanes per particle, two neighbouring columns each (one 8- or
  // 16-byte LDS read per plane, channel and row); a group holds the sums of
  // its particles h = g + NG k (k < kKP) in registers over all z-chunks
  constexpr int GL = 4;
  const int g = tid / GL, l = tid % GL;
  constexpr int NG = kPThreads / GL;
  // this thread's staged rows: (plane, channel, row) and 16-byte column
  const int cq = tid % TPR, rr = tid / TPR;
  // aligned, whole vectors
  const bool vload = (Nx % VW) == 0 && (reinterpret_cast<uintptr_t>(grid) & 15) == 0;
  size_t roff[NLD];
  bool ron[NLD];
  int rsid[NLD];
#pragma unroll
  for (int e = 0; e < NLD; ++e) {
    const int R = rr + RPP * e;
    const int r = R % kPY, t = R / kPY, ch = t % NCH, sidx = t / NCH;
    rsid[e] = sidx;
    ron[e] = R < NROW && r < th && VW * cq < tw;
    roff[e] = ch * chstride + (size_t)sidx * plane + (size_t)(ty0 + r) * Nx +
              tx0 + VW * cq;
  }

  for (int base = 0; base < nreg; base += cap) {
    const int np = min(cap, nreg - base);
    if (tid == 0) { zr[0] = dp.Nz; zr[1] = -1; }
    __syncthreads();
    int zlo = dp.Nz, zhi = -1;
    for (int h = tid; h < np; h += kPThreads) {
      const int hp = base + h;
      int a = 0, b = kPSeg;                   // segoff[a] <= hp < segoff[b]
      while (b - a > 1) {
        const int m = (a + b) >> 1;
        if (segoff[m] <= hp) a = m; else b = m;
      }
      const int p = segst[a] + (hp - segoff[a]);
      const int4 inf = pinfo[p];
      // first column and row of the window, tile-local and unwrapped so
      // that the window meets the tile
      int sx = inf.x - 3 - tx0, sy = inf.y - 3 - ty0;
      sx += sx + 6 < 0 ? Nx : (sx >= tw ? -Nx : 0);
      sy += sy + 6 < 0 ? Ny : (sy >= th ? -Ny : 0);
      pci[h] = make_int4(sx, sy, inf.z, inf.w);
      pcp[h] = p;
      // slot: tiles counted from the one holding the window's first node
      const int fx = wrap_near(inf.x - 3, Nx) / kPX;
      const int fy = wrap_near(inf.y - 3, Ny) / kPY;
      const int qx = wrap_near(tcx - fx, gxt), qy = wrap_near(tcy - fy, gyt);
      pcs[h] = qy * nqx + qx;
      zlo = min(zlo, inf.z);
      zhi = max(zhi, inf.w);
      const T* w = pw + (size_t)p * 32;
      T* d = pcw + h * kRec;
#pragma unroll
      for (int e = 0; e < 7; ++e) {
        d[e] = w[8 + e];
        d[7 + e] = w[24 + e];
        if constexpr (DT) d[14 + e] = pdw[(size_t)p * 16 + 8 + e];
      }
    }
    if (zhi >= 0) {
      atomicMin(&zr[0], zlo);
      atomicMax(&zr[1], zhi);
    }
    __syncthreads();
    const int c_first = zr[0], c_last = zr[1];
    // per particle k of the group and column e of the lane's pair: sums over
    // rows and planes with the x weight left out (it is applied once at the
    // end).  Curl route: M (3) and D (3) channels.  Derivative route: M (3),
    // then v Z - w Y, w X, u Z, u Y, v X with X = psi_D phi_D(y),
    // Y = psi_D phi_D'(y), Z = psi_D' phi_D(y) (Omega = (1/2) u x grad
    // Delta_D takes the x weights phi_D, phi_D' per term).
    constexpr int NA = DT ? 8 : NOUT;
    T sacc[kKP][2][NA];
#pragma unroll
    for (int k = 0; k < kKP; ++k)
#pragma unroll
      for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int a = 0; a < NA; ++a) sacc[k][e][a] = T(0);
    // staging is software pipelined: the next chunk's rows are loaded into
    // registers while the current chunk is interpolated from LDS
    vec pre[NLD];
    T prez[NZS];
    const bool zstager = tid < np;
    const int pz_src = zstager ? pcp[tid] : 0;
    const T* zsrc = psi + (size_t)pz_src * 2 * dp.Nz;
    const T* dsrc = DT ? dpsi + (size_t)pz_src * dp.Nz : nullptr;
    auto fetch = [&](int c0) {
      const int nz = min(ZC, c_last - c0 + 1);
      const T* gb = grid + (size_t)c0 * plane;
#pragma unroll
      for (int e = 0; e < NLD; ++e) {
        if (ron[e] && rsid[e] < nz) {
          if (vload) {
            pre[e] = *reinterpret_cast<const vec*>(gb + roff[e]);
          } else {
#pragma unroll
            for (int v = 0; v < VW; ++v)
              pre[e][v] = VW * cq + v < tw ? gb[roff[e] + v] : T(0);
          }
        }
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
      for (int e = 0; e < NLD; ++e)
        if (ron[e] && rsid[e] < nz)
          *reinterpret_cast<vec*>(G + (rr + RPP * e) * kPX + VW * cq) = pre[e];
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
#pragma unroll
      for (int k = 0; k < kKP; ++k) {
        const int h = g + NG * k;
        if (h >= np) continue;
        // (first window column, first row, z window), tile-local, in one
        // 16-byte read; without z overlap the row range is empty
        const int4 geo = pci[h];
        const bool zin = (geo.w >= c0) & (geo.z <= c0 + nz - 1);
        const int sy = geo.y;
        // the lane's column pair: both in the tile or both outside (tile
        // widths are even)
        const int e0 = (geo.x & ~1) + 2 * l;
        const bool xon = (unsigned)e0 < (unsigned)tw;
        const int ec = xon ? e0 : 0;
        const int ra = max(sy, 0), rb = zin ? min(sy + 6, th - 1) : ra - 1;
        const T* w = pcw + h * kRec;
        const T* zs = pz + h * NZS;
        T pm[ZC], pd[ZC], pq[ZC];
#pragma unroll
        for (int sidx = 0; sidx < ZC; ++sidx) {
          // read unconditionally (the staged row of particle h), then select
          const T zm = zs[sidx], zd = zs[ZC + sidx];
          const bool ok = (sidx < nz) & xon;
          pm[sidx] = ok ? q[sidx] * zm : T(0);
          pd[sidx] = ok ? q[sidx] * zd : T(0);
          if constexpr (DT) {
            const T zq = zs[2 * ZC + sidx];
            pq[sidx] = ok ? q[sidx] * zq : T(0);
          }
        }
        // the window's seven rows, unrolled (rows outside the tile skipped)
#pragma unroll
        for (int ry = ra; ry < ra + 7; ++ry) if (ry <= rb) {
          const int dy = ry - sy;
          const T wym = w[dy], wyd = w[7 + dy];
          T wyq = T(0);
          if constexpr (DT) wyq = w[14 + dy];
#pragma unroll
          for (int sidx = 0; sidx < ZC; ++sidx) {
            if (sidx < nz) {
              using v2 = typename V8<T>::type;
              constexpr int CS = kPY * kPX;
              const T* gp = G + (sidx * NCH * kPY + ry) * kPX + ec;
              const T m = pm[sidx] * wym;
              if constexpr (DT) {
                const T X = pd[sidx] * wyd, Y = pd[sidx] * wyq, Z = pq[sidx] * wyd;
                const v2 u = *reinterpret_cast<const v2*>(gp);
                const v2 v = *reinterpret_cast<const v2*>(gp + CS);
                const v2 ww = *reinterpret_cast<const v2*>(gp + 2 * CS);
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                  T* a = sacc[k][e];
                  a[0] += m * u[e];
                  a[1] += m * v[e];
                  a[2] += m * ww[e];
                  a[3] += v[e] * Z - ww[e] * Y;
                  a[4] += ww[e] * X;
                  a[5] += u[e] * Z;
                  a[6] += u[e] * Y;
                  a[7] += v[e] * X;
                }
              } else {
                const T d = pd[sidx] * wyd;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                  const v2 gv = *reinterpret_cast<const v2*>(gp + c * CS);
                  sacc[k][0][c] += m * gv[0];
                  sacc[k][1][c] += m * gv[1];
                }
                if constexpr (NCH == 6) {
#pragma unroll
                  for (int c = 0; c < 3; ++c) {
                    const v2 gv = *reinterpret_cast<const v2*>(gp + (3 + c) * CS);
                    sacc[k][0][3 + c] += d * gv[0];
                    sacc[k][1][3 + c] += d * gv[1];
                  }
                }
              }
            }
          }
        }
      }
      __syncthreads();
    }
    // x weights of the lane's columns, the sums over the group's four lanes
    // (fixed order), and the partial sums of this tile
    const int nslot = nqx * nqy;
#pragma unroll
    for (int k = 0; k < kKP; ++k) {
      const int h = g + NG * k;
      const bool on = h < np;
      const int hc = on ? h : 0;
      const int sx = pci[hc].x;
      const int e0 = (sx & ~1) + 2 * l;
      const int p = pcp[hc];
      const T* w = pw + (size_t)p * 32;
      T o[NOUT];
#pragma unroll
      for (int a = 0; a < NOUT; ++a) o[a] = T(0);
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int dx = e0 + e - sx;                     // window offset
        const bool in = e0 >= 0 && e0 < tw && dx >= 0 && dx < 7;
        const int dxc = in ? dx : 0;
        const T wxm = in ? w[dxc] : T(0), wxd = in ? w[16 + dxc] : T(0);
        const T* a = sacc[k][e];
        o[0] += wxm * a[0];
        o[1] += wxm * a[1];
        o[2] += wxm * a[2];
        if constexpr (DT) {
          const T wxq = in ? pdw[(size_t)p * 16 + dxc] : T(0);
          o[3] += wxd * a[3];
          o[4] += wxq * a[4] - wxd * a[5];
          o[5] += wxd * a[6] - wxq * a[7];
        } else if constexpr (NCH == 6) {
          o[3] += wxd * a[3];
          o[4] += wxd * a[4];
          o[5] += wxd * a[5];
        }
      }
#pragma unroll
      for (int m = 1; m < GL; m <<= 1)
#pragma unroll
        for (int a = 0; a < NOUT; ++a) o[a] += __shfl_xor(o[a], m, GL);
      if (on && l == 0) {
        T* dst = part + ((size_t)p * nslot + pcs[h]) * NOUT;
#pragma unroll
        for (int a = 0; a < NOUT; ++a) dst[a] = o[a];
      }
    }
    __syncthreads();
  }
}

// Sum of a particle's tile slots in slot order; NaN for particles outside
// the domain (sorted to the end).  Omega is halved on the derivative route.
template <typename T, int NOUT, bool DT>
__global__ void __launch_bounds__(256)
k_interp_sum(DevParams dp, int n, const uint32_t* __restrict__ skeys,
             const int* __restrict__ perm, const int4* __restrict__ pinfo,
             const T* __restrict__ part, int nqx, int nqy, T* __restrict__ U,
             T* __restrict__ Om) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int j = perm[i];
  if (skeys[i] >= (uint32_t)dp.ncells) {
    const T nan = T(NAN);
    U[3 * (size_t)j + 0] = U[3 * (size_t)j + 1] = U[3 * (size_t)j + 2] = nan;
    if (Om) Om[3 * (size_t)j + 0] = Om[3 * (size_t)j + 1] = Om[3 * (size_t)j + 2] = nan;
    return;
  }
  const int Nx = dp.Nx, Ny = dp.Ny;
  const int gxt = (Nx + kPX - 1) / kPX, gyt = (Ny + kPY - 1) / kPY;
  const int4 inf = pinfo[i];
  const int fx = wrap_near(inf.x - 3, Nx) / kPX, fy = wrap_near(inf.y - 3, Ny) / kPY;
  // tiles met by the window, as offsets from the first one
  unsigned mx = 0, my = 0;
#pragma unroll
  for (int d = 0; d < 7; ++d) {
    mx |= 1u << wrap_near(wrap_near(inf.x - 3 + d, Nx) / kPX - fx, gxt);
    my |= 1u << wrap_near(wrap_near(inf.y - 3 + d, Ny) / kPY - fy, gyt);
  }
  T s[NOUT];
#pragma unroll
  for (int e = 0; e < NOUT; ++e) s[e] = T(0);
  const int nslot = nqx * nqy;
  const T* src = part + (size_t)i * nslot * NOUT;
  for (int qy = 0; qy < nqy; ++qy) {
    if (!((my >> qy) & 1u)) continue;
    for (int qx = 0; qx < nqx; ++qx) {
      if (!((mx >> qx) & 1u)) continue;
      const T* ps = src + (qy * nqx + qx) * NOUT;
#pragma unroll
      for (int e = 0; e < NOUT; ++e) s[e] += ps[e];
    }
  }
  U[3 * (size_t)j + 0] = s[0];
  U[3 * (size_t)j + 1] = s[1];
  U[3 * (size_t)j + 2] = s[2];
  if constexpr (NOUT == 6) {
    if (Om) {
      const T half = DT ? T(0.5) : T(1);
      Om[3 * (size_t)j + 0] = half * s[3];
      Om[3 * (size_t)j + 1] = half * s[4];
      Om[3 * (size_t)j + 2] = half * s[5];
    }
  }
}

// Tiles a 7-node window can meet along an axis of n nodes cut into tiles of
// width t: 1 with one tile, 3 when a window can span a whole narrow last
// tile (narrower than 6 nodes, with at least three tiles), else 2.
int tiles_met(int n, int t) {
  const int nt = (n + t - 1) / t;
  if (nt == 1) return 1;
  const int last = n - t * (nt - 1);
  return (nt >= 3 && last < 6) ? 3 : 2;
}

template <typename T, int ZC, int NCH, bool DT>
size_t part_lds(int cap) {
  constexpr int NOUT = (NCH == 6 || DT) ? 6 : 3;
  constexpr int NZS = (DT ? 3 : 2) * ZC;
  return (size_t)ZC * NCH * kPY * kPX * sizeof(T) +
         (size_t)cap * (PRec<DT>::n + NZS) * sizeof(T) +
         (size_t)cap * (16 + 4 + 4);
}

template <typename T, int ZC, int NCH, bool DT>
void part_launch(const fcmdp_solver* s, int n, const T* grid, T* U, T* Om, int cap,
                 int nqx, int nqy, hipStream_t st) {
  constexpr int NOUT = (NCH == 6 || DT) ? 6 : 3;
  const DevParams& dp = s->dp;
  T* part = reinterpret_cast<T*>(s->spec);
  const dim3 g(((dp.Nx + kPX - 1) / kPX) * ((dp.Ny + kPY - 1) / kPY));
  const size_t lds = part_lds<T, ZC, NCH, DT>(cap);
  hipLaunchKernelGGL((k_interp_part<T, ZC, NCH, DT>), g, dim3(kPThreads), lds, st, dp, s->band, s->cell_start,
                     s->pinfo, (const T*)s->pw, (const T*)s->psi, (const T*)s->quad,
                     grid, DT ? (const T*)s->pdw : nullptr,
                     DT ? (const T*)s->dpsi : nullptr, part, cap, nqx, nqy);
  hipLaunchKernelGGL((k_interp_sum<T, NOUT, DT>), dim3((n + 255) / 256), dim3(256), 0,
                     st, dp, n, s->keyA, s->valA, s->pinfo, (const T*)part, nqx, nqy, U,
                     NOUT == 6 ? Om : nullptr);
}

template <typename T>
hipError_t part_impl(const fcmdp_solver* s, int n, const T* grid, T* U, T* Om,
                     hipStream_t st) {
  const DevParams& dp = s->dp;
  const int nqx = tiles_met(dp.Nx, kPX), nqy = tiles_met(dp.Ny, kPY);
  // particles cached per pass: a monolayer at area fraction 0.5 has ~0.22
  // particles per xy cell, ~185 in a tile's 38 x 22 cells; denser tiles
  // take several passes.  One plane per chunk keeps the LDS of a workgroup
  // small (35 KB in FP32, 64 KB in FP64), so that several share a CU:
  // the kernel waits on LDS and memory latency more than on either's rate.
  constexpr int ZC = 1;
  const int cap = kKP * (kPThreads / 4);
  if (Om && dp.dt_omega)
    part_launch<T, ZC, 3, true>(s, n, grid, U, Om, cap, nqx, nqy, st);
  else if (Om && dp.nch_out == 6)
    part_launch<T, ZC, 6, false>(s, n, grid, U, Om, cap, nqx, nqy, st);
  else
    part_launch<T, ZC, 3, false>(s, n, grid, U, nullptr, cap, nqx, nqy, st);
  return hipGetLastError();
}

}  // namespace

bool interp_part_fits(const fcmdp_solver* s, int n) {
  const DevParams& dp = s->dp;
  // a tile's particle region (38 x 22 cells) must not wrap onto itself, and
  // the partial sums must fit in the spectrum buffer (free after the
  // inverse transforms)
  if (dp.Nx < kPRW || dp.Ny < kPRH) return false;
  const size_t T = s->mixed ? 4 : 8;
  const size_t nslot = (size_t)tiles_met(dp.Nx, kPX) * tiles_met(dp.Ny, kPY);
  const size_t need = nslot * 6 * (size_t)n * T;
  const size_t spec = 6 * (size_t)dp.Nz * dp.Nkx * dp.Ny * 2 * T;
  return need <= spec;
}

hipError_t launch_interp_part(const fcmdp_solver* s, int n, const void* grid, void* U,
                              void* Omega, hipStream_t st) {
  if (s->mixed)
    return part_impl<float>(s, n, (const float*)grid, (float*)U, (float*)Omega, st);
  return part_impl<double>(s, n, (const double*)grid, (double*)U, (double*)Omega, st);
}

}  // namespace fcmdp
