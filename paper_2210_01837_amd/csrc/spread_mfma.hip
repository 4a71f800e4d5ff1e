// Matrix-core spreading of the FP32 grid (step 1 of Sec. 3.4; eq. fcm with
// the wall images of eq. kernelnearwall), for the forces (monopole kernel)
// and the torques (dipole kernel) of a mixed-precision apply.
//
// For a tile of 16 grid columns and a chunk of 20 z-planes the spread is a
// product of two small dense matrices, one pair per ES kernel:
//   grid[col][(z, ch)] = sum_p W[col][p] V[p][(z, ch)]
//   W[col][p]      = phi(x_a - x_p) phi(y_b - y_p)   (zero off the 7 x 7 footprint)
//   V[p][(z, ch)]  = F_p[ch] psi_p(z_c)              (folded z weights: the
//                                                    particle and its images)
// over the particles p of the cells whose kernels reach the tile, taken in
// cell-sorted order, four per v_mfma_f32_16x16x4f32 step.  The gather spread
// it replaces has every lane of a wavefront walk every particle near its
// 8 x 8 patch, of which a quarter reach the lane's column; here a step costs
// one matrix instruction per block of 16 (z, ch) slots, and the lanes only
// build the operands.  The matrix unit's accumulation order is fixed, so the
// grid is the same on every run.
//
// Layout of the operands (wave64): A[i][k] = W of tile column i and step
// particle k comes from lane i + 16k; B[k][n] from lane n + 16k; D[4(l/16) +
// r][l%16] is register r of lane l.  Slot n < 15 is channel n % 3 of planes
// c0 + 4 (n / 3) + b in block b = 0..3, so lane l finishes with four
// neighbouring x columns of one (channel, plane, row) per block: one 16-byte
// store each.  Slot 15 is unused.
//
// Work layout: the grid is cut into strips 16 columns wide and blocks of 8
// rows; a tile row (16 columns of one grid row) draws on the particles of
// the 22 x 7 cells around it, which in cell-sorted order are one contiguous
// slice of its block's region (22 x 14 cells).  Each workgroup walks a run
// of blocks down a strip and keeps the region's particle records in an LDS
// ring: moving to the next block stages only its 8 new cell rows, and does
// so (16-byte loads straight from global memory into LDS) while the current
// block's matrix steps run.  Blocks whose region holds more particles than
// the ring are staged in batches.
#include "fcmdp_internal.h"

namespace fcmdp {

namespace {

typedef float sf4 __attribute__((ext_vector_type(4)));

constexpr int kSZ = 20;          // planes per chunk
constexpr int kSNB = 4;          // blocks of 16 slots per kernel
constexpr int kSW = 16;          // strip (and tile row) width in x

// Staged record of a particle, in 16-byte pieces (floats in brackets):
// pieces 0-7 x/y weights [0, 32) (M x, M y, D x, D y; 8 each), 8-9 forces
// and torques [32, 40), 10 node base [40, 44) (ix, iy as int bits), 11-15
// monopole z weights of the chunk [44, 64), 16-20 dipole z weights
// [64, 84).  With torques through the kernel derivative (DT) also 21-25
// the dipole's z-derivative weights [84, 104) and 26-29 its x/y derivative
// weights [104, 120) (D' x, D' y; 8 each).  The LDS ring holds kCap
// records (three workgroups per CU).
template <bool DT> struct SRec {
  static constexpr int kSlots = DT ? 32 : 24;
  static constexpr int kLen = 4 * kSlots;
  static constexpr int kCap = DT ? 96 : 128;
  static constexpr int kZ = DT ? 3 : 2;          // z-weight rows
  static __device__ __forceinline__ int slot(int s) { return (unsigned)s % kCap; }
};

__device__ __forceinline__ int lane_value(int x, int l) {
  return __builtin_amdgcn_readlane(x, l);
}

__device__ __forceinline__ int lane_prefix(int v, int lane) {
  int incl = v;                            // inclusive prefix over lanes
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int t = __shfl_up(incl, d);
    if (lane >= d) incl += t;
  }
  return incl;
}

// A lane's parts: A column j of a tile row (x = xb + j), B / D slot j
// (channel ch, plane group zg), D rows 4g .. 4g + 3 (x = xo .. xo + 3).
struct Roles {
  int g, j, a, ch, zg, xo;
  bool inside, slot;
};

__device__ __forceinline__ Roles lane_roles(int lane, int xb, int Nx) {
  Roles r;
  r.g = lane >> 4;
  r.j = lane & 15;
  r.a = xb + r.j;
  r.inside = r.a < Nx;
  r.slot = r.j < 15;
  r.ch = r.j % 3;
  r.zg = r.slot ? r.j / 3 : 0;
  r.xo = xb + 4 * r.g;
  return r;
}

// Matrix steps of tile row y over staged particles [s0, s1); particle k's
// record is in ring slot k - base.  DT: the three force channels
// receive F phi_M phi_M psi_M + (1/2) grad Delta_D x tau, one weight matrix
// per term of grad Delta_D = (phi_D' phi_D psi_D, phi_D phi_D' psi_D,
// phi_D phi_D psi_D') (same slots, one accumulator set).
// wrap: the block's particle region crosses a periodic seam (offsets are
// then taken modulo the grid size; elsewhere they already lie in range).
// The B operand needs no zeroing: a particle that is out of range, or a
// step slot past the end, has a zero A column, and every ring slot holds a
// record (finite values), so its products vanish; slot 15 is never stored.
template <int NCH, bool DT>
__device__ __forceinline__ void tile_steps(const float (*rec)[SRec<DT>::kLen], int s0,
                                           int s1, int base, int y, const Roles& ro,
                                           int Nx, int Ny, bool wrap, sf4 (&acc)[2][kSNB]) {
  for (int k0 = s0; k0 < s1; k0 += 4) {
    const int k = k0 + ro.g;
    const bool have = k < s1;
    const float* rk = rec[SRec<DT>::slot(have ? k - base : 0)];
    const int ix = __float_as_int(rk[40]), iy = __float_as_int(rk[41]);
    int dx = ro.a - ix + 3;
    int dy = y - iy + 3;
    if (wrap) {                    // wave-uniform
      if (dx < 0) dx += Nx; else if (dx >= Nx) dx -= Nx;
      if (dy < 0) dy += Ny; else if (dy >= Ny) dy -= Ny;
    }
    const bool ok = have && ro.inside && (unsigned)dx <= 6u && (unsigned)dy <= 6u;
    const int dxs = ok ? dx : 0, dys = ok ? dy : 0;
    if constexpr (DT) {
      // A: the four weight products of the tile column; B: coefficient of
      // channel ch times the z weight row of the term
      const float g0 = rk[36], g1 = rk[37], g2 = rk[38];
      const float am = rk[dxs] * rk[8 + dys];                   // phi_M phi_M
      const float aa = rk[104 + dxs] * rk[24 + dys];            // phi_D' phi_D
      const float ab = rk[16 + dxs] * rk[112 + dys];            // phi_D phi_D'
      const float ac = rk[16 + dxs] * rk[24 + dys];             // phi_D phi_D
      const float cm = rk[32 + ro.ch];
      // (1/2) grad Delta_D x tau by channel: x: a_b g2 - a_c' g1,
      // y: -a_a g2 + a_c' g0, z: a_a g1 - a_b g0 (halved)
      const float ca = ro.ch == 0 ? 0.f : (ro.ch == 1 ? -0.5f * g2 : 0.5f * g1);
      const float cb = ro.ch == 0 ? 0.5f * g2 : (ro.ch == 1 ? 0.f : -0.5f * g0);
      const float cc = ro.ch == 0 ? -0.5f * g1 : (ro.ch == 1 ? 0.5f * g0 : 0.f);
      const sf4 zm = *reinterpret_cast<const sf4*>(rk + 44 + 4 * ro.zg);
      const sf4 zd = *reinterpret_cast<const sf4*>(rk + 64 + 4 * ro.zg);
      const sf4 zq = *reinterpret_cast<const sf4*>(rk + 84 + 4 * ro.zg);
      const float avm = ok ? am : 0.f, ava = ok ? aa : 0.f;
      const float avb = ok ? ab : 0.f, avc = ok ? ac : 0.f;
#pragma unroll
      for (int bl = 0; bl < kSNB; ++bl) {
        const float bm = cm * zm[bl];
        const float ba = ca * zd[bl];
        const float bb = cb * zd[bl];
        const float bc = cc * zq[bl];
        acc[0][bl] = __builtin_amdgcn_mfma_f32_16x16x4f32(avm, bm, acc[0][bl], 0, 0, 0);
        acc[0][bl] = __builtin_amdgcn_mfma_f32_16x16x4f32(ava, ba, acc[0][bl], 0, 0, 0);
        acc[0][bl] = __builtin_amdgcn_mfma_f32_16x16x4f32(avb, bb, acc[0][bl], 0, 0, 0);
        acc[0][bl] = __builtin_amdgcn_mfma_f32_16x16x4f32(avc, bc, acc[0][bl], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int pt = 0; pt < (NCH == 6 ? 2 : 1); ++pt) {
        const float w = rk[16 * pt + dxs] * rk[16 * pt + 8 + dys];
        const float av = ok ? w : 0.f;
        const float f = rk[32 + 4 * pt + ro.ch];
        const sf4 zw = *reinterpret_cast<const sf4*>(rk + 44 + kSZ * pt + 4 * ro.zg);
#pragma unroll
        for (int bl = 0; bl < kSNB; ++bl) {
          const float bv = f * zw[bl];
          acc[pt][bl] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[pt][bl], 0, 0, 0);
        }
      }
    }
  }
}

// Every band plane of the chunk of tile row y, zeros included.
template <int NCH>
__device__ __forceinline__ void tile_store(float* __restrict__ grid,
                                           const sf4 (&acc)[2][kSNB], int c0, int lo,
                                           int hi, int y, const Roles& ro, int Nx,
                                           int Ny, size_t plane, size_t chstride,
                                           bool vst) {
  if (!ro.slot || y >= Ny || ro.xo >= Nx) return;
  const size_t col = (size_t)y * Nx + ro.xo;
#pragma unroll
  for (int bl = 0; bl < kSNB; ++bl) {
    const int z = c0 + 4 * ro.zg + bl;
    if (z < lo || z > hi) continue;
#pragma unroll
    for (int pt = 0; pt < (NCH == 6 ? 2 : 1); ++pt) {
      const sf4 v = acc[pt][bl];
      float* dst = grid + (size_t)(ro.ch + 3 * pt) * chstride + z * plane + col;
      if (vst) {
        *reinterpret_cast<sf4*>(dst) = v;
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (ro.xo + r < Nx) dst[r] = v[r];
      }
    }
  }
}

__device__ __forceinline__ void wait_loads() {
  // the direct loads write LDS behind the compiler's back
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// NCH = 6: forces and torques; 3: forces only, or (DT) forces with the
// torques through the derivative of the dipole kernel.  Blocks of BY rows
// (8, or 16 for sparse particles: more work per staged row).
template <int NCH, int BY, bool DT>
__global__ void __launch_bounds__(256)
k_spread_mfma(DevParams dp, const int* __restrict__ band,
              const int* __restrict__ cell_start, const int4* __restrict__ pinfo,
              const float* __restrict__ pw, const float* __restrict__ pf,
              const float* __restrict__ psi, const float* __restrict__ pdw,
              const float* __restrict__ dpsi, float* __restrict__ grid, int nseg) {
  static_assert(!DT || NCH == 3, "derivative torques spread three channels");
  using R = SRec<DT>;
  constexpr int kSlots = R::kSlots, kSRec = R::kLen, kCap = R::kCap;
  constexpr int kBY = BY, kTPW = BY / 4;
  constexpr int kRows = BY + 6;            // cell rows of a block's region
  static_assert(2 * kRows <= 64 && 2 * BY + 7 <= 64, "lanes per segment, rows in rs");
  __shared__ __align__(16) float rec[kCap][kSRec];
  __shared__ int rs[64];      // stream index of the first particle of row r (r mod 64)
  __shared__ int pidx[kCap];  // batched staging: batch index -> particle
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int Nx = dp.Nx, Ny = dp.Ny, Nz = dp.Nz;
  const int gx = (Nx + kSW - 1) / kSW, nby = (Ny + kBY - 1) / kBY;
  // block bi = sx * nby + by (strip sx, block row by).  nseg = 0: the
  // workgroups share this strip-major sequence evenly.  nseg > 0: workgroup
  // w takes row segment w / gx of strip w % gx, so that all strips advance
  // through the same rows together and neighbouring strips' pieces of a
  // 128-byte line are written at about the same time (rows of Nx floats
  // that are not a whole number of lines put every strip's 64-byte piece
  // across two lines).
  const int nblk = gx * nby, nwg = gridDim.x;
  const int w = xcd_tile(blockIdx.x, nwg);
  int bA, bB;
  if (nseg > 0) {
    const int sxw = w % gx, sg = w / gx;
    bA = sxw * nby + (int)((long long)sg * nby / nseg);
    bB = sxw * nby + (int)((long long)(sg + 1) * nby / nseg);
  } else {
    bA = (int)((long long)w * nblk / nwg);
    bB = (int)((long long)(w + 1) * nblk / nwg);
  }
  const int lo = band[0], hi = band[1];
  const size_t plane = (size_t)Nx * Ny;
  const size_t chstride = plane * Nz;
  const bool vec = (Nz & 3) == 0;          // 16-byte aligned z-weight rows
  const bool vst = (Nx & 3) == 0;          // 16-byte aligned grid rows

  for (int c0 = vec ? (lo & ~3) : lo; c0 <= hi; c0 += kSZ) {
    // piece `lane` of a record (lanes < kSlots): source and bytes per particle
    const char* pbase;
    unsigned pstride;
    bool pon;
    {
      const int part = lane < kSlots ? lane : kSlots - 1;
      if (part < 8) {
        pbase = reinterpret_cast<const char*>(pw + 4 * part); pstride = 128;
        pon = NCH == 6 || DT || part < 4;
      } else if (part < 10) {
        pbase = reinterpret_cast<const char*>(pf + 4 * (part - 8)); pstride = 32;
        pon = NCH == 6 || DT || part == 8;
      } else if (part == 10) {
        pbase = reinterpret_cast<const char*>(pinfo); pstride = 16;
        pon = true;
      } else if (part < 11 + 5 * R::kZ) {
        // z weights: monopole, dipole, (DT) dipole derivative rows of the chunk
        const int u = part - 11, h = u / 5, uu = u - 5 * h;
        const int z = c0 + 4 * uu;
        const int zc = z < Nz ? z : Nz - 4;      // past Nz: never stored
        if (h < 2) {
          pbase = reinterpret_cast<const char*>(psi + h * Nz + zc); pstride = 8u * Nz;
        } else {
          pbase = reinterpret_cast<const char*>(dpsi + zc); pstride = 4u * Nz;
        }
        pon = vec && (NCH == 6 || DT || h == 0);
      } else if (DT && part < 30) {
        // x/y weights of the dipole kernel's derivative
        pbase = reinterpret_cast<const char*>(pdw + 4 * (part - 26)); pstride = 64;
        pon = true;
      } else {
        pbase = reinterpret_cast<const char*>(pinfo); pstride = 16;
        pon = false;
      }
      pon = pon && lane < kSlots;
    }
    // z-weight rows that are not 16-byte aligned: one float per lane
    // (lanes < 20 per row: monopole, dipole, dipole derivative)
    const float* zbase;
    unsigned zstride;
    bool zon;
    {
      const int h = lane / kSZ, z = c0 + lane - kSZ * h;
      const int zc = z < Nz ? z : Nz - 1;
      if (h < 2) {
        zbase = psi + h * Nz + zc; zstride = 2u * Nz;
      } else {
        zbase = dpsi + zc; zstride = Nz;
      }
      zon = !vec && lane < (NCH == 6 ? 2 : DT ? 3 : 1) * kSZ;
    }
    // stage particle p's record in ring slot s (s uniform)
    auto put = [&](int s, int p) {
      float* dst = rec[R::slot(s)];
      if (pon)
        __builtin_amdgcn_global_load_lds(pbase + (size_t)p * pstride,
                                         (__attribute__((address_space(3))) void*)dst,
                                         16, 0, 0);
      if (zon)
        __builtin_amdgcn_global_load_lds(zbase + (size_t)p * zstride,
                                         (__attribute__((address_space(3))) void*)(dst + 44),
                                         4, 0, 0);
    };

    int S = 0;                 // stream index of the next staged particle
    bool ring = false;         // the ring holds the current block's region
    int cur_sx = -1;
    int nm_st = 0, nm_ct = 0;  // the next block's new rows (lanes < 16)
    for (int bi = bA; bi < bB; ++bi) {
      const int sx = bi / nby, by = bi - sx * nby;
      const int xb = sx * kSW, yb = by * kBY;
      if (sx != cur_sx) ring = false;      // a new strip: start over
      cur_sx = sx;
      const Roles ro = lane_roles(lane, xb, Nx);
      // the block's particle region (cells xb - 3 .. xb + 18, rows yb - 3 ..
      // yb + kBY + 2) crosses a periodic seam
      const bool seam = xb < 3 || xb + kSW + 3 > Nx || yb < 3 || yb + kBY + 3 > Ny;
      // the strip's cells xb - 3 .. xb + 18, split at the periodic seam
      const int xs = wrap_index(xb - 3, Nx);
      const int xe0 = xs + kSW + 6 <= Nx ? xs + kSW + 6 : Nx;
      const int xe1 = xs + kSW + 6 - xe0;
      // segment (lane & 1) of cell row ra + (lane >> 1), lanes < 2n: first
      // particle and count
      auto row_meta = [&](int ra, int n, int& st, int& ct) {
        st = 0;
        ct = 0;
        if (lane < 2 * n) {
          const int row = wrap_index(ra + (lane >> 1), Ny) * Nx;
          const int sg = lane & 1;
          const int ca = sg ? 0 : xs, cb = sg ? xe1 : xe0;
          if (ca < cb) {
            st = cell_start[row + ca];
            ct = cell_start[row + cb] - st;
          }
        }
      };
      // append rows ra .. ra + n - 1 to the stream: their starts (and the
      // end) in rs, their records into the ring (each wavefront takes every
      // fourth segment)
      auto add_rows = [&](int ra, int n, int st, int ct) {
        const int incl = lane_prefix(ct, lane);
        const int excl = incl - ct;
        const int tot = lane_value(incl, 63);
        const int e2 = __shfl(excl, (2 * lane) & 63);
        if (wv == 0 && lane <= n) rs[(ra + lane) & 63] = S + e2;
        for (int l = wv; l < 2 * n; l += 4) {
          const int sst = lane_value(st, l), sc = lane_value(ct, l);
          const int se = lane_value(excl, l);
          for (int k = 0; k < sc; ++k) put(S + se + k, sst + k);
        }
        S += tot;
      };
      // the next block (and the one after) continue down the same strip
      auto follows = [&](int d) { return bi + d < bB && (bi + d) / nby == sx; };
      const bool more = follows(1);

      if (!ring) {
        int st, ct;
        row_meta(yb - 3, kRows, st, ct);
        const int incl = lane_prefix(ct, lane);
        const int tot = lane_value(incl, 63);
        if (tot <= kCap) {
          S = 0;
          add_rows(yb - 3, kRows, st, ct);
          ring = true;
          if (more) row_meta(yb + kBY + 3, kBY, nm_st, nm_ct);
          wait_loads();
          __syncthreads();
        } else {
          // a dense region: every batch again for each tile row
          const int excl = incl - ct;
          for (int tt = 0; tt < kTPW; ++tt) {
            const int t = wv * kTPW + tt;
            const int y = yb + t;
            const int r0 = lane_value(excl, 2 * t), r1 = lane_value(excl, 2 * (t + 7));
            sf4 acc[2][kSNB];
#pragma unroll
            for (int pt = 0; pt < 2; ++pt)
#pragma unroll
              for (int q = 0; q < kSNB; ++q) acc[pt][q] = sf4{0.f, 0.f, 0.f, 0.f};
            for (int base = 0; base < tot; base += kCap) {
              const int cnt = tot - base < kCap ? tot - base : kCap;
              if (lane < 2 * kRows) {
                const int k0 = base - excl > 0 ? base - excl : 0;
                const int k1 = base + cnt - excl < ct ? base + cnt - excl : ct;
                if (wv == 0)
                  for (int k = k0; k < k1; ++k) pidx[excl + k - base] = st + k;
              }
              __syncthreads();
              for (int q = wv; q < cnt; q += 4) put(q, pidx[q]);
              wait_loads();
              __syncthreads();
              if (y < Ny)
                tile_steps<NCH, DT>(rec, r0 > base ? r0 : base,
                                    r1 < base + cnt ? r1 : base + cnt, base, y, ro, Nx,
                                    Ny, true, acc);
              __syncthreads();             // the batch is read
            }
            tile_store<NCH>(grid, acc, c0, lo, hi, y, ro, Nx, Ny, plane, chstride, vst);
          }
          continue;                        // ring stays empty
        }
      }

      // the ring holds this block's region: stage the next block's new rows
      // now if they fit beside it, else after this block
      int nst2 = 0, nct2 = 0;
      bool pend = false;
      if (more) {
        const int cn = lane_value(lane_prefix(nm_ct, lane), 63);
        if (S + cn - rs[(yb - 3) & 63] <= kCap)
          add_rows(yb + kBY + 3, kBY, nm_st, nm_ct);
        else
          pend = true;
        if (follows(2)) row_meta(yb + 2 * kBY + 3, kBY, nst2, nct2);
      }
#pragma unroll
      for (int tt = 0; tt < kTPW; ++tt) {
        sf4 acc[2][kSNB];
#pragma unroll
        for (int pt = 0; pt < 2; ++pt)
#pragma unroll
          for (int q = 0; q < kSNB; ++q) acc[pt][q] = sf4{0.f, 0.f, 0.f, 0.f};
        const int y = yb + wv * kTPW + tt;
        if (y < Ny)
          tile_steps<NCH, DT>(rec, rs[(y - 3) & 63], rs[(y + 4) & 63], 0, y, ro, Nx, Ny,
                              seam, acc);
        // the next rows' loads were issued before the steps (and the first
        // tile row's stores one tile row ago): wait before the last stores
        if (tt == kTPW - 1) wait_loads();
        tile_store<NCH>(grid, acc, c0, lo, hi, y, ro, Nx, Ny, plane, chstride, vst);
      }
      __syncthreads();
      if (pend) {
        const int cn = lane_value(lane_prefix(nm_ct, lane), 63);
        if (S + cn - rs[(yb + kBY - 3) & 63] <= kCap) {
          add_rows(yb + kBY + 3, kBY, nm_st, nm_ct);
          wait_loads();
          __syncthreads();
        } else {
          ring = false;
        }
      }
      if (!more) ring = false;
      nm_st = nst2;
      nm_ct = nct2;
    }
    __syncthreads();                       // before the next chunk's staging
  }
}

}  // namespace

bool spread_mfma_fits(const fcmdp_solver* s) {
  // a block's region (22 cells wide, 14 rows at least) must not wrap onto
  // itself
  return s->dp.Nx >= kSW + 6 && s->dp.Ny >= 8 + 6;
}

template <int NCH, int BY, bool DT = false>
static void spread_mfma_impl(const fcmdp_solver* s, void* grid, hipStream_t st) {
  const int gx = (s->dp.Nx + kSW - 1) / kSW, nby = (s->dp.Ny + BY - 1) / BY;
  const int nblk = gx * nby;
  const int cus = s->num_cu > 0 ? s->num_cu : 256;
  int nwg = s->spread_workgroups > 0 ? s->spread_workgroups : 3 * cus;
  // strips side by side when grid rows are not whole 128-byte lines (and
  // when asked); the segments per strip then keep every workgroup resident
  const bool aligned = ((size_t)s->dp.Nx * sizeof(float)) % 128 == 0;
  int nseg = 0;
  if (s->spread_order == 2 || (s->spread_order == 0 && !aligned)) {
    nseg = nwg / gx;
    if (nseg < 1) nseg = 1;
    if (nseg > nby) nseg = nby;
    nwg = gx * nseg;
  }
  if (nwg > nblk) nwg = nblk;
  hipLaunchKernelGGL((k_spread_mfma<NCH, BY, DT>), dim3(nwg), dim3(256), 0, st, s->dp,
                     s->band, s->cell_start, s->pinfo, (const float*)s->pw,
                     (const float*)s->pf, (const float*)s->psi,
                     DT ? (const float*)s->pdw : nullptr,
                     DT ? (const float*)s->dpsi : nullptr, (float*)grid, nseg);
}

hipError_t launch_spread_mfma(const fcmdp_solver* s, int n, void* grid, hipStream_t st) {
  // 16-row blocks when a region and the next block's rows (22 x 38 cells)
  // hold about three quarters of the ring or fewer, so that the next rows
  // still load beside the current block
  const bool dt = s->dp.dt_torque != 0;
  int by = s->spread_block_rows;
  if (by == 0) {
    const double fill = 0.78 * (dt ? SRec<true>::kCap : SRec<false>::kCap);
    by = (double)n * (22.0 * 38.0) <= fill * (double)s->dp.Nx * s->dp.Ny ? 16 : 8;
  }
  if (s->dp.Ny < 16 + 6) by = 8;
  if (dt) {
    by == 16 ? spread_mfma_impl<3, 16, true>(s, grid, st)
             : spread_mfma_impl<3, 8, true>(s, grid, st);
    return hipGetLastError();
  }
  const bool dip = s->dp.nch_in == 6;
  if (by == 16)
    dip ? spread_mfma_impl<6, 16>(s, grid, st) : spread_mfma_impl<3, 16>(s, grid, st);
  else
    dip ? spread_mfma_impl<6, 8>(s, grid, st) : spread_mfma_impl<3, 8>(s, grid, st);
  return hipGetLastError();
}

}  // namespace fcmdp
