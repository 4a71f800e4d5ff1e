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
#include "fcmdp_internal.h"

namespace fcmdp {

namespace {

typedef float sf4 __attribute__((ext_vector_type(4)));

// staged record: 24 pieces of 16 bytes (floats [0, 96)): [0, 32) x/y
// weights (M x, M y, D x, D y; 8 each), [32, 40) forces and torques,
// [40, 44) node base (ix, iy, as int bits), [44, 64) monopole z weights of
// the chunk, [64, 84) dipole z weights, [84, 96) unused
constexpr int kSlots = 24;
constexpr int kSRec = 4 * kSlots;
constexpr int kSZ = 20;      // planes per chunk
constexpr int kSNB = 4;      // blocks of 16 slots per kernel
constexpr int kSW = 16;      // block (and tile) width in x

__device__ __forceinline__ int lane_value(int x, int l) {
  return __builtin_amdgcn_readlane(x, l);
}

template <int BY> struct SpreadCap;            // staged particles per batch
template <> struct SpreadCap<8> { static constexpr int n = 96; };
template <> struct SpreadCap<16> { static constexpr int n = 128; };

// NCH = 6: forces and torques; 3: forces only.  A workgroup owns a block of
// 16 x BY grid columns; its four wavefronts take BY / 4 tile rows each.
template <int NCH, int BY>
__global__ void __launch_bounds__(256)
k_spread_mfma(DevParams dp, const int* __restrict__ band,
              const int* __restrict__ cell_start, const int4* __restrict__ pinfo,
              const float* __restrict__ pw, const float* __restrict__ pf,
              const float* __restrict__ psi, float* __restrict__ grid) {
  constexpr int kRows = BY + 6;            // cell rows of the block's region
  constexpr int TPW = BY / 4;              // tile rows per wavefront
  constexpr int CAP = SpreadCap<BY>::n;
  static_assert(2 * kRows <= 64, "one lane per row segment");
  __shared__ __align__(16) float rec[CAP][kSRec];
  __shared__ int pidx[CAP];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int Nx = dp.Nx, Ny = dp.Ny, Nz = dp.Nz;
  const int gx = (Nx + kSW - 1) / kSW;
  const int gy = (Ny + BY - 1) / BY;
  const int blk = xcd_tile(blockIdx.x, gx * gy);
  const int xb = (blk % gx) * kSW, yb = (blk / gx) * BY;
  const int lo = band[0], hi = band[1];
  const size_t plane = (size_t)Nx * Ny;
  const size_t chstride = plane * Nz;

  // the region: cell rows yb - 3 .. yb + BY + 2 and cells xb - 3 .. xb + 18
  // of each (the grid is at least that large), split at the periodic seam;
  // lane 2r + s holds segment s of row r: its first particle and count
  const int xs = wrap_index(xb - 3, Nx);
  const int xe0 = xs + kSW + 6 <= Nx ? xs + kSW + 6 : Nx;
  const int xe1 = xs + kSW + 6 - xe0;      // cells [0, xe1) after the seam
  int sstart = 0, scnt = 0;
  if (lane < 2 * kRows) {
    const int r = lane >> 1, sg = lane & 1;
    const int row = wrap_index(yb - 3 + r, Ny) * Nx;
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
  const int soff = incl - scnt;            // staged-list index of the segment
  const int total = lane_value(incl, 63);
  // tile row t draws on region rows t .. t + 6: one contiguous slice
  auto row_start = [&](int r) { return r < kRows ? lane_value(soff, 2 * r) : total; };

  // operand roles: A column j of the tile row, B / D slot j
  const int g = lane >> 4, j = lane & 15;
  const int a = xb + j;
  const bool inside = a < Nx;
  const bool slot = j < 15;
  const int ch = j % 3, zg = slot ? j / 3 : 0;
  const int xo = xb + 4 * g;               // D: x columns xo .. xo + 3
  const bool vec = (Nz & 3) == 0;          // 16-byte aligned z-weight rows
  const bool vst = (Nx & 3) == 0;          // 16-byte aligned grid rows
  const int nbatch = (total + CAP - 1) / CAP;

  // stage particles [base, base + cnt) of the region's list for chunk c0
  auto stage = [&](int c0, int base, int cnt) {
    __syncthreads();                       // the previous batch is read
    // staged-list index -> particle
    if (wv == 0 && lane < 2 * kRows) {
      const int k0 = base - soff > 0 ? base - soff : 0;
      const int k1 = base + cnt - soff < scnt ? base + cnt - soff : scnt;
      for (int k = k0; k < k1; ++k) pidx[soff + k - base] = sstart + k;
    }
    __syncthreads();
    // records: piece e of the batch (particle e / 24, piece e % 24) is one
    // 16-byte load straight from global memory into LDS at byte 16 e, so
    // every load of the batch is in flight at once; consecutive lanes read
    // consecutive pieces of a particle.  Pieces: x/y weights (8), forces
    // and torques (2), node base (1), z weights of the chunk (5 monopole,
    // 5 dipole), unused (3).
    const int nel = cnt * kSlots;
    for (int e0 = wv * 64; e0 < nel; e0 += 256) {
      const int e = e0 + lane;
      const int idx = e / kSlots, part = e - idx * kSlots;
      const int p = pidx[e < nel ? idx : 0];
      const float* src;
      bool on;
      if (part < 8) {
        src = pw + (size_t)p * 32 + 4 * part;
        on = NCH == 6 || part < 4;
      } else if (part < 10) {
        src = pf + (size_t)p * 8 + 4 * (part - 8);
        on = NCH == 6 || part == 8;
      } else if (part == 10) {
        src = reinterpret_cast<const float*>(pinfo + p);
        on = true;
      } else {
        const int u = part - 11, h = u >= 5 ? 1 : 0, uu = u - 5 * h;
        const int z = c0 + 4 * uu;
        // planes past Nz read a clamped address (never stored)
        src = psi + (size_t)p * 2 * Nz + h * Nz + (z < Nz ? z : Nz - 4);
        on = vec && part < 21 && (NCH == 6 || h == 0);
      }
      if (on && e < nel)
        __builtin_amdgcn_global_load_lds(
            src, (__attribute__((address_space(3))) void*)(&rec[0][0] + 4 * e0), 16, 0, 0);
    }
    if (!vec) {
      // z-weight rows not 16-byte aligned: one float per thread and load
      constexpr int kZ = NCH == 6 ? 2 * kSZ : kSZ;
      for (int e = tid; e < cnt * kZ; e += 256) {
        const int idx = e / kZ, sl = e - idx * kZ;
        const int h = sl >= kSZ ? 1 : 0, z = c0 + sl - kSZ * h;
        const int p = pidx[idx];
        rec[idx][44 + sl] = psi[(size_t)p * 2 * Nz + h * Nz + (z < Nz ? z : Nz - 1)];
      }
    }
    // the direct loads write LDS behind the compiler's back: wait for them
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
  };

  for (int c0 = vec ? (lo & ~3) : lo; c0 <= hi; c0 += kSZ) {
    // one batch (the usual case): staged once for all tile rows; dense
    // regions: every batch again for each tile row
    if (nbatch <= 1) stage(c0, 0, total);
    for (int tt = 0; tt < TPW; ++tt) {
      const int t = wv * TPW + tt;
      const int y = yb + t;
      sf4 acc[2][kSNB];
#pragma unroll
      for (int pt = 0; pt < 2; ++pt)
#pragma unroll
        for (int k = 0; k < kSNB; ++k) acc[pt][k] = sf4{0.f, 0.f, 0.f, 0.f};
      for (int bt = 0; bt < nbatch; ++bt) {
        const int base = bt * CAP;
        const int cnt = total - base < CAP ? total - base : CAP;
        if (nbatch > 1) stage(c0, base, cnt);
        if (y >= Ny) continue;
        // this tile row's particles within the batch
        int s0 = row_start(t), s1 = row_start(t + 7);
        s0 = s0 > base ? s0 : base;
        s1 = s1 < base + cnt ? s1 : base + cnt;
        for (int k0 = s0; k0 < s1; k0 += 4) {
          const int k = k0 + g;
          const bool have = k < s1;
          const float* rk = &rec[have ? k - base : 0][0];
          const int ix = __float_as_int(rk[40]), iy = __float_as_int(rk[41]);
          int dx = a - ix + 3;
          if (dx < 0) dx += Nx; else if (dx >= Nx) dx -= Nx;
          int dy = y - iy + 3;
          if (dy < 0) dy += Ny; else if (dy >= Ny) dy -= Ny;
          const bool ok = have && inside && (unsigned)dx <= 6u && (unsigned)dy <= 6u;
          const int dxs = ok ? dx : 0, dys = ok ? dy : 0;
          const bool bok = have && slot;
#pragma unroll
          for (int pt = 0; pt < (NCH == 6 ? 2 : 1); ++pt) {
            const float w = rk[16 * pt + dxs] * rk[16 * pt + 8 + dys];
            const float av = ok ? w : 0.f;
            const float f = rk[32 + 4 * pt + ch];
            const sf4 zw = *reinterpret_cast<const sf4*>(rk + 44 + kSZ * pt + 4 * zg);
#pragma unroll
            for (int bl = 0; bl < kSNB; ++bl) {
              const float bv = bok ? f * zw[bl] : 0.f;
              acc[pt][bl] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[pt][bl], 0, 0, 0);
            }
          }
        }
      }
      // every band plane of the chunk, zeros included
      if (!slot || y >= Ny || xo >= Nx) continue;
      const size_t col = (size_t)y * Nx + xo;
#pragma unroll
      for (int bl = 0; bl < kSNB; ++bl) {
        const int z = c0 + 4 * zg + bl;
        if (z < lo || z > hi) continue;
#pragma unroll
        for (int pt = 0; pt < (NCH == 6 ? 2 : 1); ++pt) {
          const sf4 v = acc[pt][bl];
          float* dst = grid + (size_t)(ch + 3 * pt) * chstride + z * plane + col;
          if (vst) {
            *reinterpret_cast<sf4*>(dst) = v;
          } else {
#pragma unroll
            for (int r = 0; r < 4; ++r)
              if (xo + r < Nx) dst[r] = v[r];
          }
        }
      }
    }
  }
}

template <int NCH, int BY>
void spread_mfma_impl(const fcmdp_solver* s, void* grid, hipStream_t st) {
  const int gx = (s->dp.Nx + kSW - 1) / kSW;
  const int gy = (s->dp.Ny + BY - 1) / BY;
  hipLaunchKernelGGL((k_spread_mfma<NCH, BY>), dim3(gx * gy), dim3(256), 0, st,
                     s->dp, s->band, s->cell_start, s->pinfo,
                     (const float*)s->pw, (const float*)s->pf,
                     (const float*)s->psi, (float*)grid);
}

}  // namespace

bool spread_mfma_fits(const fcmdp_solver* s) {
  // the block's region (22 cells wide, BY + 6 rows) must not wrap onto
  // itself
  const int by = s->spread_block_rows;
  return s->dp.Nx >= kSW + 6 && s->dp.Ny >= by + 6;
}

hipError_t launch_spread_mfma(const fcmdp_solver* s, void* grid, hipStream_t st) {
  const bool dip = s->dp.nch_in == 6;
  if (s->spread_block_rows == 16)
    dip ? spread_mfma_impl<6, 16>(s, grid, st) : spread_mfma_impl<3, 16>(s, grid, st);
  else
    dip ? spread_mfma_impl<6, 8>(s, grid, st) : spread_mfma_impl<3, 8>(s, grid, st);
  return hipGetLastError();
}

}  // namespace fcmdp
