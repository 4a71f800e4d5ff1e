// Internal declarations shared by the HIP translation units of libfcmdp.
//
// Data layout in HBM (one solver):
//   grid      real    [6][Nz][Ny][Nx]         (T = double or float)
//   spectrum  complex [6][Nz][Nkx][Ny]        Nkx = Nx/2+1, ky fastest
//   particle records, in cell-sorted order:
//     pinfo   int4    [cap]                   (ix, iy, c_first, c_last)
//     pw      T       [cap][32]               x/y ES weights, M then D
//     pf      T       [cap][8]                F (3), pad, torque (3), pad
//     psi     T       [cap][2][Nz]            folded z weights, M then D,
//                                             zero outside the z window
//   torques through the kernel derivative (torque_route DERIVATIVE):
//     pdw     T       [cap][16]               phi_D' along x (7), along y (7)
//     dpsi    T       [cap][Nz]               psi_D', the folded z derivative
//   exact low-wavenumber vertical force (mixed slit channel only):
//     psi64   double  [cap][R][Nz]            folded M (and, with derivative
//                                             torques, D) z weights in FP64
//     fzlo    float   [Nz][Ny][Nx]            f_z - (float)f_z of the FP64
//                                             accumulated vertical force
//     lowk_part double2 [Nz][G][ns+1][2ns+1]  DFT of f_z over x (nx = 0..ns)
//                                             and over the 64-row group g of
//                                             y (ny = -ns..ns)
//     lowk_coef double2 [(ns+1)(2ns+1)][Nz]   its Chebyshev coefficients
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstddef>
#include <vector>

#include "../../include/fcmdp.h"

namespace fcmdp {

constexpr int kMaxNz = 64;
constexpr int kMaxStages = 24;
constexpr size_t kLdsBudget = 160 * 1024;   // LDS per workgroup on gfx950
constexpr int kWin = 7;        // ES window per axis: offsets -3..3 (w = 4, 6)

template <typename T> struct Cplx;
template <> struct Cplx<float> { using type = float2; };
template <> struct Cplx<double> { using type = double2; };
template <typename T> using cplx_t = typename Cplx<T>::type;

struct FFTPlan {
  int n = 0;                    // transform length
  int nstages = 0;
  int radix[kMaxStages] = {0};
};

// The row-owned transforms hold all butterflies of one thread for a stage in
// registers: at most wave_nbi_cap(R) butterflies of radix R per thread, so a
// stage of length N needs ceil(N / (R * threads per row)) <= cap.
__host__ __device__ constexpr int wave_nbi_cap(bool fp32, int R) {
  return (fp32 ? 24 : 12) / R < 1 ? 1
         : (fp32 ? 24 : 12) / R > 8 ? 8 : (fp32 ? 24 : 12) / R;
}

// Parameters the device kernels need (passed by value).
struct DevParams {
  int geometry;                 // 0 bottom wall, 1 slit channel
  int Nx, Ny, Nz, Nkx;
  int ncells;                   // Nx*Ny
  int ZW;                       // z-window slots per particle
  int half_w;                   // w/2 (3 for w = 6)
  // channels carried by the grid and spectrum of the current apply: 6 with
  // torques (in) or angular velocities (out), 3 for forces / velocities only
  int nch_in, nch_out;
  double Lx, Ly, H, h, alpha, eta;
  double beta_m, beta_d, inv_norm_m, inv_norm_d;
  double slip0, slipH;          // slit channel slip lengths (0 = no slip)
  double wall0[2], wallH[2];    // uniform wall velocities (x, y)
  // non-uniform wall velocities: unnormalised xy DFT of u^W, v^W at z = 0,
  // then at z = H, [4][Nkx][Ny] complex in the solver's precision (Nyquist
  // entries zero); nullptr = none
  const void* wallspec;
  // exact low-wavenumber vertical force: columns with |nx|, |ny| <= lowk_ns
  // take the FP64 Chebyshev coefficients of f_z from lowk_coef and FP64
  // correction node functions; -1 = off for this launch
  int lowk_ns;
  const double2* lowk_coef;
  // torques through the kernel derivative: route chosen at creation, and
  // for the current apply whether torques are spread (dt_torque) and
  // angular velocities interpolated (dt_omega) that way; tstar_d is the
  // truncation point of the dipole kernel's derivative
  int torque_deriv, dt_torque, dt_omega;
  double tstar_d;
};

// rows of y per workgroup of the low-wavenumber x transform
constexpr int kLowkRows = 64;
// largest low-wavenumber square half-width (four 16-column tiles of the
// x transform)
constexpr int kLowkMaxNs = 31;

}  // namespace fcmdp

struct fcmdp_solver {
  fcmdp_params p;
  fcmdp::DevParams dp;
  bool mixed = false;
  int device = 0;
  int64_t cap = 0;
  double norm_m = 0, norm_d = 0;
  int key_passes = 0;
  int nblk_cap = 0;

  // device buffers: every workspace buffer below is carved from `arena`,
  // every table from `tables` (one stream-ordered allocation each)
  void* arena = nullptr;
  void* tables = nullptr;
  void* grid = nullptr;
  void* spec = nullptr;
  uint32_t* keyA = nullptr;
  uint32_t* keyB = nullptr;
  int* valA = nullptr;
  int* valB = nullptr;
  uint32_t* hist = nullptr;
  int* cell_start = nullptr;
  int4* pinfo = nullptr;
  void* pw = nullptr;
  void* pf = nullptr;
  void* psi = nullptr;
  int* band = nullptr;          // [2]: first and last z-node touched
  // exact low-wavenumber vertical force (layouts above); lowk_ns = 0: off
  int lowk_ns = 0;
  bool no_lowk = false;         // variant switch (tests, measurement)
  double* psi64 = nullptr;
  void* pdw = nullptr;          // derivative-route records (layouts above)
  void* dpsi = nullptr;
  float* fzlo = nullptr;
  double2* lowk_part = nullptr;
  double2* lowk_coef = nullptr;
  double2* lowk_ex = nullptr;   // e^{-2 pi i nx a / Nx}, [Nx][ns+1]
  double2* lowk_ey = nullptr;   // e^{-2 pi i m / Ny}, [Ny]
  void* wallspec = nullptr;     // see DevParams::wallspec; kept once set
  unsigned int* nbad = nullptr;

  // tables (device)
  double* zc = nullptr;         // node heights [Nz]
  void* quad = nullptr;         // h^2 * Clenshaw-Curtis weights [Nz] (T)
  double* dct_f = nullptr;      // forward Chebyshev transform, [c][n]
  double* dct_i = nullptr;      // inverse, T_n(s_c), [c][n]
  float* dct_f32 = nullptr;     // float copies for the MFMA transforms
  float* dct_i32 = nullptr;
  double* dftc = nullptr;       // cos/sin tables of the small prime DFTs
  void* tw_x = nullptr;         // e^{-2 pi i m/(Nx/2)}, m < Nx/2 (complex T)
  void* tw_y = nullptr;         // e^{-2 pi i m/Ny}
  void* tw_r = nullptr;         // e^{-2 pi i k/Nx}, k <= Nx/2
  fcmdp::FFTPlan plan_x, plan_y;
  int dft_off[32] = {0};        // offset of prime P's table in dftc
  // row-owned transforms (x rows of Nx/2, y rows of Ny) when every stage
  // fits the register budget with at most 256 threads per row; rows per
  // workgroup and threads per row of each pass
  fcmdp::FFTPlan wplan_x, wplan_y;
  bool wave_x = false, wave_y = false;
  int rows_x = 0, rows_y = 0, tpr_x = 0, tpr_y = 0;
  int codelet_x = -1, codelet_y = -1;   // fixed-plan kernels, -1 = none
  void* dftc_t = nullptr;       // dftc converted to T

  // use the one-thread-per-column solver even when Nz <= 32 (tests)
  bool force_generic_columns = false;
  // use the one-thread-per-particle interpolation (tests)
  bool force_simple_interp = false;
  // home-particle interpolation tiles with a staged halo instead of the
  // partial sums over aligned tiles
  bool force_halo_interp = false;
  // use the untiled gather spread (tests)
  bool force_simple_spread = false;
  // use the per-patch gather spread instead of the matrix-core spread of the
  // FP32 grid (tests), the workgroups of the latter (0: three per CU, the
  // number that fit at once) and its rows per block (0: by density)
  bool force_wave_spread = false;
  int spread_workgroups = 0;
  int spread_block_rows = 0;
  int spread_order = 0;         // 0: by row alignment, 1: strip-major, 2: strips side by side
  // use the per-lane FP64 Chebyshev transforms in the mixed path (tests)
  bool force_vector_dct = false;
  // use the workgroup-per-row-batch transforms (tests)
  bool force_generic_fft = false;
  // launch one workgroup per y row instead of the persistent row loop (tests)
  bool force_no_pipeline = false;
  int num_cu = 0;               // compute units of the device

  // Lanczos square root: Krylov basis [kmax + 1][3 n] (T) and the partial
  // sums of its reductions (double), grown on demand
  void* lz_basis = nullptr;
  size_t lz_bytes = 0;
  double* lz_red = nullptr;

  // tracing: events of applies not yet summed, 7 per apply
  bool profiling = false;
  std::vector<hipEvent_t> events;
};

namespace fcmdp {

// --- launchers implemented in the .hip translation units -----------------
// prep.hip
hipError_t launch_prep(const fcmdp_solver* s, int n, const void* pos,
                       hipStream_t st);
hipError_t launch_sort(const fcmdp_solver* s, int n, hipStream_t st);
hipError_t launch_records(const fcmdp_solver* s, int n, const void* pos,
                          const void* F, const void* T, hipStream_t st);
hipError_t launch_set_band(const fcmdp_solver* s, int lo, int hi,
                           hipStream_t st);
hipError_t launch_fill(void* ptr, size_t bytes, hipStream_t st);
// spread_interp.hip
hipError_t launch_spread(const fcmdp_solver* s, int n, void* grid, hipStream_t st);
// spread_mfma.hip: the FP32 grid's spread on the matrix cores (grids of at
// least 22 x 14 nodes)
bool spread_mfma_fits(const fcmdp_solver* s);
hipError_t launch_spread_mfma(const fcmdp_solver* s, int n, void* grid, hipStream_t st);
hipError_t launch_interp(const fcmdp_solver* s, int n, const void* grid,
                         void* U, void* Omega, hipStream_t st);
// interp_part.hip: interpolation over aligned 32 x 16 tiles with per-tile
// partial sums kept in the spectrum buffer (grids of at least 38 x 22 nodes
// and partial sums that fit there)
bool interp_part_fits(const fcmdp_solver* s, int n);
hipError_t launch_interp_part(const fcmdp_solver* s, int n, const void* grid,
                              void* U, void* Omega, hipStream_t st);
// lowk.hip: exact FP64 Chebyshev coefficients of the vertical force density
// at the low wavenumbers (from the spread's f_z and fzlo planes)
hipError_t launch_lowk(const fcmdp_solver* s, const void* grid, hipStream_t st);
// whether the apply's launches use the exact low-wavenumber vertical force
bool lowk_active(const fcmdp_solver* s);
// wall.hip: spectra of non-uniform wall velocities [nw][2][Ny][Nx] into
// s->wallspec (uses the grid, the spectrum and the band as scratch; the
// caller sets three input channels)
hipError_t launch_wall_spectrum(const fcmdp_solver* s, const void* wall,
                                hipStream_t st);
// fft.hip
hipError_t launch_fft_forward(const fcmdp_solver* s, const void* grid,
                              void* spec, hipStream_t st);
hipError_t launch_fft_inverse(const fcmdp_solver* s, void* spec, void* grid,
                              hipStream_t st);
// index of a fixed-plan kernel for length n (its plan and threads per row are
// written to plan / tpr), or -1
int fft_codelet(int n, bool fp32, FFTPlan* plan, int* tpr);
// LDS elements per row of the row-owned transforms of length n (x: Nx/2,
// with room for the Nyquist element; y: Ny) for fixed plan `codelet` (-1:
// run-time plan)
int fft_lds_row(int codelet, int n, bool x);
// columns.hip (dispatches to columns_seg.hip for Nz <= 32)
hipError_t launch_columns(const fcmdp_solver* s, const void* spec_in,
                          void* spec_out, hipStream_t st);
hipError_t launch_columns_seg(const fcmdp_solver* s, const void* spec_in,
                              void* spec_out, hipStream_t st);

// --- small device helpers ------------------------------------------------
// Workgroups are dealt to the 8 XCDs round-robin (workgroup w runs on XCD
// w mod 8), and each XCD has its own L2.  Renumber them so that XCD x works
// through one contiguous range of tiles, in order: neighbouring tiles, which
// share halo data, then meet in the same L2 at about the same time.
__device__ inline int xcd_tile(int w, int ntiles) {
  constexpr int kXcd = 8;
  const int x = w % kXcd, local = w / kXcd;
  const int per = ntiles / kXcd, extra = ntiles % kXcd;
  return x < extra ? x * (per + 1) + local
                   : extra * (per + 1) + (x - extra) * per + local;
}

__host__ __device__ inline int wrap_index(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// z-node window [cA, cB] of a particle at height z: exactly the Chebyshev
// nodes with |z_c - z| <= alpha (the support of the envelope; the wall images
// only reach nodes inside this range).  An analytic first guess from the
// node formula is corrected against the node table with the same double
// comparison the envelope uses.  cB < cA means no node (cannot happen for
// particles inside the domain).
__device__ inline void z_window(const DevParams& dp, const double* zc,
                                double z, int* cA, int* cB) {
  const double N1 = dp.Nz - 1;
  const double zhi = fmin(dp.H, z + dp.alpha);
  const double sh = fmin(1.0, fmax(-1.0, 2.0 * zhi / dp.H - 1.0));
  int a = (int)ceil(N1 / M_PI * acos(sh));
  a = a < 0 ? 0 : (a > dp.Nz - 1 ? dp.Nz - 1 : a);
  while (a > 0 && fabs(zc[a - 1] - z) <= dp.alpha) --a;
  while (a < dp.Nz - 1 && fabs(zc[a] - z) > dp.alpha && zc[a] > z) ++a;
  int b = a;
  while (b + 1 < dp.Nz && fabs(zc[b + 1] - z) <= dp.alpha) ++b;
  if (fabs(zc[a] - z) > dp.alpha) b = a - 1;   // empty
  // the host sizes ZW so that this clamp never removes a supported node
  if (b > a + dp.ZW - 1) b = a + dp.ZW - 1;
  *cA = a;
  *cB = b;
}

}  // namespace fcmdp
