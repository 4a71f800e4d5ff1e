// Particle preparation: domain checks and cell keys, the z-band of touched
// Chebyshev planes, a stable LSD radix sort of particles by xy cell, cell
// start offsets, and per-particle ES weight records in sorted order.
//
// The sort makes every later reduction order a function of the input alone
// (particles of one cell keep their input order), so spreading is
// deterministic without atomics.
#include "fcmdp_internal.h"
#include "es.h"

namespace fcmdp {

// ----------------------------------------------------------------------------
// prep: keys, band, domain errors
// ----------------------------------------------------------------------------
template <typename Tin>
__global__ void __launch_bounds__(256)
k_prep(DevParams dp, int n, const Tin* __restrict__ pos,
       const double* __restrict__ zc, uint32_t* __restrict__ keys,
       int* __restrict__ band, unsigned int* __restrict__ nbad) {
  __shared__ int s_lo, s_hi, s_bad;
  if (threadIdx.x == 0) {
    s_lo = dp.Nz;
    s_hi = -1;
    s_bad = 0;
  }
  __syncthreads();
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) {
    const double x = (double)pos[3 * (size_t)j + 0];
    const double y = (double)pos[3 * (size_t)j + 1];
    const double z = (double)pos[3 * (size_t)j + 2];
    bool ok = isfinite(x) && isfinite(y) && isfinite(z) && z >= 0.0;
    if (ok) ok = dp.geometry == 0 ? (z + dp.alpha <= dp.H) : (z <= dp.H);
    if (!ok) {
      keys[j] = (uint32_t)dp.ncells;
      atomicAdd(&s_bad, 1);
    } else {
      int ix, iy;
      double fx, fy;
      cell_of(wrap_coord(x, dp.Lx), dp.h, dp.Nx, &ix, &fx);
      cell_of(wrap_coord(y, dp.Ly), dp.h, dp.Ny, &iy, &fy);
      keys[j] = (uint32_t)(iy * dp.Nx + ix);
      int cA, cB;
      z_window(dp, zc, z, &cA, &cB);
      if (cB >= cA) {
        atomicMin(&s_lo, cA);
        atomicMax(&s_hi, cB);
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    // the band only widens, so a workgroup whose planes are already inside
    // it skips the (contended) atomics
    if (s_hi >= 0) {
      const int glo = __atomic_load_n(&band[0], __ATOMIC_RELAXED);
      const int ghi = __atomic_load_n(&band[1], __ATOMIC_RELAXED);
      if (s_lo < glo) atomicMin(&band[0], s_lo);
      if (s_hi > ghi) atomicMax(&band[1], s_hi);
    }
    if (s_bad) atomicAdd(nbad, (unsigned)s_bad);
  }
}

__global__ void k_init_band(int* band, unsigned int* nbad, int lo, int hi,
                            int reset_bad) {
  band[0] = lo;
  band[1] = hi;
  if (reset_bad) *nbad = 0u;
}

hipError_t launch_prep(const fcmdp_solver* s, int n, const void* pos,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_init_band, dim3(1), dim3(1), 0, st, s->band, s->nbad,
                     s->dp.Nz, -1, 1);
  if (n == 0) return hipGetLastError();
  dim3 grid((n + 255) / 256);
  if (s->mixed)
    hipLaunchKernelGGL(k_prep<float>, grid, dim3(256), 0, st, s->dp, n,
                       (const float*)pos, s->zc, s->keyA, s->band, s->nbad);
  else
    hipLaunchKernelGGL(k_prep<double>, grid, dim3(256), 0, st, s->dp, n,
                       (const double*)pos, s->zc, s->keyA, s->band, s->nbad);
  return hipGetLastError();
}

hipError_t launch_set_band(const fcmdp_solver* s, int lo, int hi,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_init_band, dim3(1), dim3(1), 0, st, s->band, s->nbad,
                     lo, hi, 0);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// zero fill (a kernel rather than a memset so that it is safe inside
// captured graphs)
// ----------------------------------------------------------------------------
__global__ void k_fill_zero(uint4* p, size_t n16, unsigned char* tail,
                            size_t ntail) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
  if (blockIdx.x == 0 && threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

hipError_t launch_fill(void* ptr, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  const size_t n16 = bytes / 16;
  const size_t ntail = bytes - n16 * 16;
  size_t blocks = (n16 + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, st,
                     (uint4*)ptr, n16, (unsigned char*)ptr + n16 * 16, ntail);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Stable LSD radix sort, 8-bit digits.  One block sorts 2048 consecutive
// items per pass: 4 waves x 8 rounds x 64 lanes.  Stable ranks inside a
// 64-item chunk come from eight ballots (lanes with an equal digit), chunk
// counts are prefix-summed per digit in LDS, and block offsets come from a
// digit-major exclusive scan of all block histograms.
// ----------------------------------------------------------------------------
constexpr int kSortThreads = 256;
constexpr int kSortItems = 2048;
constexpr int kSortChunks = kSortItems / 64;   // 32

__global__ void __launch_bounds__(kSortThreads)
k_radix_hist(int n, const uint32_t* __restrict__ keys, int shift, int nblk,
             uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int base = blockIdx.x * kSortItems;
  for (int i = threadIdx.x; i < kSortItems; i += kSortThreads) {
    const int g = base + i;
    if (g < n) atomicAdd(&h[(keys[g] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

__global__ void __launch_bounds__(kSortThreads)
k_radix_scatter(int n, const uint32_t* __restrict__ kin,
                const int* __restrict__ vin, uint32_t* __restrict__ kout,
                int* __restrict__ vout, int shift, int nblk,
                const uint32_t* __restrict__ offs, int first_pass) {
  __shared__ uint32_t cnt[kSortChunks][256];
  __shared__ uint32_t boff[256];
  const int t = threadIdx.x;
  for (int i = t; i < kSortChunks * 256; i += kSortThreads)
    (&cnt[0][0])[i] = 0u;
  boff[t] = offs[t * nblk + blockIdx.x];
  __syncthreads();

  const int lane = t & 63;
  const int wave = t >> 6;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint32_t key[8];
  int val[8];
  int dig[8];
  int rank[8];
  const int base = blockIdx.x * kSortItems;
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int q = wave * 8 + r;
    const int g = base + q * 64 + lane;
    const bool active = g < n;
    uint32_t k = active ? kin[g] : 0u;
    int v = active ? (first_pass ? g : vin[g]) : 0;
    const int d = (int)((k >> shift) & 255u);
    uint64_t mask = __ballot(active);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t bal = __ballot(((d >> b) & 1) != 0);
      mask &= ((d >> b) & 1) ? bal : ~bal;
    }
    key[r] = k;
    val[r] = v;
    dig[r] = active ? d : -1;
    rank[r] = __popcll(mask & lt_mask);
    if (active && (mask & lt_mask) == 0ull)   // lowest lane of this digit
      cnt[q][d] = (uint32_t)__popcll(mask);
  }
  __syncthreads();
  {  // per digit: exclusive prefix over chunks
    uint32_t run = 0;
    for (int q = 0; q < kSortChunks; ++q) {
      const uint32_t c = cnt[q][t];
      cnt[q][t] = run;
      run += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    if (dig[r] < 0) continue;
    const int q = wave * 8 + r;
    const uint32_t dst = boff[dig[r]] + cnt[q][dig[r]] + (uint32_t)rank[r];
    kout[dst] = key[r];
    vout[dst] = val[r];
  }
}

// Digit-major exclusive scan of the block histograms in two launches:
// (1) block d scans the nblk counts of digit d and records the digit total;
// (2) block d adds the totals of all smaller digits.
__global__ void __launch_bounds__(256)
k_scan_digit(uint32_t* __restrict__ hist, int nblk, uint32_t* __restrict__ tot) {
  __shared__ uint32_t part[256];
  uint32_t* a = hist + (size_t)blockIdx.x * nblk;
  const int t = threadIdx.x;
  uint32_t carry = 0;
  for (int base = 0; base < nblk; base += 256) {
    const int i = base + t;
    const uint32_t v = i < nblk ? a[i] : 0u;
    part[t] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const uint32_t u = t >= off ? part[t - off] : 0u;
      __syncthreads();
      part[t] += u;
      __syncthreads();
    }
    if (i < nblk) a[i] = carry + part[t] - v;
    carry += part[255];
    __syncthreads();
  }
  if (t == 0) tot[blockIdx.x] = carry;
}

__global__ void __launch_bounds__(256)
k_scan_add(uint32_t* __restrict__ hist, int nblk, const uint32_t* __restrict__ tot) {
  __shared__ uint32_t off;
  if (threadIdx.x == 0) {
    uint32_t s = 0;
    for (int d = 0; d < (int)blockIdx.x; ++d) s += tot[d];
    off = s;
  }
  __syncthreads();
  uint32_t* a = hist + (size_t)blockIdx.x * nblk;
  for (int i = threadIdx.x; i < nblk; i += 256) a[i] += off;
}

// cell_start[c] = first sorted position with key >= c, for c = 0..ncells
__global__ void k_cell_start(int n, int ncells, const uint32_t* __restrict__ keys,
                             int* __restrict__ cell_start) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c > ncells) return;
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (keys[mid] < (uint32_t)c) lo = mid + 1; else hi = mid;
  }
  cell_start[c] = lo;
}

hipError_t launch_sort(const fcmdp_solver* s, int n, hipStream_t st) {
  const int ncells = s->dp.ncells;
  if (n > 0) {
    const int nblk = (n + kSortItems - 1) / kSortItems;
    uint32_t* kin = s->keyA;
    uint32_t* kout = s->keyB;
    int* vin = s->valA;
    int* vout = s->valB;
    for (int pass = 0; pass < s->key_passes; ++pass) {
      const int shift = 8 * pass;
      hipLaunchKernelGGL(k_radix_hist, dim3(nblk), dim3(kSortThreads), 0, st,
                         n, kin, shift, nblk, s->hist);
      hipLaunchKernelGGL(k_scan_digit, dim3(256), dim3(256), 0, st, s->hist,
                         nblk, s->hist + 256 * (size_t)s->nblk_cap);
      hipLaunchKernelGGL(k_scan_add, dim3(256), dim3(256), 0, st, s->hist,
                         nblk, s->hist + 256 * (size_t)s->nblk_cap);
      hipLaunchKernelGGL(k_radix_scatter, dim3(nblk), dim3(kSortThreads), 0,
                         st, n, kin, vin, kout, vout, shift, nblk, s->hist,
                         pass == 0 ? 1 : 0);
      uint32_t* tk = kin; kin = kout; kout = tk;
      int* tv = vin; vin = vout; vout = tv;
    }
    // the result lives in keyA/valA when the pass count is even
    if (kin != s->keyA) {
      hipMemcpyAsync(s->keyA, kin, sizeof(uint32_t) * n,
                     hipMemcpyDeviceToDevice, st);
      hipMemcpyAsync(s->valA, vin, sizeof(int) * n, hipMemcpyDeviceToDevice,
                     st);
    }
  }
  hipLaunchKernelGGL(k_cell_start, dim3((ncells + 1 + 255) / 256), dim3(256),
                     0, st, n, ncells, s->keyA, s->cell_start);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// per-particle records in sorted order
// ----------------------------------------------------------------------------
// Four lanes build the records of one sorted particle and write each as
// whole 16-byte vectors (no LDS staging, so occupancy is limited by registers
// only and the scattered reads of the unsorted inputs overlap across many
// wavefronts).  The folded z weights are stored densely over all Nz nodes
// (zero outside the particle's window), so readers index them by node
// without window arithmetic.
__device__ __forceinline__ void store4(float* p, float a, float b, float c, float d) {
  *reinterpret_cast<float4*>(p) = make_float4(a, b, c, d);
}
__device__ __forceinline__ void store4(double* p, double a, double b, double c,
                                       double d) {
  reinterpret_cast<double2*>(p)[0] = make_double2(a, b);
  reinterpret_cast<double2*>(p)[1] = make_double2(c, d);
}

template <typename Tin, typename T>
__global__ void __launch_bounds__(256)
k_records(DevParams dp, int n, const uint32_t* __restrict__ skeys,
          const int* __restrict__ perm, const Tin* __restrict__ pos,
          const Tin* __restrict__ F, const Tin* __restrict__ Tq,
          const double* __restrict__ zc, int4* __restrict__ pinfo,
          T* __restrict__ pw, T* __restrict__ pf, T* __restrict__ psi,
          double* __restrict__ psi64, T* __restrict__ pdw, T* __restrict__ dpsi) {
  // four lanes per particle (its quad): lane q writes x/y weight part q,
  // the z weights of the node groups q, q + 4, ... (four nodes each) and
  // its share of the other records, so that the kernel evaluations of one
  // particle run in four independent chains
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = gid >> 2, q = gid & 3;
  if (i >= n) return;
  const int Nz = dp.Nz;
  // FP64 z weights: the monopole's, and with torques spread through the
  // kernel derivative also the dipole's (the spread's FP64 vertical force
  // then carries their torque part)
  const int rows64 = dp.dt_torque ? 2 : 1;
  T* w = pw + (size_t)i * 32;
  T* f = pf + (size_t)i * 8;
  T* ps = psi + (size_t)i * 2 * Nz;
  double* ps64 = psi64 ? psi64 + (size_t)i * rows64 * Nz : nullptr;
  T* dw = pdw ? pdw + (size_t)i * 16 : nullptr;
  T* dps = dpsi ? dpsi + (size_t)i * Nz : nullptr;
  if (skeys[i] >= (uint32_t)dp.ncells) {
    // outside the domain: zero records (never read by the grid kernels)
    for (int e = 8 * q; e < 8 * q + 8; e += 4) store4(w + e, T(0), T(0), T(0), T(0));
    if (q < 2) store4(f + 4 * q, T(0), T(0), T(0), T(0));
    for (int e = q; e < 2 * Nz; e += 4) ps[e] = T(0);
    if (ps64)
      for (int e = q; e < rows64 * Nz; e += 4) ps64[e] = 0.0;
    if (dw)
      for (int e = q; e < 16; e += 4) dw[e] = T(0);
    if (dps)
      for (int e = q; e < Nz; e += 4) dps[e] = T(0);
    return;
  }
  const int j = perm[i];
  const double x = wrap_coord((double)pos[3 * (size_t)j + 0], dp.Lx);
  const double y = wrap_coord((double)pos[3 * (size_t)j + 1], dp.Ly);
  const double z = (double)pos[3 * (size_t)j + 2];
  int ix, iy;
  double fx, fy;
  cell_of(x, dp.h, dp.Nx, &ix, &fx);
  cell_of(y, dp.h, dp.Ny, &iy, &fy);
  int cA, cB;
  z_window(dp, zc, z, &cA, &cB);
  if (q == 0) pinfo[i] = make_int4(ix, iy, cA, cB);
  if (q < 2) {
    // forces (q = 0) and torques (q = 1), padded to four
    const Tin* src = q == 0 ? F : Tq;
    T a = T(0), b = T(0), c = T(0);
    if (src) {
      a = (T)src[3 * (size_t)j + 0];
      b = (T)src[3 * (size_t)j + 1];
      c = (T)src[3 * (size_t)j + 2];
    }
    store4(f + 4 * q, a, b, c, T(0));
  }
  // x or y weights of the M or D kernel (part q), 7 (eighth slot zero)
  {
    const double off = q & 1 ? fy : fx;
    const double beta = q < 2 ? dp.beta_m : dp.beta_d;
    const double inv = q < 2 ? dp.inv_norm_m : dp.inv_norm_d;
    T v[8];
#pragma unroll
    for (int d = 0; d < kWin; ++d)
      v[d] = es_eval<T>(((double)(d - 3) - off) * dp.h, dp.alpha, beta, inv);
    v[7] = T(0);
    store4(w + 8 * q, v[0], v[1], v[2], v[3]);
    store4(w + 8 * q + 4, v[4], v[5], v[6], v[7]);
  }
  // derivative of the dipole kernel along x (q = 0) and y (q = 1), truncated
  if (dw && q < 2) {
    const double off = q ? fy : fx;
    T v[8];
#pragma unroll
    for (int d = 0; d < kWin; ++d)
      v[d] = es_deval<T>(((double)(d - 3) - off) * dp.h, dp.alpha, dp.beta_d,
                         dp.inv_norm_d, dp.tstar_d);
    v[7] = T(0);
    store4(dw + 8 * q, v[0], v[1], v[2], v[3]);
    store4(dw + 8 * q + 4, v[4], v[5], v[6], v[7]);
  }
  // folded z weights
  const double zim_top = 2.0 * dp.H - z;
  auto zw = [&](int c, T& pm, T& pd) {
    pm = T(0);
    pd = T(0);
    if (c < cA || c > cB) return;
    const double zcv = zc[c];
    pm = es_eval<T>(zcv - z, dp.alpha, dp.beta_m, dp.inv_norm_m) -
         es_eval<T>(zcv + z, dp.alpha, dp.beta_m, dp.inv_norm_m);
    pd = es_eval<T>(zcv - z, dp.alpha, dp.beta_d, dp.inv_norm_d) -
         es_eval<T>(zcv + z, dp.alpha, dp.beta_d, dp.inv_norm_d);
    if (dp.geometry == 1) {
      pm -= es_eval<T>(zcv - zim_top, dp.alpha, dp.beta_m, dp.inv_norm_m);
      pd -= es_eval<T>(zcv - zim_top, dp.alpha, dp.beta_d, dp.inv_norm_d);
    }
  };
  if (Nz % 4 == 0) {
    // node groups of four: groups q, q + 4, ... of this lane
    for (int c = 4 * q; c < Nz; c += 16) {
      T pm[4], pd[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) zw(c + e, pm[e], pd[e]);
      store4(ps + c, pm[0], pm[1], pm[2], pm[3]);
      store4(ps + Nz + c, pd[0], pd[1], pd[2], pd[3]);
    }
  } else {
    for (int c = q; c < Nz; c += 4) zw(c, ps[c], ps[Nz + c]);
  }
  // the monopole z weights once more in FP64 (the exact low-wavenumber
  // vertical force of the mixed slit channel)
  if (ps64) {
    for (int row = 0; row < rows64; ++row) {
      const double beta = row ? dp.beta_d : dp.beta_m;
      const double inv = row ? dp.inv_norm_d : dp.inv_norm_m;
      auto p64 = [&](int c) {
        if (c < cA || c > cB) return 0.0;
        const double zcv = zc[c];
        double pm = es_eval<double>(zcv - z, dp.alpha, beta, inv) -
                    es_eval<double>(zcv + z, dp.alpha, beta, inv);
        if (dp.geometry == 1) pm -= es_eval<double>(zcv - zim_top, dp.alpha, beta, inv);
        return pm;
      };
      double* dst = ps64 + (size_t)row * Nz;
      if (Nz % 2 == 0) {
        // 16-byte stores (an even Nz keeps every row 16-byte aligned); node
        // pairs q, q + 4, ... of this lane
        double2* r2 = reinterpret_cast<double2*>(dst);
        for (int c = 2 * q; c < Nz; c += 8) r2[c / 2] = make_double2(p64(c), p64(c + 1));
      } else {
        for (int c = q; c < Nz; c += 4) dst[c] = p64(c);
      }
    }
  }
  // z derivative of the folded dipole kernel: the direct term's derivative
  // and the mirror images' (phi'(z_c - z) - phi'(z_c + z), minus
  // phi'(z_c - (2H - z)) between two walls)
  if (dps) {
    for (int c = q; c < Nz; c += 4) {
      T d = T(0);
      if (c >= cA && c <= cB) {
        const double zcv = zc[c];
        d = es_deval<T>(zcv - z, dp.alpha, dp.beta_d, dp.inv_norm_d, dp.tstar_d) -
            es_deval<T>(zcv + z, dp.alpha, dp.beta_d, dp.inv_norm_d, dp.tstar_d);
        if (dp.geometry == 1)
          d -= es_deval<T>(zcv - zim_top, dp.alpha, dp.beta_d, dp.inv_norm_d,
                           dp.tstar_d);
      }
      dps[c] = d;
    }
  }
}

template <typename Tin, typename T>
static void records_impl(const fcmdp_solver* s, int n, const void* pos,
                         const void* F, const void* Tq, hipStream_t st) {
  hipLaunchKernelGGL((k_records<Tin, T>), dim3((4 * (size_t)n + 255) / 256), dim3(256), 0,
                     st, s->dp, n, s->keyA, s->valA, (const Tin*)pos,
                     (const Tin*)F, (const Tin*)Tq, s->zc, s->pinfo,
                     (T*)s->pw, (T*)s->pf, (T*)s->psi,
                     s->dp.lowk_ns >= 0 ? s->psi64 : nullptr,
                     (s->dp.dt_torque || s->dp.dt_omega) ? (T*)s->pdw : nullptr,
                     (s->dp.dt_torque || s->dp.dt_omega) ? (T*)s->dpsi : nullptr);
}

hipError_t launch_records(const fcmdp_solver* s, int n, const void* pos,
                          const void* F, const void* T, hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (s->mixed)
    records_impl<float, float>(s, n, pos, F, T, st);
  else
    records_impl<double, double>(s, n, pos, F, T, st);
  return hipGetLastError();
}

}  // namespace fcmdp
