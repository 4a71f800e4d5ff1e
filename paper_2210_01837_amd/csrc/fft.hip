// xy Fourier transforms (step 2 and step 7 of Sec. 3.4, the periodic part of
// the paper's 3D FFT), hand-written mixed-radix Stockham FFTs in LDS.
//
//  forward: x-pass  real rows (Nx) -> half spectrum (Nx/2+1), written
//           transposed so that y becomes the contiguous axis:
//              grid[p][y][x]  ->  spec[p][kx][y]
//           y-pass  complex rows of length Ny, in place (contiguous).
//  inverse: y-pass (sign +) in place, then the complex-to-real x-pass that
//           reads the transposed layout back into real rows.
//
// The real transforms use the standard packing of a length-Nx real row into
// a length-Nx/2 complex sequence z_n = x_{2n} + i x_{2n+1}, one complex FFT,
// and a split step with the twiddles e^{-2 pi i k/Nx}.  Only planes inside the
// particle band [band[0], band[1]] are transformed.  All transforms are
// unnormalised; the 1/(Nx Ny) factor is applied by the column solve.
#include "fcmdp_internal.h"

namespace fcmdp {

template <typename C> __device__ inline C cmul(C a, C b) {
  C r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
template <typename C> __device__ inline C cadd(C a, C b) {
  C r; r.x = a.x + b.x; r.y = a.y + b.y; return r;
}
template <typename C> __device__ inline C csub(C a, C b) {
  C r; r.x = a.x - b.x; r.y = a.y - b.y; return r;
}
// multiply by (sign * i)
template <typename C, typename T> __device__ inline C cmul_si(C a, T sign) {
  C r; r.x = -sign * a.y; r.y = sign * a.x; return r;
}
template <typename C, typename T> __device__ inline C cscale(C a, T s) {
  C r; r.x = a.x * s; r.y = a.y * s; return r;
}

// ---- small DFTs: y_k = sum_q v_q e^{sign 2 pi i q k / R} --------------------
template <typename T, typename C>
__device__ inline void dft2(C* v) {
  const C a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <typename T, typename C>
__device__ inline void dft4(C* v, T sign) {
  const C s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
  const C s13 = cadd(v[1], v[3]), d13 = cmul_si<C, T>(csub(v[1], v[3]), sign);
  v[0] = cadd(s02, s13);
  v[2] = csub(s02, s13);
  v[1] = cadd(d02, d13);
  v[3] = csub(d02, d13);
}

template <typename T, typename C>
__device__ inline void dft8(C* v, T sign) {
  C e[4] = {v[0], v[2], v[4], v[6]};
  C o[4] = {v[1], v[3], v[5], v[7]};
  dft4<T, C>(e, sign);
  dft4<T, C>(o, sign);
  const T r = T(0.70710678118654752440084436210484903928);
  C w1; w1.x = r; w1.y = sign * r;
  C w3; w3.x = -r; w3.y = sign * r;
  const C t0 = o[0];
  const C t1 = cmul(o[1], w1);
  const C t2 = cmul_si<C, T>(o[2], sign);
  const C t3 = cmul(o[3], w3);
  v[0] = cadd(e[0], t0); v[4] = csub(e[0], t0);
  v[1] = cadd(e[1], t1); v[5] = csub(e[1], t1);
  v[2] = cadd(e[2], t2); v[6] = csub(e[2], t2);
  v[3] = cadd(e[3], t3); v[7] = csub(e[3], t3);
}

// radix 16 as two radix-8 halves (even / odd inputs) and one twiddled
// radix-2 combination
template <typename T, typename C>
__device__ inline void dft16(C* v, T sign) {
  C e[8], o[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) { e[m] = v[2 * m]; o[m] = v[2 * m + 1]; }
  dft8<T, C>(e, sign);
  dft8<T, C>(o, sign);
  // cos and sin of pi k / 8, k = 0..7
  const T c[8] = {T(1), T(0.92387953251128675613), T(0.70710678118654752440),
                  T(0.38268343236508977173), T(0), T(-0.38268343236508977173),
                  T(-0.70710678118654752440), T(-0.92387953251128675613)};
  const T sn[8] = {T(0), T(0.38268343236508977173), T(0.70710678118654752440),
                   T(0.92387953251128675613), T(1), T(0.92387953251128675613),
                   T(0.70710678118654752440), T(0.38268343236508977173)};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    C w; w.x = c[k]; w.y = sign * sn[k];
    const C t = cmul(o[k], w);
    v[k] = cadd(e[k], t);
    v[k + 8] = csub(e[k], t);
  }
}

// odd prime P: pair terms j and P-j; cs[2m], cs[2m+1] = cos, sin(2 pi m/P)
template <typename T, typename C, int P>
__device__ inline void dft_prime(C* v, const T* cs, T sign) {
  constexpr int Hh = (P - 1) / 2;
  C a[Hh], b[Hh];
  C y0 = v[0];
#pragma unroll
  for (int j = 1; j <= Hh; ++j) {
    a[j - 1] = cadd(v[j], v[P - j]);
    b[j - 1] = csub(v[j], v[P - j]);
    y0 = cadd(y0, a[j - 1]);
  }
  C out[P];
  out[0] = y0;
#pragma unroll
  for (int k = 1; k <= Hh; ++k) {
    C A = v[0];
    C B; B.x = T(0); B.y = T(0);
#pragma unroll
    for (int j = 1; j <= Hh; ++j) {
      const int m = (j * k) % P;
      const T c = cs[2 * m], s = cs[2 * m + 1];
      A.x += a[j - 1].x * c; A.y += a[j - 1].y * c;
      B.x += b[j - 1].x * s; B.y += b[j - 1].y * s;
    }
    const C iB = cmul_si<C, T>(B, sign);
    out[k] = cadd(A, iB);
    out[P - k] = csub(A, iB);
  }
#pragma unroll
  for (int k = 0; k < P; ++k) v[k] = out[k];
}

// One Stockham stage over nrows transforms of length N stored row-major.
template <typename T, int R>
__device__ inline void fft_stage(const cplx_t<T>* __restrict__ src,
                                 cplx_t<T>* __restrict__ dst, int N, int Ns,
                                 int nrows, const cplx_t<T>* __restrict__ tw,
                                 const double* __restrict__ cs_d, T sign) {
  using C = cplx_t<T>;
  const int nb = N / R;
  const int twstep = N / (Ns * R);
  T cs[2 * R];
  if constexpr (R != 2 && R != 4 && R != 8) {
#pragma unroll
    for (int m = 0; m < 2 * R; ++m) cs[m] = (T)cs_d[m];
  }
  const int total = nrows * nb;
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int r = idx / nb;
    const int j = idx - r * nb;
    const int base = r * N;
    C v[R];
#pragma unroll
    for (int q = 0; q < R; ++q) v[q] = src[base + j + q * nb];
    const int k = j % Ns;
    if (Ns > 1) {
#pragma unroll
      for (int q = 1; q < R; ++q) {
        C w = tw[q * k * twstep];
        w.y *= -sign;            // tw holds e^{-i...}; sign=-1 keeps it
        v[q] = cmul(v[q], w);
      }
    }
    if constexpr (R == 2) dft2<T, C>(v);
    else if constexpr (R == 4) dft4<T, C>(v, sign);
    else if constexpr (R == 8) dft8<T, C>(v, sign);
    else dft_prime<T, C, R>(v, cs, sign);
    const int out = (j - k) * R + k;
#pragma unroll
    for (int q = 0; q < R; ++q) dst[base + out + q * Ns] = v[q];
  }
}

// In-LDS FFT of nrows rows; returns the buffer holding the result.
template <typename T>
__device__ cplx_t<T>* fft_lds(cplx_t<T>* a, cplx_t<T>* b, int N,
                              const FFTPlan& plan, int nrows,
                              const cplx_t<T>* __restrict__ tw,
                              const double* __restrict__ dftc,
                              const int* __restrict__ dft_off, T sign) {
  cplx_t<T>* src = a;
  cplx_t<T>* dst = b;
  int Ns = 1;
  for (int s = 0; s < plan.nstages; ++s) {
    const int R = plan.radix[s];
    const double* cs = dftc + dft_off[R];
    switch (R) {
      case 2: fft_stage<T, 2>(src, dst, N, Ns, nrows, tw, cs, sign); break;
      case 3: fft_stage<T, 3>(src, dst, N, Ns, nrows, tw, cs, sign); break;
      case 4: fft_stage<T, 4>(src, dst, N, Ns, nrows, tw, cs, sign); break;
      case 5: fft_stage<T, 5>(src, dst, N, Ns, nrows, tw, cs, sign); break;
      case 7: fft_stage<T, 7>(src, dst, N, Ns, nrows, tw, cs, sign); break;
      case 8: fft_stage<T, 8>(src, dst, N, Ns, nrows, tw, cs, sign); break;
      case 11: fft_stage<T, 11>(src, dst, N, Ns, nrows, tw, cs, sign); break;
      case 13: fft_stage<T, 13>(src, dst, N, Ns, nrows, tw, cs, sign); break;
      case 17: fft_stage<T, 17>(src, dst, N, Ns, nrows, tw, cs, sign); break;
      default: break;
    }
    __syncthreads();
    cplx_t<T>* t = src; src = dst; dst = t;
    Ns *= R;
  }
  return src;
}

struct DftOff { int off[32]; };

// ---- x-pass, real -> half spectrum, transposed write -------------------------
template <typename T>
__global__ void __launch_bounds__(256)
k_fft_x_r2c(DevParams dp, FFTPlan plan, const int* __restrict__ band,
            const T* __restrict__ grid, cplx_t<T>* __restrict__ spec,
            const cplx_t<T>* __restrict__ tw, const cplx_t<T>* __restrict__ rtw,
            const double* __restrict__ dftc, DftOff doff, int rows) {
  using C = cplx_t<T>;
  extern __shared__ unsigned char lds_raw[];
  C* bufA = reinterpret_cast<C*>(lds_raw);
  const int M = dp.Nx / 2;
  C* bufB = bufA + rows * M;
  const int p = blockIdx.y;
  const int c = p % dp.Nz;
  if (c < band[0] || c > band[1]) return;
  const int y0 = blockIdx.x * rows;
  const int nr = min(rows, dp.Ny - y0);
  const C* src = reinterpret_cast<const C*>(grid + ((size_t)p * dp.Ny + y0) * dp.Nx);
  for (int idx = threadIdx.x; idx < nr * M; idx += blockDim.x) bufA[idx] = src[idx];
  __syncthreads();
  C* Z = fft_lds<T>(bufA, bufB, M, plan, nr, tw, dftc, doff.off, T(-1));
  const size_t pbase = (size_t)p * dp.Nkx * dp.Ny;
  for (int idx = threadIdx.x; idx < nr * (M + 1); idx += blockDim.x) {
    const int k = idx / nr;
    const int r = idx - k * nr;
    const C zk = Z[r * M + (k == M ? 0 : k)];
    C zc = Z[r * M + (k == 0 ? 0 : M - k)];
    zc.y = -zc.y;
    const C e = cscale(cadd(zk, zc), T(0.5));
    const C d = csub(zk, zc);
    C o; o.x = T(0.5) * d.y; o.y = T(-0.5) * d.x;      // -i d / 2
    spec[pbase + (size_t)k * dp.Ny + y0 + r] = cadd(e, cmul(rtw[k], o));
  }
}

// ---- y-pass, in place, contiguous rows ------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
k_fft_y(DevParams dp, FFTPlan plan, const int* __restrict__ band,
        cplx_t<T>* __restrict__ spec, const cplx_t<T>* __restrict__ tw,
        const double* __restrict__ dftc, DftOff doff, int rows, T sign) {
  using C = cplx_t<T>;
  extern __shared__ unsigned char lds_raw[];
  C* bufA = reinterpret_cast<C*>(lds_raw);
  C* bufB = bufA + rows * dp.Ny;
  const int p = blockIdx.y;
  const int c = p % dp.Nz;
  if (c < band[0] || c > band[1]) return;
  const int k0 = blockIdx.x * rows;
  const int nr = min(rows, dp.Nkx - k0);
  C* row = spec + ((size_t)p * dp.Nkx + k0) * dp.Ny;
  for (int idx = threadIdx.x; idx < nr * dp.Ny; idx += blockDim.x) bufA[idx] = row[idx];
  __syncthreads();
  C* res = fft_lds<T>(bufA, bufB, dp.Ny, plan, nr, tw, dftc, doff.off, sign);
  for (int idx = threadIdx.x; idx < nr * dp.Ny; idx += blockDim.x) row[idx] = res[idx];
}

// ---- x-pass, half spectrum -> real, transposed read -----------------------
template <typename T>
__global__ void __launch_bounds__(256)
k_fft_x_c2r(DevParams dp, FFTPlan plan, const int* __restrict__ band,
            const cplx_t<T>* __restrict__ spec, T* __restrict__ grid,
            const cplx_t<T>* __restrict__ tw, const cplx_t<T>* __restrict__ rtw,
            const double* __restrict__ dftc, DftOff doff, int rows) {
  using C = cplx_t<T>;
  extern __shared__ unsigned char lds_raw[];
  const int M = dp.Nx / 2;
  C* bufA = reinterpret_cast<C*>(lds_raw);        // rows * M
  C* bufB = bufA + rows * M;                        // rows * (M + 1)
  const int p = blockIdx.y;
  const int c = p % dp.Nz;
  if (c < band[0] || c > band[1]) return;
  const int y0 = blockIdx.x * rows;
  const int nr = min(rows, dp.Ny - y0);
  const size_t pbase = (size_t)p * dp.Nkx * dp.Ny;
  for (int idx = threadIdx.x; idx < nr * (M + 1); idx += blockDim.x) {
    const int k = idx / nr;
    const int r = idx - k * nr;
    bufB[r * (M + 1) + k] = spec[pbase + (size_t)k * dp.Ny + y0 + r];
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < nr * M; idx += blockDim.x) {
    const int r = idx / M;
    const int k = idx - r * M;
    C xk = bufB[r * (M + 1) + k];
    C xm = bufB[r * (M + 1) + (M - k)];
    if (k == 0) { xk.y = T(0); xm.y = T(0); }
    xm.y = -xm.y;                                   // conj(X_{M-k})
    const C A = cadd(xk, xm);
    const C B = csub(xk, xm);
    C w = rtw[k];
    w.y = -w.y;                                     // e^{+2 pi i k/Nx}
    const C wb = cmul(w, B);
    C z; z.x = A.x - wb.y; z.y = A.y + wb.x;        // A + i w B
    bufA[r * M + k] = z;
  }
  __syncthreads();
  C* res = fft_lds<T>(bufA, bufB, M, plan, nr, tw, dftc, doff.off, T(1));
  C* dst = reinterpret_cast<C*>(grid + ((size_t)p * dp.Ny + y0) * dp.Nx);
  for (int idx = threadIdx.x; idx < nr * M; idx += blockDim.x) dst[idx] = res[idx];
}

// ---- row-owned in-place transforms ------------------------------------------
// TPR threads (one to four wavefronts) own one row in LDS.  A Stockham stage
// first reads every butterfly input of the thread into registers and then
// writes the outputs back in place.  Butterfly j of a stage belongs to thread
// j mod TPR, so the loop trip counts are uniform and there are no index
// divisions by the row count.  With TPR = 64 the row is private to one
// wavefront, whose LDS accesses complete in issue order, and stages need no
// workgroup barrier; with more threads per row all rows of the workgroup
// step through the (identical) stage sequence together.


__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int TPR>
__device__ __forceinline__ void row_sync() {
  if constexpr (TPR == 64) wave_sync();
  else __syncthreads();
}

// One Stockham stage of radix R on a row owned by TPR threads; each thread
// holds up to NB butterflies in registers.  Rows are stored unpadded
// (run-time plans).
template <typename T, int R, int TPR, int NB>
__device__ __forceinline__ void stage_body(cplx_t<T>* row, int N, int Ns, int t,
                                           const cplx_t<T>* __restrict__ tw,
                                           const T* __restrict__ cs, T sign) {
  using C = cplx_t<T>;
  const int nb = N / R;
  const int twstep = N / (Ns * R);
  C v[NB][R];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int j = t + TPR * i;
    if (j < nb) {
#pragma unroll
      for (int q = 0; q < R; ++q) v[i][q] = row[j + q * nb];
    }
  }
  row_sync<TPR>();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int j = t + TPR * i;
    if (j < nb) {
      C* x = v[i];
      const int k = j % Ns;
      if (Ns > 1) {
#pragma unroll
        for (int q = 1; q < R; ++q) {
          C w = tw[q * k * twstep];
          w.y *= -sign;
          x[q] = cmul(x[q], w);
        }
      }
      if constexpr (R == 2) dft2<T, C>(x);
      else if constexpr (R == 4) dft4<T, C>(x, sign);
      else if constexpr (R == 8) dft8<T, C>(x, sign);
      else if constexpr (R == 16) dft16<T, C>(x, sign);
      else dft_prime<T, C, R>(x, cs, sign);
      const int out = (j - k) * R + k;
#pragma unroll
      for (int q = 0; q < R; ++q) row[out + q * Ns] = x[q];
    }
  }
  row_sync<TPR>();
}

// Generic plans: the radix is chosen at run time.  Not inlined: with every
// radix inlined into one stage loop the register allocator keeps the union
// of all stages' live ranges.
template <typename T, int R, int TPR>
__device__ __noinline__ void wstage(cplx_t<T>* row, int N, int Ns, int t,
                                    const cplx_t<T>* __restrict__ tw,
                                    const T* __restrict__ cs, T sign) {
  stage_body<T, R, TPR, wave_nbi_cap(sizeof(T) == 4, R)>(row, N, Ns, t, tw, cs, sign);
}

template <typename T, int TPR>
__device__ __forceinline__ void row_fft(cplx_t<T>* row, int N,
                                        const FFTPlan& plan, int t,
                                        const cplx_t<T>* __restrict__ tw,
                                        const T* __restrict__ dftc,
                                        const int* dft_off, T sign) {
  int Ns = 1;
  for (int s = 0; s < plan.nstages; ++s) {
    const int R = plan.radix[s];
    const T* cs = dftc + dft_off[R];
    switch (R) {
      case 2: wstage<T, 2, TPR>(row, N, Ns, t, tw, cs, sign); break;
      case 3: wstage<T, 3, TPR>(row, N, Ns, t, tw, cs, sign); break;
      case 4: wstage<T, 4, TPR>(row, N, Ns, t, tw, cs, sign); break;
      case 5: wstage<T, 5, TPR>(row, N, Ns, t, tw, cs, sign); break;
      case 7: wstage<T, 7, TPR>(row, N, Ns, t, tw, cs, sign); break;
      case 8: wstage<T, 8, TPR>(row, N, Ns, t, tw, cs, sign); break;
      case 11: wstage<T, 11, TPR>(row, N, Ns, t, tw, cs, sign); break;
      case 13: wstage<T, 13, TPR>(row, N, Ns, t, tw, cs, sign); break;
      case 16: wstage<T, 16, TPR>(row, N, Ns, t, tw, cs, sign); break;
      case 17: wstage<T, 17, TPR>(row, N, Ns, t, tw, cs, sign); break;
      default: break;
    }
    Ns *= R;
  }
}

struct GenericRows {
  template <typename T, int TPR>
  __device__ __forceinline__ static void run(cplx_t<T>* row, int N, const FFTPlan& plan, int t,
                             const cplx_t<T>* __restrict__ tw,
                             const T* __restrict__ dftc, const DftOff& doff,
                             T sign) {
    row_fft<T, TPR>(row, N, plan, t, tw, dftc, doff.off, sign);
  }
  // LDS elements a row of n occupies
  __host__ __device__ static constexpr int span(int n) { return n; }
};

// ---- fixed plans ("codelets") ----------------------------------------------
// The stage sequence is a template argument (stage code = 16 R + NB); stages
// are inlined one after another, so registers are allocated per stage and
// nothing goes through a call stack.
//
// Between stages s and s + 1 the row is stored in LDS with the layout
//   element i at i + (i / B) * pad          (B a power of two),
// chosen per boundary at compile time.  B divides both the read stride of
// stage s + 1 (N / R_{s+1}) and the write stride of stage s (or every
// radix-R_s block of stage s lies within one B-segment), so that every
// butterfly input and output sits at a constant offset from one address per
// butterfly; the pad spreads the strided writes of stage s (lanes R_s
// elements apart for the first stage) over the LDS banks.  Before the first
// and after the last stage the row is unpadded.
struct RowLay {
  int B, pad;
};

// bank conflicts of one access of 64 lanes to 8-byte elements at the given
// element indices: 64 four-byte banks, 32 lanes per cycle
constexpr int lds_conflicts(const int* idx) {
  int cost = 0;
  for (int g = 0; g < 2; ++g) {
    int cnt[64] = {};
    int worst = 0;
    for (int l = 32 * g; l < 32 * g + 32; ++l) {
      if (idx[l] < 0) continue;
      for (int h = 0; h < 2; ++h) {
        const int b = (2 * idx[l] + h) & 63;
        if (++cnt[b] > worst) worst = cnt[b];
      }
    }
    cost += worst;
  }
  return cost;
}

constexpr int lay_at(RowLay L, int i) { return i + (i / L.B) * L.pad; }

// layout after a stage of radix R with input stride Ns (next stage reads
// with stride nbn) in a row of length N
constexpr RowLay choose_lay(int N, int R, int Ns, int nbn) {
  RowLay best{N, 0};                                // unpadded
  int best_cost = 1 << 30;
  for (int B = 1; B < N; B *= 2) {
    const bool write_lin = Ns % B == 0 || B % (Ns * R) == 0;
    const bool read_lin = nbn % B == 0;
    if (!write_lin || !read_lin) continue;
    // at most one pad element per eight, so that rows grow by 12.5% at most
    const int max_pad = B >= 8 ? B / 8 : 1;
    for (int pad = 0; pad <= max_pad; ++pad) {
      const RowLay L{B, pad};
      int w[64] = {}, r[64] = {};
      for (int t = 0; t < 64; ++t) {
        const int k = t % Ns;
        const int out = (t - k) * R + k;            // stage output, q = 0
        w[t] = t < N / R ? lay_at(L, out) : -1;
        r[t] = t < nbn ? lay_at(L, t) : -1;         // next stage input, q = 0
      }
      // conflicts first, then the smallest row
      const int cost = (lds_conflicts(w) + lds_conflicts(r)) * (1 << 20) +
                       lay_at(L, N - 1);
      if (cost < best_cost) {
        best_cost = cost;
        best = L;
      }
    }
  }
  return best;
}

template <int... Codes>
struct CodeletLayout {
  static constexpr int kStages = sizeof...(Codes);
  static constexpr int kRad[kStages] = {(Codes >> 4)...};
  static constexpr int kN = (1 * ... * (Codes >> 4));
  struct Table {
    RowLay lay[kStages + 1];                        // lay[s]: input of stage s
    int span;
    constexpr Table() : lay(), span(kN) {
      lay[0] = RowLay{kN, 0};
      int Ns = 1;
      for (int s = 0; s < kStages; ++s) {
        if (s + 1 < kStages)
          lay[s + 1] = choose_lay(kN, kRad[s], Ns, kN / kRad[s + 1]);
        else
          lay[s + 1] = RowLay{kN, 0};
        const int e = lay_at(lay[s + 1], kN - 1) + 1;
        if (e > span) span = e;
        Ns *= kRad[s];
      }
    }
  };
  static constexpr Table kTable = Table();
};

// One stage of a fixed plan: every size is a compile-time constant, inputs
// in layout LI, outputs in layout LO.
template <typename T, int R, int TPR, int NB, int N, int NS, int BI, int PI, int BO,
          int PO>
__device__ __forceinline__ void stage_fixed(cplx_t<T>* row, int t,
                                            const cplx_t<T>* __restrict__ tw,
                                            const T* __restrict__ cs, T sign) {
  using C = cplx_t<T>;
  constexpr RowLay LI{BI, PI}, LO{BO, PO};
  constexpr int nb = N / R;
  constexpr int twstep = N / (NS * R);
  static_assert(nb % BI == 0 || BI >= N, "stage input layout not linear");
  static_assert(NS % BO == 0 || BO % (NS * R) == 0 || BO >= N,
                "stage output layout not linear");
  constexpr int rstep = lay_at(LI, nb);             // offset of input q = 1
  constexpr int wstep = NS % BO == 0 ? lay_at(LO, NS) : NS;
  C v[NB][R];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int j = t + TPR * i;
    if (j < nb) {
      const int base = (int)((unsigned)j / BI) * PI + j;
#pragma unroll
      for (int q = 0; q < R; ++q) v[i][q] = row[base + q * rstep];
    }
  }
  row_sync<TPR>();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int j = t + TPR * i;
    if (j < nb) {
      C* x = v[i];
      const int k = j % NS;
      if constexpr (NS > 1) {
#pragma unroll
        for (int q = 1; q < R; ++q) {
          C w = tw[q * k * twstep];
          w.y *= -sign;
          x[q] = cmul(x[q], w);
        }
      }
      if constexpr (R == 2) dft2<T, C>(x);
      else if constexpr (R == 4) dft4<T, C>(x, sign);
      else if constexpr (R == 8) dft8<T, C>(x, sign);
      else if constexpr (R == 16) dft16<T, C>(x, sign);
      else dft_prime<T, C, R>(x, cs, sign);
      const int out = (j - k) * R + k;
      const int base = (int)((unsigned)out / BO) * PO + out;
#pragma unroll
      for (int q = 0; q < R; ++q) row[base + q * wstep] = x[q];
    }
  }
  row_sync<TPR>();
}

template <typename T, int TPR, typename Lay, int S, int NS, int Code, int... Rest>
__device__ __forceinline__ void run_codes(cplx_t<T>* row, int t,
                                          const cplx_t<T>* __restrict__ tw,
                                          const T* __restrict__ dftc,
                                          const DftOff& doff, T sign) {
  constexpr int R = Code >> 4, NB = Code & 15;
  constexpr RowLay LI = Lay::kTable.lay[S], LO = Lay::kTable.lay[S + 1];
  stage_fixed<T, R, TPR, NB, Lay::kN, NS, LI.B, LI.pad, LO.B, LO.pad>(
      row, t, tw, dftc + doff.off[R], sign);
  if constexpr (sizeof...(Rest) > 0)
    run_codes<T, TPR, Lay, S + 1, NS * R, Rest...>(row, t, tw, dftc, doff, sign);
}

template <int... Codes>
struct FixedRows {
  using Lay = CodeletLayout<Codes...>;
  static constexpr int kN = Lay::kN;                // transform length
  template <typename T, int TPR>
  __device__ __forceinline__ static void run(cplx_t<T>* row, int, const FFTPlan&, int t,
                             const cplx_t<T>* __restrict__ tw,
                             const T* __restrict__ dftc, const DftOff& doff,
                             T sign) {
    run_codes<T, TPR, Lay, 0, 1, Codes...>(row, t, tw, dftc, doff, sign);
  }
  __host__ __device__ static constexpr int span(int n) {
    return n > Lay::kTable.span ? n : Lay::kTable.span;
  }
};

// LDS row stride of the x passes (Nx/2 + 1 elements at least, odd so that the
// transposed accesses of 16 rows fall into different banks)
template <typename Run>
__host__ __device__ constexpr int x_stride(int M) {
  return Run::span(M + 1) | 1;
}

// split step of the real transform: X_k from Z_k and Z_{M-k} (w = e^{-2 pi i k/Nx})
template <typename C>
__device__ inline C r2c_post(C zk, C zm, C w) {
  using T = decltype(zk.x);
  zm.y = -zm.y;
  const C e = cscale(cadd(zk, zm), T(0.5));
  const C d = csub(zk, zm);
  C o; o.x = T(0.5) * d.y; o.y = T(-0.5) * d.x;      // -i d / 2
  return cadd(e, cmul(w, o));
}

// inverse split step: Z_k from X_k and X_{M-k} (w = e^{-2 pi i k/Nx})
template <typename C>
__device__ inline C c2r_pre(C xk, C xm, C w) {
  xm.y = -xm.y;                                   // conj(X_{M-k})
  const C A = cadd(xk, xm);
  const C B = csub(xk, xm);
  w.y = -w.y;                                     // e^{+2 pi i k/Nx}
  const C wb = cmul(w, B);
  C z; z.x = A.x - wb.y; z.y = A.y + wb.x;        // A + i w B
  return z;
}

// x-pass, real rows -> half spectrum, ROWS rows per workgroup, written
// transposed as ROWS-long runs of consecutive y.
template <typename T, int ROWS, int TPR, typename Run>
__global__ void __launch_bounds__(ROWS * TPR)
k_fftw_x_r2c(DevParams dp, FFTPlan plan, const int* __restrict__ band,
             const T* __restrict__ grid, cplx_t<T>* __restrict__ spec,
             const cplx_t<T>* __restrict__ tw, const cplx_t<T>* __restrict__ rtw,
             const T* __restrict__ dftc, DftOff doff) {
  using C = cplx_t<T>;
  extern __shared__ unsigned char lds_raw[];
  C* lds = reinterpret_cast<C*>(lds_raw);
  const int M = dp.Nx / 2;
  const int S = x_stride<Run>(M);                   // row stride in LDS
  const int p = blockIdx.y;
  const int c = p % dp.Nz;
  if (c < band[0] || c > band[1]) return;           // whole workgroup
  const int y0 = blockIdx.x * ROWS;
  const int nr = min(ROWS, dp.Ny - y0);
  const int wr = __builtin_amdgcn_readfirstlane(threadIdx.x / TPR);
  const int t = threadIdx.x % TPR;
  C* row = lds + wr * S;
  // rows past the grid edge (tail workgroup) transform a copy of row y0
  const int y = wr < nr ? y0 + wr : y0;
  const C* src = reinterpret_cast<const C*>(grid + ((size_t)p * dp.Ny + y) * dp.Nx);
#pragma unroll 4
  for (int i = t; i < M; i += TPR) row[i] = src[i];
  row_sync<TPR>();
  Run::template run<T, TPR>(row, M, plan, t, tw, dftc, doff, T(-1));
  for (int k = t; k <= M / 2; k += TPR) {
    const C zk = row[k];
    if (k == 0) {
      row[0] = r2c_post(zk, zk, rtw[0]);
      row[M] = r2c_post(zk, zk, rtw[M]);
    } else {
      const C zm = row[M - k];
      row[k] = r2c_post(zk, zm, rtw[k]);
      if (M - k != k) row[M - k] = r2c_post(zm, zk, rtw[M - k]);
    }
  }
  __syncthreads();
  const size_t pbase = (size_t)p * dp.Nkx * dp.Ny;
  if constexpr (ROWS % 2 == 0 && sizeof(T) == 4) {
    // two consecutive rows per thread: one 16-byte store (y0 and Ny even)
    for (int idx = threadIdx.x; idx < (M + 1) * (ROWS / 2); idx += ROWS * TPR) {
      const int k = idx / (ROWS / 2);
      const int r = 2 * (idx % (ROWS / 2));
      C* dst = spec + pbase + (size_t)k * dp.Ny + y0 + r;
      const C a = lds[r * S + k], b = lds[(r + 1) * S + k];
      if (r + 1 < nr && (dp.Ny & 1) == 0) {
        *reinterpret_cast<float4*>(dst) = make_float4(a.x, a.y, b.x, b.y);
      } else {
        if (r < nr) dst[0] = a;
        if (r + 1 < nr) dst[1] = b;
      }
    }
  } else {
    for (int idx = threadIdx.x; idx < (M + 1) * ROWS; idx += ROWS * TPR) {
      const int k = idx / ROWS;
      const int r = idx % ROWS;
      if (r < nr) spec[pbase + (size_t)k * dp.Ny + y0 + r] = lds[r * S + k];
    }
  }
}

// y-pass, in place on contiguous rows of length Ny.
template <typename T, int ROWS, int TPR, typename Run>
__global__ void __launch_bounds__(ROWS * TPR)
k_fftw_y(DevParams dp, FFTPlan plan, const int* __restrict__ band,
         cplx_t<T>* __restrict__ spec, const cplx_t<T>* __restrict__ tw,
         const T* __restrict__ dftc, DftOff doff, T sign) {
  using C = cplx_t<T>;
  extern __shared__ unsigned char lds_raw[];
  const int p = blockIdx.y;
  const int c = p % dp.Nz;
  if (c < band[0] || c > band[1]) return;
  const int wr = __builtin_amdgcn_readfirstlane(threadIdx.x / TPR);
  const int t = threadIdx.x % TPR;
  const int kx = blockIdx.x * ROWS + wr;
  const bool live = kx < dp.Nkx;
  if (TPR == 64 && !live) return;                   // a whole wavefront
  const int N = dp.Ny;
  C* row = reinterpret_cast<C*>(lds_raw) + wr * Run::span(N);
  C* g = spec + ((size_t)p * dp.Nkx + (live ? kx : 0)) * N;
#pragma unroll 4
  for (int i = t; i < N; i += TPR) row[i] = g[i];
  row_sync<TPR>();
  Run::template run<T, TPR>(row, N, plan, t, tw, dftc, doff, sign);
  if (live) {
#pragma unroll 4
    for (int i = t; i < N; i += TPR) g[i] = row[i];
  }
}

// y-pass as a persistent loop: workgroup g (one wavefront) transforms the
// band rows g, g + G, ... and loads the next row into registers while the
// current one is transformed in LDS, so that every wavefront keeps memory
// requests in flight through its arithmetic.  Fixed-length plans only.
template <typename T, typename Run>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 8)))
k_fftw_y_pipe(DevParams dp, FFTPlan plan, const int* __restrict__ band,
              cplx_t<T>* __restrict__ spec, const cplx_t<T>* __restrict__ tw,
              const T* __restrict__ dftc, DftOff doff, T sign, int nch) {
  using C = cplx_t<T>;
  constexpr int N = Run::kN;                        // == dp.Ny
  constexpr int PER = (N + 63) / 64;
  extern __shared__ unsigned char lds_raw[];
  C* row = reinterpret_cast<C*>(lds_raw);
  const int lo = band[0], hi = band[1];
  if (lo > hi) return;
  const int P = hi - lo + 1;
  const int total = nch * P * dp.Nkx;               // band rows
  const int t = threadIdx.x;
  int r = blockIdx.x;
  if (r >= total) return;
  // row r: kx fastest, then band plane, then channel
  auto row_ptr = [&](int rr) {
    const int kx = rr % dp.Nkx, q = rr / dp.Nkx;
    const int ch = q / P, c = lo + q - ch * P;
    return spec + ((size_t)(ch * dp.Nz + c) * dp.Nkx + kx) * N;
  };
  C pre[PER];
  {
    const C* g = row_ptr(r);
#pragma unroll
    for (int i = 0; i < PER; ++i)
      if (t + 64 * i < N) pre[i] = g[t + 64 * i];
  }
  for (; r < total; r += gridDim.x) {
    C* g = row_ptr(r);
#pragma unroll
    for (int i = 0; i < PER; ++i)
      if (t + 64 * i < N) row[t + 64 * i] = pre[i];
    const int rn = r + gridDim.x;
    if (rn < total) {
      const C* gn = row_ptr(rn);
#pragma unroll
      for (int i = 0; i < PER; ++i)
        if (t + 64 * i < N) pre[i] = gn[t + 64 * i];
    }
    wave_sync();
    // the tables and the lane index are opaque to the optimiser inside the
    // loop, so that table loads and LDS addresses are not hoisted out of it
    // (which would hold every twiddle and address of the plan in registers)
    const C* twl = tw;
    const T* csl = dftc;
    int tl = t;
    asm volatile("" : "+s"(twl), "+s"(csl), "+v"(tl));
    Run::template run<T, 64>(row, N, plan, tl, twl, csl, doff, sign);
#pragma unroll
    for (int i = 0; i < PER; ++i)
      if (t + 64 * i < N) g[t + 64 * i] = row[t + 64 * i];
    wave_sync();
  }
}

// x-pass, half spectrum -> real rows, reading ROWS-long runs of the
// transposed layout.
template <typename T, int ROWS, int TPR, typename Run>
__global__ void __launch_bounds__(ROWS * TPR)
k_fftw_x_c2r(DevParams dp, FFTPlan plan, const int* __restrict__ band,
             const cplx_t<T>* __restrict__ spec, T* __restrict__ grid,
             const cplx_t<T>* __restrict__ tw, const cplx_t<T>* __restrict__ rtw,
             const T* __restrict__ dftc, DftOff doff) {
  using C = cplx_t<T>;
  extern __shared__ unsigned char lds_raw[];
  C* lds = reinterpret_cast<C*>(lds_raw);
  const int M = dp.Nx / 2;
  const int S = x_stride<Run>(M);                   // row stride in LDS
  const int p = blockIdx.y;
  const int c = p % dp.Nz;
  if (c < band[0] || c > band[1]) return;
  const int y0 = blockIdx.x * ROWS;
  const int nr = min(ROWS, dp.Ny - y0);
  const size_t pbase = (size_t)p * dp.Nkx * dp.Ny;
  if constexpr (ROWS % 2 == 0 && sizeof(T) == 4) {
    // two consecutive rows per thread: one 16-byte load (y0 and Ny even)
    const int total = (M + 1) * (ROWS / 2);
    if (nr == ROWS && (dp.Ny & 1) == 0) {
      // whole workgroup: a thread issues all of its loads (nine cover the
      // half spectrum of 2176-point rows) before the first LDS store
      constexpr int kB = 9;
      for (int base = threadIdx.x; base < total; base += kB * ROWS * TPR) {
        float4 v[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) {
          const int idx = min(base + u * ROWS * TPR, total - 1);   // in bounds
          const int k = idx / (ROWS / 2);
          const int r = 2 * (idx % (ROWS / 2));
          v[u] = *reinterpret_cast<const float4*>(spec + pbase + (size_t)k * dp.Ny + y0 + r);
        }
#pragma unroll
        for (int u = 0; u < kB; ++u) {
          const int idx = base + u * ROWS * TPR;
          if (idx < total) {
            const int k = idx / (ROWS / 2);
            const int r = 2 * (idx % (ROWS / 2));
            lds[r * S + k] = make_float2(v[u].x, v[u].y);
            lds[(r + 1) * S + k] = make_float2(v[u].z, v[u].w);
          }
        }
      }
    } else {
      for (int idx = threadIdx.x; idx < total; idx += ROWS * TPR) {
        const int k = idx / (ROWS / 2);
        const int r = 2 * (idx % (ROWS / 2));
        const C* src = spec + pbase + (size_t)k * dp.Ny + y0;
        C a, b;
        if (r + 1 < nr && (dp.Ny & 1) == 0) {
          const float4 v = *reinterpret_cast<const float4*>(src + r);
          a.x = v.x; a.y = v.y; b.x = v.z; b.y = v.w;
        } else {
          // rows past the grid edge transform a copy of row y0
          a = src[r < nr ? r : 0];
          b = src[r + 1 < nr ? r + 1 : 0];
        }
        lds[r * S + k] = a;
        lds[(r + 1) * S + k] = b;
      }
    }
  } else {
    for (int idx = threadIdx.x; idx < (M + 1) * ROWS; idx += ROWS * TPR) {
      const int k = idx / ROWS;
      const int r = idx % ROWS;
      // rows past the grid edge transform a copy of row y0
      lds[r * S + k] = spec[pbase + (size_t)k * dp.Ny + y0 + (r < nr ? r : 0)];
    }
  }
  __syncthreads();
  const int wr = __builtin_amdgcn_readfirstlane(threadIdx.x / TPR);
  const int t = threadIdx.x % TPR;
  C* row = lds + wr * S;
  for (int k = t; k <= M / 2; k += TPR) {
    if (k == 0) {
      C x0 = row[0], xm = row[M];
      x0.y = T(0);
      xm.y = T(0);
      row[0] = c2r_pre(x0, xm, rtw[0]);
    } else {
      const C xk = row[k], xm = row[M - k];
      row[k] = c2r_pre(xk, xm, rtw[k]);
      if (M - k != k) row[M - k] = c2r_pre(xm, xk, rtw[M - k]);
    }
  }
  row_sync<TPR>();
  Run::template run<T, TPR>(row, M, plan, t, tw, dftc, doff, T(1));
  if (wr < nr) {
    C* dst = reinterpret_cast<C*>(grid + ((size_t)p * dp.Ny + y0 + wr) * dp.Nx);
#pragma unroll 4
    for (int i = t; i < M; i += TPR) dst[i] = row[i];
  }
}

template <typename T, int ROWS, int TPR, typename Run>
static void launch_wave_x(bool fwd, const fcmdp_solver* s, const void* in,
                          void* out, const DftOff& doff, hipStream_t st) {
  using C = cplx_t<T>;
  const DevParams& dp = s->dp;
  const int M = dp.Nx / 2;
  const size_t lds = (size_t)ROWS * x_stride<Run>(M) * sizeof(C);
  dim3 g((dp.Ny + ROWS - 1) / ROWS, (fwd ? dp.nch_in : dp.nch_out) * dp.Nz);
  const T* cs = (const T*)s->dftc_t;
  if (fwd)
    hipLaunchKernelGGL((k_fftw_x_r2c<T, ROWS, TPR, Run>), g, dim3(ROWS * TPR),
                       lds, st, dp, s->wplan_x, s->band, (const T*)in, (C*)out,
                       (const C*)s->tw_x, (const C*)s->tw_r, cs, doff);
  else
    hipLaunchKernelGGL((k_fftw_x_c2r<T, ROWS, TPR, Run>), g, dim3(ROWS * TPR),
                       lds, st, dp, s->wplan_x, s->band, (const C*)in, (T*)out,
                       (const C*)s->tw_x, (const C*)s->tw_r, cs, doff);
}

template <typename T, int TPR, typename Run>
static void wave_x_rows(bool fwd, const fcmdp_solver* s, const void* in,
                        void* out, const DftOff& doff, hipStream_t st) {
  // rows per workgroup, capped by 1024 threads
  const int r = s->rows_x * TPR > 1024 ? 1024 / TPR : s->rows_x;
  switch (r) {
    case 16: launch_wave_x<T, 16, 64, Run>(fwd, s, in, out, doff, st); break;
    case 12: launch_wave_x<T, 12, 64, Run>(fwd, s, in, out, doff, st); break;
    case 8: launch_wave_x<T, 8, TPR, Run>(fwd, s, in, out, doff, st); break;
    case 4: launch_wave_x<T, 4, TPR, Run>(fwd, s, in, out, doff, st); break;
    case 2: launch_wave_x<T, 2, TPR, Run>(fwd, s, in, out, doff, st); break;
    default: launch_wave_x<T, 1, TPR, Run>(fwd, s, in, out, doff, st); break;
  }
}

template <typename T, int ROWS, int TPR, typename Run>
static void launch_wave_y(const fcmdp_solver* s, void* spec, const DftOff& doff,
                          T sign, hipStream_t st) {
  using C = cplx_t<T>;
  const DevParams& dp = s->dp;
  const size_t lds = (size_t)ROWS * Run::span(dp.Ny) * sizeof(C);
  dim3 g((dp.Nkx + ROWS - 1) / ROWS, (sign < 0 ? dp.nch_in : dp.nch_out) * dp.Nz);
  hipLaunchKernelGGL((k_fftw_y<T, ROWS, TPR, Run>), g, dim3(ROWS * TPR), lds, st,
                     dp, s->wplan_y, s->band, (C*)spec, (const C*)s->tw_y,
                     (const T*)s->dftc_t, doff, sign);
}

template <typename T, int TPR, typename Run>
static void wave_y_rows(const fcmdp_solver* s, void* spec, const DftOff& doff,
                        T sign, hipStream_t st) {
  const int r = s->rows_y * TPR > 1024 ? 1024 / TPR : s->rows_y;
  switch (r) {
    case 8: launch_wave_y<T, 8, TPR, Run>(s, spec, doff, sign, st); break;
    case 4: launch_wave_y<T, 4, TPR, Run>(s, spec, doff, sign, st); break;
    case 2: launch_wave_y<T, 2, TPR, Run>(s, spec, doff, sign, st); break;
    default: launch_wave_y<T, 1, TPR, Run>(s, spec, doff, sign, st); break;
  }
}

// Persistent y-pass: as many one-wavefront workgroups as stay resident (LDS
// and registers allow eight per compute unit).
template <typename T, typename Run>
static void wave_y_pipe(const fcmdp_solver* s, void* spec, const DftOff& doff,
                        T sign, hipStream_t st) {
  using C = cplx_t<T>;
  const DevParams& dp = s->dp;
  const size_t lds = (size_t)Run::span(dp.Ny) * sizeof(C);
  const int per_cu = (int)std::min<size_t>(8, kLdsBudget / lds);
  const int g = std::max(1, s->num_cu) * std::max(1, per_cu);
  hipLaunchKernelGGL((k_fftw_y_pipe<T, Run>), dim3(g), dim3(64), lds, st, dp,
                     s->wplan_y, s->band, (C*)spec, (const C*)s->tw_y,
                     (const T*)s->dftc_t, doff, sign,
                     sign < 0 ? dp.nch_in : dp.nch_out);
}

// Codelets compiled for the transform lengths of the large workloads (single
// precision, 64 threads per row).  codelet_table[i] must agree with the
// FixedRows instance that wave_x / wave_y launch for index i.
struct CodeletDesc { int n; int tpr; int nst; int code[6]; };
static const CodeletDesc kCodelets[] = {
    {1088, 64, 3, {8 * 16 + 3, 8 * 16 + 3, 17 * 16 + 1}},           // 2176 / 2
    {2176, 64, 3, {16 * 16 + 3, 8 * 16 + 5, 17 * 16 + 2}},          // 2176
    {384, 64, 3, {16 * 16 + 1, 8 * 16 + 1, 3 * 16 + 2}},            // 768 / 2
    {768, 64, 4, {4 * 16 + 3, 8 * 16 + 2, 8 * 16 + 2, 3 * 16 + 4}},  // 768
    {1350, 64, 6, {3 * 16 + 8, 3 * 16 + 8, 3 * 16 + 8, 5 * 16 + 5,    // 2700 / 2
                   5 * 16 + 5, 2 * 16 + 11}},
    {2700, 64, 6, {3 * 16 + 15, 3 * 16 + 15, 3 * 16 + 15, 5 * 16 + 9,  // 2700
                   5 * 16 + 9, 4 * 16 + 11}},
};
using Codelet0 = FixedRows<8 * 16 + 3, 8 * 16 + 3, 17 * 16 + 1>;
using Codelet1 = FixedRows<16 * 16 + 3, 8 * 16 + 5, 17 * 16 + 2>;
using Codelet2 = FixedRows<16 * 16 + 1, 8 * 16 + 1, 3 * 16 + 2>;
using Codelet3 = FixedRows<4 * 16 + 3, 8 * 16 + 2, 8 * 16 + 2, 3 * 16 + 4>;
// (odd radices first: 2.6 -> 1.9 ms per forward transform of the
// forces-only layer against the power-of-two radix first)
using Codelet4 = FixedRows<3 * 16 + 8, 3 * 16 + 8, 3 * 16 + 8, 5 * 16 + 5,
                           5 * 16 + 5, 2 * 16 + 11>;
using Codelet5 = FixedRows<3 * 16 + 15, 3 * 16 + 15, 3 * 16 + 15, 5 * 16 + 9,
                           5 * 16 + 9, 4 * 16 + 11>;

template <typename T>
static void wave_x(bool fwd, const fcmdp_solver* s, const void* in, void* out,
                   const DftOff& doff, hipStream_t st) {
  switch (s->codelet_x) {
    case 0: wave_x_rows<T, 64, Codelet0>(fwd, s, in, out, doff, st); return;
    case 1: wave_x_rows<T, 64, Codelet1>(fwd, s, in, out, doff, st); return;
    case 2: wave_x_rows<T, 64, Codelet2>(fwd, s, in, out, doff, st); return;
    case 3: wave_x_rows<T, 64, Codelet3>(fwd, s, in, out, doff, st); return;
    case 4: wave_x_rows<T, 64, Codelet4>(fwd, s, in, out, doff, st); return;
    case 5: wave_x_rows<T, 64, Codelet5>(fwd, s, in, out, doff, st); return;
    default: break;
  }
  switch (s->tpr_x) {
    case 64: wave_x_rows<T, 64, GenericRows>(fwd, s, in, out, doff, st); break;
    case 128: wave_x_rows<T, 128, GenericRows>(fwd, s, in, out, doff, st); break;
    default: wave_x_rows<T, 256, GenericRows>(fwd, s, in, out, doff, st); break;
  }
}

template <typename T>
static void wave_y(const fcmdp_solver* s, void* spec, const DftOff& doff,
                   T sign, hipStream_t st) {
  if (!s->force_no_pipeline) {
    switch (s->codelet_y) {
      case 0: wave_y_pipe<T, Codelet0>(s, spec, doff, sign, st); return;
      case 1: wave_y_pipe<T, Codelet1>(s, spec, doff, sign, st); return;
      case 2: wave_y_pipe<T, Codelet2>(s, spec, doff, sign, st); return;
      case 3: wave_y_pipe<T, Codelet3>(s, spec, doff, sign, st); return;
      case 4: wave_y_pipe<T, Codelet4>(s, spec, doff, sign, st); return;
      case 5: wave_y_pipe<T, Codelet5>(s, spec, doff, sign, st); return;
      default: break;
    }
  }
  switch (s->codelet_y) {
    case 0: wave_y_rows<T, 64, Codelet0>(s, spec, doff, sign, st); return;
    case 1: wave_y_rows<T, 64, Codelet1>(s, spec, doff, sign, st); return;
    case 2: wave_y_rows<T, 64, Codelet2>(s, spec, doff, sign, st); return;
    case 3: wave_y_rows<T, 64, Codelet3>(s, spec, doff, sign, st); return;
    case 4: wave_y_rows<T, 64, Codelet4>(s, spec, doff, sign, st); return;
    case 5: wave_y_rows<T, 64, Codelet5>(s, spec, doff, sign, st); return;
    default: break;
  }
  switch (s->tpr_y) {
    case 64: wave_y_rows<T, 64, GenericRows>(s, spec, doff, sign, st); break;
    case 128: wave_y_rows<T, 128, GenericRows>(s, spec, doff, sign, st); break;
    default: wave_y_rows<T, 256, GenericRows>(s, spec, doff, sign, st); break;
  }
}

int fft_lds_row(int codelet, int n, bool x) {
  switch (codelet) {
    case 0: return x ? x_stride<Codelet0>(n) : Codelet0::span(n);
    case 1: return x ? x_stride<Codelet1>(n) : Codelet1::span(n);
    case 2: return x ? x_stride<Codelet2>(n) : Codelet2::span(n);
    case 3: return x ? x_stride<Codelet3>(n) : Codelet3::span(n);
    case 4: return x ? x_stride<Codelet4>(n) : Codelet4::span(n);
    case 5: return x ? x_stride<Codelet5>(n) : Codelet5::span(n);
    default: return x ? x_stride<GenericRows>(n) : GenericRows::span(n);
  }
}

int fft_codelet(int n, bool fp32, FFTPlan* plan, int* tpr) {
  if (!fp32) return -1;
  for (int i = 0; i < (int)(sizeof(kCodelets) / sizeof(kCodelets[0])); ++i) {
    const CodeletDesc& c = kCodelets[i];
    if (c.n != n) continue;
    plan->n = n;
    plan->nstages = c.nst;
    for (int k = 0; k < c.nst; ++k) plan->radix[k] = c.code[k] >> 4;
    *tpr = c.tpr;
    return i;
  }
  return -1;
}

static int rows_for(int len, size_t elem, int bufs_extra, int maxrows) {
  // two ping-pong buffers of rows*len complex words within kLdsBudget
  size_t per = 2 * (size_t)len * elem + (size_t)bufs_extra * elem;
  int r = (int)(kLdsBudget / per);
  if (r < 1) r = 1;
  if (r > maxrows) r = maxrows;
  return r;
}

template <typename T>
static hipError_t fwd_impl(const fcmdp_solver* s, const T* grid, void* spec,
                           hipStream_t st) {
  using C = cplx_t<T>;
  const DevParams& dp = s->dp;
  DftOff doff;
  for (int i = 0; i < 32; ++i) doff.off[i] = s->dft_off[i];
  const int M = dp.Nx / 2;
  const int planes = dp.nch_in * dp.Nz;
  constexpr bool kRowOwned = sizeof(T) == 4;       // single precision only
  if (kRowOwned && s->wave_x && !s->force_generic_fft) {
    if constexpr (kRowOwned) wave_x<T>(true, s, grid, spec, doff, st);
  } else {
    int rows = rows_for(M, sizeof(C), 0, 16);
    if (rows > dp.Ny) rows = dp.Ny;
    size_t lds = 2 * (size_t)rows * M * sizeof(C);
    hipLaunchKernelGGL(k_fft_x_r2c<T>, dim3((dp.Ny + rows - 1) / rows, planes),
                       dim3(256), lds, st, dp, s->plan_x, s->band, grid, (C*)spec,
                       (const C*)s->tw_x, (const C*)s->tw_r, s->dftc, doff, rows);
  }
  if (kRowOwned && s->wave_y && !s->force_generic_fft) {
    if constexpr (kRowOwned) wave_y<T>(s, spec, doff, T(-1), st);
    return hipGetLastError();
  }
  int ry = rows_for(dp.Ny, sizeof(C), 0, 16);
  if (ry > dp.Nkx) ry = dp.Nkx;
  size_t lds = 2 * (size_t)ry * dp.Ny * sizeof(C);
  hipLaunchKernelGGL(k_fft_y<T>, dim3((dp.Nkx + ry - 1) / ry, planes),
                     dim3(256), lds, st, dp, s->plan_y, s->band, (C*)spec,
                     (const C*)s->tw_y, s->dftc, doff, ry, T(-1));
  return hipGetLastError();
}

template <typename T>
static hipError_t inv_impl(const fcmdp_solver* s, void* spec, T* grid,
                           hipStream_t st) {
  using C = cplx_t<T>;
  const DevParams& dp = s->dp;
  DftOff doff;
  for (int i = 0; i < 32; ++i) doff.off[i] = s->dft_off[i];
  const int M = dp.Nx / 2;
  const int planes = dp.nch_out * dp.Nz;
  constexpr bool kRowOwned = sizeof(T) == 4;       // single precision only
  if (kRowOwned && s->wave_y && !s->force_generic_fft) {
    if constexpr (kRowOwned) wave_y<T>(s, spec, doff, T(1), st);
  } else {
    int ry = rows_for(dp.Ny, sizeof(C), 0, 16);
    if (ry > dp.Nkx) ry = dp.Nkx;
    size_t lds = 2 * (size_t)ry * dp.Ny * sizeof(C);
    hipLaunchKernelGGL(k_fft_y<T>, dim3((dp.Nkx + ry - 1) / ry, planes),
                       dim3(256), lds, st, dp, s->plan_y, s->band, (C*)spec,
                       (const C*)s->tw_y, s->dftc, doff, ry, T(1));
  }
  if (kRowOwned && s->wave_x && !s->force_generic_fft) {
    if constexpr (kRowOwned) wave_x<T>(false, s, spec, grid, doff, st);
    return hipGetLastError();
  }
  int rows = rows_for(M, sizeof(C), 1, 16);
  if (rows > dp.Ny) rows = dp.Ny;
  size_t lds = (size_t)rows * (2 * M + 1) * sizeof(C);
  hipLaunchKernelGGL(k_fft_x_c2r<T>, dim3((dp.Ny + rows - 1) / rows, planes),
                     dim3(256), lds, st, dp, s->plan_x, s->band, (const C*)spec,
                     grid, (const C*)s->tw_x, (const C*)s->tw_r, s->dftc, doff,
                     rows);
  return hipGetLastError();
}

hipError_t launch_fft_forward(const fcmdp_solver* s, const void* grid,
                              void* spec, hipStream_t st) {
  return s->mixed ? fwd_impl<float>(s, (const float*)grid, spec, st)
                  : fwd_impl<double>(s, (const double*)grid, spec, st);
}

hipError_t launch_fft_inverse(const fcmdp_solver* s, void* spec, void* grid,
                              hipStream_t st) {
  return s->mixed ? inv_impl<float>(s, spec, (float*)grid, st)
                  : inv_impl<double>(s, spec, (double*)grid, st);
}

}  // namespace fcmdp
