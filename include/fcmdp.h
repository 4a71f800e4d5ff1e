/*
 * fcmdp.h -- C ABI of the MI355X (gfx950) doubly-periodic FCM mobility apply.
 *
 * Method: Hashemi et al., "Computing hydrodynamic interactions in confined
 * doubly-periodic geometries in linear time" (arXiv 2210.01837).
 *
 * Given N particles in a box periodic in x and y, either above one no-slip
 * wall at z = 0 ("bottom wall") or between no-slip walls at z = 0 and z = H
 * ("slit channel"), with forces F and torques T, the library computes the
 * particle velocities U and angular velocities Omega,
 *
 *     [U; Omega] = M [F; T]                         (eq. grandmob, Sec. 4)
 *
 * where M is the FCM mobility of Sec. 2 (eqs. fcm, kernelnearwall,
 * getpartvel, getpartvort) with the exponential-of-semicircle envelope of
 * Sec. 3.5 (eqs. es, es-scalar), evaluated by the spectral Stokes solver of
 * Sec. 3.4: spreading, xy FFT + Chebyshev transform, per-wavenumber BVP
 * solves (Sec. 3.1), wall correction (Sec. 3.2, App. A), k = 0 mode
 * (Sec. 3.3), inverse transforms and interpolation.  Torques enter through a
 * spectral curl (the paper's GPU route, Sec. 3.4).
 *
 * Conventions
 *   - Lengths: full periods Lx, Ly (x in [0, Lx), y in [0, Ly)); the grid
 *     is x_a = a*Lx/Nx, y_b = b*Ly/Ny (hx must equal hy) and the Chebyshev
 *     extrema z_c = (H/2)(1 + cos(pi c/(Nz-1))), c = 0..Nz-1 (c = 0 is z=H).
 *   - ES support alpha = w*h/2 (Sec. 3.5); beta_m and beta_d are absolute
 *     (e.g. 1.327*6 and 2.216*6 for w = 6, Table 1).
 *   - Particle arrays are row-major [n][3] in DEVICE memory, owned by the
 *     caller: double in FCMDP_FP64 mode, float in FCMDP_MIXED mode (FP32
 *     spreading, FFTs and interpolation; FP64 per-wavenumber solves).
 *   - All entry points are asynchronous on the HIP stream passed in (NULL =
 *     the default stream) unless stated otherwise; no host synchronisation
 *     happens inside an apply.
 *   - A solver is not thread safe: one call in flight per solver.
 *
 * Errors: every function returns FCMDP_OK (0) or a negative code;
 * fcmdp_strerror() names it.  No C++ exception crosses this ABI.
 */
#ifndef FCMDP_H
#define FCMDP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fcmdp_solver fcmdp_solver;

enum { FCMDP_BOTTOM_WALL = 0, FCMDP_SLIT_CHANNEL = 1 };
enum { FCMDP_FP64 = 0, FCMDP_MIXED = 1 };
enum {
  FCMDP_OK = 0,
  FCMDP_EINVAL = -1,   /* bad argument or unsupported size */
  FCMDP_EDOMAIN = -2,  /* particles outside the fluid domain (see status) */
  FCMDP_ENOMEM = -3,   /* device allocation failed */
  FCMDP_EHIP = -4,     /* a HIP runtime call failed */
  FCMDP_ECAPACITY = -5 /* n larger than the solver's max_particles */
};

typedef struct {
  int geometry;        /* FCMDP_BOTTOM_WALL or FCMDP_SLIT_CHANNEL */
  double Lx, Ly, H;    /* periods and channel height / domain top */
  int Nx, Ny, Nz;      /* grid; Nx, Ny even, >= 8, factors in {2,3,5,7,11,13,17};
                          8 <= Nz <= 64 */
  int w;               /* ES support in grid cells: 4 or 6 (the kernels hold a
                          7-point window) */
  double beta_m, beta_d; /* ES shape parameters, monopole and dipole */
  double eta;          /* viscosity > 0 */
  int precision;       /* FCMDP_FP64 or FCMDP_MIXED */
  int64_t max_particles; /* capacity of the particle workspace */
  double slip0, slipH; /* slip lengths of the walls at z = 0 and z = H (App. A,
                          partial slip u - l0 du/dz = u^W at z = 0, u + lH
                          du/dz = u^W at z = H): Nz <= 32; a bottom wall
                          takes l0 only (slipH = 0); 0 = no slip */
  double wall0[2];     /* uniform (x, y) velocity of the wall at z = 0 */
  double wallH[2];     /* ... of the slit channel's wall at z = H (zero for a
                          bottom wall); nonzero wall velocities need
                          Nz <= 32 */
  int torque_route;    /* FCMDP_TORQUE_CURL: torques spread as the dipole
                          density g and Omega = (1/2) curl u, both curls taken
                          spectrally (six channels through the transforms and
                          the solve; the paper's GPU route).
                          FCMDP_TORQUE_DERIVATIVE: the force density gets
                          (1/2) grad Delta_D x tau and Omega = (1/2) sum
                          u x grad Delta_D with the truncated derivative of
                          the dipole ES kernel (Sec. 3.4, last paragraph and
                          its footnotes; three channels through the
                          transforms and the solve).  Nz <= 32. */
} fcmdp_params;

enum { FCMDP_TORQUE_CURL = 0, FCMDP_TORQUE_DERIVATIVE = 1 };

/*
 * Create a solver: validates p, derives h, alpha, the ES normalisations, the
 * Chebyshev tables and FFT plans, and allocates all device workspace on the
 * current HIP device, ~ (2*6*Nz*Ny*Nx real words + particle buffers), see
 * fcmdp_workspace_bytes.  The workspace is allocated and the tables are
 * uploaded in stream order on hip_stream (NULL = the default stream), and
 * the call returns once hip_stream has completed them: it waits for that
 * stream only, never for the whole device, so applies in flight on other
 * streams keep running.  The solver may then be used on any stream.
 * Returns EINVAL for invalid parameters, ENOMEM/EHIP on allocation failure.
 */
int fcmdp_create_solver(const fcmdp_params* p, void* hip_stream,
                        fcmdp_solver** out);

/* Device bytes a solver with parameters p needs for n particles (host only). */
int fcmdp_workspace_bytes(const fcmdp_params* p, int64_t n, size_t* bytes);

/*
 * The mobility apply (F, T) -> (U, Omega) for n particles.
 *   pos, F: [n][3] device arrays (double in FP64 mode, float in MIXED mode).
 *   T:      torques, or NULL for none: the torque (dipole) channels are then
 *           neither spread, transformed nor read by the solve (the
 *           forces-only apply of Sec. 5 carries three channels).
 *   U:      output velocities [n][3].
 *   Omega:  output angular velocities [n][3], or NULL to skip: the solve
 *           then returns the three velocity channels only and the inverse
 *           transform and interpolation carry three channels.
 * x and y are wrapped periodically.  Particles with z < 0, z > H (slit
 * channel) or z + alpha > H (bottom wall; the forcing must vanish above the
 * computational top) are skipped: their outputs are NaN and fcmdp_status()
 * reports EDOMAIN after the stream has been synchronised.
 * n = 0 is valid (no work).  Returns ECAPACITY if n > max_particles.
 */
int fcmdp_apply_mobility(fcmdp_solver* s, int64_t n, const void* pos,
                         const void* F, const void* T, void* U, void* Omega,
                         void* hip_stream);

/* After the stream of the last apply has completed: FCMDP_OK, or EDOMAIN
 * with *n_bad (if non-NULL) set to the number of skipped particles. */
int fcmdp_status(fcmdp_solver* s, int64_t* n_bad);

/* Release all device memory of s in stream order on hip_stream (NULL = the
 * default stream); does not block the host or the device.  The caller
 * orders every apply on s before hip_stream (same stream, or an event wait)
 * and does not use s afterwards. */
void fcmdp_destroy_solver(fcmdp_solver* s, void* hip_stream);

const char* fcmdp_strerror(int code);

/*
 * Brownian displacements g = M^{1/2} W (Sec. 5.2) by the Lanczos process in
 * the Krylov space of the translational mobility M, i.e. the forces-only
 * apply F -> U of fcmdp_apply_mobility (T = NULL, Omega = NULL), which is
 * symmetric positive definite up to discretisation error.
 *   pos, W, g:  [n][3] device arrays of the solver's element type; W holds
 *               the random vector (e.g. i.i.d. N(0, 1)), g receives
 *               |W| V_k T_k^{1/2} e_1 (V_k the orthonormal Krylov basis, T_k
 *               the Lanczos tridiagonal matrix).  g must not alias W.
 *   max_iter:   1..64 iterations (one mobility apply each).
 *   tol:        stop once |g_k - g_{k-1}| / |g_{k-1}| < tol (k >= 2); 0 runs
 *               all max_iter iterations.
 *   iters, rel_change (optional): iterations used and the last relative
 *               change.
 * Blocking on the host (a few synchronisations of the stream per iteration);
 * the Krylov basis ((max_iter + 1) * 3n words) is allocated on first use and
 * kept with the solver.  W = 0 gives g = 0 and *iters = 0.  Particles outside
 * the domain make the applies, and so g, NaN (fcmdp_status reports them).
 * Returns EINVAL for bad arguments, ECAPACITY if n > max_particles, ENOMEM,
 * EHIP, or an error of the mobility apply.
 */
int fcmdp_lanczos_sqrt(fcmdp_solver* s, int64_t n, const void* pos,
                       const void* W, void* g, int max_iter, double tol,
                       int* iters, double* rel_change, void* hip_stream);

/*
 * fcmdp_lanczos_sqrt without any device allocation, for callers that cannot
 * allocate (tight serving loops, code that must not call hipMalloc): the
 * Krylov basis and the reduction partial sums live in a fixed 64 MiB device
 * array of the library, one per GPU, held until the process ends, instead of
 * the solver's on-demand buffers.  Same arguments, results and errors as
 * fcmdp_lanczos_sqrt (its arithmetic, bit for bit), plus ECAPACITY when the
 * basis ((max_iter + 1) * 3n words, rounded up to 64 per vector) and the
 * partial sums (~260 KiB) do not fit in that array: about 64 iterations at
 * n = 86,000 or 8 iterations at n = 660,000 in MIXED mode, half of that in
 * FP64.  Every call on a GPU shares that GPU's array: calls that overlap on
 * one GPU (different streams or host threads) race and must be serialised
 * by the caller.  The mobility applies inside use the solver's own
 * workspace, allocated when the solver was created.
 */
int fcmdp_lanczos_sqrt_noalloc(fcmdp_solver* s, int64_t n, const void* pos,
                               const void* W, void* g, int max_iter, double tol,
                               int* iters, double* rel_change, void* hip_stream);

/*
 * Non-uniform tangential wall velocities u^W(x, y) (eq. bcnoslip0 for the
 * bottom wall; App. A, eqs. bcslip and u0uHformula for the slit channel):
 *   wall: device array [nw][2][Ny][Nx] of (u^W, v^W) at the grid nodes
 *         x_a = a Lx / Nx, y_b = b Ly / Ny of the wall at z = 0 and, for the
 *         slit channel (nw = 2), of the wall at z = H (nw = 1 for the bottom
 *         wall).  Element type as for the particle arrays (float in MIXED,
 *         double in FP64 mode).  Read on `hip_stream` during this call only.
 *         NULL removes the field (walls back to the uniform params.wall0 /
 *         wallH).
 * The field adds to the uniform wall velocities of fcmdp_params and applies
 * to every later fcmdp_apply_mobility, fcmdp_stage_solve and Lanczos call
 * of this solver: its unnormalised xy DFT (Nyquist modes dropped) enters the
 * correction's boundary data at every wavenumber and its mean the k = 0
 * mode.  Computed on `hip_stream` with the solver's own transforms; the
 * spectrum (4 (Nx/2+1) Ny complex words) is allocated on first use
 * (stream-ordered) and kept with the solver.  Like every call on one
 * solver, it must be ordered with the solver's other calls.  Returns
 * EINVAL for s == NULL or Nz > 32 (the eight-lane column kernels), EHIP.
 */
int fcmdp_set_wall_velocity(fcmdp_solver* s, const void* wall, void* hip_stream);

/* Derived quantities of a solver (host only): out[0] = h, out[1] = alpha,
 * out[2] = ES normalisation integral of the monopole kernel, out[3] = of the
 * dipole kernel (the integral in eq. es-scalar). */
int fcmdp_solver_info(const fcmdp_solver* s, double out[4]);

/*
 * Per-stage timing with HIP events on the apply's stream (tracing).  When
 * enabled, every fcmdp_apply_mobility brackets its stages with events:
 *   0 particle prep + sort + records, 1 spread, 2 forward xy FFT,
 *   3 column solve, 4 inverse xy FFT, 5 interpolation.
 * fcmdp_stage_times() waits for the recorded events, returns the summed
 * milliseconds per stage in ms[0..5], the z-band of the last apply in
 * ms[6] (first node) and ms[7] (last node), the number of applies timed in
 * *napplies, and resets the accumulators.  Blocking (host side).
 */
int fcmdp_set_profiling(fcmdp_solver* s, int enable);
int fcmdp_stage_times(fcmdp_solver* s, double ms[8], int64_t* napplies);

/*
 * Kernel variants.  Every step has a default kernel chosen at creation from
 * the sizes; the alternatives below compute the same quantities with a
 * different parallel decomposition and exist for cross-checks and tuning.
 * value: 0/1 for the switches; for the FFT row counts a power of two, or 12
 * for the x pass (rows per workgroup of the wave-per-row x and y passes,
 * 0 = default), rejected with FCMDP_EINVAL if the rows do not fit in LDS;
 * for the spread's workgroups 1..65535, block rows 8 or 16 and block order
 * 1 or 2 (0 = default), else FCMDP_EINVAL.
 * Not thread safe with respect to applies on the same solver.
 */
enum {
  FCMDP_VARIANT_GENERIC_FFT = 0,     /* workgroup-per-row-batch transforms */
  FCMDP_VARIANT_FFT_ROWS_X = 1,      /* rows per workgroup, x pass (1..16) */
  FCMDP_VARIANT_FFT_ROWS_Y = 2,      /* rows per workgroup, y pass (1..8) */
  FCMDP_VARIANT_SIMPLE_SPREAD = 3,   /* thread-per-column gather spread */
  FCMDP_VARIANT_SIMPLE_INTERP = 4,   /* thread-per-particle interpolation */
  FCMDP_VARIANT_GENERIC_COLUMNS = 5, /* thread-per-wavenumber column solve */
  FCMDP_VARIANT_VECTOR_DCT = 6,      /* FP64 Chebyshev transforms in MIXED */
  FCMDP_VARIANT_NO_CODELET = 7,      /* run-time-plan row transforms even
                                        where a fixed-plan kernel exists */
  FCMDP_VARIANT_NO_PIPELINE = 8,     /* one workgroup per y row instead of
                                        the persistent row loop that loads
                                        the next row during a transform */
  FCMDP_VARIANT_NO_LOWK = 9,         /* MIXED slit channel: take the vertical
                                        force of the kH < 1 columns from the
                                        FP32 path too (no FP64 route) */
  FCMDP_VARIANT_WAVE_SPREAD = 10,    /* MIXED: per-patch gather spread on the
                                        vector units instead of the matrix-core
                                        spread of the FP32 grid */
  FCMDP_VARIANT_SPREAD_WORKGROUPS = 11, /* MIXED: workgroups of the
                                        matrix-core spread, which share its
                                        blocks evenly (1..65535; 0 = default,
                                        three per CU: as many as fit at once) */
  FCMDP_VARIANT_SPREAD_BLOCK_ROWS = 12, /* MIXED: grid rows per block of the
                                        matrix-core spread (8 or 16; 0 =
                                        default, chosen by particle density) */
  FCMDP_VARIANT_SPREAD_ORDER = 13,   /* MIXED: block order of the matrix-core
                                        spread: 1 strip-major, shared evenly;
                                        2 neighbouring strips side by side;
                                        0 = default: 1 if grid rows are whole
                                        128-byte lines, else 2 */
  FCMDP_VARIANT_HALO_INTERP = 14     /* interpolation by workgroups that own
                                        the particles of 26 x 26 cells and
                                        stage their planes with a 3-node halo,
                                        instead of partial sums over aligned
                                        32 x 16 tiles (read once) added per
                                        particle in a fixed order */
};
int fcmdp_set_variant(fcmdp_solver* s, int key, int value);

/*
 * Stage entry points (the steps of Sec. 3.4 one at a time, on caller
 * buffers; used for per-stage parity tests).  Real element type is double
 * in FP64 mode and float in MIXED mode.  Layouts:
 *   grid:     real    [6][Nz][Ny][Nx]   channels (fx, fy, fz, gx, gy, gz) on
 *             the way in (monopole density f and dipole density g, eq. fcm)
 *             and (u, v, w, ox, oy, oz) on the way out, omega = curl(u)/2.
 *   spectrum: complex [6][Nz][Nx/2+1][Ny] (interleaved re, im; ky fastest),
 *             the unnormalised xy DFT of the grid per z-node.
 * Only z-nodes c in [c_lo, c_hi] are read or written by the transform and
 * solve stages (the band of planes that particle kernels touch).
 */

/* Step 1: spread (eq. fcm with the images of eq. kernelnearwall); writes the
 * whole grid (zero outside the particles' kernels).  The stage entry points
 * use the six-channel (spectral-curl) layouts: a solver created with
 * FCMDP_TORQUE_DERIVATIVE refuses fcmdp_stage_spread and fcmdp_stage_interp
 * with EINVAL. */
int fcmdp_stage_spread(fcmdp_solver* s, int64_t n, const void* pos,
                       const void* F, const void* T, void* grid,
                       void* hip_stream);

/* Step 2 (xy part): forward real-to-complex 2-D DFT of planes c_lo..c_hi. */
int fcmdp_stage_fft_forward(fcmdp_solver* s, const void* grid, void* spectrum,
                            int c_lo, int c_hi, void* hip_stream);

/* Steps 2 (z part) to 6 and the vorticity curl: per-wavenumber solve from
 * the node values of f and g (planes c_lo..c_hi, zero elsewhere) to the node
 * values of u and omega on planes c_lo..c_hi, scaled by 1/(Nx*Ny) so that
 * fcmdp_stage_fft_inverse yields physical values.  Nyquist modes are zero.
 * spectrum_out may be spectrum_in (in place: every column is read whole
 * before its results are written). */
int fcmdp_stage_solve(fcmdp_solver* s, const void* spectrum_in,
                      void* spectrum_out, int c_lo, int c_hi,
                      void* hip_stream);

/* Step 7 (xy part): inverse complex-to-real 2-D DFT (unnormalised) of planes
 * c_lo..c_hi. */
int fcmdp_stage_fft_inverse(fcmdp_solver* s, const void* spectrum, void* grid,
                            int c_lo, int c_hi, void* hip_stream);

/* Step 8: interpolation (eqs. getpartvel, getpartvort) of u and omega from
 * the grid (all planes may be read).  The solver's own spectrum buffer holds
 * the per-tile partial sums, so its contents are not kept. */
int fcmdp_stage_interp(fcmdp_solver* s, int64_t n, const void* pos,
                       const void* grid, void* U, void* Omega,
                       void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* FCMDP_H */
