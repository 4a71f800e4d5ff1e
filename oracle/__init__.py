"""CPU oracle for the doubly-periodic FCM mobility apply -- TEST INFRASTRUCTURE.

A plain, slow, float64 NumPy implementation of the method of Hashemi et al.,
"Computing hydrodynamic interactions in confined doubly-periodic geometries in
linear time" (arXiv 2210.01837), written from the paper:

* ``kernel``  -- the exponential-of-semicircle (ES) envelope (Sec. 3.5,
  eqs. es, es-scalar) and its normalisation.
* ``cheb``    -- the Chebyshev extrema grid, the Chebyshev transform (DCT-I,
  the paper's 2Nz-2 even-extension FFT), Chebyshev differentiation and
  integration, Clenshaw-Curtis weights (Sec. 3.4).
* ``bvp``     -- the per-wavenumber two-point boundary value problems with
  Dirichlet-to-Neumann (Robin) conditions in the integrated Chebyshev form
  (Sec. 3.1, 3.3, 3.4; discretisation reading documented in bvp.py).
* ``stokes``  -- the Fourier-Chebyshev Stokes solve, steps 2-7 of Sec. 3.4:
  DP solve, bottom-wall / slit-channel correction (Sec. 3.2, App. A),
  k = 0 mode (Sec. 3.3, App. A.2), vorticity by a spectral curl.
* ``fcm``     -- spreading with wall images (eqs. fcm, kernelnearwall),
  interpolation (eqs. getpartvel, getpartvort) and the whole apply.
* ``lanczos`` -- Brownian displacements M^{1/2} W by the Lanczos process
  (Sec. 5.2) on top of the forces-only apply.
* ``torque_deriv`` -- the second torque route of Sec. 3.4 (last paragraph
  and its footnotes): torques spread, and angular velocities interpolated,
  through the truncated derivative of the dipole ES kernel instead of a
  spectral curl.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library and never calls
it; the product path must not route through it.

Parity pins: every function here is checked in ``tests/test_oracle_*.py``
against closed forms, invariants, library routines or brute force.  Absolute
mobility values against the paper's figures are "parity unpinned" because the
figures' data are not part of the paper's text.
"""
from .kernel import ESKernel, es_normalization, phi  # noqa: F401
from . import cheb, bvp, stokes, fcm, lanczos, torque_deriv  # noqa: F401
from .fcm import Solver, apply_mobility  # noqa: F401
