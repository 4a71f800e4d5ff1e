"""Per-wavenumber two-point boundary value problems in z (Sec. 3.1, 3.3, 3.4).

Every k != 0 solve of the DP subproblem has the form

    y''(z) - k^2 y(z) = r(z)  on [0, H],
    (d/dz + k) y(H) = g_H,    (d/dz - k) y(0) = g_0,

(pressure: eq. poissonfs with the Dirichlet-to-Neumann maps of eq. DtoNmapp;
velocities: eq. momentumfs with eqs. DtoNmapuv and DtoNmapw).  The k = 0 mode
of the tangential velocity solves y'' = -f/eta with Dirichlet/Neumann
(bottom wall, eq. bvp-u-k0-bcs) or Dirichlet/Dirichlet (slit channel with no
slip, eq. bvp-uv-k0-sc) conditions.

Discretisation (reading; the paper defers the solver to the Greengard-style
spectral-integration method of its reference on DP electrostatics and says
only that the systems are pentadiagonal): in s = 2z/H - 1 the equation reads
y_ss - kappa^2 y = (H^2/4) r with kappa = k H / 2.  Applying the double
antiderivative B^2 to it and keeping rows m = 2..Nz-1 gives

    y_m - kappa^2 (B^2 y)_m = (H^2/4) (B^2 r)_m,

(exact for the Chebyshev polynomial y of degree Nz-1, because B^2 y_ss
reproduces y in rows m >= 2).  Rows 0 and 1 are the two boundary conditions:

    sum_n (n^2 + kappa) y_n          = (H/2) g_H      (T_n(1)=1, T_n'(1)=n^2)
    sum_n (-1)^(n+1) (n^2 + kappa) y_n = (H/2) g_0    (T_n(-1)=(-1)^n,
                                                       T_n'(-1)=(-1)^(n+1) n^2)

The interior rows have bands at -2, 0, +2 only (pentadiagonal with zero odd
bands).  The oracle assembles this Nz x Nz system densely and solves it with
LU (numpy.linalg.solve); no banded structure is exploited here.
"""
from __future__ import annotations

import numpy as np

from . import cheb


def robin_matrices(kappa: np.ndarray, N: int) -> np.ndarray:
    """Dense system matrices A[k] (shape (K, N, N)) for kappa[k] > 0."""
    kappa = np.asarray(kappa, dtype=np.float64)
    n = np.arange(N, dtype=np.float64)
    B2 = cheb.b2_matrix(N)
    A = np.empty((kappa.size, N, N))
    A[:, 2:, :] = np.eye(N)[None, 2:, :] - kappa[:, None, None] ** 2 * B2[None, 2:, :]
    A[:, 0, :] = n[None, :] ** 2 + kappa[:, None]
    sgn = np.where(np.arange(N) % 2 == 1, 1.0, -1.0)    # (-1)^(n+1)
    A[:, 1, :] = sgn[None, :] * (n[None, :] ** 2 + kappa[:, None])
    return A


def robin_rhs(r: np.ndarray, g_H, g_0, H: float) -> np.ndarray:
    """Right-hand sides (K, N) for coefficient arrays r (K, N) of the source."""
    N = r.shape[-1]
    B2 = cheb.b2_matrix(N)
    b = (H * H / 4.0) * (r @ B2.T)
    b[:, 0] = 0.5 * H * np.asarray(g_H)
    b[:, 1] = 0.5 * H * np.asarray(g_0)
    return b


def solve(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Solve the real systems A x = b for complex right-hand sides b."""
    rhs = np.stack([b.real, b.imag], axis=-1)
    x = np.linalg.solve(A, rhs)
    return x[..., 0] + 1j * x[..., 1]


def zero_mode_matrix(N: int, geometry: str, H: float = 1.0, slip0: float = 0.0,
                     slipH: float = 0.0) -> np.ndarray:
    """System for y'' = rhs at k = 0.

    Rows m >= 2: y_m = (H^2/4)(B^2 rhs)_m.  Row 1: y(0) - l_0 y'(0) = 0
    with the slip length l_0 of the wall at z = 0 (eq. bvp-uv-k0-sc; l_0 = 0:
    no slip).  Row 0: bottom wall y'(H) = 0, i.e. sum n^2 y_n = 0; slit
    channel y(H) + l_H y'(H) = 0.  With T_n(+-1) = (+-1)^n and
    T_n'(+-1) = (+-1)^(n+1) n^2, d/dz = (2/H) d/ds.  Reading: a bottom wall
    with slip takes the same condition at z = 0 as the slit channel's lower
    wall.
    """
    n = np.arange(N, dtype=np.float64)
    sgn = np.where(np.arange(N) % 2 == 0, 1.0, -1.0)
    A = np.eye(N)
    if geometry == "bw":
        A[0, :] = n ** 2
        A[1, :] = sgn - slip0 * (2.0 / H) * (-sgn) * n ** 2
    else:
        A[0, :] = 1.0 + slipH * (2.0 / H) * n ** 2
        A[1, :] = sgn - slip0 * (2.0 / H) * (-sgn) * n ** 2
    return A


def zero_mode_solve(rhs_coeffs: np.ndarray, H: float, geometry: str,
                    slip0: float = 0.0, slipH: float = 0.0, g0: complex = 0.0,
                    gH: complex = 0.0) -> np.ndarray:
    """Coefficients y of y'' = rhs (rhs given as Chebyshev coefficients);
    g0 and gH are the right-hand sides of the wall conditions (the wall
    velocities of eqs. bcnoslip0fs and bvp-uv-k0-sc; gH = 0 for a bottom
    wall, whose top condition is y'(H) = 0)."""
    N = rhs_coeffs.shape[-1]
    B2 = cheb.b2_matrix(N)
    b = (H * H / 4.0) * (B2 @ rhs_coeffs)
    b[0] = gH
    b[1] = g0
    A = zero_mode_matrix(N, geometry, H, slip0, slipH)
    return solve(A[None], b[None])[0]
