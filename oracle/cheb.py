"""Chebyshev machinery in z, Sec. 3.4 (solver description and its footnote on
the Chebyshev/Fourier compatibility).

Grid: type-2 Chebyshev (extrema) points including both ends,
    s_c = cos(pi c / (Nz-1)),  z_c = (H/2)(1 + s_c),  c = 0..Nz-1,
so c = 0 is the top z = H and c = Nz-1 is the bottom wall z = 0.

Transform: Chebyshev coefficients of the interpolant through the nodes.  The
paper obtains them with an FFT of the even extension to 2Nz-2 points; that is
exactly the type-I discrete cosine transform written out below.
"""
from __future__ import annotations

import numpy as np


def nodes(Nz: int, H: float):
    """Return (s_c, z_c) of the Chebyshev extrema grid on [0, H]."""
    c = np.arange(Nz)
    s = np.cos(np.pi * c / (Nz - 1))
    return s, 0.5 * H * (1.0 + s)


def dct1_matrix(Nz: int) -> np.ndarray:
    """M[n, c] with a_n = sum_c M[n, c] f_c (interpolant coefficients).

    a_n = (2/(Nz-1)) g_n sum''_c f_c cos(pi n c/(Nz-1)), where sum'' halves
    the c = 0 and c = Nz-1 terms and g_0 = g_{Nz-1} = 1/2, g_n = 1 otherwise.
    """
    N1 = Nz - 1
    n = np.arange(Nz)[:, None]
    c = np.arange(Nz)[None, :]
    M = np.cos(np.pi * n * c / N1) * (2.0 / N1)
    M[:, 0] *= 0.5
    M[:, -1] *= 0.5
    M[0, :] *= 0.5
    M[-1, :] *= 0.5
    return M


def idct1_matrix(Nz: int) -> np.ndarray:
    """P[c, n] = T_n(s_c) = cos(pi n c/(Nz-1)): coefficients -> node values."""
    N1 = Nz - 1
    c = np.arange(Nz)[:, None]
    n = np.arange(Nz)[None, :]
    return np.cos(np.pi * n * c / N1)


def dct1(f: np.ndarray, axis: int = 0) -> np.ndarray:
    """Node values -> Chebyshev coefficients along ``axis``."""
    f = np.moveaxis(f, axis, 0)
    a = np.tensordot(dct1_matrix(f.shape[0]), f, axes=(1, 0))
    return np.moveaxis(a, 0, axis)


def idct1(a: np.ndarray, axis: int = 0) -> np.ndarray:
    """Chebyshev coefficients -> node values along ``axis``."""
    a = np.moveaxis(a, axis, 0)
    f = np.tensordot(idct1_matrix(a.shape[0]), a, axes=(1, 0))
    return np.moveaxis(f, 0, axis)


def deriv(a: np.ndarray, H: float, axis: int = 0) -> np.ndarray:
    """Coefficients of d/dz of the Chebyshev series a (z in [0, H]).

    Uses the standard recurrence in s: c_{n-1} b_{n-1} = b_{n+1} + 2 n a_n
    for n = Nz-1..1 with b_{Nz} = b_{Nz-1} = 0, c_0 = 2, c_n = 1 (n > 0);
    then d/dz = (2/H) d/ds.
    """
    a = np.moveaxis(np.asarray(a), axis, 0)
    N = a.shape[0]
    b = np.zeros_like(a)
    for n in range(N - 1, 0, -1):
        nxt = b[n + 1] if n + 1 < N else 0.0
        val = nxt + 2.0 * n * a[n]
        b[n - 1] = val / 2.0 if n - 1 == 0 else val
    return np.moveaxis(b * (2.0 / H), 0, axis)


def integ_B(N: int) -> np.ndarray:
    """Matrix of the Chebyshev antiderivative operator B on N coefficients.

    (B sigma)_n = (c_{n-1} sigma_{n-1} - sigma_{n+1}) / (2n), n >= 1, with
    sigma_j = 0 for j >= N; row 0 (the free constant) is left zero.  The
    result is truncated to N coefficients.
    """
    B = np.zeros((N, N))
    for n in range(1, N):
        B[n, n - 1] += (2.0 if n - 1 == 0 else 1.0) / (2.0 * n)
        if n + 1 < N:
            B[n, n + 1] -= 1.0 / (2.0 * n)
    return B


def b2_matrix(N: int) -> np.ndarray:
    """Rows m >= 2 of the double antiderivative B^2 on N coefficients.

    (B^2 s)_m = c_{m-2} s_{m-2}/(4m(m-1)) - s_m/(2(m^2-1)) + s_{m+2}/(4m(m+1))
    with s_j = 0 for j >= N.  Rows 0 and 1 (integration constants) are zero.
    """
    B2 = np.zeros((N, N))
    for m in range(2, N):
        B2[m, m - 2] = (2.0 if m - 2 == 0 else 1.0) / (4.0 * m * (m - 1))
        B2[m, m] = -1.0 / (2.0 * (m * m - 1))
        if m + 2 < N:
            B2[m, m + 2] = 1.0 / (4.0 * m * (m + 1))
    return B2


def cc_weights(Nz: int, H: float) -> np.ndarray:
    """Clenshaw-Curtis weights on the extrema grid of [0, H].

    By definition the weights integrate the Chebyshev interpolant exactly:
    w_c = (H/2) sum_n M[n, c] int_{-1}^{1} T_n(s) ds, with
    int T_n = 2/(1-n^2) for even n and 0 for odd n.
    """
    n = np.arange(Nz)
    iT = np.zeros(Nz)
    even = n % 2 == 0
    iT[even] = 2.0 / (1.0 - n[even].astype(float) ** 2)
    return 0.5 * H * (dct1_matrix(Nz).T @ iT)


def eval_series(a: np.ndarray, s: np.ndarray) -> np.ndarray:
    """Evaluate sum_n a_n T_n(s) at arbitrary s in [-1, 1] (for tests)."""
    n = np.arange(a.shape[0])
    return np.cos(np.outer(np.arccos(np.clip(s, -1, 1)), n)) @ a
