"""Helpers for GPU-vs-oracle parity tests (the oracle side of each stage).

Only tests import this module.  Inputs come from the seeded generators in
``workloads``; expected values come from ``oracle`` only.
"""
from __future__ import annotations

import numpy as np

from oracle import cheb, fcm, stokes


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64 if not np.iscomplexobj(a) else np.complex128)
    b = np.asarray(b)
    den = np.linalg.norm(b.ravel())
    if den == 0:
        return float(np.linalg.norm(a.ravel()))
    return float(np.linalg.norm((a - b).ravel()) / den)


def particle_err(a, b):
    """Largest error of one particle's vector, relative to the RMS particle
    vector of the reference: max_j |a_j - b_j| / sqrt(mean_j |b_j|^2) for
    (N, 3) arrays (a single particle far off shows here even when the
    norm-wise error is small)."""
    a = np.asarray(a, dtype=np.float64).reshape(-1, 3)
    b = np.asarray(b, dtype=np.float64).reshape(-1, 3)
    rms = np.sqrt(np.mean(np.sum(b * b, axis=1)))
    d = np.sqrt(np.max(np.sum((a - b) ** 2, axis=1)))
    return float(d / rms) if rms > 0 else float(d)


def max_rel(a, b):
    den = np.max(np.abs(b))
    return float(np.max(np.abs(np.asarray(a) - b)) / (den if den > 0 else 1.0))


def band_of(solver: fcm.Solver, pos):
    """First and last Chebyshev node touched by any particle's z-kernel
    (on [max(0, z-alpha), min(H, z+alpha)])."""
    zc = solver.zc
    a = solver.alpha
    H = solver.box.H
    lo = np.maximum(0.0, pos[:, 2] - a)
    hi = np.minimum(H, pos[:, 2] + a)
    inside = (zc[None, :] >= lo[:, None]) & (zc[None, :] <= hi[:, None])
    cs = np.nonzero(inside.any(axis=0))[0]
    return int(cs.min()), int(cs.max())


def oracle_spread(box, pos, F, T):
    s = fcm.Solver(box)
    f, g = s.spread(s.wrap(pos), F, T)
    return np.concatenate([f, g], axis=0)


def oracle_fft_forward(box, grid, lo, hi):
    """rfft2 per plane, laid out [6][Nz][Nkx][Ny]; planes outside the band 0."""
    g = np.zeros_like(grid)
    g[:, lo:hi + 1] = grid[:, lo:hi + 1]
    spec = np.fft.rfft2(g, axes=(-2, -1))              # [6][Nz][Ny][Nkx]
    return np.transpose(spec, (0, 1, 3, 2))


def oracle_solve(box, spec_in, lo, hi):
    """Node values (band) of f, g in xy Fourier space -> node values of u and
    omega, times 1/(Nx Ny); layout [6][Nz][Nkx][Ny]."""
    x = np.zeros_like(spec_in)
    x[:, lo:hi + 1] = spec_in[:, lo:hi + 1]
    x = np.transpose(x, (0, 1, 3, 2))                  # [6][Nz][Ny][Nkx]
    coef = cheb.dct1(x, axis=1)
    uh, omh = stokes.solve_coefficients(box, coef[:3], coef[3:])
    out = cheb.idct1(np.concatenate([uh, omh], axis=0), axis=1)
    out = out / (box.Nx * box.Ny)
    res = np.zeros_like(out)
    res[:, lo:hi + 1] = out[:, lo:hi + 1]
    return np.transpose(res, (0, 1, 3, 2))


def oracle_fft_inverse(box, spec, lo, hi):
    """Unnormalised inverse 2-D real DFT of the band planes."""
    x = np.transpose(spec, (0, 1, 3, 2))               # [6][Nz][Ny][Nkx]
    out = np.fft.irfft2(x, s=(box.Ny, box.Nx), axes=(-2, -1)) * (box.Nx * box.Ny)
    res = np.zeros_like(out)
    res[:, lo:hi + 1] = out[:, lo:hi + 1]
    return res


def oracle_interp(box, pos, grid):
    s = fcm.Solver(box)
    return s.interp(s.wrap(pos), grid[:3], grid[3:])


def oracle_apply(box, pos, F, T, sample=None):
    return fcm.Solver(box).apply(pos, F, T, sample=sample)
