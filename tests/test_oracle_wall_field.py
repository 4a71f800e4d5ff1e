"""Pins of the oracle's non-uniform wall velocities u^W(x, y) (eq. bcnoslip0;
App. A, eqs. bcslip and u0uHformula): the wall data enter the correction's
boundary conditions at every wavenumber.

The references are closed forms derived here from a stream function, not
from the oracle's correction formulas: a wall mode cos(k.x) drives a Stokes
flow with stream function psi(z) cos(k.x) along k (psi a combination of
e^{-kz}, z e^{-kz}, e^{kz}, z e^{kz}, the biharmonic modes) and a
pressure-free shear e^{+-kz} cos(k.x) across k.
"""
import numpy as np
import pytest
from dataclasses import replace

import oracle
from oracle import cheb, stokes
from workloads import Box


def _grid(box):
    h = box.Lx / box.Nx
    x = np.arange(box.Nx) * h
    y = np.arange(box.Ny) * (box.Ly / box.Ny)
    _, zc = cheb.nodes(box.Nz, box.H)
    Z, Y, X = np.meshgrid(zc, y, x, indexing="ij")
    return X, Y, Z


def _wall_mode(box, nx, ny, a0, aH=(0.0, 0.0)):
    """(nw, 2, Ny, Nx) wall field (a_x, a_y) cos(kx x + ky y) on each wall."""
    X, Y, _ = _grid(box)
    kx, ky = 2 * np.pi * nx / box.Lx, 2 * np.pi * ny / box.Ly
    c = np.cos(kx * X[0] + ky * Y[0])
    walls = [a0] if box.geometry == "bw" else [a0, aH]
    return np.stack([np.stack([w[0] * c, w[1] * c]) for w in walls])


def _field(box, wall):
    z = np.zeros((3, box.Nz, box.Ny, box.Nx))
    return stokes.stokes_solve(box, z, z, wall)


def _closed_form(box, nx, ny, a0, aH=(0.0, 0.0)):
    """Velocity at the grid nodes driven by the wall modes (stream function
    solution; slip lengths l0, lH of the box)."""
    X, Y, Z = _grid(box)
    kx, ky = 2 * np.pi * nx / box.Lx, 2 * np.pi * ny / box.Ly
    k = np.hypot(kx, ky)
    ex, ey = kx / k, ky / k                 # along k
    tx, ty = -ey, ex                        # across k
    th = kx * X + ky * Y
    L0, T0 = a0[0] * ex + a0[1] * ey, a0[0] * tx + a0[1] * ty
    LH, TH = aH[0] * ex + aH[1] * ey, aH[0] * tx + aH[1] * ty
    l0, lH, H = box.slip0, box.slipH, box.H
    if box.geometry == "bw":
        # psi = A z e^{-kz}: psi(0) = 0, bounded; psi'(0) - l0 psi''(0) = L0
        # with psi'(0) = A, psi''(0) = -2 k A
        A = L0 / (1 + 2 * k * l0)
        psi = A * Z * np.exp(-k * Z)
        dpsi = A * (1 - k * Z) * np.exp(-k * Z)
        vt = T0 / (1 + k * l0) * np.exp(-k * Z)
    else:
        # psi = A e^{-kz} + B z e^{-kz} + C e^{k(z-H)} + D z e^{k(z-H)}
        def basis(z):
            em, ep = np.exp(-k * z), np.exp(k * (z - H))
            f = np.array([em, z * em, ep, z * ep])
            d1 = np.array([-k * em, (1 - k * z) * em, k * ep, (1 + k * z) * ep])
            d2 = np.array([k * k * em, (k * k * z - 2 * k) * em, k * k * ep,
                           (2 * k + k * k * z) * ep])
            return f, d1, d2
        f0, p0, q0 = basis(0.0)
        fH, pH, qH = basis(H)
        M = np.array([f0, p0 - l0 * q0, fH, pH + lH * qH])
        A = np.linalg.solve(M, [0.0, L0, 0.0, LH])
        f, d1, _ = basis(Z)
        psi = np.tensordot(A, f, 1)
        dpsi = np.tensordot(A, d1, 1)
        # transverse shear E e^{-kz} + G e^{k(z-H)} with the Robin conditions
        M2 = np.array([[1 + k * l0, np.exp(-k * H) * (1 - k * l0)],
                       [np.exp(-k * H) * (1 - k * lH), 1 + k * lH]])
        E, G = np.linalg.solve(M2, [T0, TH])
        vt = E * np.exp(-k * Z) + G * np.exp(k * (Z - H))
    ul = dpsi * np.cos(th)
    w = k * psi * np.sin(th)
    vt = vt * np.cos(th)
    return np.stack([ul * ex + vt * tx, ul * ey + vt * ty, w])


BW = Box("bw", 16.0, 12.0, 8.0, 24, 18, 24)
SC = Box("sc", 16.0, 12.0, 6.0, 24, 18, 24)


@pytest.mark.parametrize("nx,ny,a0", [(2, 0, (1.0, 0.0)), (2, 0, (0.0, 1.0)),
                                      (1, -2, (0.7, -0.4)), (3, 1, (0.2, 0.9))])
def test_bottom_wall_mode_matches_stream_function(nx, ny, a0):
    u, om = _field(BW, _wall_mode(BW, nx, ny, a0))
    ref = _closed_form(BW, nx, ny, a0)
    assert np.max(np.abs(u - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("l0", [0.4, 2.5])
@pytest.mark.parametrize("nx,ny,a0", [(2, 0, (1.0, 0.0)), (1, -2, (0.7, -0.4))])
def test_bottom_wall_mode_with_slip_matches_stream_function(l0, nx, ny, a0):
    box = replace(BW, slip0=l0)
    u, _ = _field(box, _wall_mode(box, nx, ny, a0))
    ref = _closed_form(box, nx, ny, a0)
    assert np.max(np.abs(u - ref)) < 1e-11 * max(1.0, np.max(np.abs(ref)))


def test_bottom_wall_mode_vorticity():
    # u = U (1 - kz) e^{-kz} cos kx, w = U k z e^{-kz} sin kx:
    # (1/2) curl u has the y component -U k e^{-kz} cos kx
    U0, nx = 0.8, 2
    _, om = _field(BW, _wall_mode(BW, nx, 0, (U0, 0.0)))
    X, Y, Z = _grid(BW)
    k = 2 * np.pi * nx / BW.Lx
    ref = -U0 * k * np.exp(-k * Z) * np.cos(k * X)
    assert np.max(np.abs(om[1] - ref)) < 1e-9
    assert np.max(np.abs(om[0])) < 1e-12 and np.max(np.abs(om[2])) < 1e-12


@pytest.mark.parametrize("slip", [(0.0, 0.0), (0.5, 0.0), (0.3, 1.2)])
@pytest.mark.parametrize("nx,ny,a0,aH", [(2, 0, (1.0, 0.0), (0.0, 0.0)),
                                         (1, -1, (0.3, 0.6), (-0.5, 0.2)),
                                         (0, 2, (0.0, 0.0), (1.0, 0.4))])
def test_slit_channel_modes_match_stream_function(slip, nx, ny, a0, aH):
    box = replace(SC, slip0=slip[0], slipH=slip[1])
    u, _ = _field(box, _wall_mode(box, nx, ny, a0, aH))
    ref = _closed_form(box, nx, ny, a0, aH)
    assert np.max(np.abs(u - ref)) < 1e-11 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("geometry", ["bw", "sc"])
def test_wall_field_superposes_with_particles(geometry):
    box = BW if geometry == "bw" else SC
    rng = np.random.default_rng(5)
    alpha = 3 * box.Lx / box.Nx
    pos = np.column_stack([rng.uniform(0, box.Lx, 8), rng.uniform(0, box.Ly, 8),
                           rng.uniform(0.4, box.H - alpha - 0.1, 8)])
    F, T = rng.standard_normal((8, 3)), rng.standard_normal((8, 3))
    nw = 1 if geometry == "bw" else 2
    wall = rng.standard_normal((nw, 2, box.Ny, box.Nx))
    s = oracle.Solver(box)
    U1, O1 = s.apply(pos, F, T, wall=wall)
    U2, O2 = s.apply(pos, F, T)
    U3, O3 = s.apply(pos, 0 * F, 0 * T, wall=wall)
    np.testing.assert_allclose(U1, U2 + U3, atol=1e-12)
    np.testing.assert_allclose(O1, O2 + O3, atol=1e-12)
    assert np.linalg.norm(U3) > 1e-3


@pytest.mark.parametrize("geometry", ["bw", "sc"])
def test_uniform_field_equals_uniform_wall_velocity(geometry):
    box = BW if geometry == "bw" else SC
    rng = np.random.default_rng(6)
    pos = np.column_stack([rng.uniform(0, box.Lx, 5), rng.uniform(0, box.Ly, 5),
                           rng.uniform(1.0, 4.0, 5)])
    F, T = rng.standard_normal((5, 3)), rng.standard_normal((5, 3))
    w0, wH = (0.3, -0.2), ((0.0, 0.0) if geometry == "bw" else (0.1, 0.5))
    walls = [w0] if geometry == "bw" else [w0, wH]
    field = np.stack([np.stack([np.full((box.Ny, box.Nx), c) for c in w])
                      for w in walls])
    U1, O1 = oracle.Solver(box).apply(pos, F, T, wall=field)
    U2, O2 = oracle.Solver(replace(box, wall0=w0, wallH=wH)).apply(pos, F, T)
    np.testing.assert_allclose(U1, U2, atol=1e-12)
    np.testing.assert_allclose(O1, O2, atol=1e-12)


def test_nyquist_wall_mode_is_dropped():
    X, _, _ = _grid(BW)
    alt = np.cos(np.pi * np.arange(BW.Nx))[None, :] * np.ones((BW.Ny, 1))
    wall = np.stack([np.stack([alt, 0 * alt])])
    u, _ = _field(BW, wall)
    assert np.max(np.abs(u)) < 1e-13


def test_wall_shape_checked():
    with pytest.raises(ValueError):
        stokes.wall_spectrum(SC, np.zeros((1, 2, SC.Ny, SC.Nx)))
