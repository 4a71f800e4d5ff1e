"""Pins for the oracle's slit channel with partial slip (App. A).

Slip lengths l_0, l_H enter the correction's boundary rows (eq.
6eqs-for-constants), its boundary data (eq. u0uHformula) and the k = 0 mode
(eq. bvp-uv-k0-sc).  What fixes them: the total velocity field satisfies
u - l_0 du/dz = 0 at z = 0 and u + l_H du/dz = 0 at z = H (and w = 0) for
every Fourier mode, to rounding; l = 0 gives the no-slip operator; the
k = 0 mode matches the closed-form solution of y'' = r with Robin
conditions; the mobility stays symmetric and positive, and more slip lets a
particle move faster parallel to the walls.
"""
import numpy as np
import pytest
from dataclasses import replace

import oracle
from oracle import bvp, cheb, stokes
from workloads import Box

BOX = Box("sc", 16.0, 16.0, 7.0, 24, 24, 24)


def _particles(n=6, seed=0):
    rng = np.random.default_rng(seed)
    pos = np.column_stack([rng.uniform(0, 16, n), rng.uniform(0, 16, n),
                           rng.uniform(0.4, 6.6, n)])
    return pos, rng.standard_normal((n, 3)), rng.standard_normal((n, 3))


@pytest.mark.parametrize("l0,lH", [(0.5, 2.0), (3.0, 0.0), (0.0, 1.0)])
def test_total_field_satisfies_the_slip_conditions(l0, lH):
    box = replace(BOX, slip0=l0, slipH=lH)
    s = oracle.Solver(box)
    pos, F, T = _particles()
    f, g = s.spread(s.wrap(pos), F, T)
    Fh = stokes.forward_transform(box, f)
    Gh = stokes.forward_transform(box, g)
    uh, _ = stokes.solve_coefficients(box, Fh, Gh)        # (3, Nz, Ny, Nkx)
    N = box.Nz
    n = np.arange(N)
    n2 = n.astype(float) ** 2
    alt = np.where(n % 2 == 0, 1.0, -1.0)
    at0 = lambda a: np.tensordot(alt, a, axes=(0, 0))               # noqa: E731
    atH = lambda a: a.sum(axis=0)                                   # noqa: E731
    d0 = lambda a: (2 / box.H) * np.tensordot(-alt * n2, a, axes=(0, 0))  # noqa: E731
    dH = lambda a: (2 / box.H) * np.tensordot(n2, a, axes=(0, 0))   # noqa: E731
    # values at the walls are exact (the walls are nodes of the interpolated
    # correction); its derivative there differs from the analytic one by
    # the interpolation error of e^{-kz} at the largest k (measured 3e-9 of
    # the field's scale at Nz = 24): a wrong sign or factor of l gives O(1)
    scale = np.abs(uh).max()
    for c in (0, 1):
        assert np.abs(at0(uh[c]) - l0 * d0(uh[c])).max() < 1e-7 * scale
        assert np.abs(atH(uh[c]) + lH * dH(uh[c])).max() < 1e-7 * scale
    assert np.abs(at0(uh[2])).max() < 1e-12 * scale
    assert np.abs(atH(uh[2])).max() < 1e-12 * scale


def test_zero_slip_is_no_slip():
    pos, F, T = _particles(seed=1)
    U0, O0 = oracle.Solver(BOX).apply(pos, F, T)
    U1, O1 = oracle.Solver(replace(BOX, slip0=0.0, slipH=0.0)).apply(pos, F, T)
    assert np.array_equal(U0, U1) and np.array_equal(O0, O1)


def test_zero_mode_robin_closed_form():
    """y'' = 1 on [0, H] with y(0) - l0 y'(0) = 0, y(H) + lH y'(H) = 0:
    y = z^2/2 + a z + b with b = l0 a and H^2/2 + a H + b + lH (H + a) = 0."""
    H, l0, lH, N = 5.0, 0.7, 1.3, 16
    rhs = np.zeros(N)
    rhs[0] = 1.0
    y = bvp.zero_mode_solve(rhs.astype(complex), H, "sc", l0, lH).real
    a = -(H * H / 2 + lH * H) / (H + l0 + lH)
    b = l0 * a
    _, zc = cheb.nodes(N, H)
    got = cheb.eval_series(y, 2 * zc / H - 1)
    np.testing.assert_allclose(got, zc ** 2 / 2 + a * zc + b, atol=1e-12)


def test_slip_mobility_symmetric_positive_and_faster():
    pos = np.array([[5.3, 7.1, 2.2], [9.0, 8.4, 4.1], [12.2, 3.3, 3.0]])
    rng = np.random.default_rng(4)
    a, b = rng.standard_normal((2, 3, 3))
    z = np.zeros((3, 3))
    s = oracle.Solver(replace(BOX, slip0=1.0, slipH=1.0))
    Ua, _ = s.apply(pos, a, z)
    Ub, _ = s.apply(pos, b, z)
    aMa = np.sum(a * Ua)
    assert aMa > 0
    assert abs(np.sum(a * Ub) - np.sum(b * Ua)) < 1e-4 * aMa
    # one particle pulled along x: slip walls resist less than no-slip ones
    e = np.zeros((3, 3))
    e[0, 0] = 1.0
    U_ns, _ = oracle.Solver(BOX).apply(pos, e, z)
    U_sl, _ = s.apply(pos, e, z)
    assert U_sl[0, 0] > U_ns[0, 0] * 1.01


def test_couette_flow_between_moving_walls():
    """No particles forcing (F = T = 0), walls moving at U0 and UH: the grid
    velocity is the linear profile (exactly, at the nodes) and a particle
    away from the walls moves with the fluid at its height (to the kernel's
    quadrature accuracy); with slip the profile is u(z) = a z + b with
    b - l0 a = U0 and a H + b + lH a = UH."""
    for l0, lH in ((0.0, 0.0), (0.8, 1.5)):
        box = replace(BOX, wall0=(0.3, -0.2), wallH=(1.0, 0.5), slip0=l0,
                      slipH=lH)
        s = oracle.Solver(box)
        pos = np.array([[5.1, 6.2, 3.5], [11.3, 2.4, 2.9], [8.8, 13.1, 4.2]])
        z = np.zeros((3, 3))
        f, g = s.spread(s.wrap(pos), z, z)
        uh, _ = stokes.solve_coefficients(box, stokes.forward_transform(box, f),
                                          stokes.forward_transform(box, g))
        u = stokes.inverse_transform(box, uh)
        for c in (0, 1):
            U0, UH = box.wall0[c], box.wallH[c]
            a = (UH - U0) / (box.H + l0 + lH)
            b = U0 + l0 * a
            prof = a * s.zc + b
            np.testing.assert_allclose(u[c], prof[:, None, None] + 0 * u[c],
                                       atol=1e-12)
        U, _ = s.apply(pos, z, z)
        for c in (0, 1):
            U0, UH = box.wall0[c], box.wallH[c]
            a = (UH - U0) / (box.H + l0 + lH)
            np.testing.assert_allclose(U[:, c], a * pos[:, 2] + U0 + l0 * a,
                                       rtol=2e-3, atol=2e-3)
        assert np.abs(U[:, 2]).max() < 1e-12


def test_bottom_wall_moving():
    """A bottom wall moving at U0 under an open top drags the whole fluid:
    u = U0 everywhere (y'' = 0, y(0) = U0, y'(H) = 0)."""
    box = Box("bw", 16.0, 16.0, 8.0, 24, 24, 24, wall0=(0.7, 0.0))
    s = oracle.Solver(box)
    pos = np.array([[5.1, 6.2, 3.5]])
    z = np.zeros((1, 3))
    U, _ = s.apply(pos, z, z)
    assert U[0, 0] == pytest.approx(0.7, rel=2e-3) and abs(U[0, 1]) < 1e-12


# --- bottom wall with a slip length (the slit channel's condition at z = 0
# with the decaying modes only) ----------------------------------------------

BW = Box("bw", 16.0, 16.0, 8.0, 24, 24, 24)


@pytest.mark.parametrize("l0", [0.5, 3.0])
def test_bottom_wall_total_field_satisfies_the_slip_condition(l0):
    box = replace(BW, slip0=l0)
    s = oracle.Solver(box)
    rng = np.random.default_rng(21)
    pos = np.column_stack([rng.uniform(0, 16, 6), rng.uniform(0, 16, 6),
                           rng.uniform(0.4, 5.5, 6)])
    F, T = rng.standard_normal((6, 3)), rng.standard_normal((6, 3))
    f, g = s.spread(s.wrap(pos), F, T)
    uh, _ = stokes.solve_coefficients(box, stokes.forward_transform(box, f),
                                      stokes.forward_transform(box, g))
    n = np.arange(box.Nz)
    alt = np.where(n % 2 == 0, 1.0, -1.0)
    at0 = lambda a: np.tensordot(alt, a, axes=(0, 0))               # noqa: E731
    d0 = lambda a: (2 / box.H) * np.tensordot(-alt * n.astype(float) ** 2, a,
                                              axes=(0, 0))          # noqa: E731
    scale = np.abs(uh).max()
    for c in (0, 1):
        assert np.abs(at0(uh[c]) - l0 * d0(uh[c])).max() < 1e-7 * scale
    assert np.abs(at0(uh[2])).max() < 1e-12 * scale


def test_bottom_wall_zero_mode_robin_closed_form():
    """y'' = 1 on [0, H] with y(0) - l0 y'(0) = 0 and y'(H) = 0:
    y = z^2/2 - H z - l0 H."""
    H, l0, N = 5.0, 0.7, 16
    rhs = np.zeros(N)
    rhs[0] = 1.0
    y = bvp.zero_mode_solve(rhs.astype(complex), H, "bw", l0, 0.0).real
    _, zc = cheb.nodes(N, H)
    got = cheb.eval_series(y, 2 * zc / H - 1)
    np.testing.assert_allclose(got, zc ** 2 / 2 - H * zc - l0 * H, atol=1e-12)


def test_bottom_wall_slip_mobility_symmetric_positive_and_faster():
    pos = np.array([[5.3, 7.1, 2.2], [9.0, 8.4, 4.1], [12.2, 3.3, 3.0]])
    rng = np.random.default_rng(5)
    a, b = rng.standard_normal((2, 3, 3))
    z = np.zeros((3, 3))
    s = oracle.Solver(replace(BW, slip0=1.5))
    Ua, _ = s.apply(pos, a, z)
    Ub, _ = s.apply(pos, b, z)
    aMa = np.sum(a * Ua)
    assert aMa > 0
    assert abs(np.sum(a * Ub) - np.sum(b * Ua)) < 1e-4 * aMa
    e = np.zeros((3, 3))
    e[0, 0] = 1.0
    U_ns, _ = oracle.Solver(BW).apply(pos, e, z)
    U_sl, _ = s.apply(pos, e, z)
    assert U_sl[0, 0] > U_ns[0, 0] * 1.01


def test_bottom_wall_slip_length_at_the_top_is_refused():
    with pytest.raises(ValueError):
        oracle.Solver(replace(BW, slipH=1.0))
