"""Pins for the oracle's forces-only apply with kernel width m = 4 (Sec. 5).

The paper's one timed configuration applies forces only (the monopole
kernel, m = 4).  What fixes the oracle there: the ES kernel's partition of
unity on the grid; the far-from-wall self mobility against the classical
point-particle wall series with the radius that the paper's m = 4 table
(forces only) gives for its optimal beta; periodicity (a configuration tiled
k x k times on a k times larger box with the same grid spacing has the
one-replica solution repeated, which is how the tiled 663,552-particle layer
is checked); symmetry and positivity of the mobility; and the workload
generator's tiling itself.
"""
import numpy as np
import pytest

import oracle
import workloads
from oracle import kernel
from workloads import Box


@pytest.mark.parametrize("beta_over_m,tol", [(1.785, 2e-3), (1.87, 1e-3)])
def test_es_grid_partition_of_unity_m4(beta_over_m, tol):
    h = 1.0
    a = 2 * h
    beta = beta_over_m * 4
    I = kernel.es_normalization(a, beta)
    for x0 in np.linspace(0, h, 21):
        xi = h * np.arange(-10, 11)
        assert h * kernel.phi(xi - x0, a, beta, I).sum() == pytest.approx(1.0, abs=tol)


def test_self_mobility_m4_matches_wall_series():
    """Bottom wall, forces only, m = 4 and beta/m = 1.785 (the paper's
    optimum for m = 4 with forces only), z = 10 h: within 1% of the wall
    series for the tabulated radius R_h = 1.205 h, and outside 1% for a
    radius 1.7% larger or smaller."""
    Rh = 1.205
    box = Box("bw", 144.0, 144.0, 30.0, 144, 144, 48, w=4, beta_m=1.785 * 4,
              beta_d=1.785 * 4)
    s = oracle.Solver(box)
    z = 10.0
    pos = np.array([[72.3, 72.17, z]])
    e = np.eye(3)
    Ux, _ = s.apply(pos, e[[0]], np.zeros((1, 3)))
    Uz, _ = s.apply(pos, e[[2]], np.zeros((1, 3)))

    def series(R):
        a = R / z
        par = 1 - 9 / 16 * a + 1 / 8 * a ** 3 - 45 / 256 * a ** 4 - 1 / 16 * a ** 5
        perp = 1 - 9 / 8 * a + 1 / 2 * a ** 3
        return par / (6 * np.pi * R), perp / (6 * np.pi * R)

    par, perp = series(Rh)
    assert Ux[0, 0] == pytest.approx(par, rel=0.01)
    assert Uz[0, 2] == pytest.approx(perp, rel=0.01)
    for wrong in (0.983 * Rh, 1.017 * Rh):
        assert abs(Ux[0, 0] / series(wrong)[0] - 1) > 0.01


@pytest.mark.parametrize("geometry", ["bw", "sc"])
def test_tiled_configuration_gives_replicated_solution(geometry):
    """k x k copies of a configuration on a k times larger box with the same
    grid spacing: the forcing is periodic with the small box's period, so
    the discrete solution (and every particle's velocity) is the one-replica
    solution repeated, to rounding."""
    H = 6.0
    base = Box(geometry, 12.0, 12.0, H, 12, 12, 16, w=4, beta_m=1.87 * 4,
               beta_d=1.87 * 4)
    big = Box(geometry, 36.0, 36.0, H, 36, 36, 16, w=4, beta_m=1.87 * 4,
              beta_d=1.87 * 4)
    rng = np.random.default_rng(7)
    n = 5
    zhi = H - 2.1 if geometry == "bw" else H - 0.3
    pos = np.column_stack([rng.uniform(0, 12, n), rng.uniform(0, 12, n),
                           rng.uniform(0.3, zhi, n)])
    F = rng.standard_normal((n, 3))
    T = np.zeros((n, 3))
    U1, _ = oracle.Solver(base).apply(pos, F, T)
    ptile, Ftile, Ttile = workloads._tile(pos, F, T, 12.0, 12.0, 3)
    U3, _ = oracle.Solver(big).apply(ptile, Ftile, Ttile)
    np.testing.assert_allclose(U3, np.tile(U1, (9, 1)),
                               atol=1e-12 * np.abs(U1).max())


@pytest.mark.parametrize("geometry", ["bw", "sc"])
def test_forces_only_mobility_symmetric_and_positive(geometry):
    box = Box(geometry, 24.0, 24.0, 9.0, 24, 24, 32, w=4, beta_m=1.87 * 4,
              beta_d=1.87 * 4)
    s = oracle.Solver(box)
    rng = np.random.default_rng(11)
    n = 4
    zhi = 9.0 - 2.1 if geometry == "bw" else 8.7
    pos = np.column_stack([rng.uniform(0, 24, n), rng.uniform(0, 24, n),
                           rng.uniform(0.5, zhi, n)])
    a, b = rng.standard_normal((2, n, 3))
    zero = np.zeros((n, 3))
    Ua, _ = s.apply(pos, a, zero)
    Ub, _ = s.apply(pos, b, zero)
    aMa = np.sum(a * Ua)
    # symmetric only up to discretisation error; measured 2.7e-4 (bw) and
    # 5.4e-4 (sc) of a.M.a here, about the same at Nz = 64 (the m = 4 kernel
    # is cut off where it is still e^-7.5 ~ 6e-4 of its peak)
    assert abs(np.sum(a * Ub) - np.sum(b * Ua)) < 2e-3 * aMa
    assert aMa > 0


def test_m663k_layer_is_the_m2048_replica_tiled_exactly():
    p1, F1, T1 = workloads.particles("m2048")
    p2, F2, T2 = workloads.particles("m663k")
    r = workloads.M_REPLICAS
    assert len(p2) == r * r * len(p1) == 663552
    d = p2.reshape(r * r, len(p1), 3) - p1[None]
    # whole periods in x and y, same heights and forces; no torques
    assert np.all(np.mod(d[:, :, :2], 150.0) == 0) and np.all(d[:, :, 2] == 0)
    assert np.array_equal(F2.reshape(r * r, -1, 3), np.broadcast_to(F1, (r * r,) + F1.shape))
    assert not T1.any() and not T2.any()
    # float32-exact (the mixed path reads the same numbers as the oracle)
    assert np.array_equal(p2.astype(np.float32).astype(np.float64), p2)
    wl = workloads.WORKLOADS["m663k"]
    alpha = wl.box.w * wl.box.h / 2
    assert p2[:, 2].min() > 0 and p2[:, 2].max() + alpha < wl.box.H
    # area fraction N pi R_h^2 / L^2 of the paper's replicated layer (~0.4)
    assert 2048 * np.pi * workloads.M_RH ** 2 / 150.0 ** 2 == pytest.approx(0.388, abs=0.002)
