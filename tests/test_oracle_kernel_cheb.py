"""Pins for the oracle's ES kernel (Sec. 3.5) and Chebyshev machinery (Sec. 3.4).

Each check compares against something other than the oracle itself: an
independent quadrature (scipy), closed forms, or NumPy's Chebyshev module.
"""
import json
import os

import numpy as np
import pytest
from numpy.polynomial import chebyshev as C
from scipy import integrate

from oracle import cheb, kernel

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _quad_norm(alpha, beta):
    f = lambda t: np.exp(beta * (np.sqrt(max(0.0, 1 - (t / alpha) ** 2)) - 1))  # noqa: E731
    return integrate.quad(f, -alpha, alpha, epsabs=1e-13, epsrel=1e-13, limit=200)[0]


@pytest.mark.parametrize("alpha,beta", [(2.0, 7.962), (2.0, 13.296), (1.0, 4.0),
                                        (3.5, 20.0), (0.7, 1.0)])
def test_es_normalization_matches_adaptive_quadrature(alpha, beta):
    assert kernel.es_normalization(alpha, beta) == pytest.approx(
        _quad_norm(alpha, beta), rel=1e-12)


def test_es_phi_shape():
    a, b = 2.0, 7.962
    I = kernel.es_normalization(a, b)
    t = np.linspace(-2.5, 2.5, 1001)
    p = kernel.phi(t, a, b, I)
    np.testing.assert_array_equal(p, kernel.phi(-t, a, b, I))  # even
    assert kernel.phi(0.0, a, b, I) == pytest.approx(1.0 / I)
    assert np.all(p[np.abs(t) > a] == 0.0)                    # compact support
    # inclusive edge |t| = alpha: e^{-beta}/I, not zero
    assert kernel.phi(a, a, b, I) == pytest.approx(np.exp(-b) / I, rel=1e-14)
    # unit integral by an independent rule
    tt = np.linspace(-a, a, 200001)
    assert integrate.simpson(kernel.phi(tt, a, b, I), x=tt) == pytest.approx(1.0, abs=2e-6)


def test_es_grid_partition_of_unity():
    """h sum_i phi(x_i - x0) ~ 1 at the paper's Table 1 parameters (m = 6)."""
    h = 2.0 / 3.0
    a = 3 * h
    for beta, tol in ((7.962, 1e-3), (13.296, 1e-5)):
        I = kernel.es_normalization(a, beta)
        for x0 in np.linspace(0, h, 11):
            xi = h * np.arange(-10, 11)
            assert h * kernel.phi(xi - x0, a, beta, I).sum() == pytest.approx(1.0, abs=tol)


def test_table1_parameters_golden():
    with open(os.path.join(GOLD, "table1_es_m6.json")) as f:
        t1 = json.load(f)
    import workloads
    assert workloads.BETA_M == pytest.approx(t1["m"] * t1["betaM_over_m"])
    assert workloads.BETA_D == pytest.approx(t1["m"] * t1["betaD_over_m"])


@pytest.mark.parametrize("Nz", [8, 17, 32, 48])
def test_dct1_exact_on_chebyshev_polynomials(Nz):
    s, _ = cheb.nodes(Nz, 5.0)
    for n in range(Nz):
        f = np.cos(n * np.arccos(s))
        a = cheb.dct1(f)
        e = np.zeros(Nz)
        e[n] = 1.0
        np.testing.assert_allclose(a, e, atol=1e-13)
    x = np.random.default_rng(0).standard_normal((Nz, 3))
    np.testing.assert_allclose(cheb.idct1(cheb.dct1(x)), x, atol=1e-13)


def test_nodes_orientation():
    s, z = cheb.nodes(32, 12.0)
    assert z[0] == pytest.approx(12.0) and z[-1] == pytest.approx(0.0, abs=1e-14)
    assert np.all(np.diff(z) < 0)


@pytest.mark.parametrize("Nz,H", [(9, 1.0), (32, 12.0), (48, 10.0)])
def test_clenshaw_curtis_exact_on_polynomials(Nz, H):
    _, z = cheb.nodes(Nz, H)
    w = cheb.cc_weights(Nz, H)
    for p in range(Nz):
        assert w @ z ** p == pytest.approx(H ** (p + 1) / (p + 1), rel=1e-12)
    assert np.all(w > 0)


@pytest.mark.parametrize("N,H", [(8, 2.0), (32, 12.0), (48, 10.0)])
def test_derivative_matches_numpy_chebder(N, H):
    a = np.random.default_rng(1).standard_normal(N)
    ref = np.zeros(N)
    ref[: N - 1] = C.chebder(a) * (2.0 / H)
    np.testing.assert_allclose(cheb.deriv(a, H), ref, rtol=1e-12, atol=1e-10)


def test_integration_operators_match_numpy_chebint():
    N = 20
    a = np.random.default_rng(2).standard_normal(N)
    a[-2:] = 0.0          # degree N-3 so that antiderivatives fit in N terms
    ref = C.chebint(a)[:N]
    mine = cheb.integ_B(N) @ a
    np.testing.assert_allclose(mine[1:], ref[1:], atol=1e-14)   # row 0 free
    ref2 = C.chebint(a, 2)[:N]
    np.testing.assert_allclose((cheb.b2_matrix(N) @ a)[2:], ref2[2:], atol=1e-14)
    # B^2 undoes two derivatives in rows m >= 2 (exact for degree N-1)
    y = np.random.default_rng(3).standard_normal(N)
    y2 = np.zeros(N)
    y2[: N - 2] = C.chebder(y, 2)
    np.testing.assert_allclose((cheb.b2_matrix(N) @ y2)[2:], y[2:], atol=1e-12)
