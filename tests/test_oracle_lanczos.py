"""Pins for the oracle's Lanczos square root (Sec. 5.2).

The Krylov process is pinned on matrices whose square root is known
(eigendecomposition), on its exact termination for a matrix with few distinct
eigenvalues, and on the mobility itself: the converged result equals the
square root of the (symmetrised) dense translational mobility, and on the
replicated bottom-wall layer it converges to three digits within a few
applies (the paper's measure of convergence).
"""
import numpy as np
import pytest

import oracle
import workloads
from oracle import lanczos
from workloads import Box


def _sqrtm_apply(A, W):
    lam, Q = np.linalg.eigh(A)
    return Q @ (np.sqrt(lam) * (Q.T @ W))


def test_converges_to_the_matrix_square_root():
    rng = np.random.default_rng(3)
    n = 40
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.exp(rng.uniform(np.log(1e-2), 0.0, n))
    A = (Q * lam) @ Q.T
    W = rng.standard_normal(n)
    g, k, _ = lanczos.lanczos_sqrt(lambda x: A @ x, W, max_iter=n, tol=0.0)
    ref = _sqrtm_apply(A, W)
    assert np.linalg.norm(g - ref) / np.linalg.norm(ref) < 1e-10
    # fewer iterations: the error falls as the Krylov space grows
    errs = [np.linalg.norm(lanczos.lanczos_sqrt(lambda x: A @ x, W, m, 0.0)[0] - ref)
            for m in (4, 8, 16)]
    assert errs[0] > errs[1] > errs[2]


def test_terminates_exactly_on_few_eigenvalues():
    rng = np.random.default_rng(4)
    n = 30
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.repeat([0.5, 2.0, 7.0], n // 3)
    A = (Q * lam) @ Q.T
    W = rng.standard_normal(n)
    g, k, _ = lanczos.lanczos_sqrt(lambda x: A @ x, W, max_iter=20, tol=0.0)
    assert k == 3
    ref = _sqrtm_apply(A, W)
    assert np.linalg.norm(g - ref) / np.linalg.norm(ref) < 1e-12


def test_zero_vector():
    g, k, ch = lanczos.lanczos_sqrt(lambda x: x, np.zeros(6))
    assert k == 0 and not g.any()


@pytest.mark.parametrize("geometry", ["bw", "sc"])
def test_mobility_square_root_matches_dense(geometry):
    box = Box(geometry, 16.0, 16.0, 7.0, 16, 16, 16, w=4, beta_m=7.48,
              beta_d=7.48)
    rng = np.random.default_rng(5)
    n = 5
    zhi = 7.0 - 2.2 if geometry == "bw" else 6.5
    pos = np.column_stack([rng.uniform(0, 16, n), rng.uniform(0, 16, n),
                           rng.uniform(1.0, zhi, n)])
    s = oracle.Solver(box)
    mv = lanczos.translational_matvec(s, pos)
    M = np.column_stack([mv(e) for e in np.eye(3 * n)])
    S = 0.5 * (M + M.T)
    assert np.linalg.eigvalsh(S).min() > 0
    W = rng.standard_normal(3 * n)
    g, k, _ = lanczos.lanczos_sqrt(mv, W, max_iter=3 * n, tol=1e-12)
    ref = _sqrtm_apply(S, W)
    # M is symmetric to ~1e-4 at m = 4; the square roots agree to that level
    assert np.linalg.norm(g - ref) / np.linalg.norm(ref) < 2e-3


def test_replicated_layer_converges_to_three_digits():
    """The paper reports fewer than ten iterations for three digits on its
    roller layers (height distribution shown only in a figure); on this
    build's reading of the layer (a second layer at 3.3 R_h) the relative
    change reaches 1e-3 after 14 iterations (measured), well within 16."""
    wl = workloads.WORKLOADS["m2048"]
    pos, _, _ = workloads.particles("m2048")
    s = oracle.Solver(wl.box)
    W = workloads.random_array((wl.n, 3), 20)
    g, k, ch = lanczos.lanczos_sqrt(lanczos.translational_matvec(s, s.wrap(pos)),
                                    W, max_iter=16, tol=1e-3)
    assert ch < 1e-3 and k <= 16
