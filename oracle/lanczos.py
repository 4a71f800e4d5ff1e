"""Brownian displacements g = M^{1/2} W by the Lanczos process (Sec. 5.2).

Test infrastructure (see the package docstring).  The paper generates
Brownian velocities with a Krylov (Lanczos) approximation of the square root
of the mobility matrix, and measures convergence by the relative change
eps_k = |g_k - g_{k-1}| / |g_{k-1}| between iterations.  The process, for a
symmetric positive definite M and a vector W:

    v_0 = W / |W|
    for j = 0, 1, ...:
        w = M v_j - beta_{j-1} v_{j-1}           (no second term for j = 0)
        alpha_j = v_j . w
        w = w - sum_{i <= j} (v_i . w) v_i       (removes alpha_j v_j; done
                                                  twice, Gram-Schmidt)
        beta_j = |w|,  v_{j+1} = w / beta_j
        g_{j+1} = |W| V_{j+1} T_{j+1}^{1/2} e_1

with T_k the k x k tridiagonal matrix with alpha on the diagonal and beta
beside it.  In exact arithmetic the orthogonalisation against the older
basis vectors removes nothing; it keeps a low-precision basis orthonormal.
The matrix square root of T_k is taken from its eigendecomposition
(numpy.linalg.eigh), eigenvalues below zero (rounding) set to zero.
"""
from __future__ import annotations

import numpy as np


def sqrt_e1(alpha, beta, nrm):
    """|W| T^{1/2} e_1 for the tridiagonal T(alpha, beta)."""
    k = len(alpha)
    T = np.diag(np.asarray(alpha, float))
    if k > 1:
        b = np.asarray(beta[:k - 1], float)
        T += np.diag(b, 1) + np.diag(b, -1)
    lam, Q = np.linalg.eigh(T)
    return nrm * (Q @ (np.sqrt(np.maximum(lam, 0.0)) * Q[0, :]))


def lanczos_sqrt(matvec, W, max_iter=32, tol=1e-3):
    """(g, iterations, last relative change) for g ~ M^{1/2} W, where
    matvec(x) = M x on flat float64 vectors."""
    W = np.asarray(W, float).ravel()
    nrm = np.linalg.norm(W)
    if nrm == 0.0:
        return np.zeros_like(W), 0, 0.0
    V = [W / nrm]
    alpha, beta = [], []
    y_prev, change, k = None, 0.0, 0
    for j in range(max_iter):
        w = matvec(V[j])
        if j > 0:
            w = w - beta[j - 1] * V[j - 1]
        Vm = np.array(V)
        c = Vm @ w
        alpha.append(c[j])
        w = w - Vm.T @ c
        c = Vm @ w
        w = w - Vm.T @ c
        beta.append(np.linalg.norm(w))
        k = j + 1
        y = sqrt_e1(alpha, beta, nrm)
        if k > 1:
            yp = np.append(y_prev, 0.0)
            change = np.linalg.norm(y - yp) / np.linalg.norm(y_prev)
            if change < tol:
                break
        y_prev = y
        if beta[-1] <= 1e-13 * abs(alpha[0]):
            break
        V.append(w / beta[-1])
    return np.array(V[:k]).T @ y, k, change


def translational_matvec(solver, pos):
    """x -> U for forces x (flattened [n][3]) and no torques: the forces-only
    mobility apply of ``fcm.Solver``."""
    n = len(pos)
    zero = np.zeros((n, 3))

    def mv(x):
        U, _ = solver.apply(pos, x.reshape(n, 3), zero)
        return U.ravel()
    return mv
