"""Exponential-of-semicircle (ES) envelope, Sec. 3.5, eqs. (es) and (es-scalar).

phi(t; alpha, beta) = exp(beta*(sqrt(1-(t/alpha)^2) - 1)) / I   for |t| <= alpha
                    = 0                                          otherwise,
I = integral over [-alpha, alpha] of the unnormalised envelope.

The support is inclusive (|t/alpha| <= 1, as printed).  alpha = w*h/2 with w
the number of grid cells in the support (Sec. 3.5: "we typically take
alpha = hm/2").
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def es_normalization(alpha: float, beta: float, npts: int = 200) -> float:
    """I(alpha, beta) by Gauss-Legendre quadrature after t = alpha*sin(theta).

    With t = alpha sin(theta) the integrand becomes
    alpha * exp(beta (cos theta - 1)) cos theta on [-pi/2, pi/2], which is
    analytic, so Gauss-Legendre converges exponentially.
    """
    x, wq = np.polynomial.legendre.leggauss(npts)
    theta = 0.5 * np.pi * x
    f = np.exp(beta * (np.cos(theta) - 1.0)) * np.cos(theta)
    return float(alpha * 0.5 * np.pi * np.sum(wq * f))


def phi(t, alpha: float, beta: float, norm: float):
    """Normalised scalar ES kernel evaluated elementwise (float64)."""
    t = np.asarray(t, dtype=np.float64)
    r = t / alpha
    inside = np.abs(t) <= alpha
    one_minus_r2 = np.where(inside, (1.0 - r) * (1.0 + r), 0.0)
    return np.where(inside, np.exp(beta * (np.sqrt(one_minus_r2) - 1.0)) / norm,
                    0.0)


@dataclass(frozen=True)
class ESKernel:
    """Monopole (M) and dipole (D) ES envelopes sharing the support alpha."""
    alpha: float
    beta_m: float
    beta_d: float

    @property
    def norm_m(self) -> float:
        return es_normalization(self.alpha, self.beta_m)

    @property
    def norm_d(self) -> float:
        return es_normalization(self.alpha, self.beta_d)

    def phi_m(self, t):
        return phi(t, self.alpha, self.beta_m, self.norm_m)

    def phi_d(self, t):
        return phi(t, self.alpha, self.beta_d, self.norm_d)
