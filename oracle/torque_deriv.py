"""Torques through the derivative of the ES kernel (Sec. 3.4, last paragraph,
and its two footnotes) -- the second way the paper gives to spread torques and
interpolate angular velocities, without the dipole density and without a
spectral curl.

Spread (eq. fcm, the curl moved onto the kernel): the force density is

    f(x) = sum_j F_j Delta_M(x - r_j) + (1/2) grad Delta_D(x - r_j) x tau_j,

(curl(tau Delta) = grad(Delta) x tau for a constant tau).  Interpolation
(eq. getpartvort, integrated by parts; the wall term vanishes because u = 0
where Delta_D does not):

    Omega_j = (1/2) int curl(u) Delta_D  =  (1/2) int u x grad Delta_D,

with the same trapezoid x Clenshaw-Curtis quadrature as the linear
velocity.  Spreading and interpolation are therefore adjoint.

The kernel derivative (footnotes):
* grad Delta_D uses a different scalar function along each axis:
  (phi'(x) phi(y) psi(z), phi(x) phi'(y) psi(z), phi(x) phi(y) psi'(z)).
* phi' is unbounded at the edge of the support; it is set to zero for
  |t| > t*, the point beyond its maximum where |phi'| is smallest.  With
  r = t / alpha and s = sqrt(1 - r^2), d/dr log(r e^{beta (s - 1)} / s) = 0
  reduces to beta s^3 - beta s + 1 = 0; t* = alpha sqrt(1 - s*^2) with s*
  the smaller of its two roots in (0, 1) (the larger is the maximum).
* Near a wall the z derivative's mirror image enters with a positive sign:
  the mirror of phi'(z - z_j) is phi'(-z - z_j) = -phi'(z + z_j), and adding
  it gives psi'(z) = phi'(z - z_j) - phi'(z + z_j) (minus phi'(z - (2H - z_j))
  for the slit channel's top wall), the z derivative of the folded kernel
  psi itself, which vanishes with psi when the particle sits on the wall.
"""
from __future__ import annotations

import numpy as np

from . import fcm, stokes
from .kernel import phi


def truncation_point(alpha: float, beta: float) -> float:
    """t* of the truncated derivative (footnote reading above)."""
    roots = np.roots([beta, 0.0, -beta, 1.0])
    s = np.sort([r.real for r in roots if abs(r.imag) < 1e-12 and 0 < r.real < 1])
    if len(s) == 0:          # |phi'| has no interior minimum: keep the support
        return alpha
    return alpha * float(np.sqrt(1.0 - s[0] ** 2))


def dphi(t, alpha: float, beta: float, norm: float, tstar: float):
    """phi'(t), truncated to zero for |t| > t* (elementwise, float64)."""
    t = np.asarray(t, dtype=np.float64)
    keep = np.abs(t) <= tstar
    r = np.where(keep, t / alpha, 0.0)
    s = np.sqrt(np.where(keep, (1.0 - r) * (1.0 + r), 1.0))
    val = phi(np.where(keep, t, 0.0), alpha, beta, norm) * beta * (-r / alpha) / s
    return np.where(keep, val, 0.0)


class DerivativeSolver(fcm.Solver):
    """The mobility apply with torques spread, and angular velocities
    interpolated, through the derivative of the dipole ES kernel."""

    def __init__(self, box):
        super().__init__(box)
        self.tstar = truncation_point(self.alpha, box.beta_d)

    def _axis_dweights(self, x, L, N):
        """Indices (P, 9), phi_D and its truncated derivative on a 9-point
        window around x (derivative with respect to the grid coordinate)."""
        h = self.h
        u = x / h
        a = np.floor(u)[:, None] + np.arange(-4, 5)[None, :]
        t = (a - u[:, None]) * h      # node offset, as in fcm.Solver
        b = self.box
        return (a.astype(np.int64) % N, phi(t, self.alpha, b.beta_d, self.norm_d),
                dphi(t, self.alpha, b.beta_d, self.norm_d, self.tstar))

    def _z_dweights(self, z):
        """Folded psi_D and its z derivative psi_D' on all nodes, (P, Nz)."""
        b = self.box
        zc = self.zc[None, :]
        zj = z[:, None]
        args = [(zc - zj, 1.0), (zc + zj, -1.0)]
        if b.geometry == "sc":
            args.append((zc - (2.0 * b.H - zj), -1.0))
        psi = sum(sg * phi(t, self.alpha, b.beta_d, self.norm_d) for t, sg in args)
        dpsi = sum(sg * dphi(t, self.alpha, b.beta_d, self.norm_d, self.tstar)
                   for t, sg in args)
        return psi, dpsi

    def _grad_stencil(self, pos):
        """Flat indices and the three components of grad Delta_D, each
        (P, Nz, 9, 9)."""
        b = self.box
        ia, px, dpx = self._axis_dweights(pos[:, 0], b.Lx, b.Nx)
        ib, py, dpy = self._axis_dweights(pos[:, 1], b.Ly, b.Ny)
        psi, dpsi = self._z_dweights(pos[:, 2])
        c = np.arange(b.Nz)
        idx = ((c[None, :, None, None] * b.Ny + ib[:, None, :, None]) * b.Nx
               + ia[:, None, None, :])
        gx = psi[:, :, None, None] * py[:, None, :, None] * dpx[:, None, None, :]
        gy = psi[:, :, None, None] * dpy[:, None, :, None] * px[:, None, None, :]
        gz = dpsi[:, :, None, None] * py[:, None, :, None] * px[:, None, None, :]
        return idx, (gx, gy, gz)

    def spread_forces(self, pos, F, T, chunk=1024):
        """Force density f = sum F Delta_M + (1/2) grad Delta_D x tau,
        shape (3, Nz, Ny, Nx)."""
        b = self.box
        size = b.Nz * b.Ny * b.Nx
        out = np.zeros((3, size))
        for lo in range(0, pos.shape[0], chunk):
            sl = slice(lo, lo + chunk)
            idx, wgt = self._stencil(pos[sl], "m")
            for i in range(3):
                out[i] += np.bincount(idx.ravel(),
                                      weights=(wgt * F[sl, i][:, None, None, None]).ravel(),
                                      minlength=size)
            idx, (gx, gy, gz) = self._grad_stencil(pos[sl])
            tx, ty, tz = (T[sl, i][:, None, None, None] for i in range(3))
            # (1/2) grad Delta x tau
            comp = (0.5 * (gy * tz - gz * ty), 0.5 * (gz * tx - gx * tz),
                    0.5 * (gx * ty - gy * tx))
            for i in range(3):
                out[i] += np.bincount(idx.ravel(), weights=comp[i].ravel(),
                                      minlength=size)
        return out.reshape(3, b.Nz, b.Ny, b.Nx)

    def interp_velocities(self, pos, u, chunk=1024):
        """U = h^2 sum w u Delta_M and Omega = (1/2) h^2 sum w u x grad Delta_D."""
        b = self.box
        P = pos.shape[0]
        U = np.zeros((P, 3))
        Om = np.zeros((P, 3))
        quad = (self.h * self.h * self.wc)[None, :, None, None]
        uf = u.reshape(3, -1)
        for lo in range(0, P, chunk):
            sl = slice(lo, lo + chunk)
            idx, wgt = self._stencil(pos[sl], "m")
            wq = wgt * quad
            for i in range(3):
                U[sl, i] = np.sum(uf[i][idx] * wq, axis=(1, 2, 3))
            idx, (gx, gy, gz) = self._grad_stencil(pos[sl])
            ux, uy, uz = (uf[i][idx] * quad for i in range(3))
            Om[sl, 0] = 0.5 * np.sum(uy * gz - uz * gy, axis=(1, 2, 3))
            Om[sl, 1] = 0.5 * np.sum(uz * gx - ux * gz, axis=(1, 2, 3))
            Om[sl, 2] = 0.5 * np.sum(ux * gy - uy * gx, axis=(1, 2, 3))
        return U, Om

    def velocity_field(self, f):
        """Fluid velocity at the nodes from the force density f (no dipole
        density, no vorticity)."""
        Fh = stokes.forward_transform(self.box, f)
        uh, _ = stokes.solve_coefficients(self.box, Fh, np.zeros_like(Fh))
        return stokes.inverse_transform(self.box, uh)

    def apply(self, pos, F, T, sample=None):
        pos = self.wrap(pos)
        f = self.spread_forces(pos, np.asarray(F, float), np.asarray(T, float))
        u = self.velocity_field(f)
        tgt = pos if sample is None else pos[sample]
        return self.interp_velocities(tgt, u)
