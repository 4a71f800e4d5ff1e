"""Spreading, interpolation and the whole FCM mobility apply (Secs. 2, 3.4).

Spread (step 1 of Sec. 3.4, eq. fcm with the wall images of eq.
kernelnearwall):

    f_i(x_a, y_b, z_c) = sum_j F_{j,i} phi_M(x_a - x_j) phi_M(y_b - y_j) psi_M(z_c; z_j)
    g_i(x_a, y_b, z_c) = sum_j tau_{j,i} phi_D(...) phi_D(...) psi_D(z_c; z_j)

with x and y offsets taken as minimum images (periodic box) and the folded z
kernel psi(z_c; z_j) = phi(z_c - z_j) - phi(z_c + z_j) (image about z = 0;
the slit channel also subtracts phi(z_c - (2H - z_j)), the image about
z = H).  The image is applied to every particle: for z_j > alpha it
contributes nothing on [0, H], which is the paper's "z_j < z_im" rule with
z_im = alpha.  The body force is f + (1/2) curl g.

Interpolation (step 8, eqs. getpartvel and getpartvort, trapezoid rule in
x, y and Clenshaw-Curtis in z):

    U_j     = h^2 sum_{a,b,c} w_c u(x_a, y_b, z_c) phi_M phi_M psi_M
    Omega_j = h^2 sum_{a,b,c} w_c omega(x_a, y_b, z_c) phi_D phi_D psi_D

with omega = (1/2) curl u.
"""
from __future__ import annotations

import numpy as np

from . import cheb, stokes
from .kernel import ESKernel


class Solver:
    """Derived quantities of one box/grid/kernel choice (Sec. 3.4, 3.5)."""

    def __init__(self, box):
        self.box = box
        if abs(box.Lx / box.Nx - box.Ly / box.Ny) > 1e-12 * box.Lx / box.Nx:
            raise ValueError("the oracle requires hx == hy")
        if box.slip0 < 0 or box.slipH < 0:
            raise ValueError("slip lengths are >= 0")
        if box.geometry == "bw" and box.slipH:
            raise ValueError("a bottom wall has no slip length at z = H")
        if box.geometry == "bw" and any(box.wallH):
            raise ValueError("a bottom wall has no wall at z = H")
        self.h = box.Lx / box.Nx
        self.alpha = 0.5 * box.w * self.h        # alpha = m h / 2 (Sec. 3.5)
        self.kernel = ESKernel(self.alpha, box.beta_m, box.beta_d)
        self.norm_m = self.kernel.norm_m
        self.norm_d = self.kernel.norm_d
        self.s, self.zc = cheb.nodes(box.Nz, box.H)
        self.wc = cheb.cc_weights(box.Nz, box.H)

    # --- per-particle separable weights ---------------------------------
    def _axis_weights(self, x, L, N, beta, norm):
        """Indices (P, 9) and kernel values on a 9-point window around x.

        The support |t| <= alpha = 3h holds at most 7 grid points; the
        9-point window contains it for any rounding of floor(x/h).  The
        node offset t = x_a - x is taken as (a - x/h) h: a - x/h is exact in
        floating point (a and x/h agree to a few units), so a particle lying
        exactly on a grid node keeps both edge nodes |t| = alpha of the
        closed support (eq. es).  Periodicity acts on the index only.
        """
        h = self.h
        u = x / h
        i0 = np.floor(u)
        a = i0[:, None] + np.arange(-4, 5)[None, :]
        t = (a - u[:, None]) * h
        from .kernel import phi
        return a.astype(np.int64) % N, phi(t, self.alpha, beta, norm)

    def _z_weights(self, z, beta, norm):
        """Folded z kernel psi(z_c; z_j) on all nodes, shape (P, Nz)."""
        from .kernel import phi
        zc = self.zc[None, :]
        zj = z[:, None]
        psi = phi(zc - zj, self.alpha, beta, norm) - phi(zc + zj, self.alpha, beta, norm)
        if self.box.geometry == "sc":
            psi = psi - phi(zc - (2.0 * self.box.H - zj), self.alpha, beta, norm)
        return psi

    def _stencil(self, pos, which):
        b = self.box
        beta, norm = ((b.beta_m, self.norm_m) if which == "m"
                      else (b.beta_d, self.norm_d))
        ia, wx = self._axis_weights(pos[:, 0], b.Lx, b.Nx, beta, norm)
        ib, wy = self._axis_weights(pos[:, 1], b.Ly, b.Ny, beta, norm)
        psi = self._z_weights(pos[:, 2], beta, norm)
        c = np.arange(b.Nz)
        idx = ((c[None, :, None, None] * b.Ny + ib[:, None, :, None]) * b.Nx
               + ia[:, None, None, :])
        wgt = psi[:, :, None, None] * wy[:, None, :, None] * wx[:, None, None, :]
        return idx, wgt

    # --- step 1 ------------------------------------------------------------
    def spread(self, pos, F, T, chunk=2048):
        """Monopole density f and dipole density g, each (3, Nz, Ny, Nx)."""
        b = self.box
        size = b.Nz * b.Ny * b.Nx
        out = np.zeros((6, size))
        for lo in range(0, pos.shape[0], chunk):
            sl = slice(lo, lo + chunk)
            for which, vec, off in (("m", F, 0), ("d", T, 3)):
                idx, wgt = self._stencil(pos[sl], which)
                nz = wgt != 0.0
                flat_idx = idx[nz]
                for i in range(3):
                    val = (wgt * vec[sl, i][:, None, None, None])[nz]
                    out[off + i] += np.bincount(flat_idx, weights=val,
                                                minlength=size)
        out = out.reshape(6, b.Nz, b.Ny, b.Nx)
        return out[:3], out[3:]

    # --- step 8 ------------------------------------------------------------
    def interp(self, pos, u, om, chunk=2048):
        """Particle velocities U and angular velocities Omega, each (P, 3)."""
        b = self.box
        P = pos.shape[0]
        U = np.zeros((P, 3))
        Om = np.zeros((P, 3))
        quad = self.h * self.h * self.wc        # trapezoid x Clenshaw-Curtis
        uf = u.reshape(3, -1)
        of = om.reshape(3, -1)
        for lo in range(0, P, chunk):
            sl = slice(lo, lo + chunk)
            for which, field, out in (("m", uf, U), ("d", of, Om)):
                idx, wgt = self._stencil(pos[sl], which)
                wq = wgt * quad[None, :, None, None]
                for i in range(3):
                    out[sl, i] = np.sum(field[i][idx] * wq, axis=(1, 2, 3))
        return U, Om

    def wrap(self, pos):
        """Wrap x and y into [0, L) (periodic directions)."""
        p = np.array(pos, dtype=np.float64, copy=True)
        p[:, 0] = np.mod(p[:, 0], self.box.Lx)
        p[:, 1] = np.mod(p[:, 1], self.box.Ly)
        return p

    def apply(self, pos, F, T, sample=None, wall=None):
        """The mobility apply (F, T) -> (U, Omega) (eq. grandmob).

        ``sample``: optional index array; only those particles are
        interpolated (every particle is still spread).  ``wall``: optional
        tangential wall velocities at the walls' grid nodes, shape
        (nw, 2, Ny, Nx) (eq. bcnoslip0; App. A, eq. u0uHformula).
        """
        pos = self.wrap(pos)
        f, g = self.spread(pos, np.asarray(F, float), np.asarray(T, float))
        u, om = stokes.stokes_solve(self.box, f, g, wall)
        del f, g
        tgt = pos if sample is None else pos[sample]
        return self.interp(tgt, u, om)


def apply_mobility(box, pos, F, T, sample=None):
    """Convenience wrapper: Solver(box).apply(pos, F, T)."""
    return Solver(box).apply(pos, F, T, sample=sample)
