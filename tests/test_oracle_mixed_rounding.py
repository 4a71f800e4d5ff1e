"""Where the mixed-precision error of the slit channel comes from: FP32
rounding emulated inside the FP64 oracle (CPU only).

The mixed path stores the spread densities, their xy spectra and their
Chebyshev coefficients in FP32.  Here the oracle's FP64 values of one channel
are rounded to FP32 after the spread, after the xy DFT and after the
Chebyshev transform (single roundings, the least the FP32 path does), on
sub-boxes of the 1448 x 1448 x 12 monolayer with the same density, grid
spacing and gap, and the resulting velocities are compared with the
unrounded oracle:

* rounding the vertical force f_z costs far more than rounding a horizontal
  force channel (the roller layer's f_z is large and its rough-in-z rounding
  noise meets the slit channel's strong small-kH response);
* at a fixed number of particles that error grows as the box gets longer,
  i.e. as its smallest kH falls (0.42 in a 181 x 181 box, 0.10 in 724 x 45):
  it is set by the smallest wavenumbers, so it keeps growing with the box
  (kH = 0.052 at 1448 x 1448);
* taking f_z of the columns with |nx|, |ny| <= ceil(L / (2 pi H)) (every
  kH < 1) without rounding removes most of it -- the FP64 route of the mixed
  slit channel.

Measured here (norm-wise over U, N = 16384): f_z rounded 2.9e-7 (181 x 181),
2.0e-6 (362 x 90.5), 6.2e-6 (724 x 45.25); f_x rounded 1e-9 in all three.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import cheb, fcm, stokes


def _r32(a):
    if np.iscomplexobj(a):
        return a.astype(np.complex64).astype(np.complex128)
    return a.astype(np.float32).astype(np.float64)


class _Case:
    """One sub-box: spread and transforms once, then solves per variant."""

    def __init__(self, fx, fy):
        box, pos, F, T = workloads.sub_box("sc1m", fx, fy)
        self.box = box
        self.s = fcm.Solver(box)
        self.pos = self.s.wrap(pos)
        f, g = self.s.spread(self.pos, F, T)
        self.grid = np.concatenate([f, g])
        self.coef = cheb.dct1(np.fft.rfft2(self.grid, axes=(-2, -1)), axis=1)
        self.ref = self._finish(self.coef)

    def _finish(self, coef):
        uh, omh = stokes.solve_coefficients(self.box, coef[:3], coef[3:])
        u = stokes.inverse_transform(self.box, uh)
        om = stokes.inverse_transform(self.box, omh)
        return self.s.interp(self.pos, u, om)

    def rounded(self, ch):
        """Chebyshev coefficients of channel ch after single FP32 roundings of
        its grid values, its xy spectrum and its coefficients."""
        spec = _r32(np.fft.rfft2(_r32(self.grid[ch]), axes=(-2, -1)))
        return _r32(cheb.dct1(spec, axis=0))

    def error(self, ch, exact_ns=None):
        coef = self.coef.copy()
        rc = self.rounded(ch)
        if exact_ns is not None:
            b = self.box
            nx = np.arange(b.Nx // 2 + 1)[None, :]
            ny = np.fft.fftfreq(b.Ny, d=1.0 / b.Ny)[:, None]
            sq = (nx <= exact_ns) & (np.abs(ny) <= exact_ns)
            rc = np.where(sq[None], self.coef[ch], rc)
        coef[ch] = rc
        U, _ = self._finish(coef)
        return float(np.linalg.norm(U - self.ref[0]) / np.linalg.norm(self.ref[0]))


@pytest.fixture(scope="module")
def cases():
    # 16384 particles each: 181 x 181 (272^2 grid) and 724 x 45.25 (1088 x 68)
    return {"square": _Case(8, 8), "long": _Case(2, 32)}


def test_vertical_force_rounding_dominates_and_grows(cases):
    e_sq = cases["square"].error(2)
    e_long = cases["long"].error(2)
    e_fx = cases["long"].error(0)
    print(f"f_z rounded: 181 x 181 {e_sq:.2e}, 724 x 45 {e_long:.2e}; "
          f"f_x rounded (724 x 45) {e_fx:.2e}")
    # f_z against f_x: more than two orders of magnitude
    assert e_long > 100 * e_fx
    # same particle count and density, smaller kH: several times the error
    assert e_long > 5.0 * e_sq


def test_low_wavenumber_square_carries_the_vertical_force_error(cases):
    c = cases["long"]
    ns = math.ceil(max(c.box.Lx, c.box.Ly) / (2 * math.pi * c.box.H) - 1e-12)
    full = c.error(2)
    outside = c.error(2, exact_ns=ns)
    print(f"ns = {ns}: f_z rounded everywhere {full:.2e}, outside the square "
          f"{outside:.2e}")
    assert outside < full / 10
