"""Pins for the oracle's per-wavenumber solves (Secs. 3.1-3.3, App. A).

* manufactured Robin BVP solutions converge spectrally (discretisation);
* k = 0 closed forms (double integrals) for both geometries;
* the DP solution of one Fourier mode agrees with the whole-line Green's
  function convolution computed by brute-force quadrature (this pins the
  Dirichlet-to-Neumann maps, eqs. DtoNmapp, DtoNmapuv, DtoNmapw);
* the wall corrections enforce no slip and incompressibility;
* torque-only forcing is divergence free (zero pressure source).
"""
import numpy as np
import pytest

from oracle import bvp, cheb, stokes
from workloads import Box


def _y(z):
    g = np.exp(-(z - 3.0) ** 2)
    gp = -2.0 * (z - 3.0) * g
    gpp = (4.0 * (z - 3.0) ** 2 - 2.0) * g
    y = g * np.cos(z)
    yp = gp * np.cos(z) - g * np.sin(z)
    ypp = gpp * np.cos(z) - 2.0 * gp * np.sin(z) - g * np.cos(z)
    return y, yp, ypp


def test_robin_bvp_manufactured_spectral_convergence():
    H, k = 8.0, 0.9
    errs = []
    for Nz in (16, 24, 32, 48, 64):
        _, z = cheb.nodes(Nz, H)
        y, yp, ypp = _y(z)
        r = cheb.dct1(ypp - k * k * y)
        yH, ypH, _ = _y(np.array([H]))
        y0, yp0, _ = _y(np.array([0.0]))
        A = bvp.robin_matrices(np.array([0.5 * k * H]), Nz)
        b = bvp.robin_rhs(r[None].astype(complex), ypH + k * yH, yp0 - k * y0, H)
        sol = bvp.solve(A, b)[0]
        errs.append(np.max(np.abs(cheb.idct1(sol).real - y)))
    assert errs[0] > errs[2] > errs[-1]
    assert errs[-1] < 1e-11


@pytest.mark.parametrize("geometry", ["bw", "sc"])
def test_zero_mode_closed_forms(geometry):
    H, Nz = 6.0, 24
    _, z = cheb.nodes(Nz, H)
    P = np.polynomial.Polynomial
    f = P([0.3, -1.0, 0.5, 0.2])             # f(z), cubic
    sol = bvp.zero_mode_solve(-cheb.dct1(f(z)).astype(complex), H, geometry)
    if geometry == "bw":
        # u(z) = int_0^z int_{z'}^H f dz'' dz'
        F1 = f.integ()
        inner = F1(H) - F1                     # int_{z'}^H f
        ref = inner.integ()(z) - inner.integ()(0.0)
    else:
        # u(z) = (z/H) int_0^H (H - z') f dz' - int_0^z (z - z') f dz'
        zz = P([0, 1])
        c = ((H - zz) * f).integ()
        A = (c(H) - c(0.0)) / H
        ref = A * z - np.array([((zi - zz) * f).integ()(zi) - ((zi - zz) * f).integ()(0.0)
                                for zi in z])
    np.testing.assert_allclose(cheb.idct1(sol).real, ref, atol=1e-12)


# --- DP solve vs whole-line Green's function ---------------------------------

_GL = np.polynomial.legendre.leggauss(160)


def _gauss_legendre(a, b):
    x, w = _GL
    return 0.5 * (b - a) * x + 0.5 * (b + a), 0.5 * (b - a) * w


def _conv(z, src, k, H, deriv=False):
    """int_0^H G(z - z') src(z') dz' with G = -e^{-k|z|}/(2k) (or dG/dz)."""
    out = np.zeros(len(z), complex)
    for i, zi in enumerate(z):
        for a, b in ((0.0, zi), (zi, H)):
            if b - a <= 0:
                continue
            x, w = _gauss_legendre(a, b)
            d = zi - x
            if deriv:
                g = 0.5 * np.sign(d) * np.exp(-k * np.abs(d))
            else:
                g = -np.exp(-k * np.abs(d)) / (2 * k)
            out[i] += np.sum(w * g * src(x))
    return out


def test_dp_solve_matches_whole_line_green_function():
    H, eta = 8.0, 1.0
    kx, ky = 0.7, -0.4
    k = np.hypot(kx, ky)
    cx, cy, cz = 0.8 + 0.3j, -0.5 + 1.1j, 0.4 - 0.7j
    bump = lambda z: np.exp(-(z - 4.0) ** 2 / 0.6)               # noqa: E731
    dbump = lambda z: -2.0 * (z - 4.0) / 0.6 * bump(z)          # noqa: E731
    fx = lambda z: cx * bump(z)                                   # noqa: E731
    fy = lambda z: cy * bump(z)                                   # noqa: E731
    fz = lambda z: cz * bump(z)                                   # noqa: E731
    s = lambda z: 1j * kx * fx(z) + 1j * ky * fy(z) + cz * dbump(z)  # noqa: E731
    p = lambda z: _conv(np.atleast_1d(z), s, k, H)                 # noqa: E731
    dp = lambda z: _conv(np.atleast_1d(z), s, k, H, deriv=True)    # noqa: E731
    p0, pH = p(0.0)[0], p(H)[0]

    Nz = 64       # spectral convergence: 2.5e-5, 2.5e-9, 2e-14 at Nz = 32, 48, 64
    _, zc = cheb.nodes(Nz, H)
    box = Box("bw", 10.0, 10.0, H, 8, 8, Nz)
    F = [cheb.dct1(g(zc))[None] for g in (fx, fy, fz)]
    pp, uu, vv, ww = stokes.dp_solve(box, np.array([kx]), np.array([ky]), *F)
    np.testing.assert_allclose(cheb.idct1(pp[0]), p(zc), atol=1e-10, rtol=0)

    # u: whole-line source (i kx p - fx)/eta; p continues as p0 e^{kz} below 0
    # and pH e^{-k(z-H)} above H (closed-form tails of the convolution).
    ru = lambda z: (1j * kx * p(z) - fx(z)) / eta                 # noqa: E731
    uref = (_conv(zc, ru, k, H)
            - 1j * kx * p0 / (2 * k * eta) * np.exp(-k * zc) / (2 * k)
            - 1j * kx * pH / (4 * k * k * eta) * np.exp(-k * (H - zc)))
    np.testing.assert_allclose(cheb.idct1(uu[0]), uref, atol=1e-10, rtol=0)
    rw = lambda z: (dp(z) - fz(z)) / eta                          # noqa: E731
    wref = (_conv(zc, rw, k, H)
            - k * p0 / (2 * k * eta) * np.exp(-k * zc) / (2 * k)
            + k * pH / (4 * k * k * eta) * np.exp(-k * (H - zc)))
    np.testing.assert_allclose(cheb.idct1(ww[0]), wref, atol=1e-10, rtol=0)


# --- corrections -----------------------------------------------------------

def _random_column(Nz, H, seed):
    rng = np.random.default_rng(seed)
    _, zc = cheb.nodes(Nz, H)
    amp = rng.standard_normal((3, 2)) @ np.array([1.0, 1j])
    bump = np.exp(-(zc - 0.45 * H) ** 2 / 1.5)
    return [cheb.dct1(a * bump)[None] for a in amp]


@pytest.mark.parametrize("geometry", ["bw", "sc"])
@pytest.mark.parametrize("kxy", [(0.05, 0.02), (0.7, -0.4), (3.0, 2.5)])
def test_correction_enforces_no_slip_and_continuity(geometry, kxy):
    H, Nz = 10.0, 48
    box = Box(geometry, 10.0, 10.0, H, 8, 8, Nz)
    kx, ky = np.array([kxy[0]]), np.array([kxy[1]])
    F = _random_column(Nz, H, 7)
    _, u, v, w = stokes.dp_solve(box, kx, ky, *F)
    uc, vc, wc = stokes.correction_nodes(box, kx, ky, u, v, w)
    tot = [a + cheb.dct1(c, axis=-1) for a, c in ((u, uc), (v, vc), (w, wc))]
    alt = (-1.0) ** np.arange(Nz)
    scale = max(np.abs(a).max() for a in (u, v, w))
    for a in tot:
        assert abs((a[0] * alt).sum()) < 1e-12 * scale          # no slip at z = 0
        if geometry == "sc":
            assert abs(a[0].sum()) < 1e-12 * scale              # no slip at z = H
    # the correction field alone is divergence free (up to its interpolation
    # error on the grid, tiny for these smooth fields)
    Dz = lambda a: cheb.deriv(a, H, axis=-1)   # noqa: E731
    cu, cv, cw = (cheb.dct1(c, axis=-1) for c in (uc, vc, wc))
    div = 1j * kx[:, None] * cu + 1j * ky[:, None] * cv + Dz(cw)
    cscale = max(np.abs(c).max() for c in (cu, cv, cw))
    assert np.abs(div).max() < 1e-9 * cscale


def test_slit_correction_reduces_to_bottom_wall_for_large_kH():
    H, Nz = 10.0, 48
    kx, ky = np.array([2.4]), np.array([1.8])      # kH = 30
    F = _random_column(Nz, H, 3)
    bw = Box("bw", 10.0, 10.0, H, 8, 8, Nz)
    sc = Box("sc", 10.0, 10.0, H, 8, 8, Nz)
    _, u, v, w = stokes.dp_solve(bw, kx, ky, *F)
    cb = stokes.correction_nodes(bw, kx, ky, u, v, w)
    cs = stokes.correction_nodes(sc, kx, ky, u, v, w)
    _, zc = cheb.nodes(Nz, H)
    lower = zc < 0.5 * H
    for a, b in zip(cb, cs):
        np.testing.assert_allclose(b[0][lower], a[0][lower], atol=1e-6 * np.abs(a).max())


def test_torque_only_body_force_is_divergence_free():
    H, Nz = 8.0, 32
    rng = np.random.default_rng(11)
    G = rng.standard_normal((3, Nz)) + 1j * rng.standard_normal((3, Nz))
    kx, ky = 0.6, -1.3
    D = lambda a: cheb.deriv(a, H)   # noqa: E731
    fx, fy, fz = (0.5 * c for c in stokes.curl(G[0], G[1], G[2], 1j * kx, 1j * ky, D))
    div = 1j * kx * fx + 1j * ky * fy + D(fz)
    assert np.abs(div).max() < 1e-13 * np.abs(G).max()
