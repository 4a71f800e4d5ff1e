"""Fourier-Chebyshev Stokes solve, steps 2-7 of Sec. 3.4.

Input: the spread monopole density f_i and dipole (torque) density g_i at the
grid nodes (x_a, y_b, z_c), a = 0..Nx-1, b = 0..Ny-1, c = 0..Nz-1 (Chebyshev
extrema in z).  The body force is f + (1/2) curl g (eq. fcm); the curl is taken
spectrally (the paper's GPU route for torques).

Output: the fluid velocity u and half its vorticity, omega = (1/2) curl u, at
the nodes.

Conventions (readings): x_a = a*h with h = Lx/Nx (full periods Lx, Ly; the
paper's Sec. 2 writes the box as [-L, L], its later sections use L for the full
side); k = 2*pi*n/L with n in FFT order; the unnormalised forward DFT and an
inverse DFT normalised by 1/(Nx*Ny); the Nyquist row and column (n = -N/2)
are set to zero; eta defaults to 1.
"""
from __future__ import annotations

import numpy as np

from . import bvp, cheb


def wavenumbers(Lx, Ly, Nx, Ny):
    """k_x (Ny, Nx/2+1), k_y (Ny, Nx/2+1) and the Nyquist mask of rfft2."""
    nx = np.arange(Nx // 2 + 1)
    ny = np.fft.fftfreq(Ny, d=1.0 / Ny)
    kx = 2.0 * np.pi * nx / Lx
    ky = 2.0 * np.pi * ny / Ly
    KX, KY = np.meshgrid(kx, ky)
    nyq = np.zeros(KX.shape, dtype=bool)
    if Nx % 2 == 0:
        nyq[:, Nx // 2] = True
    if Ny % 2 == 0:
        nyq[Ny // 2, :] = True
    return KX, KY, nyq


def curl(ax, ay, az, ikx, iky, D):
    """Spectral curl (i k_x, i k_y, d/dz via the Chebyshev derivative D)."""
    return (iky * az - D(ay), D(ax) - ikx * az, ikx * ay - iky * ax)


def dp_solve(box, kx, ky, fx, fy, fz):
    """DP subproblem for k != 0 columns (Sec. 3.1, step 3 of Sec. 3.4).

    kx, ky: (K,) wavenumbers; fx, fy, fz: (K, Nz) Chebyshev coefficients of
    the body force.  Returns Chebyshev coefficients (p, u, v, w), each (K, Nz).
    """
    H, eta, Nz = box.H, box.eta, box.Nz
    alt = (-1.0) ** np.arange(Nz)
    Dz = lambda a: cheb.deriv(a, H, axis=-1)   # noqa: E731
    k = np.sqrt(kx ** 2 + ky ** 2)
    A = bvp.robin_matrices(0.5 * k * H, Nz)
    ikx = (1j * kx)[:, None]
    iky = (1j * ky)[:, None]
    # pressure: eq. poissonfs with the Dirichlet-to-Neumann maps eq. DtoNmapp
    rp = ikx * fx + iky * fy + Dz(fz)
    zero = np.zeros(k.size)
    p = bvp.solve(A, bvp.robin_rhs(rp, zero, zero, H))
    pH = p.sum(axis=-1)          # p(z = H): T_n(1) = 1 (direct summation)
    p0 = (p * alt).sum(axis=-1)  # p(z = 0): T_n(-1) = (-1)^n
    # velocities: eq. momentumfs with eqs. DtoNmapuv and DtoNmapw
    u = bvp.solve(A, bvp.robin_rhs((ikx * p - fx) / eta,
                                   -1j * kx * pH / (2 * k * eta),
                                   1j * kx * p0 / (2 * k * eta), H))
    v = bvp.solve(A, bvp.robin_rhs((iky * p - fy) / eta,
                                   -1j * ky * pH / (2 * k * eta),
                                   1j * ky * p0 / (2 * k * eta), H))
    w = bvp.solve(A, bvp.robin_rhs((Dz(p) - fz) / eta,
                                   pH / (2 * eta), p0 / (2 * eta), H))
    return p, u, v, w


def correction_nodes(box, kx, ky, u, v, w, wall=None):
    """Wall correction velocity at the Chebyshev nodes (step 4 of Sec. 3.4).

    u, v, w: (K, Nz) coefficients of the DP velocity.  Bottom wall: the
    closed form of Sec. 3.2 (eqs. usolfs-corr-final .. wsolfs-corr-final) with
    boundary data u_corr(0) = u^W - u_DP(0) (eq. bcnoslip0: the wall moves
    tangentially with u^W, w = 0).  Slit channel: App. A.  wall: None (walls
    at rest) or (4, K) xy-DFT coefficients of u^W, v^W at z = 0 and z = H
    (the last two unused for a bottom wall).

    Bottom wall with slip length l_0 (reading: the slit channel's condition
    at z = 0, eq. bcslip0, with only the decaying modes of eqs.
    psolfs-corr-sc .. wsolfs-corr-sc): u_corr = -(i k_x / k) B z e^{-kz} +
    C_x e^{-kz}, v likewise, w_corr = B z e^{-kz} + w_0 e^{-kz}, where
    B = C_0 / (2 eta).  The slip rows give (1 + k l_0) C_x + l_0 (i k_x / k)
    B = u_0 (v likewise) and continuity at z = 0 gives B + i k_x C_x +
    i k_y C_y - k w_0 = 0, so B = (k w_0 (1 + k l_0) - i (k_x u_0 + k_y
    v_0)) / (1 + 2 k l_0); l_0 = 0 is the closed form above.  The boundary
    data carry the slip term u_0 = u^W - u_DP(0) + l_0 du_DP/dz(0).
    """
    Nz = box.Nz
    _, zc = cheb.nodes(Nz, box.H)
    alt = (-1.0) ** np.arange(Nz)
    k = np.sqrt(kx ** 2 + ky ** 2)
    if box.geometry != "bw":
        return _slit_correction(box, kx, ky, k, u, v, w, zc, alt, wall)
    kk = k[:, None]
    em = np.exp(-kk * zc[None, :])            # e^{-kz}
    u0 = -(u * alt).sum(-1)
    v0 = -(v * alt).sum(-1)
    w0 = -(w * alt).sum(-1)
    if wall is not None:
        u0, v0 = u0 + wall[0], v0 + wall[1]
    l0 = box.slip0
    if l0:
        # du/dz at z = 0: (2/H) sum T_n'(-1) a_n, T_n'(-1) = (-1)^(n+1) n^2
        n2 = np.arange(Nz, dtype=float) ** 2
        d0 = lambda a: (2.0 / box.H) * (a * (-alt) * n2).sum(-1)   # noqa: E731
        u0 = u0 + l0 * d0(u)
        v0 = v0 + l0 * d0(v)
        Bs = (k * w0 * (1.0 + k * l0) - 1j * (kx * u0 + ky * v0)) / (1.0 + 2.0 * k * l0)
        Cx = (u0 - l0 * (1j * kx / k) * Bs) / (1.0 + k * l0)
        Cy = (v0 - l0 * (1j * ky / k) * Bs) / (1.0 + k * l0)
        ze = zc[None, :] * em
        uc = -(1j * kx / k * Bs)[:, None] * ze + Cx[:, None] * em
        vc = -(1j * ky / k * Bs)[:, None] * ze + Cy[:, None] * em
        wc = Bs[:, None] * ze + w0[:, None] * em
        return uc, vc, wc
    Acoef = (1j * k * w0 + kx * u0 + ky * v0)[:, None]
    ze = zc[None, :] * em
    uc = -(kx / k)[:, None] * Acoef * ze + u0[:, None] * em
    vc = -(ky / k)[:, None] * Acoef * ze + v0[:, None] * em
    wc = ((k * w0 - 1j * kx * u0 - 1j * ky * v0)[:, None] * ze
          + w0[:, None] * em)
    return uc, vc, wc


def _dp_and_correction(box, kx, ky, fx, fy, fz, wall=None, chunk=16384):
    """k != 0 columns: DP solve plus wall correction, added in coefficient
    space after a Chebyshev transform of the nodal correction (step 6).
    wall: None or (4, K) xy-DFT coefficients of the wall velocities
    (u^W, v^W at z = 0, then at z = H)."""
    K = kx.size
    Nz = box.Nz
    u = np.empty((K, Nz), complex)
    v = np.empty((K, Nz), complex)
    w = np.empty((K, Nz), complex)
    for lo in range(0, K, chunk):
        sl = slice(lo, min(K, lo + chunk))
        _, uu, vv, ww = dp_solve(box, kx[sl], ky[sl], fx[sl], fy[sl], fz[sl])
        uc, vc, wc = correction_nodes(box, kx[sl], ky[sl], uu, vv, ww,
                                      None if wall is None else wall[:, sl])
        u[sl] = uu + cheb.dct1(uc, axis=-1)
        v[sl] = vv + cheb.dct1(vc, axis=-1)
        w[sl] = ww + cheb.dct1(wc, axis=-1)
    return u, v, w


def _slit_correction(box, kx, ky, k, uu, vv, ww, zc, alt, wall=None):
    """Slit-channel correction with slip lengths l_0, l_H (App. A; no slip
    when both are zero) and wall velocities (wall: None, or the (4, K) xy-DFT
    coefficients of u^W, v^W at z = 0 and at z = H).

    Unknowns (C0, D0, Cx, Dx, Cy, Dy, Cz, Dz) of eqs. psolfs-corr-sc ..
    wsolfs-corr-sc from the six boundary conditions (eq. 6eqs-for-constants)
    and the two continuity conditions (eq. 2eqs-for-constants).  The boundary
    data are eq. u0uHformula: u_0 = u_0^W - u_DP(0) + l_0 du_DP/dz(0), u_H =
    u_H^W - u_DP(H) - l_H du_DP/dz(H), w_0 = -w_DP(0), w_H = -w_DP(H).  Reading: the
    D-coefficients are rescaled, D~ = D e^{kH}, so every matrix entry carries
    at most e^{-kH} <= 1 (rows scaled by e^{-kH} where needed).
    """
    H, eta = box.H, box.eta
    l0, lH = box.slip0, box.slipH
    Kc = k.size
    E = np.exp(-k * H)
    # z-derivatives at the walls: T_n'(+-1) = (+-1)^(n+1) n^2, d/dz = (2/H) d/ds
    n2 = np.arange(uu.shape[-1], dtype=float) ** 2
    d0 = lambda a: (2.0 / H) * (a * (-alt) * n2).sum(-1)   # noqa: E731
    dH = lambda a: (2.0 / H) * (a * n2).sum(-1)            # noqa: E731
    u0 = -(uu * alt).sum(-1) + l0 * d0(uu)
    v0 = -(vv * alt).sum(-1) + l0 * d0(vv)
    w0 = -(ww * alt).sum(-1)
    uH = -uu.sum(-1) - lH * dH(uu)
    vH = -vv.sum(-1) - lH * dH(vv)
    wH = -ww.sum(-1)
    if wall is not None:
        u0, v0, uH, vH = u0 + wall[0], v0 + wall[1], uH + wall[2], vH + wall[3]
    M = np.zeros((Kc, 8, 8), complex)
    b = np.zeros((Kc, 8), complex)
    C0, D0, CX, DX, CY, DY, CZ, DZ = range(8)
    one = np.ones(Kc)
    # u(0) - l_0 u'(0) = u0, v likewise; w(0) = w0
    for row, kk, rhs, Cc, Dc in ((0, kx, u0, CX, DX), (1, ky, v0, CY, DY)):
        c = 1j * kk * l0 / (2.0 * eta * k)
        M[:, row, C0] = c
        M[:, row, D0] = -c * E
        M[:, row, Cc] = 1.0 + k * l0
        M[:, row, Dc] = (1.0 - k * l0) * E
        b[:, row] = rhs
    M[:, 2, CZ], M[:, 2, DZ], b[:, 2] = one, E, w0
    # u(H) + l_H u'(H) = uH, v likewise
    for row, kk, rhs, Cc, Dc in ((3, kx, uH, CX, DX), (4, ky, vH, CY, DY)):
        c = 1j * kk * H / (2.0 * eta * k)
        M[:, row, C0] = c * E * (k * lH - lH / H - 1.0)
        M[:, row, D0] = c * (k * lH + lH / H + 1.0)
        M[:, row, Cc] = E * (1.0 - k * lH)
        M[:, row, Dc] = 1.0 + k * lH
        b[:, row] = rhs
    # w(H) = wH
    M[:, 5, C0] = H * E / (2.0 * eta)
    M[:, 5, D0] = H / (2.0 * eta)
    M[:, 5, CZ] = E
    M[:, 5, DZ] = one
    b[:, 5] = wH
    # continuity at z = 0 and z = H
    M[:, 6, C0] = 1.0 / (2.0 * eta)
    M[:, 6, D0] = E / (2.0 * eta)
    M[:, 6, CX], M[:, 6, DX] = 1j * kx, 1j * kx * E
    M[:, 6, CY], M[:, 6, DY] = 1j * ky, 1j * ky * E
    M[:, 6, CZ], M[:, 6, DZ] = -k, k * E
    M[:, 7, C0] = E / (2.0 * eta)
    M[:, 7, D0] = 1.0 / (2.0 * eta)
    M[:, 7, CX], M[:, 7, DX] = 1j * kx * E, 1j * kx
    M[:, 7, CY], M[:, 7, DY] = 1j * ky * E, 1j * ky
    M[:, 7, CZ], M[:, 7, DZ] = -k * E, k
    X = np.linalg.solve(M, b[..., None])[..., 0]
    kk = k[:, None]
    z = zc[None, :]
    em = np.exp(-kk * z)           # e^{-kz}
    ep = np.exp(kk * (z - H))      # e^{kz} e^{-kH}
    c0, d0 = X[:, C0:C0 + 1], X[:, D0:D0 + 1]
    ax = (1j * kx / (2.0 * eta * k))[:, None]
    ay = (1j * ky / (2.0 * eta * k))[:, None]
    uc = -c0 * ax * z * em + d0 * ax * z * ep + X[:, CX:CX + 1] * em + X[:, DX:DX + 1] * ep
    vc = -c0 * ay * z * em + d0 * ay * z * ep + X[:, CY:CY + 1] * em + X[:, DY:DY + 1] * ep
    wc = (c0 / (2 * eta)) * z * em + (d0 / (2 * eta)) * z * ep + X[:, CZ:CZ + 1] * em + X[:, DZ:DZ + 1] * ep
    return uc, vc, wc


def wall_spectrum(box, wall):
    """xy DFT (unnormalised, like the force densities) of tangential wall
    velocities given at the grid nodes of the walls.

    wall: (nw, 2, Ny, Nx) with (u^W, v^W) of the wall at z = 0 and, for the
    slit channel (nw = 2), of the wall at z = H.  Returns (4, Ny, Nx/2+1):
    u^W(0), v^W(0), u^W(H), v^W(H).  Reading: the Nyquist modes are dropped
    like those of the forcing (a field sampled on the grid resolves only
    |n| < N/2).
    """
    wall = np.asarray(wall, dtype=np.float64)
    nw = 2 if box.geometry == "sc" else 1
    if wall.shape != (nw, 2, box.Ny, box.Nx):
        raise ValueError(f"wall velocities have shape {(nw, 2, box.Ny, box.Nx)}")
    out = np.zeros((4, box.Ny, box.Nx // 2 + 1), complex)
    out[:2 * nw] = np.fft.rfft2(wall.reshape(2 * nw, box.Ny, box.Nx),
                                axes=(-2, -1))
    _, _, nyq = wavenumbers(box.Lx, box.Ly, box.Nx, box.Ny)
    return np.where(nyq[None], 0.0, out)


def solve_coefficients(box, Fh, Gh, wall_hat=None):
    """Steps 2 (derivative part) to 6 in coefficient space.

    Fh, Gh: complex (3, Nz, Ny, Nx/2+1) Fourier-Chebyshev coefficients of the
    monopole and dipole densities.  wall_hat: None, or wall_spectrum() of
    non-uniform wall velocities (they add to the uniform box.wall0/wallH).
    Returns (uh, omh) of the same shape.
    """
    H, Nz = box.H, box.Nz
    KX, KY, nyq = wavenumbers(box.Lx, box.Ly, box.Nx, box.Ny)
    Fh = np.where(nyq[None, None], 0.0, Fh)
    Gh = np.where(nyq[None, None], 0.0, Gh)
    ikx, iky = 1j * KX[None], 1j * KY[None]
    D = lambda a: cheb.deriv(a, H, axis=0)   # noqa: E731
    # body force f + (1/2) curl g (eq. fcm), spectral curl
    cg = curl(Gh[0], Gh[1], Gh[2], ikx, iky, D)
    fx, fy, fz = (Fh[i] + 0.5 * cg[i] for i in range(3))
    shape = Fh.shape[1:]
    col = lambda a: a.reshape(Nz, -1).T     # noqa: E731  (K, Nz) columns
    kx, ky = KX.ravel(), KY.ravel()
    k2 = kx ** 2 + ky ** 2
    live = (~nyq.ravel()) & (k2 > 0)
    U = [np.zeros((kx.size, Nz), complex) for _ in range(3)]
    cx, cy, cz = col(fx), col(fy), col(fz)
    idx = np.nonzero(live)[0]
    wl = None if wall_hat is None else wall_hat.reshape(4, -1)
    uu, vv, ww = _dp_and_correction(box, kx[idx], ky[idx], cx[idx], cy[idx],
                                    cz[idx], None if wl is None else wl[:, idx])
    U[0][idx], U[1][idx], U[2][idx] = uu, vv, ww
    # Step 5: k = 0 mode (Sec. 3.3; App. A.2 for the slit channel); w = 0.
    # Uniform wall velocities enter only here: the unnormalised xy DFT of a
    # constant c is c Nx Ny at k = 0; a non-uniform field adds its mean the
    # same way (its k = 0 coefficient).
    k0 = np.nonzero(k2 == 0)[0]
    nxy = box.Nx * box.Ny
    for j in k0:
        for c, cc in ((0, cx), (1, cy)):
            g0, gH = nxy * box.wall0[c], nxy * box.wallH[c]
            if wl is not None:
                g0, gH = g0 + wl[c, j].real, gH + wl[2 + c, j].real
            U[c][j] = bvp.zero_mode_solve(-cc[j] / box.eta, H, box.geometry,
                                          box.slip0, box.slipH, g0, gH)
    uh = np.stack([U[i].T.reshape(shape) for i in range(3)])
    # vorticity: omega = (1/2) curl u in Fourier-Chebyshev space
    cu = curl(uh[0], uh[1], uh[2], ikx, iky, D)
    omh = 0.5 * np.stack(cu)
    return uh, omh


def forward_transform(box, f):
    """Step 2: xy DFT (unnormalised) and Chebyshev transform in z."""
    return cheb.dct1(np.fft.rfft2(f, axes=(-2, -1)), axis=-3)


def inverse_transform(box, fh):
    """Step 7: inverse Chebyshev transform and inverse xy DFT."""
    return np.fft.irfft2(cheb.idct1(fh, axis=-3), s=(box.Ny, box.Nx),
                         axes=(-2, -1))


def stokes_solve(box, f, g, wall=None):
    """Velocity u and (1/2) curl u at the nodes from spread densities f, g
    (wall: optional non-uniform wall velocities, see wall_spectrum)."""
    Fh = forward_transform(box, f)
    Gh = forward_transform(box, g)
    uh, omh = solve_coefficients(box, Fh, Gh,
                                 None if wall is None else wall_spectrum(box, wall))
    return inverse_transform(box, uh), inverse_transform(box, omh)
