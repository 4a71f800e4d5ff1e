"""Pins for the oracle's whole mobility operator (Secs. 2-4).

Invariants the paper's construction fixes: linearity; adjointness of spreading
and interpolation under the trapezoid x Clenshaw-Curtis inner product;
invariance under integer-cell shifts and 90-degree rotations of a square box;
the slit channel's mirror symmetry about z = H/2 (so the translation-rotation
coupling vanishes at the midplane, Sec. 4.1); zero fluid velocity at the
wall(s); zero mobility of a particle on the wall (negative images,
eq. kernelnearwall); symmetry of the mobility matrix to about five digits
(Sec. 4); positive definiteness (Sec. 1); and the absolute scale: far from the
wall the self mobilities follow the classical point-particle wall series with
the Table 1 radius R_h = 1.731 h.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import stokes
from workloads import Box

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _setup(geometry="bw", n=6, seed=0, L=16.0, N=24, H=8.0, Nz=24):
    box = Box(geometry, L, L, H, N, N, Nz)
    rng = np.random.default_rng(seed)
    alpha = 3 * L / N
    zlo, zhi = (0.3, H - alpha - 0.1) if geometry == "bw" else (0.3, H - 0.3)
    pos = np.column_stack([rng.uniform(0, L, n), rng.uniform(0, L, n),
                           rng.uniform(zlo, zhi, n)])
    return box, oracle.Solver(box), pos, rng


def test_linearity():
    box, s, pos, rng = _setup()
    F1, T1, F2, T2 = (rng.standard_normal((6, 3)) for _ in range(4))
    U1, O1 = s.apply(pos, F1, T1)
    U2, O2 = s.apply(pos, F2, T2)
    U3, O3 = s.apply(pos, F1 + 2.0 * F2, T1 + 2.0 * T2)
    np.testing.assert_allclose(U3, U1 + 2 * U2, atol=1e-13)
    np.testing.assert_allclose(O3, O1 + 2 * O2, atol=1e-13)


@pytest.mark.parametrize("geometry", ["bw", "sc"])
def test_spread_interp_adjoint(geometry):
    box, s, pos, rng = _setup(geometry)
    F, T = rng.standard_normal((6, 3)), rng.standard_normal((6, 3))
    f, g = s.spread(pos, F, T)
    u = rng.standard_normal(f.shape)
    om = rng.standard_normal(g.shape)
    U, Om = s.interp(pos, u, om)
    q = (s.h ** 2) * s.wc[None, :, None, None]
    lhs = np.sum(F * U) + np.sum(T * Om)
    rhs = np.sum(q * f * u) + np.sum(q * g * om)
    assert lhs == pytest.approx(rhs, rel=1e-13)


@pytest.mark.parametrize("L,N,k", [(1448.0, 2176, 1071), (16.0, 24, 0)])
def test_particle_on_a_grid_node_keeps_both_support_edges(L, N, k):
    # x = k h exactly (h = 181/272 makes every 17th node of the 2176-node
    # grid an FP32 value; k = 0 sits on the periodic seam): the closed
    # support |t| <= alpha = 3h (eq. es) holds seven nodes, the two edge
    # nodes with the value e^{-beta}/norm, and the spread is symmetric
    box = Box("bw", L, L, 8.0, N, N, 16)
    s = oracle.Solver(box)
    x = np.array([k * (L / N)])
    assert x[0] / s.h == k
    idx, w = s._axis_weights(x, L, N, box.beta_m, s.norm_m)
    live = w[0] != 0.0
    assert live.sum() == 7
    got = dict(zip(idx[0][live] % N, w[0][live]))
    edge = np.exp(-box.beta_m) / s.norm_m
    for d in (3, -3):
        assert got[(k + d) % N] == pytest.approx(edge, rel=1e-12)
    for d in (1, 2, 3):
        assert got[(k + d) % N] == pytest.approx(got[(k - d) % N], rel=1e-13)


def test_integer_cell_shift_invariance():
    box, s, pos, rng = _setup("sc")
    F, T = rng.standard_normal((6, 3)), rng.standard_normal((6, 3))
    U, Om = s.apply(pos, F, T)
    sh = pos.copy()
    sh[:, 0] += 5 * s.h
    sh[:, 1] -= 7 * s.h
    U2, Om2 = s.apply(sh, F, T)
    np.testing.assert_allclose(U2, U, atol=1e-12)
    np.testing.assert_allclose(Om2, Om, atol=1e-12)


def test_quarter_turn_invariance():
    box, s, pos, rng = _setup("bw")
    F, T = rng.standard_normal((6, 3)), rng.standard_normal((6, 3))
    U, Om = s.apply(pos, F, T)
    R = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    rp = pos @ R.T
    U2, Om2 = s.apply(rp, F @ R.T, T @ R.T)        # proper rotation
    np.testing.assert_allclose(U2, U @ R.T, atol=1e-12)
    np.testing.assert_allclose(Om2, Om @ R.T, atol=1e-12)


def test_slit_mirror_symmetry_and_midplane_coupling():
    box, s, pos, rng = _setup("sc")
    F, T = rng.standard_normal((6, 3)), rng.standard_normal((6, 3))
    U, Om = s.apply(pos, F, T)
    M = np.diag([1.0, 1.0, -1.0])
    mp = pos.copy()
    mp[:, 2] = box.H - pos[:, 2]
    # F is a vector, tau a pseudovector: under z -> H - z, F_z and tau_x, tau_y flip
    U2, Om2 = s.apply(mp, F @ M, -(T @ M))
    np.testing.assert_allclose(U2, U @ M, atol=1e-12)
    np.testing.assert_allclose(Om2, -(Om @ M), atol=1e-12)
    # one particle at the midplane: torque about x gives no y velocity
    p1 = np.array([[3.3, 4.1, 0.5 * box.H]])
    U1, _ = s.apply(p1, np.zeros((1, 3)), np.array([[1.0, 0.0, 0.0]]))
    assert abs(U1[0, 1]) < 1e-14


@pytest.mark.parametrize("geometry", ["bw", "sc"])
def test_fluid_velocity_vanishes_at_walls(geometry):
    box, s, pos, rng = _setup(geometry)
    F, T = rng.standard_normal((6, 3)), rng.standard_normal((6, 3))
    f, g = s.spread(pos, F, T)
    u, om = stokes.stokes_solve(box, f, g)
    scale = np.abs(u).max()
    assert np.abs(u[:, -1]).max() < 1e-13 * scale        # z = 0 node
    if geometry == "sc":
        assert np.abs(u[:, 0]).max() < 1e-13 * scale     # z = H node


@pytest.mark.parametrize("geometry", ["bw", "sc"])
def test_particle_on_wall_does_not_move(geometry):
    box, s, pos, rng = _setup(geometry)
    pos[0, 2] = 0.0
    F, T = rng.standard_normal((6, 3)), rng.standard_normal((6, 3))
    U, Om = s.apply(pos, F, T)
    assert np.all(U[0] == 0.0) and np.all(Om[0] == 0.0)
    # and its force has no effect on the others
    F2 = F.copy()
    T2 = T.copy()
    F2[0] *= -3.0
    T2[0] *= 5.0
    U2, Om2 = s.apply(pos, F2, T2)
    np.testing.assert_allclose(U2, U, atol=1e-14)
    np.testing.assert_allclose(Om2, Om, atol=1e-14)


@pytest.mark.parametrize("geometry", ["bw", "sc"])
def test_mobility_symmetric_and_positive(geometry):
    box, s, pos, rng = _setup(geometry, n=4, seed=3, L=24.0, N=36, H=9.0, Nz=48)
    a = rng.standard_normal((2, 4, 3))
    b = rng.standard_normal((2, 4, 3))
    Ua, Oa = s.apply(pos, a[0], a[1])
    Ub, Ob = s.apply(pos, b[0], b[1])
    aMb = np.sum(a[0] * Ub) + np.sum(a[1] * Ob)
    bMa = np.sum(b[0] * Ua) + np.sum(b[1] * Oa)
    aMa = np.sum(a[0] * Ua) + np.sum(a[1] * Oa)
    # the discrete operator is symmetric only up to discretisation error;
    # measured 4e-6 (bw) and 1e-5 (sc) of a.M.a here ("five digits")
    assert abs(aMb - bMa) < 2e-5 * abs(aMa)
    assert aMa > 0


def test_far_from_wall_self_mobility_matches_wall_series():
    """Bottom wall, z = 10 h = 5.8 R_h, box 144 h: within 1% of the classical
    wall series for a sphere of radius R_h = 1.731 h (Table 1)."""
    with open(os.path.join(GOLD, "table1_es_m6.json")) as f:
        Rh = json.load(f)["Rh_over_h"]
    box = Box("bw", 144.0, 144.0, 30.0, 144, 144, 48)
    s = oracle.Solver(box)
    z = 10.0
    pos = np.array([[72.3, 72.17, z]])
    e = np.eye(3)
    Ux, _ = s.apply(pos, e[[0]], np.zeros((1, 3)))
    Uz, _ = s.apply(pos, e[[2]], np.zeros((1, 3)))
    _, Wx = s.apply(pos, np.zeros((1, 3)), e[[0]])
    a = Rh / z
    par = 1 - 9 / 16 * a + 1 / 8 * a ** 3 - 45 / 256 * a ** 4 - 1 / 16 * a ** 5
    perp = 1 - 9 / 8 * a + 1 / 2 * a ** 3
    rot = 1 - 5 / 16 * a ** 3
    assert Ux[0, 0] * 6 * np.pi * Rh == pytest.approx(par, rel=0.01)
    assert Uz[0, 2] * 6 * np.pi * Rh == pytest.approx(perp, rel=0.01)
    assert Wx[0, 0] * 8 * np.pi * Rh ** 3 == pytest.approx(rot, rel=0.005)
    # a wrong radius by 1% would already fail the rotation check
    assert abs(Wx[0, 0] * 8 * np.pi * (1.01 * Rh) ** 3 - rot) > 0.005 * rot
