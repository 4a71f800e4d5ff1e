"""GPU parity of the derivative-kernel torque route (Sec. 3.4, last paragraph
and its footnotes): torques spread as (1/2) grad Delta_D x tau and angular
velocities interpolated as (1/2) sum u x grad Delta_D, three channels through
the transforms and the solve, against the oracle's DerivativeSolver."""
from dataclasses import replace

import numpy as np
import pytest

import workloads
from workloads import Box

from _parity import particle_err, rel_err
from oracle import torque_deriv

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

BOXES = {
    "bw48": Box("bw", 32.0, 32.0, 8.0, 48, 48, 32, torque_route="derivative"),
    "sc40x56": Box("sc", 20.0, 28.0, 7.0, 40, 56, 24, torque_route="derivative"),
}


def _solver(box, precision, cap):
    from paper_2210_01837_amd import Solver
    return Solver.from_box(box, precision=precision, max_particles=cap)


def _dev(a, precision):
    dt = torch.float64 if precision == "fp64" else torch.float32
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def _particles(box, n, seed):
    alpha = 3 * box.h
    zhi = box.H - alpha - 0.05 if box.geometry == "bw" else box.H - 0.2
    pos, F, T = workloads.random_particles(box, n, seed, 0.2, zhi)
    pos[0, :2] = [box.Lx - 1e-3, 0.3]
    pos[1, :2] = [0.2, box.Ly - 0.7 * box.h]
    pos[2, 2] = 0.4 * alpha
    if box.geometry == "sc":
        pos[3, 2] = box.H - 0.3 * alpha
    return pos, F, T


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", list(BOXES))
def test_apply_against_oracle(name, precision):
    box = BOXES[name]
    pos, F, T = _particles(box, 300, 81)
    if precision == "mixed":
        pos, F, T = (a.astype(np.float32).astype(np.float64) for a in (pos, F, T))
    print(f"[torque derivative] {name} {precision}", flush=True)
    rU, rO = torque_deriv.DerivativeSolver(box).apply(pos, F, T)
    s = _solver(box, precision, 512)
    U, Om = s.apply(_dev(pos, precision), _dev(F, precision), _dev(T, precision))
    U, Om = _np(U), _np(Om)
    eU, eO = rel_err(U, rU), rel_err(Om, rO)
    pU, pO = particle_err(U, rU), particle_err(Om, rO)
    print(f"  rel err U {eU:.2e} Omega {eO:.2e}; max particle {pU:.2e} {pO:.2e}",
          flush=True)
    tol = 1e-10 if precision == "fp64" else 1e-5
    assert eU < tol and eO < tol and pU < 10 * tol and pO < 10 * tol
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_channel_modes_and_forces_only(precision):
    # the route changes only what torques and Omega do: a forces-only apply
    # gives the curl route's bits, and U does not depend on whether Omega is
    # requested
    box = BOXES["sc40x56"]
    pos, F, T = _particles(box, 200, 82)
    P, Fd, Td = (_dev(a, precision) for a in (pos, F, T))
    sd = _solver(box, precision, 256)
    sc = _solver(replace(box, torque_route="curl"), precision, 256)
    U1, _ = sd.apply(P, Fd, None, want_omega=False)
    U2, _ = sc.apply(P, Fd, None, want_omega=False)
    torch.cuda.synchronize()
    assert torch.equal(U1, U2)
    U3, O3 = sd.apply(P, Fd, Td)
    U4, _ = sd.apply(P, Fd, Td, want_omega=False)
    torch.cuda.synchronize()
    assert torch.equal(U3, U4)
    # zero torques: the forces-only velocities up to the rounding of the
    # added zero torque terms
    U5, O5 = sd.apply(P, Fd, torch.zeros_like(Td))
    tol = 1e-14 if precision == "fp64" else 1e-6
    assert rel_err(_np(U5), _np(U1)) < tol
    sd.close()
    sc.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_dense_cluster(precision):
    # 400 particles in 4 x 4 cells: spread regions past the staged capacity
    box = BOXES["bw48"]
    rng = np.random.default_rng(83)
    n = 400
    pos = np.stack([10.0 + 4 * box.h * rng.random(n),
                    20.0 + 4 * box.h * rng.random(n),
                    1.0 + 3.0 * rng.random(n)], axis=1)
    F = rng.standard_normal((n, 3))
    T = rng.standard_normal((n, 3))
    if precision == "mixed":
        pos, F, T = (a.astype(np.float32).astype(np.float64) for a in (pos, F, T))
    print(f"[torque derivative dense] {precision}", flush=True)
    rU, rO = torque_deriv.DerivativeSolver(box).apply(pos, F, T)
    s = _solver(box, precision, n)
    U, Om = s.apply(_dev(pos, precision), _dev(F, precision), _dev(T, precision))
    eU, eO = rel_err(_np(U), rU), rel_err(_np(Om), rO)
    print(f"  rel err U {eU:.2e} Omega {eO:.2e}", flush=True)
    tol = 1e-10 if precision == "fp64" else 1e-5
    assert eU < tol and eO < tol
    s.close()


def test_slit_channel_monolayer_with_the_fp64_vertical_force():
    # mixed slit channel: the vertical force (with its torque part) of the
    # kH < 1 columns takes the FP64 route
    box, pos, F, T = workloads.sub_box("sc1m", 16)
    box = replace(box, torque_route="derivative")
    print(f"[torque derivative sc1m/16] N={len(pos)}", flush=True)
    rU, rO = torque_deriv.DerivativeSolver(box).apply(pos, F, T)
    s = _solver(box, "mixed", len(pos))
    res = {}
    for off in (1, 0):
        s.set_variant("no_lowk", off)
        U, Om = s.apply(_dev(pos, "mixed"), _dev(F, "mixed"), _dev(T, "mixed"))
        res[off] = (rel_err(_np(U), rU), rel_err(_np(Om), rO),
                    particle_err(_np(U), rU))
        print(f"  no_lowk={off}: U {res[off][0]:.2e} Omega {res[off][1]:.2e} "
              f"max particle {res[off][2]:.2e}", flush=True)
    assert res[0][0] < 1e-6 and res[0][1] < 1e-6 and res[0][2] < 1e-5
    s.close()


def test_stage_spread_and_interp_refused():
    from paper_2210_01837_amd import _lib
    box = BOXES["bw48"]
    pos, F, T = _particles(box, 10, 84)
    s = _solver(box, "fp64", 16)
    with pytest.raises(_lib.FcmdpError) as e:
        s.stage_spread(_dev(pos, "fp64"), _dev(F, "fp64"), _dev(T, "fp64"))
    assert e.value.code == _lib.EINVAL
    s.close()
