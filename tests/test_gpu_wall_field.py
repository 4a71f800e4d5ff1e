"""GPU parity of non-uniform wall velocities u^W(x, y) (eq. bcnoslip0;
App. A, eqs. bcslip and u0uHformula) against the oracle, in both
precisions, with particles forced as usual."""
from dataclasses import replace

import numpy as np
import pytest

import workloads
from workloads import Box

from _parity import particle_err, rel_err
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

BOXES = {
    "bw48": Box("bw", 32.0, 32.0, 8.0, 48, 48, 32),
    "sc40x56": Box("sc", 20.0, 28.0, 7.0, 40, 56, 24),
}


def _solver(box, precision, cap=512):
    from paper_2210_01837_amd import Solver
    return Solver.from_box(box, precision=precision, max_particles=cap)


def _dev(a, precision):
    dt = torch.float64 if precision == "fp64" else torch.float32
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def _inputs(box, n, seed, precision):
    alpha = 3 * box.h
    zhi = box.H - alpha - 0.05 if box.geometry == "bw" else box.H - 0.2
    pos, F, T = workloads.random_particles(box, n, seed, 0.2, zhi)
    nw = 1 if box.geometry == "bw" else 2
    wall = workloads.random_array((nw, 2, box.Ny, box.Nx), seed)
    if precision == "mixed":
        pos, F, T, wall = (a.astype(np.float32).astype(np.float64)
                           for a in (pos, F, T, wall))
    return pos, F, T, wall


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("case", ["bw48", "bw_slip", "sc40x56", "sc_slip"])
def test_apply_with_wall_field_against_oracle(case, precision):
    box = BOXES[{"sc_slip": "sc40x56", "bw_slip": "bw48"}.get(case, case)]
    if case == "sc_slip":
        box = replace(box, slip0=0.6, slipH=1.4, wall0=(0.2, 0.0))
    if case == "bw_slip":
        box = replace(box, slip0=0.9, wall0=(0.1, -0.2))
    pos, F, T, wall = _inputs(box, 120, 91, precision)
    print(f"[wall field] {case} {precision}", flush=True)
    rU, rO = oracle.Solver(box).apply(pos, F, T, wall=wall)
    s = _solver(box, precision)
    s.set_wall_velocity(_dev(wall, precision))
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
def test_replace_and_remove_the_field(precision):
    box = BOXES["sc40x56"]
    pos, F, T, wall = _inputs(box, 60, 92, precision)
    _, _, _, wall2 = _inputs(box, 60, 93, precision)
    P, Fd, Td = (_dev(a, precision) for a in (pos, F, T))
    s = _solver(box, precision)
    U0, O0 = s.apply(P, Fd, Td)
    U0, O0 = U0.clone(), O0.clone()
    s.set_wall_velocity(_dev(wall, precision))
    s.apply(P, Fd, Td)
    # a second field replaces the first
    s.set_wall_velocity(_dev(wall2, precision))
    U2, O2 = s.apply(P, Fd, Td)
    rU, rO = oracle.Solver(box).apply(pos, F, T, wall=wall2)
    tol = 1e-10 if precision == "fp64" else 1e-5
    assert rel_err(_np(U2), rU) < tol and rel_err(_np(O2), rO) < tol
    # removing it gives back the bits of the walls at rest
    s.set_wall_velocity(None)
    U3, O3 = s.apply(P, Fd, Td)
    torch.cuda.synchronize()
    assert torch.equal(U3, U0) and torch.equal(O3, O0)
    s.close()


def test_slit_channel_monolayer_with_wall_field_and_fp64_route():
    # the mixed slit channel's kH < 1 columns (FP64 vertical force) with a
    # moving-wall pattern of long wavelength on both walls
    box, pos, F, T = workloads.sub_box("sc1m", 16)
    X = np.arange(box.Nx) * box.h
    Y = np.arange(box.Ny) * box.h
    c = np.cos(2 * np.pi * (X[None, :] / box.Lx + 2 * Y[:, None] / box.Ly))
    wall = np.stack([np.stack([0.05 * c, -0.02 * c]), np.stack([0.01 * c, 0.03 * c])])
    wall = wall.astype(np.float32).astype(np.float64)
    print(f"[wall field sc1m/16] N={len(pos)}", flush=True)
    rU, rO = oracle.Solver(box).apply(pos, F, T, wall=wall)
    s = _solver(box, "mixed", len(pos))
    s.set_wall_velocity(_dev(wall, "mixed"))
    U, Om = s.apply(_dev(pos, "mixed"), _dev(F, "mixed"), _dev(T, "mixed"))
    eU, eO = rel_err(_np(U), rU), rel_err(_np(Om), rO)
    print(f"  rel err U {eU:.2e} Omega {eO:.2e}", flush=True)
    assert eU < 1e-5 and eO < 1e-5
    s.close()


def test_wall_field_refused_beyond_the_eight_lane_kernels():
    from paper_2210_01837_amd import _lib
    box = Box("sc", 20.0, 20.0, 7.0, 30, 30, 48)
    s = _solver(box, "fp64", 16)
    wall = torch.zeros((2, 2, 30, 30), dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.FcmdpError) as e:
        s.set_wall_velocity(wall)
    assert e.value.code == _lib.EINVAL
    with pytest.raises(ValueError):
        s.set_wall_velocity(wall[:1])
    s.close()
