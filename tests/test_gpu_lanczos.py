"""GPU parity of the Lanczos square root fcmdp_lanczos_sqrt (Sec. 5.2)
against the oracle's Lanczos process on the oracle's forces-only apply.

Fixed iteration counts compare the same Krylov approximation (FP64 to 1e-9,
mixed to 2e-5); with a tolerance both stop after the same number of
iterations.  On the tiled 663,552-particle layer a tiled W keeps the Krylov
space periodic, so the result is the one-replica result repeated and every
particle is checked against the oracle on one replica.
"""
import numpy as np
import pytest

import workloads
from workloads import Box

from _parity import rel_err
from oracle import fcm, lanczos

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

BOX = Box("bw", 30.0, 36.0, 9.0, 30, 36, 19, w=4, beta_m=7.48, beta_d=7.48)
SC_BOX = Box("sc", 40.0, 40.0, 8.0, 40, 40, 20, w=4, beta_m=7.48, beta_d=7.48)


def _solver(box, precision, cap):
    from paper_2210_01837_amd import Solver
    return Solver.from_box(box, precision=precision, max_particles=cap)


def _dev(a, precision):
    dt = torch.float64 if precision == "fp64" else torch.float32
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def _particles(box, n, seed):
    zhi = box.H - 2.1 if box.geometry == "bw" else box.H - 0.3
    pos, _, _ = workloads.random_particles(box, n, seed, 0.5, zhi)
    return pos


def _oracle(box, pos, W, max_iter, tol):
    s = fcm.Solver(box)
    return lanczos.lanczos_sqrt(lanczos.translational_matvec(s, s.wrap(pos)),
                                W, max_iter=max_iter, tol=tol)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("box", [BOX, SC_BOX], ids=["bw", "sc"])
def test_lanczos_fixed_iterations(box, precision):
    pos = _particles(box, 60, 31)
    W = workloads.random_array((60, 3), 32)
    if precision == "mixed":
        pos, W = (a.astype(np.float32).astype(np.float64) for a in (pos, W))
    print(f"[lanczos] {box.geometry} {precision}", flush=True)
    s = _solver(box, precision, 64)
    g, k, ch = s.lanczos_sqrt(_dev(pos, precision), _dev(W, precision),
                              max_iter=12, tol=0.0)
    rg, rk, rch = _oracle(box, pos, W, 12, 0.0)
    assert k == rk == 12
    e = rel_err(g.double().cpu().numpy().ravel(), rg)
    print(f"  rel err g {e:.3e}, change {ch:.3e} (oracle {rch:.3e})", flush=True)
    assert e < (1e-9 if precision == "fp64" else 2e-5)
    assert ch == pytest.approx(rch, rel=1e-6 if precision == "fp64" else 1e-2)


def test_lanczos_stops_like_the_oracle_and_edge_cases():
    pos = _particles(BOX, 60, 33)
    W = workloads.random_array((60, 3), 34)
    print("[lanczos] tolerance, zero vector, argument checks", flush=True)
    s = _solver(BOX, "fp64", 64)
    P = _dev(pos, "fp64")
    g, k, ch = s.lanczos_sqrt(P, _dev(W, "fp64"), max_iter=40, tol=1e-6)
    rg, rk, rch = _oracle(BOX, pos, W, 40, 1e-6)
    assert k == rk and ch < 1e-6
    assert rel_err(g.cpu().numpy().ravel(), rg) < 1e-9
    g0, k0, _ = s.lanczos_sqrt(P, torch.zeros_like(P), max_iter=5)
    assert k0 == 0 and not torch.any(g0)
    from paper_2210_01837_amd import FcmdpError
    for bad in (0, 65):
        with pytest.raises(FcmdpError):
            s.lanczos_sqrt(P, _dev(W, "fp64"), max_iter=bad)


def test_lanczos_on_the_replicated_layer():
    """A W repeated in every replica keeps the Krylov space periodic: the
    663,552-particle result is the 2048-particle result repeated."""
    pos1, _, _ = workloads.particles("m2048")
    W1 = workloads.random_array((2048, 3), 35).astype(np.float32).astype(np.float64)
    rg, rk, rch = _oracle(workloads.WORKLOADS["m2048"].box, pos1, W1, 16, 1e-3)
    r = workloads.M_REPLICAS
    for name in ("m2048", "m663k"):
        wl = workloads.WORKLOADS[name]
        pos, _, _ = workloads.particles(name)
        W = np.tile(W1, (r * r, 1)) if name == "m663k" else W1
        print(f"[lanczos layer] {name}", flush=True)
        s = _solver(wl.box, "mixed", wl.n)
        g, k, ch = s.lanczos_sqrt(_dev(pos, "mixed"), _dev(W, "mixed"),
                                  max_iter=16, tol=1e-3)
        got = g.double().cpu().numpy().reshape(-1, 2048, 3)
        e = rel_err(got, np.broadcast_to(rg.reshape(2048, 3), got.shape))
        print(f"  iterations {k} (oracle {rk}), rel err g {e:.3e}", flush=True)
        assert k == rk and e < 2e-5
        s.close()
