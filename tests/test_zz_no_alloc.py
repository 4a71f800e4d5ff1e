"""GPU: the allocation-free Lanczos entry point (fcmdp_lanczos_sqrt_noalloc)
against the allocating one, through the C ABI.

Both run the same kernels in the same order on the same solver, so g and the
iteration count must agree bit for bit; two calls in a row, the second with
fewer particles and iterations (the shared scratch array keeps the first
call's contents), in both precisions; sizes beyond the array are rejected
before any work.
"""
import ctypes

import numpy as np
import pytest

import workloads
from workloads import Box

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _lanczos(fn, s, pos, W, g, max_iter, tol):
    it = ctypes.c_int(-1)
    ch = ctypes.c_double(-1.0)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = fn(s._h, pos.shape[0], _ptr(pos), _ptr(W), _ptr(g), int(max_iter),
            float(tol), ctypes.byref(it), ctypes.byref(ch), st)
    torch.cuda.synchronize()
    return rc, it.value, ch.value


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_noalloc_lanczos_equals_allocating_entry_point(precision):
    from paper_2210_01837_amd import Solver
    from paper_2210_01837_amd import _lib
    L = _lib.lib()
    dt = torch.float32 if precision == "mixed" else torch.float64
    box = Box("sc", 48.0, 48.0, 9.0, 72, 72, 24, w=4, beta_m=7.48, beta_d=7.48)
    pos, _, _ = workloads.random_particles(box, 2000, 61, 0.4, 8.6)
    Wn = workloads.random_array((2000, 3), 62)
    s = Solver.from_box(box, precision=precision, max_particles=2000)
    for n, iters, tol in ((2000, 12, 0.0), (700, 6, 1e-3)):
        print(f"[noalloc lanczos] {precision} n={n} iterations<={iters}",
              flush=True)
        P = torch.tensor(pos[:n], dtype=dt, device="cuda")
        W = torch.tensor(Wn[:n], dtype=dt, device="cuda")
        g_ref = torch.full((n, 3), float("nan"), dtype=dt, device="cuda")
        g_new = torch.full((n, 3), float("nan"), dtype=dt, device="cuda")
        r1 = _lanczos(L.fcmdp_lanczos_sqrt, s, P, W, g_ref, iters, tol)
        r2 = _lanczos(L.fcmdp_lanczos_sqrt_noalloc, s, P, W, g_new, iters, tol)
        assert r1[0] == 0 and r2[0] == 0
        assert r1[1] == r2[1] and r1[2] == r2[2]
        assert bool(torch.isfinite(g_new).all())
        assert torch.equal(g_ref, g_new)
    s.close()


def test_noalloc_lanczos_rejects_sizes_beyond_its_array():
    from paper_2210_01837_amd import Solver
    from paper_2210_01837_amd import _lib
    L = _lib.lib()
    box = Box("bw", 64.0, 64.0, 9.0, 96, 96, 16, w=4, beta_m=7.48, beta_d=7.48)
    n = 95000
    s = Solver.from_box(box, precision="mixed", max_particles=n)
    P = torch.zeros((n, 3), dtype=torch.float32, device="cuda")
    W = torch.zeros_like(P)
    g = torch.zeros_like(P)
    # 65 basis vectors of 3n floats need 74 MB: more than the 64 MiB array
    rc, it, _ = _lanczos(L.fcmdp_lanczos_sqrt_noalloc, s, P, W, g, 64, 0.0)
    assert rc == _lib.ECAPACITY and it == -1
    s.close()
