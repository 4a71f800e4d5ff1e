"""Host-side logic of the serving loop: admission under a byte budget and the
solver pool (reuse by key, least-recently-used eviction of idle solvers)."""
import pytest

import workloads
from paper_2210_01837_amd.serving import (AdmissionQueue, SolverPool,
                                          capacity_bucket, solver_key)


def test_capacity_bucket():
    assert capacity_bucket(1) == 1024
    assert capacity_bucket(1024) == 1024
    assert capacity_bucket(1025) == 2048
    assert capacity_bucket(262144) == 262144


def test_admission_fifo_under_budget():
    q = AdmissionQueue(100)
    q.push("a", 60)
    q.push("b", 50)
    q.push("c", 10)
    assert q.head_fits()
    assert q.pop() == ("a", 60)
    assert not q.head_fits()          # b does not fit; c waits behind it
    q.release(60)
    assert q.pop() == ("b", 50)
    assert q.pop() == ("c", 10)
    assert q.in_use == 60
    with pytest.raises(ValueError):
        q.push("huge", 101)


class _Fake:
    def __init__(self, key):
        self.key = key
        self.closed = False

    def close(self):
        self.closed = True


def test_pool_reuse_and_lru_eviction():
    sizes = {"s": 30, "m": 50, "l": 80}
    pool = SolverPool(100, factory=_Fake, sizer=lambda k: sizes[k])
    a, ba = pool.get("s")
    b, bb = pool.get("m")
    assert pool.allocated == 80 and pool.created == 2
    pool.put("s", a, ba)
    pool.put("m", b, bb)
    a2, _ = pool.get("s")
    assert a2 is a and pool.created == 2          # reused, not re-created
    pool.put("s", a2, ba)
    # "l" needs 80: idle solvers go least recently used first ("m", then "s")
    c, _ = pool.get("l")
    assert b.closed and a.closed and pool.evicted == 2
    assert pool.allocated == 80
    pool.put("l", c, 80)
    pool.close()
    assert pool.allocated == 0


def test_pool_refuses_when_everything_busy():
    pool = SolverPool(100, factory=_Fake, sizer=lambda k: 60)
    pool.get("x")
    with pytest.raises(MemoryError):
        pool.get("y")


def test_solver_keys_of_the_stream():
    reqs = workloads.serving_requests(64)
    keys = {solver_key(r.box, r.n, "mixed") for r in reqs}
    assert 1 < len(keys) <= 64
    for r in reqs:
        assert r.box.Nx == r.box.Ny and r.box.Nx % 2 == 0
        assert 1024 <= r.n <= 262144


def test_pool_evicts_only_what_it_needs():
    sizes = {"s": 30, "m": 50, "l": 40}
    pool = SolverPool(100, factory=_Fake, sizer=lambda k: sizes[k])
    a, _ = pool.get("s")
    b, _ = pool.get("m")
    pool.put("m", b, 50)
    pool.put("s", a, 30)                 # "m" is now least recently used
    pool.get("l")
    assert b.closed and not a.closed and pool.evicted == 1
    assert pool.allocated == 70


def test_keys_separate_every_operator_parameter():
    from dataclasses import replace
    from paper_2210_01837_amd.serving import key_capacity, key_params
    base = workloads.Box("sc", 64.0, 64.0, 10.0, 96, 96, 32)
    variants = [replace(base, w=4, beta_m=7.48, beta_d=7.48),
                replace(base, beta_m=7.0), replace(base, beta_d=12.0),
                replace(base, eta=2.0), replace(base, slip0=0.5),
                replace(base, slipH=0.5), replace(base, wall0=(0.1, 0.0)),
                replace(base, wallH=(0.0, 0.1)), replace(base, geometry="bw"),
                replace(base, Nz=24)]
    keys = {solver_key(b, 1000, "mixed") for b in [base] + variants}
    assert len(keys) == len(variants) + 1
    assert solver_key(base, 1000, "mixed") != solver_key(base, 1000, "fp64")
    k = solver_key(variants[0], 3000, "mixed")
    kw = key_params(k)
    assert kw["w"] == 4 and kw["beta_m"] == 7.48 and kw["precision"] == "mixed"
    assert key_capacity(k) == 4096
