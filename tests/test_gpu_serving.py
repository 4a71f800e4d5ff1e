"""GPU: requests served concurrently (shared solver pool, several streams,
admission under a byte budget) give the same results as each request applied
alone, and agree with the oracle on a sample."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _jobs(count):
    from paper_2210_01837_amd.serving import Job
    reqs = workloads.serving_requests(count, nmax=20000)
    jobs = []
    for r in reqs:
        pos, F, T = workloads.request_particles(r)
        dev = [torch.tensor(a, dtype=torch.float32, device="cuda") for a in (pos, F, T)]
        jobs.append(Job(r.rid, r.box, *dev))
    return reqs, jobs


def test_served_results_equal_standalone_applies():
    from paper_2210_01837_amd import Solver
    from paper_2210_01837_amd.serving import (SolverPool, latency_summary,
                                              serve)
    reqs, jobs = _jobs(24)
    print(f"[serving] {len(jobs)} requests", flush=True)
    # a budget that forces queueing and evictions
    pool = SolverPool(6 << 30)
    arrivals = list(np.linspace(0.0, 20.0, len(jobs)))
    serve(jobs, arrivals, budget=pool.budget, streams=4, pool=pool)
    summ = latency_summary(jobs)
    assert summ["p99_ms"] >= summ["p50_ms"] > 0
    for j in jobs:
        s = Solver.from_box(j.box, precision="mixed", max_particles=j.n)
        U, Om = s.apply(j.pos, j.F, j.T)
        torch.cuda.synchronize()
        assert torch.equal(U, j.U) and torch.equal(Om, j.Omega), j.rid
        s.close()
    pool.close()


def test_served_request_matches_oracle():
    from _parity import oracle_apply, rel_err
    from paper_2210_01837_amd.serving import serve
    reqs, jobs = _jobs(3)
    serve(jobs, [0.0, 0.0, 0.0], budget=4 << 30, streams=3)
    torch.cuda.synchronize()
    i = int(np.argmin([r.n for r in reqs]))
    j, r = jobs[i], reqs[i]
    print(f"[serving oracle] request {i}: N={r.n} grid {r.box.Nx}", flush=True)
    pos, F, T = workloads.request_particles(r)
    sample = np.arange(0, r.n, max(1, r.n // 200))
    U, Om = oracle_apply(r.box, pos, F, T, sample=sample)
    assert rel_err(j.U.double().cpu().numpy()[sample], U) < 1e-5
    assert rel_err(j.Omega.double().cpu().numpy()[sample], Om) < 1e-5
