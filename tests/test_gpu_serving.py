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


def test_largest_slit_request_matches_oracle():
    # the slit-channel request with the most particles of the 512-request
    # stream (N = 256,915, 1400^2 x 32), served through the loop and checked
    # on its stored 1% oracle sample (tests/golden/make_fixtures.py)
    import os
    from _parity import particle_err, rel_err
    from paper_2210_01837_amd.serving import Job, serve
    path = os.path.join(os.path.dirname(__file__), "golden",
                        "serve_sc_max_oracle_sample.npz")
    g = np.load(path)
    r = workloads.largest_request("sc")
    print(f"[serving largest sc] N={r.n} grid {r.box.Nx}", flush=True)
    pos, F, T = workloads.request_particles(r)
    dev = [torch.tensor(a, dtype=torch.float32, device="cuda") for a in (pos, F, T)]
    jobs = serve([Job(r.rid, r.box, *dev)], [0.0], budget=16 << 30, streams=1)
    torch.cuda.synchronize()
    idx = g["index"]
    U = jobs[0].U.double().cpu().numpy()[idx]
    Om = jobs[0].Omega.double().cpu().numpy()[idx]
    eU, eO = rel_err(U, g["U"]), rel_err(Om, g["Omega"])
    pU, pO = particle_err(U, g["U"]), particle_err(Om, g["Omega"])
    print(f"  rel err U {eU:.2e} Omega {eO:.2e}; max particle {pU:.2e} {pO:.2e}",
          flush=True)
    assert eU < 1e-5 and eO < 1e-5 and pU < 1e-4 and pO < 1e-4


def test_serving_keeps_kernel_width_and_shape_apart():
    # two requests on the same box and grid, one with the forces-only
    # kernel of width 4 (its own beta): each is served by its own solver and
    # gives the bits of a standalone apply with its own parameters
    from dataclasses import replace
    from paper_2210_01837_amd import Solver
    from paper_2210_01837_amd.serving import Job, SolverPool, serve
    r = workloads.serving_requests(8, nmax=8000)[0]
    b6 = r.box
    b4 = replace(b6, w=4, beta_m=7.48, beta_d=7.48)
    pos, F, T = workloads.request_particles(r)
    dev = [torch.tensor(a, dtype=torch.float32, device="cuda") for a in (pos, F, T)]
    pool = SolverPool(4 << 30)
    jobs = [Job(0, b6, *dev), Job(1, b4, *dev)]
    serve(jobs, [0.0, 0.0], budget=pool.budget, streams=2, pool=pool)
    assert pool.created == 2
    for j, b in zip(jobs, (b6, b4)):
        s = Solver.from_box(b, precision="mixed", max_particles=j.n)
        U, Om = s.apply(*dev)
        torch.cuda.synchronize()
        assert torch.equal(U, j.U) and torch.equal(Om, j.Omega), b.w
        s.close()
    assert not torch.equal(jobs[0].U, jobs[1].U)
    pool.close()
