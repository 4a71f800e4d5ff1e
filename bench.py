"""Benchmark: particle mobility-applies per second of the MI355X DP-FCM apply.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload bw1m]

One step = one whole mobility apply (F, T) -> (U, Omega) of the workload:
particle prep + sort, ES spreading, forward xy FFT, per-wavenumber FP64
column solve (Chebyshev transform, DP BVPs, wall correction, k = 0 mode,
vorticity), inverse FFT and interpolation.  Inputs are seeded synthetic
particles already resident in HBM before the timed region.

Prints one JSON line.  `value` = N * K / (time of K steps).  The `roofline`
object describes the slowest stage (per-stage HIP events on the apply's
stream, summed over the timed region), `stages_ms` all of them; the
`cpu_baseline` object times the CPU oracle on a bounded sub-box of the same
workload (same density, same grid spacing) on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def stage_bytes(box, n, band, complex_bytes=8, real_bytes=4, torques=True,
                lowk=False, deriv=False):
    """Algorithmic HBM bytes of one launch of each stage (mixed precision).

    P = number of band planes; the real grid holds 6 channels (forces and
    torques in, velocities and angular velocities out), 3 in the
    forces-only apply and with torques through the kernel derivative
    (deriv: torques enter the spread, Omega the interpolation, through the
    three force / velocity channels).  lowk: the mixed slit channel's FP64 route for the
    vertical force of its kH < 1 columns (the spread also writes the FP32
    residual plane of f_z, which the direct x transform reads back with f_z
    itself; its small y and Chebyshev stages are negligible).
    """
    P = band[1] - band[0] + 1
    nxy = box.Nx * box.Ny
    nk = (box.Nx // 2 + 1) * box.Ny
    nch = 6 if torques and not deriv else 3
    grid = nch * P * nxy * real_bytes
    spec = nch * P * nk * complex_bytes
    particles_in = n * (36 if torques else 24)   # pos, F (, T) (float32)
    particles_out = n * (24 if torques else 12)  # U (, Omega)
    lo_plane = P * nxy * 4 if lowk else 0
    return {
        "spread": particles_in + grid + lo_plane,
        "fft_forward": grid + spec + 2 * spec + 2 * lo_plane,
        "columns": 2 * spec,
        "fft_inverse": 2 * spec + spec + grid,
        "interp": grid + n * 12 + particles_out,
    }


# the paper's one timing (Sec. 5.1): 663,552 particles, forces only, m = 4,
# 370 ms per mobility solve on a V100
PAPER_FORCES_ONLY_RATE = 663552 / 0.370


# the kernel each single-kernel stage launches once per apply
STAGE_KERNEL = {"spread": "k_spread_mfma", "columns": "k_columns_mfma",
                "interp": "k_interp_part"}


def measured_traffic(workload, kernel):
    """HBM bytes per launch from the committed rocprofv3 counters
    (profiles/traffic_<workload>.json), or None if there are none or the
    kernel's sources changed since they were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not kernel or not os.path.exists(path):
        return None
    from paper_2210_01837_amd.profiling import source_hash
    with open(path) as fh:
        t = json.load(fh)
    k = t.get("kernels", {}).get(kernel)
    if not k or k.get("source_hash") != source_hash(kernel):
        return None
    return k["bytes_per_launch"]


# MI355X: 256 CUs x 4 SIMDs at 2.4 GHz; dense peaks (TFLOP/s)
FP64_VECTOR_PEAK = 78.6
FP32_MATRIX_PEAK = 157.3
SIMDS, CLOCK_HZ = 1024, 2.4e9


def measured_compute(workload, kernel, avg_ms):
    """Arithmetic roofline of one kernel from the committed rocprofv3 FLOP
    and instruction counters (profiles/compute_<workload>.json) and the
    launch time measured here, or None if there are none or the kernel's
    sources changed since they were taken."""
    path = os.path.join(ROOT, "profiles", f"compute_{workload}.json")
    if not kernel or not os.path.exists(path):
        return None
    from paper_2210_01837_amd.profiling import source_hash
    with open(path) as fh:
        t = json.load(fh)
    k = t.get("kernels", {}).get(kernel)
    if not k or k.get("source_hash") != source_hash(kernel):
        return None
    sec = avg_ms * 1e-3
    f64 = k["fp64_vector_flops"] / sec / 1e12
    mf = k["fp32_matrix_flops"] / sec / 1e12
    out = {"bound": "alu", "unit": "TFLOP/s",
           "achieved": f64, "peak": FP64_VECTOR_PEAK,
           "frac": f64 / FP64_VECTOR_PEAK,
           "flops_fp64_per_launch": k["fp64_vector_flops"],
           "mfma_f32": {"achieved": mf, "peak": FP32_MATRIX_PEAK,
                        "frac": mf / FP32_MATRIX_PEAK},
           "source": f"profiles/compute_{workload}.json (executed FLOPs)"}
    insts = k["counters"].get("SQ_INSTS_VALU")
    if insts:
        # a wave64 VALU instruction occupies its SIMD for 4 cycles
        out["valu_issue_frac"] = insts * 4 / (SIMDS * CLOCK_HZ * sec)
    return out


def fp64_comparison(name="bw131k", steps=5):
    """Mixed vs FP64 GPU applies on the same inputs: time and agreement."""
    import numpy as np
    import torch

    import workloads
    from paper_2210_01837_amd import Solver
    wl = workloads.WORKLOADS[name]
    pos, F, T = workloads.particles(name)
    out = {"workload": name, "N": wl.n}
    res = {}
    for prec, dt in (("mixed", torch.float32), ("fp64", torch.float64)):
        s = Solver.from_box(wl.box, precision=prec, max_particles=wl.n)
        Pd, Fd, Td = (torch.tensor(a, dtype=dt, device="cuda") for a in (pos, F, T))
        U = torch.empty_like(Pd)
        Om = torch.empty_like(Pd)
        s.apply(Pd, Fd, Td, U=U, Omega=Om)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            s.apply(Pd, Fd, Td, U=U, Omega=Om)
        e1.record()
        torch.cuda.synchronize()
        out[f"ms_{prec}"] = e0.elapsed_time(e1) / steps
        res[prec] = (U.double().cpu().numpy(), Om.double().cpu().numpy())
        s.close()
    (Um, Om_m), (Ud, Od) = res["mixed"], res["fp64"]
    out["speedup_mixed_over_fp64"] = out["ms_fp64"] / out["ms_mixed"]
    out["rel_err_U_mixed_vs_fp64"] = float(np.linalg.norm(Um - Ud) / np.linalg.norm(Ud))
    out["rel_err_Omega_mixed_vs_fp64"] = float(np.linalg.norm(Om_m - Od) / np.linalg.norm(Od))
    return out


def forces_only_summary(steps=10, warmup=2):
    """The paper's timed case (Sec. 5.1): the forces-only apply (m = 4) of
    the 663,552-particle replicated layer, its accuracy against the oracle's
    one-replica values, and a Lanczos square root to three digits."""
    import numpy as np
    import torch

    import workloads
    from paper_2210_01837_amd import Solver
    wl = workloads.WORKLOADS["m663k"]
    pos, F, _ = workloads.particles("m663k")
    P = torch.tensor(pos, dtype=torch.float32, device="cuda")
    Fd = torch.tensor(F, dtype=torch.float32, device="cuda")
    U = torch.empty_like(P)
    s = Solver.from_box(wl.box, precision="mixed", max_particles=wl.n)
    for _ in range(warmup):
        s.apply(P, Fd, None, U=U, want_omega=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        s.apply(P, Fd, None, U=U, want_omega=False)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    out = {"workload": "m663k", "N": wl.n, "grid": [wl.box.Nx, wl.box.Ny, wl.box.Nz],
           "w": wl.box.w, "ms_per_apply": ms, "value": wl.n / (ms * 1e-3),
           "unit": "particle-applies/s",
           "vs_paper_v100": wl.n / (ms * 1e-3) / PAPER_FORCES_ONLY_RATE}
    gold = os.path.join(ROOT, "tests", "golden", "m2048_oracle_sample.npz")
    if os.path.exists(gold):
        gU = np.load(gold)["U"]
        Uh = U.double().cpu().numpy().reshape(-1, len(gU), 3)
        out["rel_err_U"] = float(np.linalg.norm(Uh - gU[None]) /
                                 (np.linalg.norm(gU) * np.sqrt(Uh.shape[0])))
    W = torch.tensor(workloads.random_array((wl.n, 3), 40), dtype=torch.float32,
                     device="cuda")
    g, it, ch = s.lanczos_sqrt(P, W, max_iter=32, tol=1e-3)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g, it, ch = s.lanczos_sqrt(P, W, max_iter=32, tol=1e-3, g=g)
    torch.cuda.synchronize()
    out["lanczos"] = {"iterations": it, "rel_change": ch, "tol": 1e-3,
                      "ms": (time.perf_counter() - t1) * 1e3}
    s.close()
    return out


def cpu_baseline(name, factor=4):
    """Time the oracle on a 1/factor x 1/factor sub-box of the workload, with
    every host core available to NumPy's thread pools (BLAS / OpenMP).  The
    oracle is not parallelised beyond that: NumPy's FFT and its per-particle
    loops run on one thread, so `cores` reports the threads it actually kept
    busy (process CPU time over wall time)."""
    import numpy as np  # noqa: F401
    from threadpoolctl import threadpool_info, threadpool_limits

    import workloads
    from oracle import fcm
    box, pos, F, T = workloads.sub_box(name, factor)
    avail = len(os.sched_getaffinity(0))
    with threadpool_limits(avail):
        pools = {p.get("internal_api", "?"): p.get("num_threads")
                 for p in threadpool_info()}
        c0 = time.process_time()
        t0 = time.perf_counter()
        fcm.Solver(box).apply(pos, F, T)
        dt = time.perf_counter() - t0
        busy = (time.process_time() - c0) / dt
    return {
        "value": len(pos) / dt,
        "unit": "particle-applies/s",
        "cores": round(busy, 2),
        "kind": "oracle",
        "sample": (f"one oracle apply (float64 NumPy) of a "
                   f"{box.Nx}x{box.Ny}x{box.Nz} sub-box with {len(pos)} "
                   f"particles at the same density and grid spacing as "
                   f"{name}; {dt:.1f} s"),
        "host_cores_available": avail,
        "thread_pools": pools,
    }


def slit_channel_summary(steps=10, warmup=2):
    """The slit channel at N = 1M (mixed): per-apply time and stages with the
    FP64 route for the vertical force of the kH < 1 columns (the default)
    and without it, and the accuracy of both against the stored oracle
    sample."""
    import numpy as np
    import torch

    import workloads
    from paper_2210_01837_amd import Solver
    name = "sc1m"
    wl = workloads.WORKLOADS[name]
    pos, F, T = workloads.particles(name)
    P, Fd, Td = (torch.tensor(a, dtype=torch.float32, device="cuda")
                 for a in (pos, F, T))
    U = torch.empty_like(P)
    Om = torch.empty_like(P)
    s = Solver.from_box(wl.box, precision="mixed", max_particles=wl.n)
    gold = os.path.join(ROOT, "tests", "golden", f"{name}_oracle_sample.npz")
    g = np.load(gold) if os.path.exists(gold) else None
    out = {"workload": name, "N": wl.n}
    for label, off in (("fp64_route", 0), ("fp32_only", 1)):
        s.set_variant("no_lowk", off)
        for _ in range(warmup):
            s.apply(P, Fd, Td, U=U, Omega=Om)
        torch.cuda.synchronize()
        s.stage_times()
        s.set_profiling(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            s.apply(P, Fd, Td, U=U, Omega=Om)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        s.set_profiling(False)
        stages, na, band = s.stage_times()
        r = {"ms_per_apply": ms, "value": wl.n / (ms * 1e-3),
             "stages_ms": {k: v / max(1, na) for k, v in stages.items()}}
        if g is not None:
            idx = g["index"]
            Uh = U.double().cpu().numpy()[idx]
            Oh = Om.double().cpu().numpy()[idx]
            r["rel_err_U"] = float(np.linalg.norm(Uh - g["U"]) /
                                   np.linalg.norm(g["U"]))
            r["rel_err_Omega"] = float(np.linalg.norm(Oh - g["Omega"]) /
                                       np.linalg.norm(g["Omega"]))
        out[label] = r
    s.close()
    return out


def torque_derivative_summary(name="bw1m", steps=10, warmup=2):
    """Torques through the derivative of the dipole kernel (three channels
    through the transforms and the solve) against the spectral-curl route
    (six) on the same inputs: per-apply time, stages, algorithmic bytes and
    the difference between the two discrete operators."""
    from dataclasses import replace

    import numpy as np
    import torch

    import workloads
    from paper_2210_01837_amd import Solver
    wl = workloads.WORKLOADS[name]
    pos, F, T = workloads.particles(name)
    P, Fd, Td = (torch.tensor(a, dtype=torch.float32, device="cuda")
                 for a in (pos, F, T))
    out = {"workload": name, "N": wl.n}
    res = {}
    for route in ("curl", "derivative"):
        box = replace(wl.box, torque_route=route)
        s = Solver.from_box(box, precision="mixed", max_particles=wl.n)
        U = torch.empty_like(P)
        Om = torch.empty_like(P)
        for _ in range(warmup):
            s.apply(P, Fd, Td, U=U, Omega=Om)
        torch.cuda.synchronize()
        s.stage_times()
        s.set_profiling(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            s.apply(P, Fd, Td, U=U, Omega=Om)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        s.set_profiling(False)
        stages, na, band = s.stage_times()
        nb = stage_bytes(wl.box, wl.n, band, deriv=route == "derivative",
                         lowk=wl.box.geometry == "sc")
        out[route] = {"ms_per_apply": ms, "value": wl.n / (ms * 1e-3),
                      "stages_ms": {k: v / max(1, na) for k, v in stages.items()},
                      "algorithmic_bytes": sum(nb.values())}
        res[route] = (U.double().cpu().numpy(), Om.double().cpu().numpy())
        s.close()
    out["byte_ratio"] = (out["derivative"]["algorithmic_bytes"] /
                         out["curl"]["algorithmic_bytes"])
    out["speedup"] = out["curl"]["ms_per_apply"] / out["derivative"]["ms_per_apply"]
    (Uc, Oc), (Ud, Od) = res["curl"], res["derivative"]
    out["rel_diff_U_vs_curl"] = float(np.linalg.norm(Ud - Uc) / np.linalg.norm(Uc))
    out["rel_diff_Omega_vs_curl"] = float(np.linalg.norm(Od - Oc) /
                                          np.linalg.norm(Oc))
    return out


def serving_bench(count=512, loads=(0.5, 0.8, 0.95), streams=4):
    """The mixed serving stream: per-request latency at Poisson loads given
    as fractions of the saturated request rate (all requests at t = 0)."""
    import torch

    import workloads
    from paper_2210_01837_amd import serving

    reqs = workloads.serving_requests(count)
    jobs = []
    for r in reqs:
        pos, F, T = workloads.request_particles(r)
        dev = [torch.tensor(a, dtype=torch.float32, device="cuda") for a in (pos, F, T)]
        jobs.append(serving.Job(r.rid, r.box, *dev))
    free, _ = torch.cuda.mem_get_info()
    budget = int(free * 0.6)
    pool = serving.SolverPool(budget)
    at0 = [0.0] * count
    t0 = time.perf_counter()
    serving.serve(jobs, at0, budget=budget, streams=streams, pool=pool)
    warm_s = time.perf_counter() - t0
    sat = serving.latency_summary(
        serving.serve(jobs, at0, budget=budget, streams=streams, pool=pool))
    print(f"[bench] serving saturated: {sat}", file=sys.stderr, flush=True)
    out = {"requests": count, "streams": streams, "budget_bytes": budget,
           "solvers_created": pool.created, "solvers_evicted": pool.evicted,
           "warmup_s": warm_s, "saturated": sat, "poisson": {}}
    for f in loads:
        arr = workloads.poisson_arrivals(count, f * sat["requests_per_s"]) * 1e3
        res = serving.latency_summary(
            serving.serve(jobs, list(arr), budget=budget, streams=streams,
                          pool=pool))
        print(f"[bench] serving load {f}: {res}", file=sys.stderr, flush=True)
        out["poisson"][str(f)] = res
    pool.close()
    # a budget a fifth of the stream's distinct-solver total: the pool keeps
    # evicting (stream-ordered releases) and creating (stream-ordered
    # allocations) solvers while requests run
    small = max(int(budget * 0.2), 8 << 30)
    pool = serving.SolverPool(small)
    arr = workloads.poisson_arrivals(count, 0.8 * sat["requests_per_s"]) * 1e3
    res = serving.latency_summary(
        serving.serve(jobs, list(arr), budget=small, streams=streams, pool=pool))
    res.update({"budget_bytes": small, "solvers_created": pool.created,
                "solvers_evicted": pool.evicted})
    print(f"[bench] serving load 0.8, evicting pool: {res}", file=sys.stderr,
          flush=True)
    out["poisson_evicting"] = res
    pool.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="bw1m")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-fp64-comparison", action="store_true")
    ap.add_argument("--no-forces-only", action="store_true")
    ap.add_argument("--no-slit-channel", action="store_true")
    ap.add_argument("--no-torque-derivative", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=512)
    ap.add_argument("--copy-calibrate", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for "
                         "the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must "
                          "be 1 (multi-GPU sharding is a design note only)"}))
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibrate:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4,
                          "copy_bytes_written": dst.numel() * 4,
                          "launches": 3}), flush=True)
        return

    import workloads
    from paper_2210_01837_amd import Solver

    name = args.workload
    wl = workloads.WORKLOADS[name]
    box = wl.box
    pos, F, T = workloads.particles(name)
    dt = torch.float32 if wl.precision == "mixed" else torch.float64
    P = torch.tensor(pos, dtype=dt, device="cuda")
    Fd = torch.tensor(F, dtype=dt, device="cuda")
    # forces-only workloads: no torques in, no angular velocities out
    Td = torch.tensor(T, dtype=dt, device="cuda") if wl.torques else None
    U = torch.empty_like(P)
    Om = torch.empty_like(P) if wl.torques else None
    s = Solver.from_box(box, precision=wl.precision, max_particles=wl.n)
    print(f"[bench] {name}: N={wl.n} grid {box.Nx}x{box.Ny}x{box.Nz} "
          f"{wl.precision}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        s.apply(P, Fd, Td, U=U, Omega=Om, want_omega=wl.torques)
    torch.cuda.synchronize()
    s.stage_times()                         # discard warm-up events
    s.set_profiling(True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record()
    for i in range(args.steps):
        s.apply(P, Fd, Td, U=U, Omega=Om, want_omega=wl.torques)
        ev[i + 1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    per_apply = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps))
    s.set_profiling(False)
    stages, napplies, band = s.stage_times()
    code, bad = s.status()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = wl.n / (ms_per_step * 1e-3)
    avg = {k: v / max(1, napplies) for k, v in stages.items()}
    print(f"[bench] {ms_per_step:.3f} ms/apply, stages {avg}, band {band}",
          file=sys.stderr, flush=True)

    lowk = wl.precision == "mixed" and box.geometry == "sc"
    nbytes = stage_bytes(box, wl.n, band,
                         complex_bytes=8 if wl.precision == "mixed" else 16,
                         real_bytes=4 if wl.precision == "mixed" else 8,
                         torques=wl.torques, lowk=lowk)
    # dominant stage; its kernel (one launch per apply for the columns and
    # spread stages; the interp stage is its tile kernel plus a small
    # per-particle sum) is what the roofline describes
    dom = max((k for k in nbytes), key=lambda k: avg[k])
    achieved = nbytes[dom] / (avg[dom] * 1e-3) / 1e9
    kname = STAGE_KERNEL.get(dom)
    roofline = {"bound": "hbm", "kernel": kname or dom, "achieved": achieved,
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS,
                "traffic": measured_traffic(name, kname),
                "algorithmic_bytes": nbytes[dom], "avg_ms": avg[dom]}
    comp = measured_compute(name, kname, avg[dom])
    if comp is not None:
        roofline["compute"] = comp
    stage_gbs = {k: nbytes[k] / (avg[k] * 1e-3) / 1e9 for k in nbytes}
    # the same accounting with every plane transformed (P = Nz), for
    # comparison with a full-grid implementation
    full = stage_bytes(box, wl.n, (0, box.Nz - 1),
                       complex_bytes=8 if wl.precision == "mixed" else 16,
                       real_bytes=4 if wl.precision == "mixed" else 8,
                       torques=wl.torques)
    full_grid = {"bytes": full,
                 "gbs": {k: full[k] / (avg[k] * 1e-3) / 1e9 for k in full}}

    # accuracy on the seeded 1% sample, against stored oracle values
    # (a tiled layer is compared in full with its replica's stored values:
    # its solution is the replica's solution repeated)
    acc = None
    base = {"m663k": "m2048"}.get(name, name)
    gold = os.path.join(ROOT, "tests", "golden", f"{base}_oracle_sample.npz")
    if os.path.exists(gold):
        g = np.load(gold)
        idx = g["index"]
        Ua = U.double().cpu().numpy()
        if base != name:
            Uh = Ua.reshape(-1, len(idx), 3)
            gU = np.broadcast_to(g["U"], Uh.shape)
        else:
            Uh, gU = Ua[idx], g["U"]
        acc = {"rel_err_U": float(np.linalg.norm(Uh - gU) / np.linalg.norm(gU)),
               "sample": int(Uh.size // 3)}
        if Om is not None and "Omega" in g:
            Oh = Om.double().cpu().numpy()[idx]
            acc["rel_err_Omega"] = float(np.linalg.norm(Oh - g["Omega"]) /
                                         np.linalg.norm(g["Omega"]))

    forces_only = not wl.torques
    line = {
        "metric": ("particle mobility-applies/sec, forces only, N=663,552 "
                   "replicated layer" if forces_only else
                   "particle mobility-applies/sec at N=1M single wall"),
        "value": value,
        "unit": "particle-applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "ms_per_apply_median": per_apply[len(per_apply) // 2],
        "ms_per_apply_max": per_apply[-1],
        "higher_is_better": True,
        "scaling": "weak",
        # the paper prints a number for the forces-only layer only
        "vs_baseline": (value / PAPER_FORCES_ONLY_RATE
                        if name == "m663k" else None),
        "dtype": "f32+f64" if wl.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": name, "geometry": box.geometry, "N": wl.n,
                   "grid": [box.Nx, box.Ny, box.Nz], "box": [box.Lx, box.Ly, box.H],
                   "precision": wl.precision, "w": box.w,
                   "torques": wl.torques,
                   "beta_m": box.beta_m, "beta_d": box.beta_d,
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "stages_ms": avg,
        "stages_gbs": stage_gbs,
        "full_grid_accounting": full_grid,
        "band_planes": [band[0], band[1]],
        "domain_status": [code, bad],
        "accuracy": acc,
        "paper_context": "663,552 particles (forces only, m=4) in 370 ms on a "
                         "V100, i.e. ~1.79e6 particle-applies/s (Sec. 5.1)",
    }
    if forces_only:
        # Brownian displacements M^{1/2} W on the same layer (Sec. 5.2):
        # three digits (relative change below 1e-3), a fresh N(0,1) vector
        W = torch.tensor(workloads.random_array((wl.n, 3), 40), dtype=dt,
                         device="cuda")
        g, it, ch = s.lanczos_sqrt(P, W, max_iter=32, tol=1e-3)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        g, it, ch = s.lanczos_sqrt(P, W, max_iter=32, tol=1e-3, g=g)
        torch.cuda.synchronize()
        line["lanczos"] = {"iterations": it, "rel_change": ch, "tol": 1e-3,
                           "ms": (time.perf_counter() - t2) * 1e3,
                           "ms_per_iteration": (time.perf_counter() - t2) * 1e3 / max(1, it)}
        print(f"[bench] lanczos: {line['lanczos']}", file=sys.stderr, flush=True)
        del W, g
    del P, Fd, Td, U, Om
    s.close()
    if not args.no_fp64_comparison:
        line["fp64_comparison"] = fp64_comparison()
        print(f"[bench] fp64 comparison: {line['fp64_comparison']}",
              file=sys.stderr, flush=True)
    if not args.no_slit_channel and name == "bw1m":
        line["slit_channel"] = slit_channel_summary()
        print(f"[bench] slit channel: {line['slit_channel']}", file=sys.stderr,
              flush=True)
    if not args.no_torque_derivative and name == "bw1m":
        line["torque_derivative"] = torque_derivative_summary(name)
        print(f"[bench] torque derivative: {line['torque_derivative']}",
              file=sys.stderr, flush=True)
    if not args.no_forces_only and name != "m663k":
        line["forces_only"] = forces_only_summary()
        print(f"[bench] forces only: {line['forces_only']}", file=sys.stderr,
              flush=True)
    if not args.no_serving:
        sv = serving_bench(args.serving_requests)
        line["serving"] = sv
        p = sv["poisson"].get("0.8")
        if p:
            line["latency_p50_ms"] = p["p50_ms"]
            line["latency_p99_ms"] = p["p99_ms"]
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(name)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
