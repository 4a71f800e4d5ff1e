"""Write the stored oracle values used by the large-scale GPU parity tests.

    python tests/golden/make_fixtures.py [bw131k] [bw1m] [sc1m] [m2048]
                                         [serve_sc_max]

For each workload this draws the seeded inputs (workloads.particles), runs
the CPU oracle's full apply -- every particle is spread and the whole grid is
solved -- and interpolates only the seeded 1% sample (workloads.subsample).
It stores <name>_oracle_sample.npz with the sample indices and the oracle's
U and Omega (float64).  Only oracle/ and workloads/ are used.

``serve_sc_max`` is the slit-channel request with the most particles in the
512-request serving stream (its 1% sample, seeded).

Forces-only workloads (no torques) store U only.  ``m2048`` is one replica
of the tiled ``m663k`` layer; every particle is interpolated.  Its values
also serve the tiled layer: there the forcing is periodic with the replica's
period on a grid of the same spacing, so the discrete solution is the
replica's solution repeated (checked on a small tiling in the oracle tests).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import fcm, stokes  # noqa: E402


class _Req:
    """A serving request in the shape make() expects of a workload."""

    def __init__(self, r):
        self.box, self.n, self.torques = r.box, r.n, True


def make(name: str) -> str:
    if name == "serve_sc_max":
        r = workloads.largest_request("sc")
        wl = _Req(r)
        pos, F, T = workloads.request_particles(r)
        idx = np.sort(np.random.default_rng(workloads.SEED_BASE + 107).choice(
            r.n, size=max(1, r.n // 100), replace=False))
    else:
        wl = workloads.WORKLOADS[name]
        pos, F, T = workloads.particles(name)
        idx = workloads.subsample(name) if wl.n > 4096 else np.arange(wl.n)
    s = fcm.Solver(wl.box)
    t0 = time.time()
    p = s.wrap(pos)
    f, g = s.spread(p, F, T)
    print(f"{name}: spread {time.time() - t0:.0f} s", flush=True)
    Fh = stokes.forward_transform(wl.box, f)
    del f
    Gh = stokes.forward_transform(wl.box, g)
    del g
    uh, omh = stokes.solve_coefficients(wl.box, Fh, Gh)
    del Fh, Gh
    print(f"{name}: solve {time.time() - t0:.0f} s", flush=True)
    u = stokes.inverse_transform(wl.box, uh)
    del uh
    om = stokes.inverse_transform(wl.box, omh)
    del omh
    U, Om = s.interp(p[idx], u, om)
    out = os.path.join(HERE, f"{name}_oracle_sample.npz")
    if wl.torques:
        np.savez_compressed(out, index=idx, U=U, Omega=Om)
    else:
        np.savez_compressed(out, index=idx, U=U)
    print(f"{name}: wrote {out} ({len(idx)} particles) in {time.time() - t0:.0f} s",
          flush=True)
    return out


if __name__ == "__main__":
    names = sys.argv[1:] or ["bw131k", "bw1m", "sc1m"]
    for nm in names:
        make(nm)
