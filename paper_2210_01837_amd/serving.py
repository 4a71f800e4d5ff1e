"""Serving many mobility applies of different box sizes on one GPU.

A request is one mobility apply (F, T) -> (U, Omega) for its own particle set
and periodic box (geometry, L, grid).  The server

* keeps a pool of solvers keyed by every parameter of the discrete operator
  (geometry, box, grid, kernel width and shapes, viscosity, slip lengths and
  wall velocities), the precision and the particle capacity: a solver owns
  the grid, spectrum, sort buffers and FFT plans of one shape, so a repeated
  shape reuses them (the plan cache); solvers are created and released in
  stream order on the pool's own stream, so neither stalls the requests in
  flight;
* admits requests first-in first-out while the device workspace of everything
  in flight plus the next request fits the HBM budget (fcmdp_workspace_bytes,
  the admission-control query of the C ABI), and evicts idle solvers, least
  recently used first, to make room;
* runs admitted requests concurrently, one stream each, so small requests
  that do not fill the GPU overlap;
* records each request's latency: GPU completion time minus arrival time.

Every apply runs in libfcmdp's kernels; this module only schedules them.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

from .solver import Solver, workspace_bytes


def capacity_bucket(n: int, minimum: int = 1024) -> int:
    """Particle capacity a request of n particles is served with (the next
    power of two), so that similar requests share one solver."""
    c = minimum
    while c < n:
        c *= 2
    return c


# every parameter of the discrete operator (fcmdp_params), so that requests
# differing in any of them never share a solver
_KEY_FIELDS = ("geometry", "Lx", "Ly", "H", "Nx", "Ny", "Nz", "w", "beta_m",
               "beta_d", "eta", "slip0", "slipH", "wall0", "wallH",
               "torque_route")
_DEFAULTS = {"w": 6, "beta_m": 1.327 * 6, "beta_d": 2.216 * 6, "eta": 1.0,
             "slip0": 0.0, "slipH": 0.0, "wall0": (0.0, 0.0),
             "wallH": (0.0, 0.0), "torque_route": "curl"}


def _field(box, name):
    v = getattr(box, name, _DEFAULTS.get(name))
    if name in ("geometry", "torque_route"):
        return v
    if name in ("Nx", "Ny", "Nz", "w"):
        return int(v)
    if name in ("wall0", "wallH"):
        return tuple(float(x) for x in v)
    return float(v)


def solver_key(box, n: int, precision: str):
    """(box and operator parameters, precision, particle capacity)."""
    return tuple(_field(box, f) for f in _KEY_FIELDS) + (precision,
                                                          capacity_bucket(n))


def key_params(key) -> dict:
    """Keyword arguments of Solver / workspace_bytes for a solver key."""
    kw = dict(zip(_KEY_FIELDS, key[:len(_KEY_FIELDS)]))
    kw["precision"] = key[len(_KEY_FIELDS)]
    return kw


def key_capacity(key) -> int:
    return key[len(_KEY_FIELDS) + 1]


def key_bytes(key) -> int:
    return workspace_bytes(key_capacity(key), **key_params(key))


class AdmissionQueue:
    """First-in first-out admission under a byte budget."""

    def __init__(self, budget: int):
        self.budget = int(budget)
        self.in_use = 0
        self._q = collections.deque()

    def __len__(self):
        return len(self._q)

    def push(self, item, nbytes: int):
        if nbytes > self.budget:
            raise ValueError(f"request needs {nbytes} B of workspace, more "
                             f"than the whole budget of {self.budget} B")
        self._q.append((item, int(nbytes)))

    def head_fits(self) -> bool:
        return bool(self._q) and self.in_use + self._q[0][1] <= self.budget

    def pop(self):
        item, nbytes = self._q.popleft()
        self.in_use += nbytes
        return item, nbytes

    def release(self, nbytes: int):
        self.in_use -= int(nbytes)
        assert self.in_use >= 0


class SolverPool:
    """Solvers by key; idle ones are evicted least recently used first when
    the allocated total would exceed the budget."""

    def __init__(self, budget: int, factory=None, sizer=key_bytes):
        self.budget = int(budget)
        self.allocated = 0
        self.created = 0
        self.evicted = 0
        self._idle = collections.OrderedDict()     # id -> (key, solver, bytes)
        self._factory = factory or self._make
        self._sizer = sizer
        self._setup = None          # stream of solver creation and release

    def _stream(self):
        if self._setup is None:
            import torch
            self._setup = torch.cuda.Stream()
        return self._setup

    def _make(self, key):
        # stream-ordered allocation on the pool's own stream: creating a
        # solver waits for that stream only, not for requests in flight
        return Solver(max_particles=key_capacity(key), stream=self._stream(),
                      **key_params(key))

    def _release(self, s):
        # stream-ordered release after the solver's last apply; no
        # synchronisation of the device or the host
        if hasattr(s, "close"):
            if self._factory == self._make:
                s.close(stream=self._stream())
            else:
                s.close()

    def get(self, key):
        """An idle solver for key (reused or newly created) and its bytes."""
        for sid, (k, s, b) in self._idle.items():
            if k == key:
                del self._idle[sid]
                return s, b
        need = self._sizer(key)
        while self.allocated + need > self.budget and self._idle:
            _, (k, s, b) = self._idle.popitem(last=False)
            self._release(s)
            self.allocated -= b
            self.evicted += 1
        if self.allocated + need > self.budget:
            raise MemoryError("no idle solver left to evict")
        s = self._factory(key)
        self.allocated += need
        self.created += 1
        return s, need

    def put(self, key, solver, nbytes):
        self._idle[id(solver)] = (key, solver, nbytes)

    def close(self):
        for _, s, b in self._idle.values():
            self._release(s)
            self.allocated -= b
        self._idle.clear()


@dataclass
class Job:
    rid: int
    box: object
    pos: object            # device tensors [n][3]
    F: object
    T: object
    U: object = None
    Omega: object = None
    arrival_ms: float = 0.0
    done_ms: float = 0.0
    key: tuple = field(default=None)

    @property
    def n(self):
        return int(self.pos.shape[0])

    @property
    def latency_ms(self):
        return self.done_ms - self.arrival_ms


def serve(jobs, arrival_ms, precision="mixed", budget=None, streams=4,
          pool=None):
    """Run jobs arriving at arrival_ms (host clock, from the start of the
    call) and return them with U, Omega and done_ms filled in.

    budget: device bytes for solver workspace (default: half the free HBM).
    pool: a SolverPool to reuse across calls (warm plan cache).
    """
    import torch

    if budget is None:
        free, _ = torch.cuda.mem_get_info()
        budget = free // 2
    own_pool = pool is None
    if own_pool:
        pool = SolverPool(budget)
    adm = AdmissionQueue(budget)
    free_streams = collections.deque(torch.cuda.Stream() for _ in range(streams))
    order = sorted(range(len(jobs)), key=lambda i: arrival_ms[i])
    pending = collections.deque(order)
    inflight = []
    for j, t in zip(jobs, arrival_ms):
        j.arrival_ms = float(t)
        j.key = solver_key(j.box, j.n, precision)
        if j.U is None:
            j.U = torch.empty_like(j.pos)
            j.Omega = torch.empty_like(j.pos)

    start = torch.cuda.Event(enable_timing=True)
    start.record()
    start.synchronize()
    t0 = time.perf_counter()
    while pending or len(adm) or inflight:
        now = (time.perf_counter() - t0) * 1e3
        while pending and jobs[pending[0]].arrival_ms <= now:
            j = jobs[pending.popleft()]
            adm.push(j, key_bytes(j.key))
        still = []
        for (j, s, nbytes, st, ev) in inflight:
            if ev.query():
                j.done_ms = start.elapsed_time(ev)
                pool.put(j.key, s, nbytes)
                adm.release(nbytes)
                free_streams.append(st)
            else:
                still.append((j, s, nbytes, st, ev))
        inflight = still
        while free_streams and adm.head_fits():
            j, nbytes = adm.pop()
            s, _ = pool.get(j.key)
            st = free_streams.popleft()
            s.apply(j.pos, j.F, j.T, U=j.U, Omega=j.Omega, stream=st)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(st)
            inflight.append((j, s, nbytes, st, ev))
        if not inflight and not len(adm) and pending:
            wait = jobs[pending[0]].arrival_ms - (time.perf_counter() - t0) * 1e3
            if wait > 0.2:
                time.sleep(wait * 1e-3 * 0.5)
    torch.cuda.synchronize()
    if own_pool:
        pool.close()
    return jobs


def latency_summary(jobs):
    import numpy as np
    lat = np.array([j.latency_ms for j in jobs])
    span = max(j.done_ms for j in jobs) - min(j.arrival_ms for j in jobs)
    return {"p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()),
            "makespan_ms": float(span),
            "requests": len(jobs),
            "particle_applies_per_s": float(sum(j.n for j in jobs) / (span * 1e-3)),
            "requests_per_s": float(len(jobs) / (span * 1e-3))}
