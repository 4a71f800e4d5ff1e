"""Seeded synthetic workloads for the doubly-periodic FCM mobility apply.

This module only draws inputs (positions, forces, torques, request streams) and
describes grid/box parameters.  It contains none of the method's arithmetic, so
both the CPU oracle and the GPU path can consume it without sharing code.

Recipes (all seeded with ``numpy.random.default_rng(221001837 + i)`` for
workload ``i``; draw order x, y, z, then F, then T):

* ``bw64``     -- bottom wall, FP64: N=64 on a 32x32 box, z ~ U[1.5, 5],
                  F, T ~ N(0,1); grid 48x48, Nz=32, H=8.
* ``sc4096``   -- slit channel, FP64: N=4096 on a 128x128 box, H=10,
                  z ~ U[1.2, 8.8], F, T ~ N(0,1); grid 192x192, Nz=48.
* ``bw131k``   -- bottom wall, mixed precision: N=131072 on a 512x512 box,
                  sedimented monolayer (z = 1.1 + Exp(0.3), i.e. the Boltzmann
                  density exp(-(z-1)/0.3) restricted to z >= 1.1),
                  F = (0,0,-1) + N(0,0.1^2), T = (0,1,0) + N(0,0.1^2);
                  grid 768x768, Nz=32, H=12.
* ``bw1m`` / ``sc1m`` -- the same monolayer at N=1,048,576 on a 1448x1448
                  box, grid 2176x2176, Nz=32, H=12, positions stored as FP32;
                  a seeded 1% subsample is used for oracle comparison.
* ``m2048`` / ``m663k`` -- the forces-only (monopole, kernel width m = 4)
                  performance test of Sec. 5 and its parameter table: one
                  replica of 2048 particles with L = 128.8 R_h, 150 x 150 grid
                  cells, Nz = 19, H = 9.1 R_h, beta/m = 1.87, area fraction
                  N pi R_h^2 / L^2 = 0.39; ``m663k`` tiles that replica
                  18 x 18 times (663,552 particles on 2700 x 2700 x 19).
                  Lengths are in units of the grid spacing h (R_h = 150/128.8
                  h), and x, y are multiples of 2^-11 so that the tiled
                  positions are exact in FP32: the tiled apply then equals the
                  one-replica apply replicated.  Heights (the paper shows a
                  two-layer distribution only as a figure): half the
                  particles at z/R_h = 1.1 + Exp(0.3), half at z/R_h = 3.3 +
                  N(0, 0.3^2) clipped to [2.4, 5]; F = (0,0,-1) + N(0,0.1^2)
                  (in units of the monolayer's gravity), no torques.
* ``serve``    -- 512 requests, N log-uniform in [1024, 262144], geometry
                  bottom wall or slit channel with equal odds, box side set for
                  N/L^2 = 0.4, grid spacing h = 1/1.731 (so the ES radius
                  1.731 h equals the unit particle radius), Nz=32, H=12.

The ES kernel uses width w=6 with the M&D optimum of the paper's Table 1:
beta_M = 1.327*6, beta_D = 2.216*6.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, replace

import numpy as np

SEED_BASE = 221001837
W = 6
BETA_M = 1.327 * W   # Table 1, m = 6, monopole
BETA_D = 2.216 * W   # Table 1, m = 6, dipole
RH_OVER_H = 1.731    # Table 1, m = 6

# forces-only test of Sec. 5 (lengths in units of h)
M_W = 4
M_BETA = 1.87 * M_W          # beta/m of the monopole-only performance test
M_RH = 150.0 / 128.8         # R_h in units of h (L = 128.8 R_h = 150 h)
M_H = 9.1 * M_RH
M_REPLICAS = 18


@dataclass(frozen=True)
class Box:
    """Box, grid and kernel parameters of one apply (lengths in units of a)."""
    geometry: str          # "bw" (bottom wall) or "sc" (slit channel)
    Lx: float
    Ly: float
    H: float
    Nx: int
    Ny: int
    Nz: int
    w: int = W
    beta_m: float = BETA_M
    beta_d: float = BETA_D
    eta: float = 1.0
    slip0: float = 0.0     # slip lengths of the slit channel's walls at
    slipH: float = 0.0     # z = 0 and z = H (App. A); 0 = no slip
    wall0: tuple = (0.0, 0.0)   # uniform (x, y) velocity of the wall at z = 0
    wallH: tuple = (0.0, 0.0)   # and of the slit channel's wall at z = H
    torque_route: str = "curl"  # "curl" (spectral curl) or "derivative"
                                # (derivative of the dipole kernel, Sec. 3.4)

    @property
    def h(self) -> float:
        return self.Lx / self.Nx


@dataclass(frozen=True)
class Workload:
    name: str
    index: int
    box: Box
    n: int
    precision: str         # "fp64" or "mixed"
    heights: str           # "uniform" or "monolayer"
    zlo: float = 0.0
    zhi: float = 0.0
    forces: str = "normal"  # "normal", "roller" or "gravity" (no torques)
    pos_fp32: bool = False
    torques: bool = True    # False: forces-only apply (T = None, no Omega)
    replicas: int = 1       # tile a base replica replicas x replicas times
    unit: float = 1.0       # particle radius in length units (heights)


WORKLOADS = {
    "bw64": Workload("bw64", 1, Box("bw", 32.0, 32.0, 8.0, 48, 48, 32), 64,
                     "fp64", "uniform", 1.5, 5.0),
    "sc4096": Workload("sc4096", 2, Box("sc", 128.0, 128.0, 10.0, 192, 192, 48),
                       4096, "fp64", "uniform", 1.2, 8.8),
    "bw131k": Workload("bw131k", 3, Box("bw", 512.0, 512.0, 12.0, 768, 768, 32),
                       131072, "mixed", "monolayer", forces="roller"),
    "bw1m": Workload("bw1m", 4, Box("bw", 1448.0, 1448.0, 12.0, 2176, 2176, 32),
                     1048576, "mixed", "monolayer", forces="roller", pos_fp32=True),
    "sc1m": Workload("sc1m", 4, Box("sc", 1448.0, 1448.0, 12.0, 2176, 2176, 32),
                     1048576, "mixed", "monolayer", forces="roller", pos_fp32=True),
    "m2048": Workload("m2048", 7, Box("bw", 150.0, 150.0, M_H, 150, 150, 19,
                                      w=M_W, beta_m=M_BETA, beta_d=M_BETA),
                      2048, "mixed", "bimodal", forces="gravity", torques=False,
                      unit=M_RH),
    "m663k": Workload("m663k", 7, Box("bw", 150.0 * M_REPLICAS, 150.0 * M_REPLICAS,
                                      M_H, 150 * M_REPLICAS, 150 * M_REPLICAS, 19,
                                      w=M_W, beta_m=M_BETA, beta_d=M_BETA),
                      2048 * M_REPLICAS ** 2, "mixed", "bimodal",
                      forces="gravity", torques=False, replicas=M_REPLICAS,
                      unit=M_RH),
}


def _draw(rng: np.random.Generator, n: int, L_x: float, L_y: float,
          heights: str, zlo: float, zhi: float, forces: str, unit: float = 1.0):
    x = rng.uniform(0.0, L_x, n)
    y = rng.uniform(0.0, L_y, n)
    if heights == "uniform":
        z = rng.uniform(zlo, zhi, n)
    elif heights == "bimodal":
        # two equally weighted layers (in units of the particle radius)
        low = 1.1 + rng.exponential(0.3, n)
        high = np.clip(3.3 + 0.3 * rng.standard_normal(n), 2.4, 5.0)
        z = unit * np.where(rng.uniform(size=n) < 0.5, low, high)
        # x, y on a 2^-11 lattice: exact in FP32 after tiling (|x| < 4096)
        x = np.round(x * 2048.0) / 2048.0
        y = np.round(y * 2048.0) / 2048.0
    else:
        z = 1.1 + rng.exponential(0.3, n)
    if forces == "normal":
        F = rng.standard_normal((n, 3))
        T = rng.standard_normal((n, 3))
    elif forces == "gravity":
        F = np.array([0.0, 0.0, -1.0]) + 0.1 * rng.standard_normal((n, 3))
        T = np.zeros((n, 3))
    else:
        F = np.array([0.0, 0.0, -1.0]) + 0.1 * rng.standard_normal((n, 3))
        T = np.array([0.0, 1.0, 0.0]) + 0.1 * rng.standard_normal((n, 3))
    pos = np.stack([x, y, z], axis=1)
    return pos, F, T


def _tile(pos, F, T, L_x, L_y, reps):
    """reps x reps periodic copies of one replica of side (L_x, L_y)."""
    a, b = np.meshgrid(np.arange(reps), np.arange(reps), indexing="ij")
    shift = np.stack([a.ravel() * L_x, b.ravel() * L_y,
                      np.zeros(reps * reps)], axis=1)
    pos_t = (pos[None, :, :] + shift[:, None, :]).reshape(-1, 3)
    return (pos_t, np.tile(F, (reps * reps, 1)), np.tile(T, (reps * reps, 1)))


def particles(name: str):
    """Seeded (pos, F, T) as float64 arrays of shape (N, 3).

    Mixed-precision workloads are rounded to float32 values here (and returned
    as float64 holding those exact float32 values) so that every consumer sees
    the same numbers.
    """
    wl = WORKLOADS[name]
    rng = np.random.default_rng(SEED_BASE + wl.index)
    r = wl.replicas
    Lx, Ly = wl.box.Lx / r, wl.box.Ly / r
    pos, F, T = _draw(rng, wl.n // (r * r), Lx, Ly, wl.heights, wl.zlo,
                      wl.zhi, wl.forces, wl.unit)
    if r > 1:
        pos, F, T = _tile(pos, F, T, Lx, Ly, r)
    if wl.precision == "mixed":
        pos = pos.astype(np.float32).astype(np.float64)
        F = F.astype(np.float32).astype(np.float64)
        T = T.astype(np.float32).astype(np.float64)
    return pos, F, T


def subsample(name: str, fraction: float = 0.01) -> np.ndarray:
    """Seeded sorted subsample of particle indices (the 1% oracle sample)."""
    wl = WORKLOADS[name]
    rng = np.random.default_rng(SEED_BASE + 100 + wl.index)
    k = max(1, int(round(fraction * wl.n)))
    return np.sort(rng.choice(wl.n, size=k, replace=False))


def sub_box(name: str, factor: int, factor_y: int | None = None):
    """A box 1/factor as wide in x (1/factor_y in y, default the same) with
    the same particle density, grid spacing and height.

    Used to time the CPU oracle on a bounded sample of a large workload and
    for small-box error studies; the sample is a fresh seeded draw with the
    same recipe.
    """
    wl = WORKLOADS[name]
    b = wl.box
    fy = factor if factor_y is None else factor_y
    box = replace(b, Lx=b.Lx / factor, Ly=b.Ly / fy, Nx=b.Nx // factor,
                  Ny=b.Ny // fy)
    box = replace(box, Lx=box.Nx * b.h, Ly=box.Ny * b.h)
    n = int(round(wl.n * (box.Lx * box.Ly) / (b.Lx * b.Ly)))
    rng = np.random.default_rng(SEED_BASE + 200 + wl.index)
    pos, F, T = _draw(rng, n, box.Lx, box.Ly, wl.heights, wl.zlo, wl.zhi,
                      wl.forces, wl.unit)
    if wl.precision == "mixed":
        pos = pos.astype(np.float32).astype(np.float64)
        F = F.astype(np.float32).astype(np.float64)
        T = T.astype(np.float32).astype(np.float64)
    return box, pos, F, T


def _smooth(n: int) -> bool:
    for p in (2, 3, 5, 7):
        while n % p == 0:
            n //= p
    return n == 1


def nearest_smooth_even(x: float) -> int:
    """Nearest even integer whose only prime factors are 2, 3, 5 and 7."""
    best = None
    c = max(8, int(round(x)))
    for d in range(0, 4 * c):
        for cand in (c - d, c + d):
            if cand >= 8 and cand % 2 == 0 and _smooth(cand):
                if best is None or abs(cand - x) < abs(best - x):
                    best = cand
        if best is not None and d > abs(best - x) + 1:
            break
    return best


@dataclass(frozen=True)
class Request:
    rid: int
    n: int
    box: Box
    seed: int


def serving_requests(count: int = 512, nmin: int = 1024, nmax: int = 262144,
                     area_fraction: float = 0.4, H: float = 12.0, Nz: int = 32):
    """The serving stream: per request N, geometry and a box sized for N."""
    rng = np.random.default_rng(SEED_BASE + 5)
    h0 = 1.0 / RH_OVER_H
    reqs = []
    for r in range(count):
        n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        geom = "bw" if rng.uniform() < 0.5 else "sc"
        L = math.sqrt(n / area_fraction)
        nx = nearest_smooth_even(L / h0)
        Lb = nx * h0
        reqs.append(Request(r, n, Box(geom, Lb, Lb, H, nx, nx, Nz),
                            SEED_BASE + 1000 + r))
    return reqs


def largest_request(geometry: str, count: int = 512) -> Request:
    """The request of the given geometry with the most particles in the
    serving stream of `count` requests."""
    reqs = [r for r in serving_requests(count) if r.box.geometry == geometry]
    return max(reqs, key=lambda r: r.n)


def request_particles(req: Request):
    """Monolayer particles of one serving request (float32-exact float64)."""
    rng = np.random.default_rng(req.seed)
    pos, F, T = _draw(rng, req.n, req.box.Lx, req.box.Ly, "monolayer", 0, 0,
                      "roller")
    return (pos.astype(np.float32).astype(np.float64),
            F.astype(np.float32).astype(np.float64),
            T.astype(np.float32).astype(np.float64))


def poisson_arrivals(count: int, rate: float, seed: int = SEED_BASE + 6):
    """Arrival times (seconds) of a Poisson process with the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, count))


def random_array(shape, seed: int, complex_: bool = False):
    """Seeded N(0,1) array (complex: independent real and imaginary parts);
    stage-level inputs for parity tests."""
    rng = np.random.default_rng(SEED_BASE + 300 + seed)
    a = rng.standard_normal(shape)
    if complex_:
        a = a + 1j * rng.standard_normal(shape)
    return a


def random_particles(box: Box, n: int, seed: int, zlo: float, zhi: float):
    """Seeded uniform particles in [0,Lx) x [0,Ly) x [zlo, zhi] with
    N(0,1) forces and torques."""
    rng = np.random.default_rng(SEED_BASE + 400 + seed)
    return _draw(rng, n, box.Lx, box.Ly, "uniform", zlo, zhi, "normal")
