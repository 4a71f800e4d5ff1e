"""GPU parity: every stage and the whole apply of libfcmdp against the oracle.

FP64 path: stages agree to ~1e-13 (rounding); the whole apply to 1e-10
(norm-wise relative error over the 3N-vectors U and Omega, separately).
Mixed path (FP32 spreading/FFT/interpolation, FP64 solves): 1e-5.
Sizes span several FFT factors (48 = 2^4*3, 192 = 2^6*3, 40 = 2^3*5, 56 = 2^3*7)
and ragged tiles; particle sets straddle the periodic seams and both walls.
"""
import numpy as np
import pytest

import workloads
from workloads import Box

from _parity import (band_of, max_rel, oracle_apply, oracle_fft_forward,
                     oracle_fft_inverse, oracle_interp, oracle_solve,
                     oracle_spread, particle_err, rel_err)
from oracle import fcm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _solver(box, precision, cap=1 << 16):
    from paper_2210_01837_amd import Solver
    return Solver.from_box(box, precision=precision, max_particles=cap)


def _dev(a, precision):
    dt = torch.float64 if precision == "fp64" else torch.float32
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(
        np.complex128 if t.is_complex() else np.float64)


BOXES = {
    "bw48": Box("bw", 32.0, 32.0, 8.0, 48, 48, 32),
    "sc40x56": Box("sc", 20.0, 28.0, 7.0, 40, 56, 24),
    "sc192": Box("sc", 128.0, 128.0, 10.0, 192, 192, 48),
}


def _particles(box, n, seed):
    alpha = 3 * box.h
    zhi = box.H - alpha - 0.05 if box.geometry == "bw" else box.H - 0.2
    pos, F, T = workloads.random_particles(box, n, seed, 0.2, zhi)
    # a few particles across the periodic seams and near the walls
    pos[0, :2] = [box.Lx - 1e-3, 0.3]
    pos[1, :2] = [0.2, box.Ly - 0.7 * box.h]
    pos[2, 2] = 0.4 * alpha
    if box.geometry == "sc":
        pos[3, 2] = box.H - 0.3 * alpha
    return pos, F, T


@pytest.mark.parametrize("name", ["bw48", "sc40x56"])
def test_stage_spread_fp64(name):
    box = BOXES[name]
    pos, F, T = _particles(box, 97, 1)
    print(f"[spread fp64] {name}", flush=True)
    s = _solver(box, "fp64")
    g = _np(s.stage_spread(_dev(pos, "fp64"), _dev(F, "fp64"), _dev(T, "fp64")))
    ref = oracle_spread(box, pos, F, T)
    assert rel_err(g, ref) < 1e-13
    assert max_rel(g, ref) < 1e-13


@pytest.mark.parametrize("name", ["bw48", "sc40x56"])
def test_stage_fft_roundtrip_fp64(name):
    box = BOXES[name]
    shape = (6, box.Nz, box.Ny, box.Nx)
    grid = workloads.random_array(shape, 2)
    lo, hi = 3, box.Nz - 2
    print(f"[fft fp64] {name}", flush=True)
    s = _solver(box, "fp64")
    spec = s.stage_fft_forward(_dev(grid, "fp64"), lo, hi)
    ref = oracle_fft_forward(box, grid, lo, hi)
    got = _np(spec)
    sl = slice(lo, hi + 1)
    assert rel_err(got[:, sl], ref[:, sl]) < 1e-14
    # inverse of a seeded spectrum
    sp = workloads.random_array(s.spectrum_shape(), 3, complex_=True)
    sp_t = torch.tensor(sp, dtype=torch.complex128, device="cuda")
    back = _np(s.stage_fft_inverse(sp_t, lo, hi))
    refb = oracle_fft_inverse(box, sp, lo, hi)
    assert rel_err(back[:, sl], refb[:, sl]) < 1e-13


@pytest.mark.parametrize("name", ["bw48", "sc40x56", "sc192"])
def test_stage_solve_fp64(name):
    box = BOXES[name]
    lo, hi = (2, box.Nz - 1) if box.geometry == "bw" else (0, box.Nz - 1)
    sp = workloads.random_array((6, box.Nz, box.Nx // 2 + 1, box.Ny), 4,
                                complex_=True)
    print(f"[solve fp64] {name}", flush=True)
    s = _solver(box, "fp64")
    got = _np(s.stage_solve(torch.tensor(sp, dtype=torch.complex128,
                                         device="cuda"), lo, hi))
    ref = oracle_solve(box, sp, lo, hi)
    sl = slice(lo, hi + 1)
    for ch in range(6):
        assert rel_err(got[ch, sl], ref[ch, sl]) < 1e-11, ch


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["bw48", "sc40x56"])
def test_stage_solve_in_place(name, precision):
    # the column kernels read every column whole before writing it: the
    # in-place solve gives the out-of-place bits
    box = BOXES[name]
    lo, hi = 1, box.Nz - 2
    sp = workloads.random_array((6, box.Nz, box.Nx // 2 + 1, box.Ny), 14,
                                complex_=True)
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    s = _solver(box, precision)
    a = torch.tensor(sp, dtype=dt, device="cuda")
    ref = s.stage_solve(a, lo, hi)
    b = a.clone()
    got = s.stage_solve(b, lo, hi, out=b)
    torch.cuda.synchronize()
    assert got.data_ptr() == b.data_ptr()
    assert torch.equal(got[:, lo:hi + 1], ref[:, lo:hi + 1])


@pytest.mark.parametrize("name", ["bw48", "sc40x56"])
def test_stage_interp_fp64(name):
    box = BOXES[name]
    pos, F, T = _particles(box, 61, 5)
    grid = workloads.random_array((6, box.Nz, box.Ny, box.Nx), 6)
    print(f"[interp fp64] {name}", flush=True)
    s = _solver(box, "fp64")
    U, Om = s.stage_interp(_dev(pos, "fp64"), _dev(grid, "fp64"))
    rU, rO = oracle_interp(box, pos, grid)
    assert rel_err(_np(U), rU) < 1e-13
    assert rel_err(_np(Om), rO) < 1e-13


# Shapes of the aligned-tile interpolation (32 x 16 tiles): whole and
# ragged last tiles, last tiles narrower than six nodes (a window then meets
# three tiles along that axis), and the smallest grid it takes (40 x 22).
INTERP_BOXES = {
    "bw48": BOXES["bw48"],
    "sc40x56": BOXES["sc40x56"],
    "bw68x70": Box("bw", 34.0, 35.0, 6.0, 68, 70, 16),
    "sc100x36": Box("sc", 50.0, 18.0, 6.0, 100, 36, 12),
    "bw40x22": Box("bw", 20.0, 11.0, 5.0, 40, 22, 12),
}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", list(INTERP_BOXES))
def test_stage_interp_tiles(name, precision):
    """Partial sums over aligned tiles against the oracle, the halo-tile
    kernel and itself (bit for bit on a second run)."""
    box = INTERP_BOXES[name]
    pos, F, T = _particles(box, 150, 21)
    grid = workloads.random_array((6, box.Nz, box.Ny, box.Nx), 22)
    if precision == "mixed":
        pos, grid = (a.astype(np.float32).astype(np.float64) for a in (pos, grid))
    print(f"[interp tiles] {name} {precision}", flush=True)
    s = _solver(box, precision)
    P, G = _dev(pos, precision), _dev(grid, precision)
    U, Om = s.stage_interp(P, G)
    U2, O2 = s.stage_interp(P, G)
    torch.cuda.synchronize()
    assert torch.equal(U, U2) and torch.equal(Om, O2)
    s.set_variant("halo_interp", 1)
    Uh, Oh = s.stage_interp(P, G)
    s.set_variant("halo_interp", 0)
    rU, rO = oracle_interp(box, pos, grid)
    tol = 1e-13 if precision == "fp64" else 2e-6
    for got, ref in ((U, rU), (Om, rO)):
        e, ep = rel_err(_np(got), ref), particle_err(_np(got), ref)
        print(f"  vs oracle rel {e:.3e} particle {ep:.3e}", flush=True)
        assert e < tol and ep < 4 * tol
    for got, ref in ((U, Uh), (Om, Oh)):
        e = rel_err(_np(got), _np(ref))
        print(f"  vs halo tiles rel {e:.3e}", flush=True)
        assert e < tol


@pytest.mark.parametrize("name", ["bw48", "sc40x56"])
def test_apply_fp64_small(name):
    box = BOXES[name]
    pos, F, T = _particles(box, 40, 7)
    print(f"[apply fp64] {name}", flush=True)
    s = _solver(box, "fp64")
    U, Om = s.apply(_dev(pos, "fp64"), _dev(F, "fp64"), _dev(T, "fp64"))
    rU, rO = oracle_apply(box, pos, F, T)
    assert rel_err(_np(U), rU) < 1e-10
    assert rel_err(_np(Om), rO) < 1e-10
    code, bad = s.status()
    assert code == 0 and bad == 0


@pytest.mark.parametrize("name", ["bw64", "sc4096"])
def test_apply_fp64_workloads(name):
    wl = workloads.WORKLOADS[name]
    pos, F, T = workloads.particles(name)
    print(f"[apply fp64 workload] {name}", flush=True)
    s = _solver(wl.box, "fp64", cap=wl.n)
    U, Om = s.apply(_dev(pos, "fp64"), _dev(F, "fp64"), _dev(T, "fp64"))
    rU, rO = oracle_apply(wl.box, pos, F, T)
    eU, eO = rel_err(_np(U), rU), rel_err(_np(Om), rO)
    print(f"  rel err U {eU:.3e} Omega {eO:.3e}", flush=True)
    assert eU < 1e-10 and eO < 1e-10


@pytest.mark.parametrize("name", ["bw48", "sc40x56"])
def test_apply_mixed_small(name):
    box = BOXES[name]
    pos, F, T = _particles(box, 40, 8)
    pos, F, T = (a.astype(np.float32).astype(np.float64) for a in (pos, F, T))
    print(f"[apply mixed] {name}", flush=True)
    s = _solver(box, "mixed")
    U, Om = s.apply(_dev(pos, "mixed"), _dev(F, "mixed"), _dev(T, "mixed"))
    rU, rO = oracle_apply(box, pos, F, T)
    eU, eO = rel_err(_np(U), rU), rel_err(_np(Om), rO)
    print(f"  rel err U {eU:.3e} Omega {eO:.3e}", flush=True)
    assert eU < 1e-5 and eO < 1e-5


def test_apply_deterministic_and_edge_cases():
    box = BOXES["sc40x56"]
    pos, F, T = _particles(box, 50, 9)
    print("[edge] determinism, no torque, no omega, n=0, capacity", flush=True)
    s = _solver(box, "mixed", cap=64)
    P, Fd, Td = _dev(pos, "mixed"), _dev(F, "mixed"), _dev(T, "mixed")
    U1, O1 = s.apply(P, Fd, Td)
    U2, O2 = s.apply(P, Fd, Td)
    assert torch.equal(U1, U2) and torch.equal(O1, O2)     # bitwise
    # torque-free apply equals the apply with zero torques
    U3, O3 = s.apply(P, Fd, None)
    U4, O4 = s.apply(P, Fd, torch.zeros_like(Td))
    assert torch.equal(U3, U4) and torch.equal(O3, O4)
    U5, O5 = s.apply(P, Fd, Td, want_omega=False)
    assert O5 is None and torch.equal(U5, U1)
    # empty input
    e = torch.empty((0, 3), dtype=torch.float32, device="cuda")
    s.apply(e, e, e)
    torch.cuda.synchronize()
    assert s.status() == (0, 0)
    # capacity
    from paper_2210_01837_amd import FcmdpError
    big = _dev(np.tile(pos, (2, 1)), "mixed")
    with pytest.raises(FcmdpError):
        s.apply(big, big, big)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_apply_dense_cluster(precision):
    """Hundreds of particles in a few cells: spread regions beyond the staged
    capacity (the global-memory path) and interpolation tiles with more home
    particles than one pass holds (several passes)."""
    box = BOXES["bw48"]
    pos, F, T = _particles(box, 420, 12)
    rng = np.random.default_rng(1234)
    # 400 of them in a 4 x 4-cell patch next to the periodic seam
    pos[20:, 0] = (box.Lx - 2 * box.h) + 4 * box.h * rng.random(400)
    pos[20:, 0] %= box.Lx
    pos[20:, 1] = 10.0 + 4 * box.h * rng.random(400)
    if precision == "mixed":
        pos, F, T = (a.astype(np.float32).astype(np.float64) for a in (pos, F, T))
    print(f"[dense cluster] {precision}", flush=True)
    s = _solver(box, precision)
    U, Om = s.apply(_dev(pos, precision), _dev(F, precision), _dev(T, precision))
    rU, rO = oracle_apply(box, pos, F, T)
    eU, eO = rel_err(_np(U), rU), rel_err(_np(Om), rO)
    print(f"  rel err U {eU:.3e} Omega {eO:.3e}", flush=True)
    tol = 1e-5 if precision == "mixed" else 1e-10
    assert eU < tol and eO < tol


def test_domain_errors_give_nan_and_status():
    box = BOXES["bw48"]
    pos, F, T = _particles(box, 30, 10)
    pos[4, 2] = -0.1                    # below the wall
    pos[7, 2] = box.H - 0.5             # kernel above the domain top
    print("[edge] domain errors", flush=True)
    s = _solver(box, "fp64")
    U, Om = s.apply(_dev(pos, "fp64"), _dev(F, "fp64"), _dev(T, "fp64"))
    U, Om = _np(U), _np(Om)
    assert np.all(np.isnan(U[[4, 7]])) and np.all(np.isnan(Om[[4, 7]]))
    assert s.status() == (-2, 2)
    good = np.ones(len(pos), bool)
    good[[4, 7]] = False
    rU, rO = oracle_apply(box, pos[good], F[good], T[good])
    assert rel_err(U[good], rU) < 1e-10 and rel_err(Om[good], rO) < 1e-10


def test_periodic_wrapping_of_inputs():
    box = BOXES["sc40x56"]
    pos, F, T = _particles(box, 20, 11)
    shifted = pos.copy()
    shifted[:, 0] += 3 * box.Lx
    shifted[:, 1] -= 2 * box.Ly
    print("[edge] wrapping", flush=True)
    s = _solver(box, "fp64")
    U1, O1 = s.apply(_dev(pos, "fp64"), _dev(F, "fp64"), _dev(T, "fp64"))
    U2, O2 = s.apply(_dev(shifted, "fp64"), _dev(F, "fp64"), _dev(T, "fp64"))
    assert rel_err(_np(U2), _np(U1)) < 1e-12
    assert rel_err(_np(O2), _np(O1)) < 1e-12


# --- single-precision transforms over many factorisations --------------------
# (row-owned kernels by default, the workgroup-per-row-batch kernels as the
# "generic_fft" variant); one band plane, compared with numpy's FFT in FP64 on
# the same float32-rounded input.
FFT_SIZES = [(48, 48), (40, 56), (96, 26), (90, 1000), (1536, 1000),
             (768, 768), (2176, 2176), (2700, 2700)]


def _fft_box(nx, ny, nz=8):
    h = 0.5
    return Box("bw", nx * h, ny * h, 4.0, nx, ny, nz)


@pytest.mark.parametrize("nx,ny", FFT_SIZES)
def test_stage_fft_mixed_sizes(nx, ny):
    box = _fft_box(nx, ny)
    lo = hi = 3
    nkx = nx // 2 + 1
    print(f"[fft mixed] {nx}x{ny}", flush=True)
    plane = workloads.random_array((6, ny, nx), 7).astype(np.float32)
    grid = torch.zeros((6, box.Nz, ny, nx), dtype=torch.float32, device="cuda")
    grid[:, lo] = torch.from_numpy(plane).cuda()
    ref = np.transpose(np.fft.rfft2(plane.astype(np.float64), axes=(-2, -1)),
                       (0, 2, 1))
    sp = workloads.random_array((6, nkx, ny), 8, complex_=True).astype(np.complex64)
    spec_in = torch.zeros((6, box.Nz, nkx, ny), dtype=torch.complex64, device="cuda")
    spec_in[:, lo] = torch.from_numpy(sp).cuda()
    refb = np.fft.irfft2(np.transpose(sp.astype(np.complex128), (0, 2, 1)),
                         s=(ny, nx), axes=(-2, -1)) * (nx * ny)
    s = _solver(box, "mixed", cap=16)
    results = {}
    for variant in ("default", "no_pipeline", "no_codelet", "generic_fft"):
        if variant != "default":
            s.set_variant(variant, 1)
        got = _np(s.stage_fft_forward(grid, lo, hi))
        assert rel_err(got[:, lo], ref) < 2e-6, variant
        back = _np(s.stage_fft_inverse(spec_in, lo, hi))
        assert rel_err(back[:, lo], refb) < 2e-6, variant
        # planes outside the band are neither read nor written
        assert not np.any(back[:, lo + 1])
        results[variant] = (got, back)
        if variant != "default":
            s.set_variant(variant, 0)
    # fixed-plan and run-time-plan kernels do the same butterflies (the
    # compiler may contract multiply-adds differently): agree to FP32 rounding
    sl = (slice(None), lo)
    assert rel_err(results["default"][0][sl], results["no_codelet"][0][sl]) < 1e-6
    assert rel_err(results["default"][1][sl], results["no_codelet"][1][sl]) < 1e-6
    # the persistent (prefetching) kernels run the same plan per row
    assert rel_err(results["default"][0][sl], results["no_pipeline"][0][sl]) < 1e-6
    assert rel_err(results["default"][1][sl], results["no_pipeline"][1][sl]) < 1e-6


@pytest.mark.parametrize("rows", [1, 2, 4, 8, 12, 16])
def test_stage_fft_mixed_rows_per_workgroup(rows):
    nx, ny = 1536, 1000
    box = _fft_box(nx, ny)
    lo = hi = 2
    print(f"[fft mixed rows] {rows}", flush=True)
    plane = workloads.random_array((6, ny, nx), 9).astype(np.float32)
    grid = torch.zeros((6, box.Nz, ny, nx), dtype=torch.float32, device="cuda")
    grid[:, lo] = torch.from_numpy(plane).cuda()
    s = _solver(box, "mixed", cap=16)
    base = _np(s.stage_fft_forward(grid, lo, hi))
    s.set_variant("fft_rows_x", rows)
    s.set_variant("fft_rows_y", min(rows, 8))
    got = _np(s.stage_fft_forward(grid, lo, hi))
    # same butterflies in the same order: identical bits
    assert np.array_equal(got, base)
    with pytest.raises(Exception):
        s.set_variant("fft_rows_x", 3)


# --- full-size workloads against stored oracle values ------------------------
# tests/golden/<name>_oracle_sample.npz holds the oracle's U and Omega of a
# seeded 1% particle sample (written by tests/golden/make_fixtures.py, which
# runs only the oracle).  The GPU runs the whole apply in the launch
# configuration the benchmark times and is compared on that sample.
#
# Mixed-precision tolerance: 1e-5 norm-wise in U and Omega.  The slit
# channel reaches it through the FP64 route for the vertical force of its
# kH < 1 columns (without it the FP32 rounding of f_z, amplified by the
# small-kH response of the slit channel, gives ~8e-5 at N = 1M).  The largest
# single-particle error (relative to the RMS particle velocity) must stay
# within ten times that.
GOLDEN = {"bw131k": 1e-5, "bw1m": 1e-5, "sc1m": 1e-5}


def _golden(name):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden",
                        f"{name}_oracle_sample.npz")
    if not os.path.exists(path):
        pytest.skip(f"no stored oracle sample for {name}")
    return np.load(path)


@pytest.mark.parametrize("name", ["bw1m", "sc1m"])
def test_interp_tiles_full_size_every_particle(name):
    """At N = 1M, every particle's U and Omega from the aligned-tile
    interpolation against the halo-tile kernel in the same apply (the two
    differ only in the summation order of the FP32 interpolation)."""
    wl = workloads.WORKLOADS[name]
    pos, F, T = workloads.particles(name)
    print(f"[interp tiles full size] {name} N={len(pos)}", flush=True)
    from paper_2210_01837_amd import Solver
    s = Solver.from_box(wl.box, precision="mixed", max_particles=wl.n)
    P, Fd, Td = _dev(pos, "mixed"), _dev(F, "mixed"), _dev(T, "mixed")
    U, Om = s.apply(P, Fd, Td)
    s.set_variant("halo_interp", 1)
    Uh, Oh = s.apply(P, Fd, Td)
    assert s.status() == (0, 0)
    for got, ref in ((U, Uh), (Om, Oh)):
        g, r = _np(got), _np(ref)
        assert np.all(np.isfinite(g))
        e, ep = rel_err(g, r), particle_err(g, r)
        print(f"  rel {e:.2e} max particle {ep:.2e}", flush=True)
        assert e < 1e-6 and ep < 1e-5
    s.close()


def test_spread_mfma_full_size_every_particle():
    """At N = 1M, every particle's U and Omega with the matrix-core spread
    against the per-patch gather spread in the same apply (FP32 sums in a
    different order)."""
    wl = workloads.WORKLOADS["bw1m"]
    pos, F, T = workloads.particles("bw1m")
    print(f"[spread mfma full size] bw1m N={len(pos)}", flush=True)
    from paper_2210_01837_amd import Solver
    s = Solver.from_box(wl.box, precision="mixed", max_particles=wl.n)
    P, Fd, Td = _dev(pos, "mixed"), _dev(F, "mixed"), _dev(T, "mixed")
    U, Om = s.apply(P, Fd, Td)
    s.set_variant("wave_spread", 1)
    Uw, Ow = s.apply(P, Fd, Td)
    assert s.status() == (0, 0)
    # each spread is within 2.3e-6 (U) of the oracle at this size (the
    # golden test), so the two agree to their sum; per particle 10x that,
    # as in the golden tests
    for got, ref in ((U, Uw), (Om, Ow)):
        g, r = _np(got), _np(ref)
        e, ep = rel_err(g, r), particle_err(g, r)
        print(f"  rel {e:.2e} max particle {ep:.2e}", flush=True)
        assert e < 5e-6 and ep < 5e-5
    s.close()


@pytest.mark.parametrize("name", list(GOLDEN))
def test_apply_mixed_full_size_golden(name):
    g = _golden(name)
    wl = workloads.WORKLOADS[name]
    pos, F, T = workloads.particles(name)
    print(f"[golden mixed] {name} N={len(pos)}", flush=True)
    from paper_2210_01837_amd import Solver
    s = Solver.from_box(wl.box, precision="mixed", max_particles=wl.n)
    U, Om = s.apply(_dev(pos, "mixed"), _dev(F, "mixed"), _dev(T, "mixed"))
    assert s.status() == (0, 0)
    idx = g["index"]
    assert np.array_equal(idx, workloads.subsample(name))
    Ug, Og = _np(U)[idx], _np(Om)[idx]
    eU, eO = rel_err(Ug, g["U"]), rel_err(Og, g["Omega"])
    pU, pO = particle_err(Ug, g["U"]), particle_err(Og, g["Omega"])
    print(f"  rel err U {eU:.2e} Omega {eO:.2e}; max particle {pU:.2e} "
          f"{pO:.2e}", flush=True)
    assert eU < GOLDEN[name] and eO < GOLDEN[name]
    assert pU < 10 * GOLDEN[name] and pO < 10 * GOLDEN[name]
    s.close()


@pytest.mark.parametrize("name,tol", [("bw1m", 1e-12), ("sc1m", 1e-11)])
def test_apply_fp64_full_size_golden(name, tol):
    # measured 3.3e-14 (bw1m) and 3.6e-13 (sc1m; the slit channel's kH < 0.1
    # columns amplify rounding, the oracle itself agrees with extended
    # precision to 2e-10 per column there)
    g = _golden(name)
    wl = workloads.WORKLOADS[name]
    pos, F, T = workloads.particles(name)
    print(f"[golden fp64] {name} N={len(pos)}", flush=True)
    from paper_2210_01837_amd import Solver
    s = Solver.from_box(wl.box, precision="fp64", max_particles=wl.n)
    U, Om = s.apply(_dev(pos, "fp64"), _dev(F, "fp64"), _dev(T, "fp64"))
    assert s.status() == (0, 0)
    idx = g["index"]
    Ug, Og = _np(U)[idx], _np(Om)[idx]
    eU, eO = rel_err(Ug, g["U"]), rel_err(Og, g["Omega"])
    pU, pO = particle_err(Ug, g["U"]), particle_err(Og, g["Omega"])
    print(f"  rel err U {eU:.2e} Omega {eO:.2e}; max particle {pU:.2e} "
          f"{pO:.2e}", flush=True)
    assert eU < tol and eO < tol and pU < 10 * tol and pO < 10 * tol
    s.close()


# --- forces-only apply (no torques, no angular velocities) at m = 4 ----------
# The paper's timed configuration (Sec. 5): monopole kernel of width 4,
# beta/m = 1.87; the apply then carries three channels through every stage.
M_BOXES = {
    "bw30x36_m4": Box("bw", 30.0, 36.0, 9.0, 30, 36, 19, w=4, beta_m=7.48,
                      beta_d=7.48),
    "sc40_m4": Box("sc", 40.0, 40.0, 8.0, 40, 40, 20, w=4, beta_m=7.48,
                   beta_d=7.48),
}


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("name", list(M_BOXES))
def test_apply_forces_only_m4(name, precision):
    box = M_BOXES[name]
    pos, F, _ = _particles(box, 60, 13)
    if precision == "mixed":
        pos, F = (a.astype(np.float32).astype(np.float64) for a in (pos, F))
    print(f"[forces only m=4] {name} {precision}", flush=True)
    s = _solver(box, precision)
    P, Fd = _dev(pos, precision), _dev(F, precision)
    U, Om = s.apply(P, Fd, None, want_omega=False)
    assert Om is None
    zero = np.zeros_like(F)
    rU, _ = oracle_apply(box, pos, F, zero)
    eU = rel_err(_np(U), rU)
    print(f"  rel err U {eU:.3e}", flush=True)
    assert eU < (1e-5 if precision == "mixed" else 1e-10)
    # three channels give the same bits as six with zero torques
    U6, _ = s.apply(P, Fd, torch.zeros_like(Fd))
    assert torch.equal(U, U6)
    assert s.status() == (0, 0)


def test_apply_forces_only_replicated_layer():
    """The paper's forces-only layer: 663,552 particles (18 x 18 copies of a
    2048-particle replica) on 2700 x 2700 x 19.  Its solution is the
    replica's solution repeated, so every particle is checked against the
    oracle's apply of one replica (stored values)."""
    g = _golden("m2048")
    assert np.array_equal(g["index"], np.arange(2048))
    rU = g["U"]
    for name in ("m2048", "m663k"):
        wl = workloads.WORKLOADS[name]
        pos, F, _ = workloads.particles(name)
        print(f"[forces only layer] {name} N={wl.n}", flush=True)
        s = _solver(wl.box, "mixed", cap=wl.n)
        U, Om = s.apply(_dev(pos, "mixed"), _dev(F, "mixed"), None,
                        want_omega=False)
        got = _np(U).reshape(-1, len(rU), 3)
        e = rel_err(got, np.broadcast_to(rU, got.shape))
        worst = max(rel_err(got[r], rU) for r in range(got.shape[0]))
        print(f"  rel err U {e:.3e} (worst replica {worst:.3e})", flush=True)
        assert e < 1e-5 and worst < 1e-5
        assert s.status() == (0, 0)
        s.close()
        del U


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("name", ["bw48", "sc192"])
def test_channel_modes_give_the_same_bits(name, precision):
    """Without torques (T = None) the spread, transforms and solve carry the
    three force channels; without Omega the solve returns three channels.
    Every combination gives the velocities (and, where asked, angular
    velocities) of the six-channel apply with zero torques bit for bit.
    sc192 (Nz = 48) runs the one-thread-per-column solve, bw48 the
    eight-lane one."""
    box = BOXES[name]
    pos, F, T = _particles(box, 50, 14)
    if precision == "mixed":
        pos, F, T = (a.astype(np.float32).astype(np.float64) for a in (pos, F, T))
    print(f"[channel modes] {name} {precision}", flush=True)
    s = _solver(box, precision)
    P, Fd, Td = _dev(pos, precision), _dev(F, precision), _dev(T, precision)
    Z = torch.zeros_like(Td)
    U0, O0 = s.apply(P, Fd, Z)                            # 6 in, 6 out
    U1, O1 = s.apply(P, Fd, None)                         # 3 in, 6 out
    U2, O2 = s.apply(P, Fd, None, want_omega=False)       # 3 in, 3 out
    assert torch.equal(U1, U0) and torch.equal(O1, O0)
    assert O2 is None and torch.equal(U2, U0)
    U3, O3 = s.apply(P, Fd, Td)                           # 6 in, 6 out
    U4, O4 = s.apply(P, Fd, Td, want_omega=False)         # 6 in, 3 out
    assert O4 is None and torch.equal(U4, U3)
    rU, rO = oracle_apply(box, pos, F, T)
    tol = 1e-5 if precision == "mixed" else 1e-10
    assert rel_err(_np(U4), rU) < tol and rel_err(_np(O3), rO) < tol


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("nz,geometry", [(8, "bw"), (64, "bw"), (64, "sc")])
def test_apply_smallest_and_largest_nz(nz, geometry, precision):
    """Nz = 8 and Nz = 64, the limits the library accepts (Nz > 32 runs the
    one-thread-per-column solve)."""
    box = Box(geometry, 16.0, 16.0, 6.0, 24, 24, nz)
    pos, F, T = _particles(box, 30, 15)
    if precision == "mixed":
        pos, F, T = (a.astype(np.float32).astype(np.float64) for a in (pos, F, T))
    print(f"[nz limits] {geometry} Nz={nz} {precision}", flush=True)
    s = _solver(box, precision)
    U, Om = s.apply(_dev(pos, precision), _dev(F, precision), _dev(T, precision))
    rU, rO = oracle_apply(box, pos, F, T)
    eU, eO = rel_err(_np(U), rU), rel_err(_np(Om), rO)
    print(f"  rel err U {eU:.3e} Omega {eO:.3e}", flush=True)
    tol = 1e-5 if precision == "mixed" else 1e-10
    assert eU < tol and eO < tol


# --- slit channel with partial slip (App. A) ----------------------------------
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("slip", [(0.5, 2.0), (3.0, 0.0), (0.0, 0.7)])
def test_apply_slit_channel_partial_slip(slip, precision):
    from dataclasses import replace
    box = replace(BOXES["sc40x56"], slip0=slip[0], slipH=slip[1])
    pos, F, T = _particles(box, 40, 16)
    if precision == "mixed":
        pos, F, T = (a.astype(np.float32).astype(np.float64) for a in (pos, F, T))
    print(f"[slip] {slip} {precision}", flush=True)
    s = _solver(box, precision)
    U, Om = s.apply(_dev(pos, precision), _dev(F, precision), _dev(T, precision))
    rU, rO = oracle_apply(box, pos, F, T)
    eU, eO = rel_err(_np(U), rU), rel_err(_np(Om), rO)
    print(f"  rel err U {eU:.3e} Omega {eO:.3e}", flush=True)
    tol = 1e-5 if precision == "mixed" else 1e-10
    assert eU < tol and eO < tol
    # the forces-only kernel and the FP64 eight-lane kernel take the same rows
    U2, _ = s.apply(_dev(pos, precision), _dev(F, precision), None,
                    want_omega=False)
    rU2, _ = oracle_apply(box, pos, F, np.zeros_like(T))
    assert rel_err(_np(U2), rU2) < tol


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("l0", [0.6, 3.0])
def test_apply_bottom_wall_partial_slip(l0, precision):
    # a slip length at the bottom wall (the slit channel's condition at
    # z = 0 with the decaying correction modes only)
    from dataclasses import replace
    box = replace(BOXES["bw48"], slip0=l0)
    pos, F, T = _particles(box, 40, 18)
    if precision == "mixed":
        pos, F, T = (a.astype(np.float32).astype(np.float64) for a in (pos, F, T))
    print(f"[bottom wall slip] {l0} {precision}", flush=True)
    s = _solver(box, precision)
    U, Om = s.apply(_dev(pos, precision), _dev(F, precision), _dev(T, precision))
    rU, rO = oracle_apply(box, pos, F, T)
    eU, eO = rel_err(_np(U), rU), rel_err(_np(Om), rO)
    print(f"  rel err U {eU:.3e} Omega {eO:.3e}", flush=True)
    tol = 1e-5 if precision == "mixed" else 1e-10
    assert eU < tol and eO < tol
    U2, _ = s.apply(_dev(pos, precision), _dev(F, precision), None,
                    want_omega=False)
    rU2, _ = oracle_apply(box, pos, F, np.zeros_like(T))
    assert rel_err(_np(U2), rU2) < tol
    # the slip branch changes the result: no-slip gives another answer
    U0, _ = oracle_apply(BOXES["bw48"], pos, F, T)
    assert rel_err(U0, rU) > 1e-3


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("case", ["bw", "bw_slip", "sc", "sc_slip"])
def test_apply_moving_walls(case, precision):
    """Uniform wall velocities (and slip) with particles forced as usual."""
    from dataclasses import replace
    if case in ("bw", "bw_slip"):
        box = replace(BOXES["bw48"], wall0=(0.4, -0.3))
        if case == "bw_slip":
            box = replace(box, slip0=1.2)
    else:
        box = replace(BOXES["sc40x56"], wall0=(0.3, -0.2), wallH=(-0.5, 0.6))
        if case == "sc_slip":
            box = replace(box, slip0=0.8, slipH=1.5)
    pos, F, T = _particles(box, 40, 17)
    if precision == "mixed":
        pos, F, T = (a.astype(np.float32).astype(np.float64) for a in (pos, F, T))
    print(f"[moving walls] {case} {precision}", flush=True)
    s = _solver(box, precision)
    U, Om = s.apply(_dev(pos, precision), _dev(F, precision), _dev(T, precision))
    rU, rO = oracle_apply(box, pos, F, T)
    eU, eO = rel_err(_np(U), rU), rel_err(_np(Om), rO)
    print(f"  rel err U {eU:.3e} Omega {eO:.3e}", flush=True)
    tol = 1e-5 if precision == "mixed" else 1e-10
    assert eU < tol and eO < tol


def test_apply_forces_only_replicated_layer_fp64():
    """The 663,552-particle forces-only layer on the all-FP64 path: every
    particle against the oracle's one-replica apply."""
    g = _golden("m2048")
    rU = g["U"]
    wl = workloads.WORKLOADS["m663k"]
    pos, F, _ = workloads.particles("m663k")
    print("[forces only layer fp64] m663k", flush=True)
    s = _solver(wl.box, "fp64", cap=wl.n)
    U, _ = s.apply(_dev(pos, "fp64"), _dev(F, "fp64"), None, want_omega=False)
    got = _np(U).reshape(-1, len(rU), 3)
    e = rel_err(got, np.broadcast_to(rU, got.shape))
    print(f"  rel err U {e:.3e}", flush=True)
    assert e < 1e-9
    assert s.status() == (0, 0)
    s.close()
