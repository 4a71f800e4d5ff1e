"""Python binding of the MI355X doubly-periodic FCM mobility apply.

Argument marshalling only: every step runs in libfcmdp's HIP kernels.  Torch
tensors provide device memory and the current HIP stream.
"""
from __future__ import annotations

import ctypes

from . import _lib as L

GEOMETRY = {"bw": L.BOTTOM_WALL, "sc": L.SLIT_CHANNEL,
            "bottom_wall": L.BOTTOM_WALL, "slit_channel": L.SLIT_CHANNEL}
PRECISION = {"fp64": L.FP64, "mixed": L.MIXED}


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


TORQUE_ROUTE = {"curl": L.TORQUE_CURL, "derivative": L.TORQUE_DERIVATIVE}


def make_params(geometry, Lx, Ly, H, Nx, Ny, Nz, w=6, beta_m=1.327 * 6,
                beta_d=2.216 * 6, eta=1.0, precision="mixed",
                max_particles=0, slip0=0.0, slipH=0.0, wall0=(0.0, 0.0),
                wallH=(0.0, 0.0), torque_route="curl") -> L.Params:
    arr = ctypes.c_double * 2
    return L.Params(GEOMETRY[geometry], float(Lx), float(Ly), float(H),
                    int(Nx), int(Ny), int(Nz), int(w), float(beta_m),
                    float(beta_d), float(eta), PRECISION[precision],
                    int(max_particles), float(slip0), float(slipH),
                    arr(*map(float, wall0)), arr(*map(float, wallH)),
                    TORQUE_ROUTE[torque_route])


def workspace_bytes(n, **kw) -> int:
    p = make_params(**kw)
    out = ctypes.c_size_t(0)
    L.check(L.lib().fcmdp_workspace_bytes(ctypes.byref(p), int(n),
                                          ctypes.byref(out)),
            "fcmdp_workspace_bytes")
    return out.value


class Solver:
    """create_solver(geometry, Lx, Ly, H, grid, w, beta) of the C ABI."""

    def __init__(self, geometry, Lx, Ly, H, Nx, Ny, Nz, w=6, beta_m=1.327 * 6,
                 beta_d=2.216 * 6, eta=1.0, precision="mixed",
                 max_particles=1 << 20, slip0=0.0, slipH=0.0, wall0=(0.0, 0.0),
                 wallH=(0.0, 0.0), torque_route="curl", stream=None):
        self.params = make_params(geometry, Lx, Ly, H, Nx, Ny, Nz, w, beta_m,
                                  beta_d, eta, precision, max_particles, slip0,
                                  slipH, wall0, wallH, torque_route)
        self.precision = precision
        self.Nx, self.Ny, self.Nz = int(Nx), int(Ny), int(Nz)
        self._h = ctypes.c_void_p(0)
        self._last = None          # event after the last call's device work
        L.check(L.lib().fcmdp_create_solver(ctypes.byref(self.params),
                                            _stream(stream),
                                            ctypes.byref(self._h)),
                "fcmdp_create_solver")

    @classmethod
    def from_box(cls, box, precision="mixed", max_particles=1 << 20,
                 stream=None):
        return cls(box.geometry, box.Lx, box.Ly, box.H, box.Nx, box.Ny, box.Nz,
                   box.w, box.beta_m, box.beta_d, box.eta, precision,
                   max_particles, getattr(box, "slip0", 0.0),
                   getattr(box, "slipH", 0.0), getattr(box, "wall0", (0.0, 0.0)),
                   getattr(box, "wallH", (0.0, 0.0)),
                   getattr(box, "torque_route", "curl"), stream=stream)

    def _mark(self, stream):
        """Record the end of this call's device work (close() orders the
        release of the workspace after it)."""
        import torch
        st = torch.cuda.current_stream() if stream is None else stream
        ev = torch.cuda.Event()
        ev.record(st)
        self._last = ev

    @property
    def dtype(self):
        import torch
        return torch.float64 if self.precision == "fp64" else torch.float32

    def close(self, stream=None):
        """Release the device workspace in stream order on `stream` (default:
        the current stream), after the last call's work; no device-wide
        synchronisation."""
        if self._h and self._h.value:
            import torch
            st = torch.cuda.current_stream() if stream is None else stream
            if self._last is not None:
                st.wait_event(self._last)
            L.lib().fcmdp_destroy_solver(self._h, ctypes.c_void_p(st.cuda_stream))
            self._h = ctypes.c_void_p(0)
            self._last = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        out = (ctypes.c_double * 4)()
        L.check(L.lib().fcmdp_solver_info(self._h, out), "fcmdp_solver_info")
        return {"h": out[0], "alpha": out[1], "norm_m": out[2],
                "norm_d": out[3]}

    def _check_particles(self, *ts):
        for t in ts:
            if t is None:
                continue
            if t.dtype != self.dtype or not t.is_cuda or not t.is_contiguous():
                raise TypeError("particle arrays must be contiguous device "
                                f"tensors of dtype {self.dtype}")
            if t.dim() != 2 or t.shape[1] != 3:
                raise ValueError("particle arrays must have shape (n, 3)")

    def apply(self, pos, F, T=None, U=None, Omega=None, want_omega=True,
              stream=None):
        """(U, Omega) = M (F, T); Omega is None if want_omega is False."""
        import torch
        n = pos.shape[0]
        if U is None:
            U = torch.empty((n, 3), dtype=self.dtype, device=pos.device)
        if Omega is None and want_omega:
            Omega = torch.empty((n, 3), dtype=self.dtype, device=pos.device)
        self._check_particles(pos, F, T, U, Omega)
        L.check(L.lib().fcmdp_apply_mobility(
            self._h, n, _ptr(pos), _ptr(F), _ptr(T), _ptr(U), _ptr(Omega),
            _stream(stream)), "fcmdp_apply_mobility")
        self._mark(stream)
        return U, Omega

    def lanczos_sqrt(self, pos, W, max_iter=32, tol=1e-3, g=None, stream=None):
        """g = M^{1/2} W for the translational mobility (fcmdp_lanczos_sqrt).

        Returns (g, iterations, last relative change)."""
        import torch
        n = pos.shape[0]
        if g is None:
            g = torch.empty((n, 3), dtype=self.dtype, device=pos.device)
        self._check_particles(pos, W, None, g, None)
        it = ctypes.c_int(0)
        ch = ctypes.c_double(0.0)
        L.check(L.lib().fcmdp_lanczos_sqrt(
            self._h, n, _ptr(pos), _ptr(W), _ptr(g), int(max_iter), float(tol),
            ctypes.byref(it), ctypes.byref(ch), _stream(stream)),
            "fcmdp_lanczos_sqrt")
        self._mark(stream)
        return g, it.value, ch.value

    def set_wall_velocity(self, wall, stream=None):
        """Non-uniform tangential wall velocities (fcmdp_set_wall_velocity):
        a contiguous device tensor (nw, 2, Ny, Nx) of the solver's dtype with
        (u^W, v^W) at the grid nodes of the wall at z = 0 (and at z = H for
        the slit channel, nw = 2), or None to remove the field."""
        if wall is not None:
            nw = 2 if self.params.geometry == 1 else 1
            if (wall.dtype != self.dtype or not wall.is_cuda or
                    not wall.is_contiguous()):
                raise TypeError("wall velocities must be a contiguous device "
                                f"tensor of dtype {self.dtype}")
            if tuple(wall.shape) != (nw, 2, self.Ny, self.Nx):
                raise ValueError(f"wall velocities have shape {(nw, 2, self.Ny, self.Nx)}")
        L.check(L.lib().fcmdp_set_wall_velocity(self._h, _ptr(wall), _stream(stream)),
                "fcmdp_set_wall_velocity")
        self._mark(stream)

    STAGES = ("particles", "spread", "fft_forward", "columns", "fft_inverse",
              "interp")

    VARIANTS = {"generic_fft": 0, "fft_rows_x": 1, "fft_rows_y": 2,
                "simple_spread": 3, "simple_interp": 4, "generic_columns": 5,
                "vector_dct": 6, "no_codelet": 7, "no_pipeline": 8,
                "no_lowk": 9, "wave_spread": 10, "spread_workgroups": 11,
                "spread_block_rows": 12,
                "spread_order": 13, "halo_interp": 14}

    def set_variant(self, name, value):
        """Select an alternative kernel (see fcmdp_set_variant)."""
        L.check(L.lib().fcmdp_set_variant(self._h, self.VARIANTS[name], int(value)),
                "fcmdp_set_variant")

    def set_profiling(self, enable=True):
        L.check(L.lib().fcmdp_set_profiling(self._h, int(bool(enable))),
                "fcmdp_set_profiling")

    def stage_times(self):
        """Summed ms per stage since the last call, the number of applies,
        and the z-band (first, last node) of the last apply."""
        ms = (ctypes.c_double * 8)()
        na = ctypes.c_int64(0)
        L.check(L.lib().fcmdp_stage_times(self._h, ms, ctypes.byref(na)),
                "fcmdp_stage_times")
        return (dict(zip(self.STAGES, ms[:6])), na.value,
                (int(ms[6]), int(ms[7])))

    def status(self):
        bad = ctypes.c_int64(0)
        code = L.lib().fcmdp_status(self._h, ctypes.byref(bad))
        if code not in (L.OK, L.EDOMAIN):
            L.check(code, "fcmdp_status")
        return code, bad.value

    # --- stage entry points -------------------------------------------------
    def grid_shape(self):
        return (6, self.Nz, self.Ny, self.Nx)

    def spectrum_shape(self):
        return (6, self.Nz, self.Nx // 2 + 1, self.Ny)

    def stage_spread(self, pos, F, T=None, stream=None):
        import torch
        grid = torch.empty(self.grid_shape(), dtype=self.dtype,
                           device=pos.device)
        self._check_particles(pos, F, T)
        L.check(L.lib().fcmdp_stage_spread(self._h, pos.shape[0], _ptr(pos),
                                           _ptr(F), _ptr(T), _ptr(grid),
                                           _stream(stream)),
                "fcmdp_stage_spread")
        self._mark(stream)
        return grid

    def _cplx(self):
        import torch
        return torch.complex128 if self.precision == "fp64" else torch.complex64

    @staticmethod
    def _check_buffer(t, shape, dtype, what):
        """Grids and spectra cross the ABI as raw pointers in the layouts of
        fcmdp.h: they must be contiguous device tensors of that shape."""
        if t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
            raise TypeError(f"{what} must be a contiguous device tensor of dtype "
                            f"{dtype}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{what} must have shape {tuple(shape)}")

    def stage_fft_forward(self, grid, c_lo, c_hi, stream=None):
        import torch
        self._check_buffer(grid, self.grid_shape(), self.dtype, "grid")
        spec = torch.zeros(self.spectrum_shape(), dtype=self._cplx(),
                           device=grid.device)
        L.check(L.lib().fcmdp_stage_fft_forward(self._h, _ptr(grid), _ptr(spec),
                                                c_lo, c_hi, _stream(stream)),
                "fcmdp_stage_fft_forward")
        self._mark(stream)
        return spec

    def stage_solve(self, spec, c_lo, c_hi, stream=None, out=None):
        """Column solve of planes c_lo..c_hi; `out` may be `spec` (in place)."""
        import torch
        self._check_buffer(spec, self.spectrum_shape(), self._cplx(), "spectrum")
        if out is None:
            out = torch.zeros_like(spec)
        else:
            self._check_buffer(out, self.spectrum_shape(), self._cplx(), "spectrum")
        L.check(L.lib().fcmdp_stage_solve(self._h, _ptr(spec), _ptr(out), c_lo,
                                          c_hi, _stream(stream)),
                "fcmdp_stage_solve")
        self._mark(stream)
        return out

    def stage_fft_inverse(self, spec, c_lo, c_hi, stream=None):
        import torch
        self._check_buffer(spec, self.spectrum_shape(), self._cplx(), "spectrum")
        grid = torch.zeros(self.grid_shape(), dtype=self.dtype,
                           device=spec.device)
        L.check(L.lib().fcmdp_stage_fft_inverse(self._h, _ptr(spec), _ptr(grid),
                                                c_lo, c_hi, _stream(stream)),
                "fcmdp_stage_fft_inverse")
        self._mark(stream)
        return grid

    def stage_interp(self, pos, grid, stream=None):
        import torch
        n = pos.shape[0]
        U = torch.empty((n, 3), dtype=self.dtype, device=pos.device)
        Om = torch.empty((n, 3), dtype=self.dtype, device=pos.device)
        self._check_particles(pos)
        self._check_buffer(grid, self.grid_shape(), self.dtype, "grid")
        L.check(L.lib().fcmdp_stage_interp(self._h, n, _ptr(pos), _ptr(grid),
                                           _ptr(U), _ptr(Om), _stream(stream)),
                "fcmdp_stage_interp")
        self._mark(stream)
        return U, Om
