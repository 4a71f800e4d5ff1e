"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/fcmdp.h declares, and rejects invalid parameters
before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fcmdp.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fcmdp_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_2210_01837_amd import _lib
    return _lib.lib()


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert "fcmdp_apply_mobility" in names and "fcmdp_create_solver" in names
    for n in names:
        assert hasattr(L, n), n


def test_strerror(L):
    from paper_2210_01837_amd import _lib
    for code in (0, -1, -2, -3, -4, -5):
        assert _lib.strerror(code)
    assert _lib.strerror(-99) == "unknown error"


def _params(**kw):
    from paper_2210_01837_amd import make_params
    base = dict(geometry="bw", Lx=32.0, Ly=32.0, H=8.0, Nx=48, Ny=48, Nz=32,
                precision="fp64", max_particles=64)
    base.update(kw)
    return make_params(**base)


@pytest.mark.parametrize("bad", [
    dict(Nx=47), dict(Ny=6), dict(Nz=7), dict(Nz=65), dict(Nx=38),  # 19 prime
    dict(Ly=31.0), dict(H=1.9), dict(w=8), dict(w=5), dict(w=2), dict(eta=0.0),
    dict(geometry="sc", H=3.9), dict(max_particles=-1), dict(beta_m=-1.0),
    # partial slip: non-negative, Nz <= 32, no slip length at z = H for a
    # bottom wall
    dict(slipH=0.5), dict(Nz=48, slip0=0.5), dict(geometry="sc", slipH=-1.0),
    dict(geometry="sc", Nz=48, slip0=1.0), dict(geometry="sc", slip0=float("inf")),
    # uniform wall velocities: no top wall for a bottom wall, Nz <= 32
    dict(wallH=(1.0, 0.0)), dict(Nz=48, wall0=(0.5, 0.0)),
    dict(geometry="sc", wallH=(float("nan"), 0.0)),
    # torques through the kernel derivative: three-channel kernels, Nz <= 32
    dict(Nz=48, torque_route="derivative"),
])
def test_invalid_parameters_rejected(L, bad):
    from paper_2210_01837_amd import _lib
    p = _params(**bad)
    h = ctypes.c_void_p(0)
    assert L.fcmdp_create_solver(ctypes.byref(p), None, ctypes.byref(h)) == _lib.EINVAL
    assert not h.value
    nb = ctypes.c_size_t(0)
    assert L.fcmdp_workspace_bytes(ctypes.byref(p), 10, ctypes.byref(nb)) == _lib.EINVAL


def test_workspace_bytes_scales(L):
    from paper_2210_01837_amd import workspace_bytes
    kw = dict(geometry="bw", Lx=1448.0, Ly=1448.0, H=12.0, Nx=2176, Ny=2176,
              Nz=32, precision="mixed")
    small = workspace_bytes(1000, **kw)
    big = workspace_bytes(1 << 20, **kw)
    grid = 6 * 32 * 2176 * 2176 * 4
    assert small > 2 * grid and big > small
    kw64 = dict(kw, Nx=768, Ny=768, Lx=512.0, Ly=512.0)
    assert (workspace_bytes(1 << 17, **dict(kw64, precision="fp64"))
            > workspace_bytes(1 << 17, **kw64))


def test_null_arguments(L):
    from paper_2210_01837_amd import _lib
    assert L.fcmdp_create_solver(None, None, None) == _lib.EINVAL
    assert L.fcmdp_apply_mobility(None, 1, None, None, None, None, None, None) == _lib.EINVAL
    assert L.fcmdp_status(None, None) == _lib.EINVAL
    L.fcmdp_destroy_solver(None, None)


def test_params_struct_matches_the_header():
    """The ctypes mirror of fcmdp_params has the header's fields, in order,
    with the header's C types (an ABI drift would misread every field after
    it)."""
    from paper_2210_01837_amd import _lib
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    body = re.search(r"typedef struct \{(.*?)\} fcmdp_params;", src, re.S).group(1)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        ctype, names = decl.split(None, 1)
        for nm in names.split(","):
            m = re.match(r"(\w+)(?:\[(\d+)\])?$", nm.strip())
            fields.append((m.group(1), ctype, int(m.group(2) or 0)))
    ctypes_of = {"int": ctypes.c_int, "double": ctypes.c_double,
                 "int64_t": ctypes.c_int64}
    got = [(n, t) for n, t in _lib.Params._fields_]
    assert [n for n, _ in got] == [n for n, _, _ in fields]
    for (n, t), (_, c, dim) in zip(got, fields):
        if dim:
            assert issubclass(t, ctypes.Array) and t._length_ == dim, n
            assert t._type_ is ctypes_of[c], n
        else:
            assert t is ctypes_of[c], n
