"""MI355X-native doubly-periodic FCM mobility apply (arXiv 2210.01837).

The compute path is libfcmdp.so (hand-written HIP for gfx950) behind the C
ABI in include/fcmdp.h; this package is its thin Python binding.
"""
from .solver import Solver, make_params, workspace_bytes  # noqa: F401
from ._lib import FcmdpError, lib  # noqa: F401

__all__ = ["Solver", "make_params", "workspace_bytes", "FcmdpError", "lib"]
