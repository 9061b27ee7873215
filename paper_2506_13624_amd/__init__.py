"""MI355X branch-MPC hot path: tree LQR and AL multiple-shooting iLQR in HIP.

``_lib`` binds the C ABI of ``libbmpc.so`` (same names as ``include/bmpc.h``);
``layout`` converts between node-major host arrays and device arrays in the
library's layouts.  Every compute step runs in the library's kernels; there is
no CPU fallback.
"""
from . import _lib  # noqa: F401  (raises ImportError if libbmpc.so is missing)
from ._lib import BmpcError  # noqa: F401
