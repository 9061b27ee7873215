"""ctypes binding of libbmpc.so: one Python function per C entry point, same
names, argument marshalling only.  Device arrays are passed as
``torch.Tensor`` (their ``data_ptr()``); host arrays as NumPy arrays.

The library must be built (``python -m paper_2506_13624_amd.build`` or
``__graft_entry__.build()``); importing without it raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbmpc.so")

STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "TOPOLOGY", 3: "NOT_PD", 4: "NONFINITE",
                5: "MAXITER", 6: "LINESEARCH", 7: "HIP", 8: "OOM", 9: "UNSUPPORTED"}

LAYOUT_NODE_MAJOR = 0
LAYOUT_ELEM_MAJOR = 1
RICCATI_AUTO = 0
RICCATI_LEVEL = 1
RICCATI_SEGSCAN = 2


class BmpcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"bmpc status {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


if not os.path.exists(LIB_PATH):
    raise ImportError(f"libbmpc.so is not built ({LIB_PATH}); run paper_2506_13624_amd/build.py")

lib = C.CDLL(LIB_PATH)

_vp = C.c_void_p
_i32 = C.c_int32
_pi32 = C.POINTER(C.c_int32)
_pd = C.POINTER(C.c_double)


def _sig(name, res, args):
    f = getattr(lib, name)
    f.restype = res
    f.argtypes = args
    return f


_sig("bmpc_last_error", C.c_char_p, [])
_sig("bmpc_version", _i32, [])
_sig("bmpc_device_count", _i32, [])
_sig("bmpc_tree_create", _i32, [_pi32, _i32, C.POINTER(_vp)])
_sig("bmpc_tree_destroy", None, [_vp])
_sig("bmpc_tree_info", _i32, [_vp, _pi32, _pi32, _pi32, _pi32])
_sig("bmpc_tree_segments", _i32, [_vp, _pi32])
_sig("bmpc_weights_from_probs", _i32, [_vp, _pd, _pd])
_sig("bmpc_lqr_plan_create", _i32, [_vp, _i32, _i32, _i32, C.POINTER(_vp)])
_sig("bmpc_lqr_plan_destroy", None, [_vp])
_sig("bmpc_lqr_supported", _i32, [_i32, _i32, _i32])
_sig("bmpc_lqr_solve", _i32, [_vp] + [_vp] * 16 + [_i32, _vp])
_sig("bmpc_lqr_check", _i32, [_vp, _pi32, _vp])
_sig("bmpc_profile_enable", _i32, [_i32])
_sig("bmpc_profile_read", _i32, [C.c_char_p, _pd, _pi32, _i32])


def check(status):
    if status != 0:
        raise BmpcError(status, lib.bmpc_last_error().decode())
    return status


def dptr(t):
    """Device pointer of a torch tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device array expected (torch tensor on a HIP device)")
    if not t.is_contiguous():
        raise ValueError("device array must be contiguous")
    return _vp(t.data_ptr())


def _hi32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_pi32)


def _hf64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_pd)


def stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return _vp(s.cuda_stream)


# ----------------------------------------------------------------------------
# entry points with the C names
# ----------------------------------------------------------------------------

def bmpc_version():
    return lib.bmpc_version()


def bmpc_device_count():
    return lib.bmpc_device_count()


def bmpc_tree_create(parent):
    parent, pp = _hi32(parent)
    h = _vp()
    check(lib.bmpc_tree_create(pp, len(parent), C.byref(h)))
    return h


def bmpc_tree_destroy(h):
    lib.bmpc_tree_destroy(h)


def bmpc_tree_info(h):
    v = [_i32() for _ in range(4)]
    check(lib.bmpc_tree_info(h, *[C.byref(x) for x in v]))
    return {"num_nodes": v[0].value, "num_leaves": v[1].value, "depth": v[2].value,
            "num_segments": v[3].value}


def bmpc_tree_segments(h, num_nodes):
    out = np.zeros(num_nodes, dtype=np.int32)
    check(lib.bmpc_tree_segments(h, out.ctypes.data_as(_pi32)))
    return out


def bmpc_weights_from_probs(h, leaf_prob, num_nodes):
    lp, lpp = _hf64(leaf_prob)
    out = np.zeros(num_nodes)
    check(lib.bmpc_weights_from_probs(h, lpp, out.ctypes.data_as(_pd)))
    return out


def bmpc_lqr_supported(nx, nu, variant=RICCATI_AUTO):
    return bool(lib.bmpc_lqr_supported(nx, nu, variant))


def bmpc_lqr_plan_create(tree, nx, nu, layout):
    h = _vp()
    check(lib.bmpc_lqr_plan_create(tree, nx, nu, layout, C.byref(h)))
    return h


def bmpc_lqr_plan_destroy(h):
    lib.bmpc_lqr_plan_destroy(h)


def bmpc_lqr_solve(plan, A, B, c, Q, R, M, q, r, x0, x, u, lam, K=None, k=None, P=None, p=None,
                   variant=RICCATI_AUTO, stream=None):
    args = [dptr(v) for v in (A, B, c, Q, R, M, q, r, x0, x, u, lam, K, k, P, p)]
    check(lib.bmpc_lqr_solve(plan, *args, variant, stream_ptr(stream)))


def bmpc_lqr_check(plan, stream=None):
    bad = _i32(-1)
    st = lib.bmpc_lqr_check(plan, C.byref(bad), stream_ptr(stream))
    return st, bad.value


def bmpc_profile_enable(on=True):
    check(lib.bmpc_profile_enable(1 if on else 0))


def bmpc_profile_read(cap=64):
    """Per-kernel {name: (total_ms, launches)} since the last read."""
    names = C.create_string_buffer(64 * cap)
    tot = np.zeros(cap)
    cnt = np.zeros(cap, dtype=np.int32)
    n = lib.bmpc_profile_read(names, tot.ctypes.data_as(_pd), cnt.ctypes.data_as(_pi32), cap)
    out = {}
    raw = names.raw
    for i in range(min(n, cap)):
        nm = raw[64 * i: 64 * (i + 1)].split(b"\0", 1)[0].decode()
        out[nm] = (float(tot[i]), int(cnt[i]))
    return out
