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
BLOCK_GRID = -1


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
_sig("bmpc_tree_order", _i32, [_pi32, _i32, _pi32, _pi32])
_sig("bmpc_tree_create_any", _i32, [_pi32, _i32, _pi32, C.POINTER(_vp)])
_sig("bmpc_tree_permute", _i32, [_vp, _i32, _i32, _i32, _vp, _vp, _vp])
_sig("bmpc_lqr_plan_create", _i32, [_vp, _i32, _i32, _i32, C.POINTER(_vp)])
_sig("bmpc_lqr_plan_destroy", None, [_vp])
_sig("bmpc_lqr_supported", _i32, [_i32, _i32, _i32])
_sig("bmpc_lqr_solve", _i32, [_vp] + [_vp] * 16 + [_i32, _vp])
_sig("bmpc_lqr_solve_host", _i32, [_vp] + [_pd] * 12 + [_i32, _vp])
_sig("bmpc_lqr_solve_f32", _i32, [_vp] + [_vp] * 16 + [_vp])
_sig("bmpc_lqr_solve_mixed", _i32, [_vp] + [_vp] * 12 + [_i32, _vp, _vp])
_sig("bmpc_lqr_check", _i32, [_vp, _pi32, _vp])
_sig("bmpc_profile_enable", _i32, [_i32])
_sig("bmpc_profile_read", _i32, [C.c_char_p, _pd, _pi32, _i32])
_sig("bmpc_profile_only", _i32, [C.c_char_p])


def check(status):
    if status != 0:
        raise BmpcError(status, lib.bmpc_last_error().decode())
    return status


def dptr(t, dtype=None, numel=None, name="array"):
    """Device pointer of a torch tensor (None -> NULL).  With ``dtype`` and
    ``numel`` the tensor must have that element type and hold at least that
    many elements: the kernels trust the sizes the library derives from its
    handles, so a short or mistyped array would be read past its end."""
    if t is None:
        return None
    _check_only(t, dtype, numel, name)
    if not t.is_cuda:
        raise ValueError(f"{name}: device array expected (torch tensor on a HIP device)")
    if not t.is_contiguous():
        raise ValueError(f"{name}: device array must be contiguous")
    return _vp(t.data_ptr())


def _dptrs(specs):
    """dptr over (tensor, dtype, numel, name) tuples, checking the types and
    sizes of all of them before the device placement of any."""
    for t, dtype, numel, name in specs:
        if t is not None:
            _check_only(t, dtype, numel, name)
    return [dptr(t, dtype, numel, name) for t, dtype, numel, name in specs]


def _check_only(t, dtype, numel, name):
    if dtype is not None and t.dtype != _torch_dtype(dtype):
        raise ValueError(f"{name}: element type {t.dtype}, expected {dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name}: {t.numel()} elements, at least {numel} expected")


def _torch_dtype(name):
    import torch
    return {"float64": torch.float64, "float32": torch.float32, "int16": torch.int16,
            "bfloat16": torch.bfloat16}[name]


def _bf16_ptr(t, numel, name):
    """BF16 bit patterns: int16 or bfloat16 tensors."""
    if t is not None and t.dtype == _torch_dtype("bfloat16"):
        return dptr(t, "bfloat16", numel, name)
    return dptr(t, "int16", numel, name)


# sizes behind the opaque handles, for the argument checks of dptr
_dims = {}


def _key(h):
    return h.value if isinstance(h, _vp) else int(h)


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


TO_LIBRARY_ORDER = 0
TO_CALLER_ORDER = 1


def bmpc_tree_order(parent):
    """(order, lib_parent): order[k] = caller index of library node k."""
    parent, pp = _hi32(parent)
    order = np.zeros(len(parent), dtype=np.int32)
    lib_parent = np.zeros(len(parent), dtype=np.int32)
    check(lib.bmpc_tree_order(pp, len(parent), order.ctypes.data_as(_pi32),
                              lib_parent.ctypes.data_as(_pi32)))
    return order, lib_parent


def bmpc_tree_create_any(parent):
    """(tree handle, order) for a parent array in any node order."""
    parent, pp = _hi32(parent)
    order = np.zeros(len(parent), dtype=np.int32)
    h = _vp()
    check(lib.bmpc_tree_create_any(pp, len(parent), order.ctypes.data_as(_pi32), C.byref(h)))
    return h, order


def bmpc_tree_permute(tree, direction, layout, width, src, dst, stream=None):
    n = bmpc_tree_info(tree)["num_nodes"] * width
    ps, pd = _dptrs([(src, "float64", n, "src"), (dst, "float64", n, "dst")])
    check(lib.bmpc_tree_permute(tree, direction, layout, width, ps, pd, stream_ptr(stream)))


def bmpc_lqr_supported(nx, nu, variant=RICCATI_AUTO):
    return bool(lib.bmpc_lqr_supported(nx, nu, variant))


def bmpc_lqr_plan_create(tree, nx, nu, layout):
    h = _vp()
    check(lib.bmpc_lqr_plan_create(tree, nx, nu, layout, C.byref(h)))
    _dims[_key(h)] = (bmpc_tree_info(tree)["num_nodes"], nx, nu)
    return h


def bmpc_lqr_plan_destroy(h):
    _dims.pop(_key(h), None)
    lib.bmpc_lqr_plan_destroy(h)


def bmpc_lqr_solve(plan, A, B, c, Q, R, M, q, r, x0, x, u, lam, K=None, k=None, P=None, p=None,
                   variant=RICCATI_AUTO, stream=None):
    N, n, m = _dims[_key(plan)]
    sizes = (("A", N * n * n), ("B", N * n * m), ("c", N * n), ("Q", N * n * n), ("R", N * m * m),
             ("M", N * m * n), ("q", N * n), ("r", N * m), ("x0", n), ("x", N * n), ("u", N * m),
             ("lam", N * n), ("K", N * m * n), ("k", N * m), ("P", N * n * n), ("p", N * n))
    args = _dptrs([(v, "float64", cnt, nm) for v, (nm, cnt) in zip((A, B, c, Q, R, M, q, r, x0, x, u, lam, K, k,
                                                                     P, p), sizes)])
    check(lib.bmpc_lqr_solve(plan, *args, variant, stream_ptr(stream)))


def bmpc_lqr_solve_host(plan, A, B, c, Q, R, M, q, r, x0, variant=RICCATI_AUTO, stream=None):
    """Host NumPy inputs in the plan's layout (flattened); returns host
    (x, u, lam) as flat float64 arrays in that layout."""
    N, n, m = _dims[_key(plan)]
    sizes = _lqr_sizes(plan)
    ins = []
    for v, (nm, cnt) in zip((A, B, c, Q, R, M, q, r, x0), sizes):
        a = np.ascontiguousarray(v, dtype=np.float64).reshape(-1)
        if a.size != cnt:
            raise ValueError(f"{nm}: {a.size} elements, {cnt} expected")
        ins.append(a)
    outs = [np.zeros(N * n), np.zeros(N * m), np.zeros(N * n)]
    check(lib.bmpc_lqr_solve_host(plan, *[a.ctypes.data_as(_pd) for a in ins + outs], variant,
                                  stream_ptr(stream)))
    return tuple(outs)


def _lqr_sizes(plan):
    N, n, m = _dims[_key(plan)]
    return (("A", N * n * n), ("B", N * n * m), ("c", N * n), ("Q", N * n * n), ("R", N * m * m),
            ("M", N * m * n), ("q", N * n), ("r", N * m), ("x0", n), ("x", N * n), ("u", N * m),
            ("lam", N * n), ("K", N * m * n), ("k", N * m), ("P", N * n * n), ("p", N * n))


def bmpc_lqr_solve_f32(plan, A, B, c, Q, R, M, q, r, x0, x, u, lam, K=None, k=None, P=None, p=None, stream=None):
    """FP32 tree LQR: every array float32, sizes and layout as bmpc_lqr_solve."""
    args = _dptrs([(v, "float32", cnt, nm) for v, (nm, cnt) in zip((A, B, c, Q, R, M, q, r, x0, x, u, lam, K, k,
                                                                     P, p), _lqr_sizes(plan))])
    check(lib.bmpc_lqr_solve_f32(plan, *args, stream_ptr(stream)))


LQR_REFINE_MAX = 64


def bmpc_lqr_solve_mixed(plan, A, B, c, Q, R, M, q, r, x0, x, u, lam, refine_steps, res_norms=None, stream=None):
    """FP64 tree LQR by FP32 solves with FP64 iterative refinement;
    res_norms (float64, refine_steps + 2 entries) receives the largest KKT
    residual after each FP32 solve."""
    specs = [(v, "float64", cnt, nm) for v, (nm, cnt) in zip((A, B, c, Q, R, M, q, r, x0, x, u, lam),
                                                              _lqr_sizes(plan))]
    specs.append((res_norms, "float64", refine_steps + 2, "res_norms"))
    args = _dptrs(specs)
    check(lib.bmpc_lqr_solve_mixed(plan, *args[:12], int(refine_steps), args[12], stream_ptr(stream)))


def bmpc_lqr_check(plan, stream=None):
    bad = _i32(-1)
    st = lib.bmpc_lqr_check(plan, C.byref(bad), stream_ptr(stream))
    return st, bad.value


def bmpc_profile_enable(on=True):
    check(lib.bmpc_profile_enable(1 if on else 0))


def bmpc_profile_only(name=None):
    check(lib.bmpc_profile_only(name.encode() if name else None))


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


# ----------------------------------------------------------------------------
# branch-MPC problem and solver
# ----------------------------------------------------------------------------

class bmpc_bicycle_params(C.Structure):
    _fields_ = [("wheelbase", C.c_double), ("dt", C.c_double), ("Qd", C.c_double * 4),
                ("Rd", C.c_double * 2), ("a_max", C.c_double), ("steer_max", C.c_double),
                ("obs_radius", C.c_double)]


class bmpc_settings(C.Structure):
    _fields_ = [("eps_tol", C.c_double), ("tau", C.c_double), ("omega0", C.c_double),
                ("eta0", C.c_double), ("a_omega", C.c_double), ("b_omega", C.c_double),
                ("a_eta", C.c_double), ("b_eta", C.c_double), ("rho0", C.c_double),
                ("mu0", C.c_double), ("armijo_beta", C.c_double), ("n_alpha", C.c_int32),
                ("max_outer", C.c_int32), ("max_inner", C.c_int32), ("max_ls_fail", C.c_int32),
                ("riccati_variant", C.c_int32), ("block_size", C.c_int32),
                ("max_iter_total", C.c_int32), ("ls_rounds", C.c_int32), ("hessian", C.c_int32),
                ("eig_floor", C.c_double)]


HESSIAN_GAUSS_NEWTON = 0
HESSIAN_EXACT = 1


class bmpc_stats(C.Structure):
    _fields_ = [("status", C.c_int32), ("outer_it", C.c_int32), ("inner_it", C.c_int32),
                ("ls_failures", C.c_int32), ("bad_node", C.c_int32), ("start", C.c_int32), ("r_kkt", C.c_double),
                ("viol", C.c_double), ("rho", C.c_double), ("mu", C.c_double),
                ("merit", C.c_double), ("time_ms", C.c_double * 5)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["time_ms"] = dict(zip(PHASES, list(self.time_ms)))
        return d


PHASES = ("linearise", "backward", "forward", "line_search", "update")


_sig("bmpc_settings_default", None, [C.POINTER(bmpc_settings)])
_sig("bmpc_bicycle_default", None, [C.POINTER(bmpc_bicycle_params)])
_sig("bmpc_node_refs", _i32, [_vp, _pd, _pd, C.c_double, C.c_double, _pd])
_sig("bmpc_problem_create", _i32, [_vp, C.POINTER(bmpc_bicycle_params), _pd, _pd, _pd, _pi32, _pd,
                                   C.POINTER(_vp)])
_sig("bmpc_problem_destroy", None, [_vp])
_sig("bmpc_problem_update", _i32, [_vp, _pd, _pd, _pd, _pi32, _pd])
_sig("bmpc_problem_output_width", _i32, [_vp, _pi32])
_sig("bmpc_problem_get_x0", _i32, [_vp, _pd])
_sig("bmpc_batch_start_from_network", _i32, [_vp, _vp, _i32, _i32, _vp])
_sig("bmpc_batch_state_all", _i32, [_vp, _vp, _vp, _vp, _vp, _i32, _vp])
_sig("bmpc_batch_total_nodes", C.c_int64, [_vp])
_sig("bmpc_problem_set_x0", _i32, [_vp, _pd])
_sig("bmpc_solve", _i32, [_vp, C.POINTER(bmpc_settings), _i32, _vp, _vp, _vp, _vp,
                          C.POINTER(bmpc_stats), _vp])
_sig("bmpc_linearize", _i32, [_vp, _vp, _vp, _vp, _vp, C.c_double] + [_vp] * 7 + [_pd, _vp])
_sig("bmpc_linearize_noalloc", _i32, [_vp, _vp, _vp, _vp, _vp, C.c_double] + [_vp] * 8 + [_vp])
_sig("bmpc_linearize_exact", _i32, [_vp, C.c_double, _vp, _vp, _vp, _vp, C.c_double] + [_vp] * 8 + [_pd, _vp])
NOALLOC_MAX_NODES = 2048
_sig("bmpc_batch_create", _i32, [C.POINTER(_vp), _i32, _i32, C.POINTER(_vp)])
_sig("bmpc_batch_destroy", None, [_vp])
_sig("bmpc_batch_launch", _i32, [_vp, C.POINTER(bmpc_settings), _i32, _vp])
_sig("bmpc_batch_stats", _i32, [_vp, C.POINTER(bmpc_stats), _vp])
_sig("bmpc_batch_state", _i32, [_vp, _i32, _vp, _vp, _vp, _vp, _i32, _vp])
_sig("bmpc_batch_history", _i32, [_vp, _i32, _pd, _vp])
_sig("bmpc_batch_shift", _i32, [_vp, _vp])


def bmpc_settings_default(**kw):
    s = bmpc_settings()
    lib.bmpc_settings_default(C.byref(s))
    for k, v in kw.items():
        setattr(s, k, v)
    return s


def bmpc_bicycle_default(**kw):
    p = bmpc_bicycle_params()
    lib.bmpc_bicycle_default(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def bmpc_node_refs(tree, leaf_prob, leaf_offset, dt, speed, num_nodes):
    lp, lpp = _hf64(leaf_prob)
    lo, lop = _hf64(leaf_offset)
    out = np.zeros((num_nodes, 4))
    check(lib.bmpc_node_refs(tree, lpp, lop, dt, speed, out.ctypes.data_as(_pd)))
    return out


def bmpc_problem_create(tree, prm, node_weight, node_ref, node_obs, has_obs, x0):
    w, wp = _hf64(node_weight)
    r, rp = _hf64(node_ref)
    o, op = _hf64(node_obs)
    h, hp = _hi32(has_obs)
    x, xp = _hf64(x0)
    out = _vp()
    check(lib.bmpc_problem_create(tree, C.byref(prm), wp, rp, op, hp, xp, C.byref(out)))
    _dims[_key(out)] = bmpc_tree_info(tree)["num_nodes"]
    return out


def bmpc_problem_destroy(h):
    _dims.pop(_key(h), None)
    lib.bmpc_problem_destroy(h)


def bmpc_problem_set_x0(h, x0):
    x, xp = _hf64(x0)
    check(lib.bmpc_problem_set_x0(h, xp))


def bmpc_problem_update(h, node_weight, node_ref, node_obs, has_obs, x0):
    w, wp = _hf64(node_weight)
    r, rp = _hf64(node_ref)
    o, op = _hf64(node_obs)
    hs, hp = _hi32(has_obs)
    x, xp = _hf64(x0)
    check(lib.bmpc_problem_update(h, wp, rp, op, hp, xp))


def bmpc_problem_get_x0(h):
    x = np.zeros(4)
    check(lib.bmpc_problem_get_x0(h, x.ctypes.data_as(_pd)))
    return x


def bmpc_problem_output_width(h):
    w = C.c_int32()
    check(lib.bmpc_problem_output_width(h, C.byref(w)))
    return w.value


def bmpc_solve(problem, settings, warm, x, u, lam, ye, stream=None, raise_on_status=False):
    """x, u, lam, ye: device tensors (node-major).  Returns the stats dict;
    the solver's own status is reported in stats['status']."""
    st = bmpc_stats()
    N = _dims[_key(problem)]
    status = lib.bmpc_solve(problem, C.byref(settings), warm, *_state_ptrs(N, x, u, lam, ye), C.byref(st),
                            stream_ptr(stream))
    if raise_on_status:
        check(status)
    elif status not in (0, 3, 4, 5, 6):
        check(status)
    return st.as_dict()


def bmpc_linearize(problem, x, u, lam, ye, rho, A, B, c, Q, R, q, r, stream=None):
    kv = np.zeros(2)
    N = _dims[_key(problem)]
    f = _dptrs([(v, "float64", N * w, nm) for v, w, nm in
         ((x, 4, "x"), (u, 2, "u"), (lam, 4, "lam"), (ye, 5, "ye"), (A, 16, "A"), (B, 8, "B"), (c, 4, "c"),
          (Q, 16, "Q"), (R, 4, "R"), (q, 4, "q"), (r, 2, "r"))])
    check(lib.bmpc_linearize(problem, f[0], f[1], f[2], f[3], rho, *f[4:], kv.ctypes.data_as(_pd),
                             stream_ptr(stream)))
    return float(kv[0]), float(kv[1])


def bmpc_linearize_exact(problem, eig_floor, x, u, lam, ye, rho, A, B, c, Q, R, M, q, r, stream=None):
    """bmpc_linearize with the exact Hessian and eigenvalue modification;
    M (N*2*4) receives the cross blocks."""
    kv = np.zeros(2)
    N = _dims[_key(problem)]
    f = _dptrs([(v, "float64", N * w, nm) for v, w, nm in
         ((x, 4, "x"), (u, 2, "u"), (lam, 4, "lam"), (ye, 5, "ye"), (A, 16, "A"), (B, 8, "B"), (c, 4, "c"),
          (Q, 16, "Q"), (R, 4, "R"), (M, 8, "M"), (q, 4, "q"), (r, 2, "r"))])
    check(lib.bmpc_linearize_exact(problem, float(eig_floor), f[0], f[1], f[2], f[3], rho, *f[4:],
                                   kv.ctypes.data_as(_pd), stream_ptr(stream)))
    return float(kv[0]), float(kv[1])


def bmpc_linearize_noalloc(problem, x, u, lam, ye, rho, A, B, c, Q, R, q, r, kkt_viol=None, stream=None):
    """As bmpc_linearize, with the library's fixed workspace (no device
    allocation); kkt_viol: float64 device tensor of 2 entries or None.
    Asynchronous."""
    N = _dims[_key(problem)]
    f = _dptrs([(v, "float64", N * w, nm) for v, w, nm in
                ((x, 4, "x"), (u, 2, "u"), (lam, 4, "lam"), (ye, 5, "ye"), (A, 16, "A"), (B, 8, "B"),
                 (c, 4, "c"), (Q, 16, "Q"), (R, 4, "R"), (q, 4, "q"), (r, 2, "r"))]
               + [(kkt_viol, "float64", 2, "kkt_viol")])
    check(lib.bmpc_linearize_noalloc(problem, f[0], f[1], f[2], f[3], rho, *f[4:], stream_ptr(stream)))


def bmpc_batch_create(problems, hist_cap=0):
    arr = (_vp * len(problems))(*[p.value if isinstance(p, _vp) else p for p in problems])
    out = _vp()
    check(lib.bmpc_batch_create(arr, len(problems), hist_cap, C.byref(out)))
    _dims[_key(out)] = [_dims[_key(p)] for p in problems]
    return out


def bmpc_batch_destroy(h):
    _dims.pop(_key(h), None)
    lib.bmpc_batch_destroy(h)


def bmpc_batch_launch(batch, settings, warm=0, stream=None):
    check(lib.bmpc_batch_launch(batch, C.byref(settings), warm, stream_ptr(stream)))


def bmpc_batch_stats(batch, count, stream=None):
    arr = (bmpc_stats * count)()
    check(lib.bmpc_batch_stats(batch, arr, stream_ptr(stream)))
    return [a.as_dict() for a in arr]


def _state_ptrs(N, x, u, lam, ye):
    return _dptrs([(v, "float64", N * w, nm) for v, w, nm in ((x, 4, "x"), (u, 2, "u"), (lam, 4, "lam"),
                                                               (ye, 5, "ye"))])


def bmpc_batch_state(batch, i, x=None, u=None, lam=None, ye=None, into_batch=False, stream=None):
    sizes = _dims[_key(batch)]
    if not 0 <= i < len(sizes):
        raise ValueError(f"problem index {i} outside the batch of {len(sizes)}")
    check(lib.bmpc_batch_state(batch, i, *_state_ptrs(sizes[i], x, u, lam, ye), 1 if into_batch else 0,
                               stream_ptr(stream)))


def bmpc_batch_state_all(batch, x=None, u=None, lam=None, ye=None, into_batch=False, stream=None):
    T = sum(_dims[_key(batch)])
    check(lib.bmpc_batch_state_all(batch, *_state_ptrs(T, x, u, lam, ye), 1 if into_batch else 0,
                                   stream_ptr(stream)))


def bmpc_batch_total_nodes(batch):
    return int(lib.bmpc_batch_total_nodes(batch))


def bmpc_batch_history(batch, i, hist_cap, stream=None):
    h = np.zeros((hist_cap, 6))
    check(lib.bmpc_batch_history(batch, i, h.ctypes.data_as(_pd), stream_ptr(stream)))
    return h


def bmpc_batch_start_from_network(batch, Y, rows, width, stream=None):
    """Y: float32 device tensor (rows x width)."""
    check(lib.bmpc_batch_start_from_network(batch, dptr(Y, "float32", rows * width, "Y"), rows, width,
                                            stream_ptr(stream)))


_sig("bmpc_warm_shift", _i32, [_vp, _vp, _vp, _vp, _vp, _pd, _vp])


def bmpc_warm_shift(problem, x, u, lam, ye, x0_new=None, stream=None):
    """x, u, lam, ye: device tensors, the previous solution in, the shifted
    start point out; x0_new: host array of 4 (measured state) or None."""
    N = _dims[_key(problem)]
    ptrs = _state_ptrs(N, x, u, lam, ye)
    if x0_new is not None:
        xa, xp = _hf64(x0_new)
        if xa.size != 4:
            raise ValueError("x0_new: 4 entries expected")
    else:
        xp = None
    check(lib.bmpc_warm_shift(problem, *ptrs, xp, stream_ptr(stream)))


def bmpc_batch_shift(batch, stream=None):
    check(lib.bmpc_batch_shift(batch, stream_ptr(stream)))


# ----------------------------------------------------------------------------
# warm-start network
# ----------------------------------------------------------------------------

_pf32 = C.POINTER(C.c_float)
_sig("bmpc_mlp_create", _i32, [_pi32, _i32, _i32, C.POINTER(_vp)])
_sig("bmpc_mlp_destroy", None, [_vp])
_sig("bmpc_mlp_num_params", C.c_int64, [_vp])
_sig("bmpc_mlp_set_params", _i32, [_vp, _pf32])
_sig("bmpc_mlp_get_params", _i32, [_vp, _pf32])
_sig("bmpc_mlp_set_input_map", _i32, [_vp, _pf32, _pf32])
_sig("bmpc_mlp_forward", _i32, [_vp, _vp, _i32, _vp, _vp])
_sig("bmpc_mlp_gradients", _i32, [_vp, _vp, _vp, _i32, _pf32, _pf32, _vp])
_sig("bmpc_mlp_train_step", _i32, [_vp, _vp, _vp, _i32, C.c_float, _pf32, _vp])
_sig("bmpc_gemm_bf16", _i32, [_i32, _i32, _i32, _vp, _i32, _vp, _i32, _vp, _vp])


def _hf32(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(_pf32)


def bmpc_mlp_create(widths, max_batch):
    w, pw = _hi32(widths)
    out = _vp()
    check(lib.bmpc_mlp_create(pw, len(w) - 1, max_batch, C.byref(out)))
    _dims[_key(out)] = (int(w[0]), int(w[-1]))
    return out


def bmpc_mlp_destroy(h):
    _dims.pop(_key(h), None)
    lib.bmpc_mlp_destroy(h)


def bmpc_mlp_num_params(h):
    return int(lib.bmpc_mlp_num_params(h))


def bmpc_mlp_set_params(h, params):
    p, pp = _hf32(params)
    if p.size != bmpc_mlp_num_params(h):
        raise ValueError("parameter vector of the wrong length")
    check(lib.bmpc_mlp_set_params(h, pp))


def bmpc_mlp_set_input_map(h, shift, scale):
    a, pa = _hf32(shift)
    b, pb = _hf32(scale)
    check(lib.bmpc_mlp_set_input_map(h, pa, pb))


def bmpc_mlp_get_params(h):
    p = np.zeros(bmpc_mlp_num_params(h), dtype=np.float32)
    check(lib.bmpc_mlp_get_params(h, p.ctypes.data_as(_pf32)))
    return p


def bmpc_mlp_forward(h, X, Y, stream=None):
    """X (B, w_0) and Y (B, w_L): float32 device tensors."""
    w0, wl = _dims[_key(h)]
    B = X.shape[0]
    px, py = _dptrs([(X, "float32", B * w0, "X"), (Y, "float32", B * wl, "Y")])
    check(lib.bmpc_mlp_forward(h, px, B, py, stream_ptr(stream)))


def bmpc_mlp_gradients(h, X, T, stream=None):
    g = np.zeros(bmpc_mlp_num_params(h), dtype=np.float32)
    loss = np.zeros(1, dtype=np.float32)
    w0, wl = _dims[_key(h)]
    B = X.shape[0]
    px, pt = _dptrs([(X, "float32", B * w0, "X"), (T, "float32", B * wl, "T")])
    check(lib.bmpc_mlp_gradients(h, px, pt, B,
                                 g.ctypes.data_as(_pf32),
                                 loss.ctypes.data_as(_pf32), stream_ptr(stream)))
    return float(loss[0]), g


def bmpc_mlp_train_step(h, X, T, lr, want_loss=True, stream=None):
    loss = np.zeros(1, dtype=np.float32)
    w0, wl = _dims[_key(h)]
    B = X.shape[0]
    px, pt = _dptrs([(X, "float32", B * w0, "X"), (T, "float32", B * wl, "T")])
    check(lib.bmpc_mlp_train_step(h, px, pt, B, lr,
                                  loss.ctypes.data_as(_pf32) if want_loss else None, stream_ptr(stream)))
    return float(loss[0]) if want_loss else None


def bmpc_gemm_bf16(M, N, K, A, trans_a, B, trans_b, C_out, stream=None):
    """A, B: int16/bfloat16 device tensors holding BF16 bit patterns; C_out float32."""
    check(lib.bmpc_gemm_bf16(M, N, K, _bf16_ptr(A, M * K, "A"), int(trans_a), _bf16_ptr(B, K * N, "B"),
                             int(trans_b), dptr(C_out, "float32", M * N, "C"), stream_ptr(stream)))


# ----------------------------------------------------------------------------
# launch configuration and graphs
# ----------------------------------------------------------------------------

_sig("bmpc_batch_tune", _i32, [_vp, _vp, _i32, _i32, _pi32, _pi32, _pd, _vp])
_sig("bmpc_batch_tune_candidates", _i32, [_pi32, _pi32, _i32])
_sig("bmpc_graph_begin", _i32, [_vp])
_sig("bmpc_graph_end", _i32, [_vp, C.POINTER(_vp)])
_sig("bmpc_graph_launch", _i32, [_vp, _vp])
_sig("bmpc_graph_destroy", None, [_vp])


def bmpc_batch_tune_candidates():
    n = lib.bmpc_batch_tune_candidates(None, None, 0)
    v = np.zeros(n, dtype=np.int32)
    b = np.zeros(n, dtype=np.int32)
    lib.bmpc_batch_tune_candidates(v.ctypes.data_as(_pi32), b.ctypes.data_as(_pi32), n)
    return list(zip(v.tolist(), b.tolist()))


_sig("bmpc_batch_autotune", _i32, [_vp, _vp, _i32, _i32, C.c_char_p, _pi32, _pi32, _pd, _pi32, _vp])


def bmpc_batch_autotune(batch, settings, warm=0, budget_ms=0, cache_path=None, stream=None):
    """Returns (variant, block_size, ms per inner iteration, from_cache)."""
    v, b, fc = C.c_int32(), C.c_int32(), C.c_int32()
    t = C.c_double()
    check(lib.bmpc_batch_autotune(batch, C.byref(settings), warm, int(budget_ms),
                                  cache_path.encode() if cache_path else None, C.byref(v), C.byref(b),
                                  C.byref(t), C.byref(fc), stream_ptr(stream)))
    return v.value, b.value, t.value, bool(fc.value)


def bmpc_batch_tune(batch, settings, warm=0, reps=1, stream=None):
    """Returns (variant, block_size, {(variant, block): ms per inner iteration})."""
    cands = bmpc_batch_tune_candidates()
    v, b = C.c_int32(), C.c_int32()
    ms = np.zeros(len(cands))
    check(lib.bmpc_batch_tune(batch, C.byref(settings), warm, reps, C.byref(v), C.byref(b),
                              ms.ctypes.data_as(_pd), stream_ptr(stream)))
    return v.value, b.value, dict(zip(cands, ms.tolist()))


def bmpc_graph_begin(stream):
    check(lib.bmpc_graph_begin(stream_ptr(stream)))


def bmpc_graph_end(stream):
    out = _vp()
    check(lib.bmpc_graph_end(stream_ptr(stream), C.byref(out)))
    return out


def bmpc_graph_launch(graph, stream=None):
    check(lib.bmpc_graph_launch(graph, stream_ptr(stream)))


def bmpc_graph_destroy(graph):
    lib.bmpc_graph_destroy(graph)
