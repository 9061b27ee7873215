"""CPU FP64 oracle for the branch-MPC hot path (ctypes front end).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
CPU-baseline leg of the benchmark are the only users.  The HIP library never
loads or calls anything in this package, and this package imports nothing
from the library.

The C sources (``oracle_lqr.c``, ``oracle_bmpc.c``) hold the arithmetic;
this module only converts NumPy arrays to pointers.  ``cvf.py`` holds the
conditional-value-function algebra of the parallel-scan LQR, in NumPy.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SOURCES = ["oracle_lqr.c", "oracle_bmpc.c", "oracle_hess.c", "oracle_mlp.c"]

STATUS = {0: "OK", 1: "INVALID_ARG", 2: "TOPOLOGY", 3: "NOT_PD", 4: "NONFINITE",
          5: "MAXITER", 6: "LINESEARCH"}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2; no target-specific flags so the
    library runs on any x86-64 host)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    srcs = [os.path.join(_HERE, s) for s in SOURCES if os.path.exists(os.path.join(_HERE, s))]
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wno-unused-function",
           "-o", tmp] + srcs + ["-lm", "-lpthread"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def use_native_build(out_dir=None) -> str:
    """Compile a copy of the oracle with -O3 -march=native for this host and
    load it instead of the portable build (the CPU-baseline timings use it;
    the arithmetic is the same C code)."""
    global _lib
    out_dir = out_dir or os.path.join(os.path.dirname(_HERE), "_build")
    os.makedirs(out_dir, exist_ok=True)
    path = os.path.join(out_dir, "liboracle_native.so")
    srcs = [os.path.join(_HERE, s) for s in SOURCES if os.path.exists(os.path.join(_HERE, s))]
    tmp = path + ".tmp"
    subprocess.run(["gcc", "-O3", "-march=native", "-std=c11", "-fPIC", "-shared", "-o", tmp] + srcs
                   + ["-lm", "-lpthread"], check=True)
    os.replace(tmp, path)
    _lib = C.CDLL(path)
    _declare(_lib)
    return path


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = C.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


class Model(C.Structure):
    _fields_ = [("model", C.c_int), ("wheelbase", C.c_double), ("dt", C.c_double),
                ("Qd", C.c_double * 4), ("Rd", C.c_double * 2), ("a_max", C.c_double),
                ("steer_max", C.c_double), ("obs_r", C.c_double), ("Al", C.c_double * 16),
                ("Bl", C.c_double * 8)]


class Problem(C.Structure):
    _fields_ = [("N", C.c_int), ("parent", _ip), ("weight", _dp), ("ref", _dp), ("obs", _dp),
                ("has_obs", _ip), ("x0", _dp), ("model", Model)]


class Settings(C.Structure):
    _fields_ = [("eps_tol", C.c_double), ("tau", C.c_double), ("omega0", C.c_double),
                ("eta0", C.c_double), ("a_omega", C.c_double), ("b_omega", C.c_double),
                ("a_eta", C.c_double), ("b_eta", C.c_double), ("rho0", C.c_double),
                ("mu0", C.c_double), ("armijo_beta", C.c_double), ("n_alpha", C.c_int),
                ("max_outer", C.c_int), ("max_inner", C.c_int), ("max_ls_fail", C.c_int),
                ("max_iter_total", C.c_int), ("ls_rounds", C.c_int), ("hessian", C.c_int),
                ("eig_floor", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("status", C.c_int), ("outer_it", C.c_int), ("inner_it", C.c_int),
                ("ls_failures", C.c_int), ("bad_node", C.c_int), ("start", C.c_int), ("r_kkt", C.c_double),
                ("viol", C.c_double), ("rho", C.c_double), ("mu", C.c_double),
                ("merit", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def _declare(L):
    L.orc_tree_lqr.restype = C.c_int
    L.orc_tree_lqr.argtypes = [C.c_int, C.c_int, C.c_int, _ip] + [_dp] * 9 + [_dp] * 7 + [_ip]
    L.orc_tree_lqr_ld.restype = C.c_int
    L.orc_tree_lqr_ld.argtypes = [C.c_int, C.c_int, C.c_int, _ip] + [_dp] * 9 + [_dp] * 7 + [_ip]
    L.orc_tree_lqr_f.restype = C.c_int
    L.orc_tree_lqr_f.argtypes = [C.c_int, C.c_int, C.c_int, _ip] + [_dp] * 9 + [_dp] * 7 + [_ip]
    L.orc_settings_default.argtypes = [C.POINTER(Settings)]
    L.orc_bmpc_solve.restype = C.c_int
    L.orc_bmpc_solve.argtypes = [C.POINTER(Problem), C.POINTER(Settings), C.c_int, _dp, _dp,
                                 _dp, _dp, C.POINTER(Stats), _dp, C.c_int]
    L.orc_rk4.argtypes = [C.POINTER(Model), _dp, _dp, _dp, _dp, _dp]
    L.orc_node_weights.argtypes = [C.c_int, _ip, _dp, _dp]
    L.orc_node_refs.argtypes = [C.c_int, _ip, _dp, _dp, C.c_double, C.c_double, _dp]
    L.orc_node_terms.restype = C.c_double
    L.orc_node_terms.argtypes = [C.POINTER(Problem), C.c_int, _dp, _dp, _dp, C.c_double, _dp,
                                 _dp, _dp, _dp, _dp]
    for name in ("orc_augmented_lagrangian", "orc_violation"):
        getattr(L, name).restype = C.c_double
        getattr(L, name).argtypes = [C.POINTER(Problem), _dp, _dp, _dp, C.c_double]
    L.orc_merit.restype = C.c_double
    L.orc_merit.argtypes = [C.POINTER(Problem), _dp, _dp, _dp, _dp, C.c_double, C.c_double]
    L.orc_direction.restype = C.c_int
    L.orc_direction.argtypes = [C.POINTER(Problem), _dp, _dp, _dp, _dp, C.c_double, C.c_double,
                                _dp, _dp, _dp, _dp]
    L.orc_direction_h.restype = C.c_int
    L.orc_direction_h.argtypes = [C.POINTER(Problem), _dp, _dp, _dp, _dp, C.c_double, C.c_double, C.c_int,
                                  C.c_double, _dp, _dp, _dp, _dp]
    L.orc_rk4_hessian.restype = None
    L.orc_rk4_hessian.argtypes = [C.POINTER(Model), _dp, _dp, _dp, _dp]
    L.orc_sym_eig.restype = C.c_int
    L.orc_sym_eig.argtypes = [C.c_int, _dp, _dp, _dp]
    L.orc_eig_modify.restype = C.c_int
    L.orc_eig_modify.argtypes = [C.c_int, _dp, C.c_double, _dp]
    L.orc_node_quadratic.restype = None
    L.orc_node_quadratic.argtypes = [C.POINTER(Problem), C.c_int, _dp, _dp, _dp, _dp, C.c_double, C.c_int,
                                     C.c_double, C.c_int, _dp, _dp, _dp, _dp, _dp]
    L.orc_kkt.restype = C.c_double
    L.orc_kkt.argtypes = [C.POINTER(Problem), _dp, _dp, _dp, _dp, C.c_double]
    L.orc_adjoint.argtypes = [C.POINTER(Problem), _dp, _dp, _dp, C.c_double, _dp]
    L.orc_rollout.argtypes = [C.POINTER(Problem), _dp, _dp]
    L.orc_shift.argtypes = [C.POINTER(Problem)] + [_dp] * 11
    if hasattr(L, "orc_mlp_forward"):
        _declare_mlp(L)


def _declare_mlp(L):
    for name in ("orc_bf16", "orc_gelu", "orc_gelu_prime"):
        getattr(L, name).restype = C.c_double
        getattr(L, name).argtypes = [C.c_double]
    L.orc_mlp_forward.argtypes = [C.c_int, _ip, C.c_int, _dp, _dp, C.c_int, _dp]
    L.orc_mlp_backward.argtypes = [C.c_int, _ip, C.c_int, _dp, _dp, _dp, C.c_int, _dp, _dp]
    L.orc_adam.argtypes = [C.c_long, _dp, _dp, _dp, _dp, C.c_int, C.c_double, C.c_double, C.c_double,
                           C.c_double]


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


# ----------------------------------------------------------------------------
# tree LQR
# ----------------------------------------------------------------------------

def tree_lqr(parent, A, B, c, Q, R, M, q, r, x0, extended=False, single=False):
    """Serial tree Riccati (node-major arrays).  Returns a dict with x, u, lam,
    K, k, P, p; raises on a non-OK status.  extended=True carries the
    recursion out in long double (results rounded to double); single=True in
    float (inputs rounded to float, results widened)."""
    parent = np.ascontiguousarray(parent, dtype=np.int32)
    N = len(parent)
    nx = np.shape(A)[1]
    nu = np.shape(B)[2]
    A, B, c, Q, R, M, q, r, x0 = (_f64(v) for v in (A, B, c, Q, R, M, q, r, x0))
    out = {"x": np.zeros((N, nx)), "u": np.zeros((N, nu)), "lam": np.zeros((N, nx)),
           "K": np.zeros((N, nu, nx)), "k": np.zeros((N, nu)), "P": np.zeros((N, nx, nx)),
           "p": np.zeros((N, nx))}
    bad = np.array([-1], dtype=np.int32)
    fn = lib().orc_tree_lqr_ld if extended else lib().orc_tree_lqr_f if single else lib().orc_tree_lqr
    st = fn(N, nx, nu, _i(parent), _d(A), _d(B), _d(c), _d(Q), _d(R), _d(M),
                            _d(q), _d(r), _d(x0), _d(out["x"]), _d(out["u"]), _d(out["lam"]),
                            _d(out["K"]), _d(out["k"]), _d(out["P"]), _d(out["p"]), _i(bad))
    if st != 0:
        raise OracleError(st, int(bad[0]))
    return out


def tree_lqr_inst(inst, extended=False, single=False):
    return tree_lqr(inst.parent, inst.A, inst.B, inst.c, inst.Q, inst.R, inst.M, inst.q,
                    inst.r, inst.x0, extended=extended, single=single)


class OracleError(RuntimeError):
    def __init__(self, status, node=-1):
        super().__init__(f"oracle status {STATUS.get(status, status)} (node {node})")
        self.status = status
        self.node = node


# ----------------------------------------------------------------------------
# branch-MPC problem
# ----------------------------------------------------------------------------

def default_settings(**kw) -> Settings:
    s = Settings()
    lib().orc_settings_default(C.byref(s))
    for k, v in kw.items():
        setattr(s, k, v)
    return s


def node_weights(parent, leaf_prob):
    parent = np.ascontiguousarray(parent, dtype=np.int32)
    lp = _f64(leaf_prob)
    w = np.zeros(len(parent))
    lib().orc_node_weights(len(parent), _i(parent), _d(lp), _d(w))
    return w


def node_refs(parent, leaf_prob, leaf_offset, dt, speed):
    parent = np.ascontiguousarray(parent, dtype=np.int32)
    ref = np.zeros((len(parent), 4))
    lib().orc_node_refs(len(parent), _i(parent), _d(_f64(leaf_prob)), _d(_f64(leaf_offset)),
                        dt, speed, _d(ref))
    return ref


class BmpcProblem:
    """Holds the arrays a ctypes ``Problem`` points to (keeps them alive)."""

    def __init__(self, parent, weight, ref, node_obs_xy, has_obs, x0, model: Model):
        self.parent = np.ascontiguousarray(parent, dtype=np.int32)
        self.N = len(self.parent)
        self.weight = _f64(weight)
        self.ref = _f64(ref, (self.N, 4))
        self.obs = _f64(node_obs_xy, (self.N, 2))
        self.has_obs = np.ascontiguousarray(has_obs, dtype=np.int32)
        self.x0 = _f64(x0)
        self.model = model
        self.c = Problem(self.N, _i(self.parent), _d(self.weight), _d(self.ref), _d(self.obs),
                         _i(self.has_obs), _d(self.x0), model)

    @property
    def ptr(self):
        return C.byref(self.c)


def bicycle_model(inst) -> Model:
    m = Model()
    m.model = 0
    m.wheelbase = inst.wheelbase
    m.dt = inst.dt
    for i in range(4):
        m.Qd[i] = inst.q_diag[i]
    for i in range(2):
        m.Rd[i] = inst.r_diag[i]
    m.a_max = inst.a_max
    m.steer_max = inst.steer_max
    m.obs_r = inst.obs_radius
    return m


def linear_model(Al, Bl, q_diag, r_diag, a_max=1e3, steer_max=1e3, obs_r=1.5, dt=0.1) -> Model:
    m = Model()
    m.model = 1
    m.dt = dt
    m.wheelbase = 1.0
    for i in range(4):
        m.Qd[i] = q_diag[i]
    for i in range(2):
        m.Rd[i] = r_diag[i]
    m.a_max = a_max
    m.steer_max = steer_max
    m.obs_r = obs_r
    for i, v in enumerate(np.asarray(Al, np.float64).ravel()):
        m.Al[i] = v
    for i, v in enumerate(np.asarray(Bl, np.float64).ravel()):
        m.Bl[i] = v
    return m


def problem_from_instance(inst, x0=None) -> BmpcProblem:
    w = node_weights(inst.parent, inst.leaf_prob)
    ref = node_refs(inst.parent, inst.leaf_prob, inst.leaf_offset, inst.dt, inst.ref_speed)
    has = (inst.node_obstacle >= 0).astype(np.int32)
    xy = np.zeros((inst.num_nodes, 2))
    if len(inst.obstacles):
        xy[has == 1] = inst.obstacles[inst.node_obstacle[has == 1]]
    return BmpcProblem(inst.parent, w, ref, xy, has, inst.x0 if x0 is None else x0,
                       bicycle_model(inst))


def solve(pb: BmpcProblem, settings: Settings | None = None, warm=None, hist_cap=4096, guarded=False):
    """Run the AL multiple-shooting iLQR.  ``warm`` may be a dict with any of
    x, u, lam, ye; u without x starts from the rollout of u.  ``guarded``
    keeps the cold start instead when it is better by max(KKT residual,
    violation).  Returns (state dict, stats dict, history array)."""
    st = settings if settings is not None else default_settings()
    N = pb.N
    x = np.zeros((N, 4))
    u = np.zeros((N, 2))
    lam = np.zeros((N, 4))
    ye = np.zeros((N, 5))
    bits = 0
    if warm:
        if "x" in warm and "u" in warm:
            x[:] = warm["x"]
            u[:] = warm["u"]
            bits |= 1
        elif "u" in warm:
            u[:] = warm["u"]
            bits |= 8
        if "lam" in warm:
            lam[:] = warm["lam"]
            bits |= 2
        if "ye" in warm:
            ye[:] = warm["ye"]
            bits |= 4
    if guarded:
        bits |= 16
    stats = Stats()
    hist = np.zeros((hist_cap, 6))
    lib().orc_bmpc_solve(pb.ptr, C.byref(st), bits, _d(x), _d(u), _d(lam), _d(ye),
                         C.byref(stats), _d(hist), hist_cap)
    s = stats.as_dict()
    return {"x": x, "u": u, "lam": lam, "ye": ye}, s, hist[: s["inner_it"]]


def rk4(model: Model, x, u):
    x = _f64(x)
    u = _f64(u)
    xn = np.zeros(4)
    A = np.zeros((4, 4))
    B = np.zeros((4, 2))
    lib().orc_rk4(C.byref(model), _d(x), _d(u), _d(xn), _d(A), _d(B))
    return xn, A, B


def node_terms(pb: BmpcProblem, n, x, u, ye, rho):
    g = np.zeros(5)
    gx = np.zeros(4)
    gu = np.zeros(2)
    Hxx = np.zeros((4, 4))
    Huu = np.zeros((2, 2))
    v = lib().orc_node_terms(pb.ptr, n, _d(_f64(x)), _d(_f64(u)), _d(_f64(ye)), rho, _d(g),
                             _d(gx), _d(gu), _d(Hxx), _d(Huu))
    return v, g, gx, gu, Hxx, Huu


def augmented_lagrangian(pb, x, u, ye, rho):
    return lib().orc_augmented_lagrangian(pb.ptr, _d(_f64(x)), _d(_f64(u)), _d(_f64(ye)), rho)


def merit(pb, x, u, lam, ye, rho, mu):
    return lib().orc_merit(pb.ptr, _d(_f64(x)), _d(_f64(u)), _d(_f64(lam)), _d(_f64(ye)), rho, mu)


def kkt(pb, x, u, lam, ye, rho):
    return lib().orc_kkt(pb.ptr, _d(_f64(x)), _d(_f64(u)), _d(_f64(lam)), _d(_f64(ye)), rho)


def direction(pb, x, u, lam, ye, rho, mu, hessian=0, eig_floor=1e-9):
    """One search direction at (x, u, lam): the tree-LQR step and the merit
    slope pieces.  Returns (dx, du, lam_hat, dict) with the dict holding
    gtd, dhd, lhd, dd, mu_hat, mu, dphi0, phi0.  hessian=1 takes the exact
    Hessian with eigenvalue modification."""
    N = pb.N
    dx, du, lh = np.zeros((N, 4)), np.zeros((N, 2)), np.zeros((N, 4))
    out = np.zeros(8)
    st = lib().orc_direction_h(pb.ptr, _d(_f64(x)), _d(_f64(u)), _d(_f64(lam)), _d(_f64(ye)), rho, mu,
                               int(hessian), float(eig_floor), _d(dx), _d(du), _d(lh), _d(out))
    if st != 0:
        raise OracleError(st)
    keys = ("gtd", "dhd", "lhd", "dd", "mu_hat", "mu", "dphi0", "phi0")
    return dx, du, lh, dict(zip(keys, out.tolist()))


def rk4_hessian(model: Model, x, u, mu):
    """Second derivatives (6 x 6, z = (x, u)) of mu^T F(x, u)."""
    H = np.zeros((6, 6))
    lib().orc_rk4_hessian(C.byref(model), _d(_f64(x)), _d(_f64(u)), _d(_f64(mu)), _d(H))
    return H


def sym_eig(A):
    A = _f64(A)
    n = A.shape[0]
    w, V = np.zeros(n), np.zeros((n, n))
    st = lib().orc_sym_eig(n, _d(A), _d(w), _d(V))
    if st != 0:
        raise OracleError(st)
    return w, V


def eig_modify(A, delta):
    A = _f64(A)
    n = A.shape[0]
    out = np.zeros((n, n))
    st = lib().orc_eig_modify(n, _d(A), float(delta), _d(out))
    if st != 0:
        raise OracleError(st)
    return out


def node_quadratic(pb, n, x, u, lam, ye, rho, hessian=1, eig_floor=1e-9, modify=True):
    """Quadratic model of node n: q, r, Q, R, M (whole-tree state arrays)."""
    q, r = np.zeros(4), np.zeros(2)
    Q, R, M = np.zeros((4, 4)), np.zeros((2, 2)), np.zeros((2, 4))
    lib().orc_node_quadratic(pb.ptr, int(n), _d(_f64(x)), _d(_f64(u)), _d(_f64(lam)), _d(_f64(ye)), float(rho),
                             int(hessian), float(eig_floor), int(bool(modify)), _d(q), _d(r), _d(Q), _d(R), _d(M))
    return q, r, Q, R, M


def violation(pb, x, u, ye, rho):
    return lib().orc_violation(pb.ptr, _d(_f64(x)), _d(_f64(u)), _d(_f64(ye)), rho)


def adjoint(pb, x, u, ye, rho):
    lam = np.zeros((pb.N, 4))
    lib().orc_adjoint(pb.ptr, _d(_f64(x)), _d(_f64(u)), _d(_f64(ye)), rho, _d(lam))
    return lam


def rollout(pb, u):
    x = np.zeros((pb.N, 4))
    lib().orc_rollout(pb.ptr, _d(_f64(u)), _d(x))
    return x


def shift(pb: BmpcProblem, state, x0_meas=None):
    """Shifted warm start after one simulated step (x0_meas: the measured
    next state, default the model's prediction).  Returns (new problem,
    shifted state dict)."""
    N = pb.N
    ref = np.zeros((N, 4))
    x0 = np.zeros(4)
    out = {"x": np.zeros((N, 4)), "u": np.zeros((N, 2)), "lam": np.zeros((N, 4)),
           "ye": np.zeros((N, 5))}
    st = {k: _f64(state[k]) for k in ("x", "u", "lam", "ye")}
    xa = None if x0_meas is None else _f64(x0_meas)
    xm = None if xa is None else _d(xa)
    lib().orc_shift(pb.ptr, _d(st["x"]), _d(st["u"]), _d(st["lam"]), _d(st["ye"]), xm, _d(ref), _d(x0),
                    _d(out["x"]), _d(out["u"]), _d(out["lam"]), _d(out["ye"]))
    new = BmpcProblem(pb.parent, pb.weight, ref, pb.obs, pb.has_obs, x0, pb.model)
    return new, out


# ----------------------------------------------------------------------------
# warm-start network (oracle_mlp.c)
# ----------------------------------------------------------------------------

def mlp_num_params(widths):
    w = list(widths)
    return sum(w[l] * w[l + 1] + w[l + 1] for l in range(len(w) - 1))


def bf16(x):
    """Nearest BF16 value of each entry (ties to even), as float64."""
    f = lib().orc_bf16
    a = np.asarray(x, dtype=np.float64)
    return np.array([f(float(v)) for v in a.ravel()]).reshape(a.shape)


def gelu(z):
    return lib().orc_gelu(float(z))


def gelu_prime(z):
    return lib().orc_gelu_prime(float(z))


def mlp_forward(widths, params, X, quant=True):
    w = np.ascontiguousarray(widths, dtype=np.int32)
    X = _f64(X)
    B = X.shape[0]
    Y = np.zeros((B, int(w[-1])))
    p = _f64(params)
    st = lib().orc_mlp_forward(len(w) - 1, _i(w), B, _d(p), _d(X), int(quant), _d(Y))
    if st != 0:
        raise OracleError(st)
    return Y


def mlp_loss_grad(widths, params, X, T, quant=True):
    w = np.ascontiguousarray(widths, dtype=np.int32)
    X, T, p = _f64(X), _f64(T), _f64(params)
    B = X.shape[0]
    g = np.zeros_like(p)
    loss = np.zeros(1)
    st = lib().orc_mlp_backward(len(w) - 1, _i(w), B, _d(p), _d(X), _d(T), int(quant), _d(g), _d(loss))
    if st != 0:
        raise OracleError(st)
    return float(loss[0]), g


def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step in place on float64 arrays p, m, v."""
    for a in (p, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _f64(g)
    lib().orc_adam(p.size, _d(p), _d(g), _d(m), _d(v), int(t), lr, b1, b2, eps)
