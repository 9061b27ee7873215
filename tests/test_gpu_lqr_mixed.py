"""FP32 tree LQR and the mixed-precision solve (FP32 Riccati sweeps with FP64
iterative refinement) against the oracle, through the C ABI.

Bars:
  - FP32 solve: the reference is the oracle's recursion in long double on
    the same (double) data; the GPU's relative error per array is at most 16
    times that of the oracle's own float recursion (inputs rounded to float,
    every operation in float), or 2^-20, whichever is larger: both make the
    same input roundings and differ only in the order of their float sums.
  - mixed solve: the FP64 bar of the tree LQR, relative 1e-9 per array
    (at the rounding floor of the double recursion on ill-conditioned
    subproblems), after enough refinement steps; the residual norms it
    reports agree with a host evaluation of the KKT rows.
"""
import numpy as np
import pytest

import bmpc_synth as S
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_2506_13624_amd import _lib as L  # noqa: E402
from paper_2506_13624_amd.layout import empty, from_device, to_device  # noqa: E402

from test_gpu_lqr import TREES, gauss_newton_subproblem, relerr  # noqa: E402

TOL = 1e-9
DIMS = [(3, 1), (4, 2), (6, 3)]


def _plan(inst, layout):
    tree = L.bmpc_tree_create(inst.parent)
    return tree, L.bmpc_lqr_plan_create(tree, inst.nx, inst.nu, layout)


def _shapes(inst):
    N = len(inst.parent)
    return {"x": (N, inst.nx), "u": (N, inst.nu), "lam": (N, inst.nx), "K": (N, inst.nu, inst.nx),
            "k": (N, inst.nu), "P": (N, inst.nx, inst.nx), "p": (N, inst.nx)}


def gpu_f32(inst, layout):
    tree, plan = _plan(inst, layout)
    try:
        dev = {k: to_device(getattr(inst, k), layout).float() for k in "ABcQRMqr"}
        x0 = to_device(inst.x0, layout).float()
        shp = _shapes(inst)
        out = {k: torch.zeros(int(np.prod(v)), dtype=torch.float32, device="cuda") for k, v in shp.items()}
        L.bmpc_lqr_solve_f32(plan, dev["A"], dev["B"], dev["c"], dev["Q"], dev["R"], dev["M"], dev["q"],
                             dev["r"], x0, out["x"], out["u"], out["lam"], out["K"], out["k"], out["P"], out["p"])
        st, bad = L.bmpc_lqr_check(plan)
        return {k: from_device(v, shp[k], layout).astype(np.float64) for k, v in out.items()}, st, bad
    finally:
        L.bmpc_lqr_plan_destroy(plan)
        L.bmpc_tree_destroy(tree)


def gpu_mixed(inst, layout, steps, repeat=1):
    tree, plan = _plan(inst, layout)
    try:
        dev = {k: to_device(getattr(inst, k), layout) for k in "ABcQRMqr"}
        x0 = to_device(inst.x0, layout)
        shp = _shapes(inst)
        runs = []
        for _ in range(repeat):
            out = {k: empty(shp[k]) for k in ("x", "u", "lam")}
            norms = torch.full((steps + 2,), -1.0, dtype=torch.float64, device="cuda")
            L.bmpc_lqr_solve_mixed(plan, dev["A"], dev["B"], dev["c"], dev["Q"], dev["R"], dev["M"], dev["q"],
                                   dev["r"], x0, out["x"], out["u"], out["lam"], steps, res_norms=norms)
            st, bad = L.bmpc_lqr_check(plan)
            runs.append(({k: from_device(v, shp[k], layout) for k, v in out.items()}, norms.cpu().numpy(), st,
                         bad))
        return runs if repeat > 1 else runs[0]
    finally:
        L.bmpc_lqr_plan_destroy(plan)
        L.bmpc_tree_destroy(tree)


def kkt_rows_max(inst, sol):
    """Largest |KKT row| of the tree QP at (x, u, lam): stationarity in u
    (control nodes) and x (every node, the root's lam being the multiplier
    of x_0 = x0) and the dynamics defects (root: x0 - x_0)."""
    par = inst.parent
    x, u, lam = sol["x"], sol["u"], sol["lam"]
    nch = S.num_children(par)
    worst = 0.0
    for n in range(len(par)):
        kids = np.nonzero(par == n)[0]
        gx = inst.Q[n] @ x[n] + inst.q[n] - lam[n] + sum((inst.A[j].T @ lam[j] for j in kids), 0.0)
        if nch[n] > 0:
            gx = gx + inst.M[n].T @ u[n]
            gu = inst.R[n] @ u[n] + inst.M[n] @ x[n] + inst.r[n] + sum(inst.B[j].T @ lam[j] for j in kids)
            worst = max(worst, np.abs(gu).max())
        d = inst.x0 - x[n] if par[n] < 0 else inst.A[n] @ x[par[n]] + inst.B[n] @ u[par[n]] + inst.c[n] - x[n]
        worst = max(worst, np.abs(gx).max(), np.abs(d).max())
    return worst


@pytest.mark.parametrize("layout", [L.LAYOUT_NODE_MAJOR, L.LAYOUT_ELEM_MAJOR])
@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("name", sorted(TREES))
def test_f32_solve_at_float_accuracy(name, dims, layout):
    par = TREES[name]
    print(f"f32 tree={name} N={len(par)} dims={dims} layout={layout}", flush=True)
    inst = S.lqr_on(par, dims[0], dims[1], seed=17, random_cost=True)
    ext = oracle.tree_lqr_inst(inst, extended=True)
    single = oracle.tree_lqr_inst(inst, single=True)
    g, st, bad = gpu_f32(inst, layout)
    assert st == 0, bad
    for k in ("x", "u", "lam", "K", "k", "P", "p"):
        floor = relerr(single[k], ext[k])
        e = relerr(g[k], ext[k])
        assert e <= max(2.0 ** -20, 16.0 * floor), f"{k}: {e:.3e} (oracle float {floor:.3e})"


@pytest.mark.parametrize("layout", [L.LAYOUT_NODE_MAJOR, L.LAYOUT_ELEM_MAJOR])
@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("name", sorted(TREES))
def test_mixed_solve_matches_oracle(name, dims, layout):
    par = TREES[name]
    print(f"mixed tree={name} N={len(par)} dims={dims} layout={layout}", flush=True)
    inst = S.lqr_on(par, dims[0], dims[1], seed=17, random_cost=True)
    o = oracle.tree_lqr_inst(inst)
    g, norms, st, bad = gpu_mixed(inst, layout, steps=3)
    assert st == 0, bad
    for k in ("x", "u", "lam"):
        e = relerr(g[k], o[k])
        assert e <= TOL, f"{k}: relative error {e:.3e}"
    # entry 0 is the data's largest |row|; the last one the final residual
    N = len(par)
    nch = S.num_children(par)
    data = max(np.abs(inst.q).max(), np.abs(inst.c[1:]).max() if N > 1 else 0.0, np.abs(inst.x0).max(),
               np.abs(inst.r[nch > 0]).max() if (nch > 0).any() else 0.0)
    assert norms[0] == data
    host = kkt_rows_max(inst, g)
    print(f"  residual norms {norms}, host {host:.3e}", flush=True)
    assert abs(norms[-1] - host) <= 1e-13 * data + 0.5 * host
    assert norms[-1] <= 1e-11 * data


def test_mixed_without_refinement_is_the_f32_solve_of_the_rounded_data():
    """With no refinement step the result is the FP32 solve of the data
    rounded to float, bit for bit."""
    inst = S.lqr_on(TREES["random_a"], 4, 2, seed=5, random_cost=True)
    g, norms, st, _ = gpu_mixed(inst, L.LAYOUT_ELEM_MAJOR, steps=0)
    f, st2, _ = gpu_f32(inst, L.LAYOUT_ELEM_MAJOR)
    assert st == st2 == 0
    for k in ("x", "u", "lam"):
        np.testing.assert_array_equal(g[k], f[k])
    assert len(norms) == 2 and norms[1] > 0


def test_mixed_residual_contracts_each_step():
    """Each refinement step shrinks the FP64 residual by the FP32 solve's
    relative accuracy (well below 1e-3 here), down to the double rounding
    floor; the result is bitwise reproducible."""
    inst = S.lqr_on(S.tree_parent(40, [3, 9, 20], 3), 6, 3, seed=21, random_cost=True)
    runs = gpu_mixed(inst, L.LAYOUT_NODE_MAJOR, steps=5, repeat=2)
    norms = runs[0][1]
    print(f"residual norms {norms}", flush=True)
    floor = 1e-13 * norms[0]
    for a, b in zip(norms[1:], norms[2:]):
        assert b <= 1e-3 * a or b <= floor
    for k in ("x", "u", "lam"):
        np.testing.assert_array_equal(runs[0][0][k], runs[1][0][k])
    np.testing.assert_array_equal(runs[0][1], runs[1][1])


def test_mixed_large_tree_full_size():
    """nx=4, nu=2 random data on the 4096-scenario topology (122,871 nodes):
    every element of x, u, lam within 1e-9 of the oracle."""
    par = S.large_tree(0).parent
    print(f"mixed large tree N={len(par)}", flush=True)
    inst = S.lqr_on(par, 4, 2, seed=3)
    o = oracle.tree_lqr_inst(inst)
    g, norms, st, _ = gpu_mixed(inst, L.LAYOUT_ELEM_MAJOR, steps=3)
    print(f"  residual norms {norms}", flush=True)
    assert st == 0
    for k in ("x", "u", "lam"):
        e = relerr(g[k], o[k])
        assert e <= TOL, f"{k}: relative error {e:.3e}"


@pytest.mark.parametrize("seed", [0, 1])
def test_mixed_on_single_tree_gauss_newton_subproblems(seed):
    """The solver's own subproblems (single-tree workload along the oracle's
    iteration path).  Their conditioning ranges over orders of magnitude;
    the mixed solve is held to the FP64 bar (1e-9, or four times the double
    recursion's own error against long double where that is larger) once
    its residual has stopped falling, and the number of steps that took is
    reported."""
    inst = S.single_bmpc(seed)
    pb = oracle.problem_from_instance(inst)
    for its in (0, 3, 10, 25):
        st, s, _ = oracle.solve(pb, oracle.default_settings(max_iter_total=its))
        rho = oracle.default_settings().rho0 if its == 0 else s["rho"]
        sub = gauss_newton_subproblem(inst, st, rho)
        g, norms, stt, bad = gpu_mixed(sub, L.LAYOUT_ELEM_MAJOR, steps=8)
        print(f"GN subproblem seed {seed} after {its} iterations: residual norms {norms}", flush=True)
        assert stt == 0, bad
        ext = oracle.tree_lqr_inst(sub, extended=True)
        dbl = oracle.tree_lqr_inst(sub)
        for k in ("x", "u", "lam"):
            floor = relerr(dbl[k], ext[k])
            e = relerr(g[k], ext[k])
            print(f"  {k}: mixed {e:.2e}, oracle double {floor:.2e}", flush=True)
            assert e <= max(TOL, 4.0 * floor), f"{k}: relative error {e:.3e} (oracle double {floor:.3e})"


def test_refine_steps_and_dims_validated():
    inst = S.lqr_on(TREES["fig1b"], 4, 2, seed=1)
    tree, plan = _plan(inst, L.LAYOUT_NODE_MAJOR)
    dev = {k: to_device(getattr(inst, k), L.LAYOUT_NODE_MAJOR) for k in "ABcQRMqr"}
    x0 = to_device(inst.x0, L.LAYOUT_NODE_MAJOR)
    out = [empty((len(inst.parent), n)) for n in (4, 2, 4)]
    for steps in (-1, L.LQR_REFINE_MAX + 1):
        with pytest.raises(L.BmpcError) as e:
            L.bmpc_lqr_solve_mixed(plan, *(dev[k] for k in "ABcQRMqr"), x0, *out, steps)
        assert e.value.status == 1
    L.bmpc_lqr_plan_destroy(plan)
    L.bmpc_tree_destroy(tree)
    big = S.lqr_on(TREES["fig1b"], 12, 4, seed=1)
    tree, plan = _plan(big, L.LAYOUT_NODE_MAJOR)
    dev = {k: to_device(getattr(big, k), L.LAYOUT_NODE_MAJOR) for k in "ABcQRMqr"}
    x0 = to_device(big.x0, L.LAYOUT_NODE_MAJOR)
    out = [empty((len(big.parent), n)) for n in (12, 4, 12)]
    with pytest.raises(L.BmpcError) as e:
        L.bmpc_lqr_solve_mixed(plan, *(dev[k] for k in "ABcQRMqr"), x0, *out, 2)
    assert e.value.status == 9
    L.bmpc_lqr_plan_destroy(plan)
    L.bmpc_tree_destroy(tree)


def test_f32_not_positive_definite_reports_node():
    par = TREES["fig1b"]
    inst = S.lqr_on(par, 3, 1, seed=2, random_cost=True)
    inst.R[5] = -10.0
    inst.B[7] = 0.0
    inst.B[8] = 0.0
    _, st, bad = gpu_f32(inst, L.LAYOUT_NODE_MAJOR)
    assert st == 3 and bad == 5


def test_mixed_on_large_tree_cold_start_subproblem():
    """The 4096-scenario tree's subproblem at the cold start (node weights
    down to 2e-7 against penalties of 100): the mixed solve is held to the
    FP64 bar of the double recursion on the same data."""
    inst = S.large_tree(0)
    pb = oracle.problem_from_instance(inst)
    N = inst.num_nodes
    u = np.zeros((N, 2))
    st = {"x": oracle.rollout(pb, u), "u": u, "ye": np.zeros((N, 5))}
    sub = gauss_newton_subproblem(inst, st, 100.0)
    print(f"GN subproblem large tree N={N}", flush=True)
    g, norms, stt, bad = gpu_mixed(sub, L.LAYOUT_NODE_MAJOR, steps=4)
    print(f"  residual norms {norms}", flush=True)
    assert stt == 0, bad
    ext = oracle.tree_lqr_inst(sub, extended=True)
    dbl = oracle.tree_lqr_inst(sub)
    for k in ("x", "u", "lam"):
        floor = relerr(dbl[k], ext[k])
        e = relerr(g[k], ext[k])
        print(f"  {k}: mixed {e:.2e}, oracle double {floor:.2e}", flush=True)
        assert e <= max(TOL, 4.0 * floor), f"{k}: relative error {e:.3e} (oracle double {floor:.3e})"
