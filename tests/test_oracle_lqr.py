"""Pins of the oracle's serial tree Riccati (CPU only).

Each test checks the oracle against something other than itself: a dense
KKT solve, a scenario-split QP with explicit nonanticipativity rows, the
closed-form scalar Riccati fixed point, and equivalences of tree shapes.
"""
import json
import zlib
import os

import numpy as np
import pytest

import bmpc_synth as S
import oracle
from oracle import cvf
from qp_dense import dense_tree_qp, scenario_qp


def _fig1b(golden_dir):
    with open(os.path.join(golden_dir, "fig1b_tree.json")) as f:
        return json.load(f)


def test_fig1b_topology_facts(golden_dir):
    d = _fig1b(golden_dir)
    par = np.array(d["parent"])
    st = S.stages_of(par)
    nch = S.num_children(par)
    facts = d["facts"]
    assert len(par) == d["num_nodes"]
    assert list(np.nonzero(nch == 0)[0]) == d["leaves"]
    assert par[5] == facts["parent_of_5"]
    assert [i for i in range(len(par)) if par[i] == 5] == facts["children_of_5"]
    a = 5
    while st[a] > 1:
        a = par[a]
    assert a == facts["ancestor_at_stage_1_of_5"]

    def under(n, i):
        while i > n and i >= 0:
            i = par[i]
        return i == n

    assert [i for i in range(len(par)) if st[i] == 5 and under(5, i)] == facts["descendants_at_stage_5_of_5"]
    assert list(np.nonzero(st == 3)[0]) == facts["stage_3_nodes"]


def test_fig2a_tree_paths(golden_dir):
    with open(os.path.join(golden_dir, "fig2a_tree.json")) as f:
        d = json.load(f)
    par = S.tree_parent(d["horizon"], list(range(d["robust_horizon"])), d["n_d"])
    assert int((S.num_children(par) == 0).sum()) == d["num_paths"] == d["n_d"] ** d["robust_horizon"]


TREES = {
    "fig1b": [-1, 0, 1, 1, 2, 3, 4, 5, 5, 6, 7, 8],
    "fig2a": list(S.tree_parent(4, [0, 1], 2)),
    "chain": list(S.tree_parent(7, [], 1)),
    "ternary": list(S.tree_parent(6, [1, 3], 3)),
    "single_bmpc_shape": list(S.tree_parent(20, [4], 3)),
}


@pytest.mark.parametrize("name", sorted(TREES))
@pytest.mark.parametrize("dims", [(4, 2), (3, 1), (6, 3)])
def test_tree_lqr_matches_dense_kkt(name, dims):
    nx, nu = dims
    par = np.array(TREES[name], dtype=np.int32)
    inst = S.lqr_on(par, nx, nu, seed=zlib.crc32(f"{name}{nx}".encode()) % 1000, random_cost=True)
    o = oracle.tree_lqr_inst(inst)
    x, u, lam = dense_tree_qp(par, inst.A, inst.B, inst.c, inst.Q, inst.R, inst.M, inst.q,
                              inst.r, inst.x0)
    scale = max(1.0, np.abs(x).max())
    assert np.abs(o["x"] - x).max() <= 1e-11 * scale
    assert np.abs(o["u"] - u).max() <= 1e-11 * scale
    # costates P x + p equal the KKT multipliers of the dynamics rows
    assert np.abs(o["lam"][1:] - lam[1:]).max() <= 1e-10 * max(1.0, np.abs(lam).max())
    # gains reproduce the inputs
    nch = S.num_children(par)
    for n in np.nonzero(nch > 0)[0]:
        assert np.allclose(o["K"][n] @ o["x"][n] + o["k"][n], o["u"][n], atol=1e-11 * scale)


def test_tree_lqr_config1_matches_dense_on_subtree():
    """The microbenchmark's random data on a smaller tree of the same kind
    (binary branching every 4 stages), dense KKT."""
    par = S.tree_parent(9, [0, 4, 8], 2)
    rng = np.random.Generator(np.random.PCG64(5))
    inst = S.random_lqr(par, 12, 4, rng)
    o = oracle.tree_lqr_inst(inst)
    x, u, lam = dense_tree_qp(par, inst.A, inst.B, inst.c, inst.Q, inst.R, inst.M, inst.q,
                              inst.r, inst.x0)
    assert np.abs(o["x"] - x).max() <= 1e-10 * np.abs(x).max()
    assert np.abs(o["u"] - u).max() <= 1e-10 * np.abs(u).max()


@pytest.mark.parametrize("name", ["fig1b", "fig2a", "ternary"])
def test_shared_controls_equal_scenario_form(name):
    """Nonanticipativity: the tree solution equals the scenario-split QP in
    which every path is a separate copy and the copies of a node are tied by
    explicit equality rows; the copies' inputs agree across branches."""
    par = np.array(TREES[name], dtype=np.int32)
    inst = S.lqr_on(par, 4, 2, seed=11, random_cost=True)
    nl = int((S.num_children(par) == 0).sum())
    w = np.random.Generator(np.random.PCG64(3)).dirichlet(np.ones(nl))
    o = oracle.tree_lqr_inst(inst)
    scen = scenario_qp(par, inst.A, inst.B, inst.c, inst.Q, inst.R, inst.M, inst.q, inst.r,
                       inst.x0, w)
    for (leaf, n), us in scen.items():
        assert np.allclose(us, o["u"][n], atol=1e-9), (leaf, n)


def test_scalar_chain_reaches_algebraic_riccati_closed_form():
    """Time-invariant scalar chain x+ = x + u with cost (q x^2 + r u^2)/2: the
    value P at the root of a long chain tends to the positive root of
    P^2 - q P - q r = 0, i.e. P = (q + sqrt(q^2 + 4 q r)) / 2."""
    qv, rv = 2.0, 0.5
    Nh = 200
    par = S.tree_parent(Nh, [], 1)
    N = len(par)
    A = np.ones((N, 1, 1))
    B = np.ones((N, 1, 1))
    c = np.zeros((N, 1))
    Q = np.full((N, 1, 1), qv)
    R = np.full((N, 1, 1), rv)
    R[-1] = 0
    M = np.zeros((N, 1, 1))
    q = np.zeros((N, 1))
    r = np.zeros((N, 1))
    o = oracle.tree_lqr(par, A, B, c, Q, R, M, q, r, np.array([1.0]))
    P_inf = (qv + np.sqrt(qv * qv + 4 * qv * rv)) / 2
    assert abs(o["P"][0, 0, 0] - P_inf) < 1e-12
    # optimal feedback gain of the stationary problem: K = -P/(r + P)
    assert abs(o["K"][0, 0, 0] + P_inf / (rv + P_inf)) < 1e-12


def test_duplicate_branches_equal_chain_with_summed_costs():
    """A node with two identical child subtrees is the same problem as a chain
    whose post-branch costs are doubled."""
    nx, nu = 3, 2
    chain = S.tree_parent(6, [], 1)
    ci = S.lqr_on(chain, nx, nu, seed=21, random_cost=True)
    tree = S.tree_parent(6, [2], 2)  # nodes 0..2 shared, then two copies of stages 3..6
    N = len(tree)
    st = S.stages_of(tree)
    T = {k: np.zeros((N,) + getattr(ci, k).shape[1:]) for k in "ABcQRMqr"}
    for i in range(N):
        src = int(st[i])  # chain node index == stage
        f = 1.0 if st[i] <= 2 else 0.5
        for k in "ABc":
            T[k][i] = getattr(ci, k)[src]
        for k in "QRMqr":
            T[k][i] = f * getattr(ci, k)[src]
    # the two halves carry half the cost each, so the tree equals the chain
    o_t = oracle.tree_lqr(tree, T["A"], T["B"], T["c"], T["Q"], T["R"], T["M"], T["q"], T["r"],
                          ci.x0)
    o_c = oracle.tree_lqr_inst(ci)
    for i in range(N):
        assert np.allclose(o_t["x"][i], o_c["x"][st[i]], atol=1e-11)
        assert np.allclose(o_t["u"][i], o_c["u"][st[i]], atol=1e-11)


def test_not_positive_definite_is_reported_with_node():
    par = np.array(TREES["fig1b"], dtype=np.int32)
    inst = S.lqr_on(par, 3, 2, seed=2, random_cost=True)
    inst.R[5] = -10.0 * np.eye(2)
    inst.B[7] = 0.0
    inst.B[8] = 0.0
    with pytest.raises(oracle.OracleError) as e:
        oracle.tree_lqr_inst(inst)
    assert e.value.status == 3 and e.value.node == 5


def test_bad_topology_rejected():
    par = np.array([-1, 0, 2], dtype=np.int32)
    inst = S.lqr_on(np.array([-1, 0, 1], dtype=np.int32), 2, 1, seed=1)
    with pytest.raises(oracle.OracleError) as e:
        oracle.tree_lqr(par, inst.A, inst.B, inst.c, inst.Q, inst.R, inst.M, inst.q, inst.r,
                        inst.x0)
    assert e.value.status == 2


# ----------------------------------------------------------------------------
# conditional value functions (parallel-scan algebra)
# ----------------------------------------------------------------------------

def _chain_elements(inst):
    N = len(inst.parent)
    els = []
    for k in range(N - 1):
        j = k + 1
        els.append(cvf.element(inst.A[j], inst.B[j], inst.c[j], inst.Q[k], inst.R[k], inst.M[k],
                               inst.q[k], inst.r[k]))
    els.append(cvf.value_element(inst.Q[N - 1], inst.q[N - 1]))
    return els


def test_cvf_scan_reproduces_serial_riccati():
    chain = S.tree_parent(9, [], 1)
    inst = S.lqr_on(chain, 3, 2, seed=4, random_cost=True)
    o = oracle.tree_lqr_inst(inst)
    suf = cvf.suffix_scan(_chain_elements(inst))
    for k, e in enumerate(suf):
        assert np.allclose(e[3], o["P"][k], rtol=1e-12, atol=1e-12)
        assert np.allclose(e[4], o["p"][k], rtol=1e-12, atol=1e-12)
        assert np.abs(e[0]).max() == 0.0  # terminal element absorbs the end state


def test_cvf_combine_is_associative_and_reduces_to_affine_composition():
    chain = S.tree_parent(8, [], 1)
    inst = S.lqr_on(chain, 4, 2, seed=8, random_cost=True)
    els = _chain_elements(inst)[:-1]
    seq = cvf.suffix_scan(els)[0]
    bal = cvf.balanced_fold(els)
    for a, b in zip(seq, bal):
        assert np.allclose(a, b, rtol=1e-11, atol=1e-11)
    # C = 0 and P = 0: plain composition of affine maps
    rng = np.random.default_rng(0)
    e1 = (rng.standard_normal((3, 3)), rng.standard_normal(3), np.zeros((3, 3)), np.zeros((3, 3)), np.zeros(3))
    e2 = (rng.standard_normal((3, 3)), rng.standard_normal(3), np.zeros((3, 3)), np.zeros((3, 3)), np.zeros(3))
    A, c, C, P, p = cvf.combine(e1, e2)
    assert np.allclose(A, e2[0] @ e1[0])
    assert np.allclose(c, e2[0] @ e1[1] + e2[1])


def test_cvf_inverse_transpose_identity():
    rng = np.random.default_rng(1)
    G = rng.standard_normal((4, 4))
    C = G @ G.T
    G = rng.standard_normal((4, 4))
    P = G @ G.T
    lhs = np.linalg.inv(np.eye(4) + C @ P)
    rhs = np.linalg.inv(np.eye(4) + P @ C).T
    assert np.allclose(lhs, rhs, atol=1e-12)


def test_printed_combination_signs_are_not_the_minimisation():
    """The rule with the printed signs does not reproduce the serial Riccati
    under a balanced fold (the reading implemented in ``cvf.combine`` does)."""
    chain = S.tree_parent(6, [], 1)
    inst = S.lqr_on(chain, 3, 2, seed=4, random_cost=True)
    els = _chain_elements(inst)
    o = oracle.tree_lqr_inst(inst)
    good = cvf.balanced_fold(els)
    bad = cvf.balanced_fold(els, cvf.combine_as_printed)
    assert np.allclose(good[3], o["P"][0], rtol=1e-11, atol=1e-11)
    assert np.allclose(good[4], o["p"][0], rtol=1e-11, atol=1e-11)
    # P is even in the sign of A, so the slip shows in the linear term p
    assert not np.allclose(bad[4], o["p"][0], rtol=1e-3, atol=1e-3)


def _tree_qp_kkt_residual(inst, sol):
    """Infinity norm of the KKT conditions of the tree QP at (x, u, lam),
    evaluated in long double: stationarity in u_n and x_n (n != 0) with the
    convention L = cost + sum_j lam_j^T (A_j x_p + B_j u_p + c_j - x_j), and
    the dynamics."""
    ld = np.longdouble
    par = inst.parent
    N = len(par)
    A, B, c, Q, R, M, q, r = (np.asarray(getattr(inst, k), dtype=ld) for k in "ABcQRMqr")
    x, u, lam = (np.asarray(sol[k], dtype=ld) for k in ("x", "u", "lam"))
    nch = S.num_children(par)
    res = ld(0)
    for n in range(N):
        kids = np.nonzero(par == n)[0]
        if nch[n] > 0:
            gu = R[n] @ u[n] + M[n] @ x[n] + r[n] + sum(B[j].T @ lam[j] for j in kids)
            res = max(res, np.abs(gu).max())
        if n > 0:
            gx = Q[n] @ x[n] + q[n] - lam[n] + sum((A[j].T @ lam[j] for j in kids), np.zeros(len(q[n]), ld))
            if nch[n] > 0:
                gx = gx + M[n].T @ u[n]
            res = max(res, np.abs(gx).max())
            d = A[n] @ x[par[n]] + B[n] @ u[par[n]] + c[n] - x[n]
            res = max(res, np.abs(d).max())
    return float(res)


def test_extended_precision_recursion_solves_the_same_problem_more_accurately():
    """The long-double recursion agrees with the double one to rounding on a
    well-conditioned tree; on a badly conditioned one (input weights 1e-7,
    A = I + 0.3 N(0,1)) its KKT residual, evaluated in long double, is at
    least 10 times smaller than the double recursion's (its outputs are
    rounded to double, which bounds how small it can get)."""
    par = S.tree_parent(12, [2, 6], 2)
    inst = S.lqr_on(par, 4, 2, seed=8, random_cost=True)
    d = oracle.tree_lqr_inst(inst)
    e = oracle.tree_lqr_inst(inst, extended=True)
    for k in ("x", "u", "lam", "P", "p"):
        assert np.abs(d[k] - e[k]).max() <= 1e-12 * max(1.0, np.abs(e[k]).max()), k
    bad = S.lqr_on(S.tree_parent(30, [2, 6, 14], 2), 4, 2, seed=9, a_scale=0.3, r_scale=1e-7)
    d = oracle.tree_lqr_inst(bad)
    e = oracle.tree_lqr_inst(bad, extended=True)
    rd, re = _tree_qp_kkt_residual(bad, d), _tree_qp_kkt_residual(bad, e)
    print(f"KKT residual: double {rd:.3e}, long double {re:.3e}")
    assert re * 10 <= rd


def _kkt_rows(inst, sol):
    """KKT rows of the tree QP at (x, u, lam), every node including the root:
    g_u (control nodes; zero at leaves), g_x (with -lam_n; at the root lam_0 is
    the multiplier of x_0 = x0) and the defects d (root: x0 - x_0)."""
    par = inst.parent
    N = len(par)
    x, u, lam = sol["x"], sol["u"], sol["lam"]
    nch = S.num_children(par)
    gx, gu, d = np.zeros_like(x), np.zeros_like(u), np.zeros_like(x)
    for n in range(N):
        kids = np.nonzero(par == n)[0]
        gx[n] = inst.Q[n] @ x[n] + inst.q[n] - lam[n] + sum((inst.A[j].T @ lam[j] for j in kids), 0.0)
        if nch[n] > 0:
            gx[n] += inst.M[n].T @ u[n]
            gu[n] = inst.R[n] @ u[n] + inst.M[n] @ x[n] + inst.r[n] + sum(inst.B[j].T @ lam[j] for j in kids)
        d[n] = inst.x0 - x[n] if par[n] < 0 else inst.A[n] @ x[par[n]] + inst.B[n] @ u[par[n]] + inst.c[n] - x[n]
    return gx, gu, d


def test_single_precision_recursion_is_float_accurate():
    """The float recursion (inputs rounded to float) agrees with the
    long-double one to float accuracy on well-conditioned trees, not better:
    relative errors between 1e-9 and 1e-5, and the KKT rows of its solution
    are of the same order."""
    for dims, seed in (((3, 1), 1), ((4, 2), 2), ((6, 3), 3)):
        inst = S.lqr_on(S.tree_parent(9, [1, 3, 6], 3), *dims, seed=seed, random_cost=True)
        e = oracle.tree_lqr_inst(inst, extended=True)
        f = oracle.tree_lqr_inst(inst, single=True)
        for k in ("x", "u", "lam", "K", "P"):
            err = np.abs(f[k] - e[k]).max() / np.abs(e[k]).max()
            assert 1e-9 < err < 1e-5, (dims, k, err)
        rows = _kkt_rows(inst, f)
        scale = max(np.abs(inst.q).max(), np.abs(inst.c).max(), 1.0)
        assert max(np.abs(r).max() for r in rows) < 1e-4 * scale
        assert max(np.abs(r).max() for r in _kkt_rows(inst, e)) < 1e-12 * scale


def test_iterative_refinement_with_float_solves_reaches_the_double_solution():
    """Refinement as the mixed-precision solver does it, carried out with the
    oracle's float recursion: each step solves the tree QP whose linear terms
    (q, r, c, x0) are the KKT rows of the current iterate and adds the
    solution.  The error contracts by about cond * 2^-24 per step and three
    steps reach the double-precision solution to 1e-12; with the signs of
    any one linear term flipped the iteration does not converge."""
    inst = S.lqr_on(S.tree_parent(12, [2, 6], 2), 4, 2, seed=4, random_cost=True)
    ref = oracle.tree_lqr_inst(inst, extended=True)

    def refine(flip=None, steps=3):
        z = {k: np.zeros_like(ref[k]) for k in ("x", "u", "lam")}
        errs = []
        for _ in range(steps + 1):
            gx, gu, d = _kkt_rows(inst, z)
            lin = {"q": gx, "r": gu, "c": d.copy(), "x0": d[0].copy()}
            if flip:
                lin[flip] = -lin[flip]
            dz = oracle.tree_lqr(inst.parent, inst.A, inst.B, lin["c"], inst.Q, inst.R, inst.M, lin["q"],
                                 lin["r"], lin["x0"], single=True)
            for k in z:
                z[k] = z[k] + dz[k]
            errs.append(max(np.abs(z[k] - ref[k]).max() / np.abs(ref[k]).max() for k in z))
        return errs

    errs = refine()
    print("refinement errors", errs)
    assert errs[0] > 1e-9 and errs[-1] < 1e-12
    assert all(b < 1e-3 * a or b < 1e-13 for a, b in zip(errs, errs[1:]))
    for flip in ("q", "r", "c"):
        assert refine(flip)[-1] > 1e-3, flip


# ----------------------------------------------------------------------------
# chain of masses and springs (per-scenario dynamics)
# ----------------------------------------------------------------------------

def test_mass_spring_model_conserves_energy_and_branches_take_their_constant():
    """The discretised chain (no damping, zero-order hold) keeps the
    energy 1/2 v^T v - k/2 p^T L p of a free motion (u = 0) to rounding, and
    each edge of the tree carries the matrices of its branch's spring
    constant: siblings differ, a chain below a branch repeats its edge."""
    M, k = 4, 0.8
    A, B = S.mass_spring_matrices(M, k)
    Lm = -2.0 * np.eye(M) + np.eye(M, k=1) + np.eye(M, k=-1)
    W = np.zeros((2 * M, 2 * M))
    W[:M, :M] = -k * Lm
    W[M:, M:] = np.eye(M)
    x = np.random.default_rng(0).standard_normal(2 * M)
    for _ in range(20):
        xn = A @ x
        assert abs(xn @ W @ xn - x @ W @ x) <= 1e-10 * (x @ W @ x)
        x = xn
    # an actuator pushes its two masses apart: opposite velocities, equal up
    # to what the springs transmit within the step; no net momentum at first
    # order in dt
    v = (B @ np.eye(M - 1)[0])[M:]
    assert v[0] < 0 < v[1] and abs(v[0] + v[1]) < 1e-3 * v[1] and np.all(np.abs(v[2:]) < 0.05 * v[1])
    inst = S.mass_spring_tree(M=3, robust_horizon=2, n_d=2, horizon=5)
    par = inst.parent
    nch = S.num_children(par)
    kids0 = np.nonzero(par == 0)[0]
    assert len(kids0) == 2 and not np.allclose(inst.A[kids0[0]], inst.A[kids0[1]])
    for j in range(1, len(par)):
        p = par[j]
        if p > 0 and nch[p] == 1:
            np.testing.assert_array_equal(inst.A[j], inst.A[p])


@pytest.mark.parametrize("nr", [1, 2])
def test_mass_spring_tree_lqr_matches_dense_kkt(nr):
    """The oracle's tree Riccati on small mass-spring trees (per-edge
    dynamics, random linear terms and defects) against a dense solve of the
    equality-constrained QP."""
    inst = S.mass_spring_tree(M=3, robust_horizon=nr, n_d=2, horizon=6, random_terms=True)
    o = oracle.tree_lqr_inst(inst)
    x, u = _dense(inst)
    assert np.abs(o["x"] - x).max() <= 1e-10 * max(1.0, np.abs(x).max())
    assert np.abs(o["u"] - u).max() <= 1e-10 * max(1.0, np.abs(u).max())


def _dense(inst):
    out = dense_tree_qp(inst.parent, inst.A, inst.B, inst.c, inst.Q, inst.R, inst.M, inst.q, inst.r, inst.x0)
    return out[0], out[1]


def test_mass_spring_identical_constants_make_every_scenario_the_chain():
    """With all n_d spring constants equal, the branches of the tree are
    copies: the tree LQR's inputs along every path equal those of the
    single chain whose costs after the branching carry the number of
    copies as weight (duplicate branches = chain with summed weights)."""
    inst = S.mass_spring_tree(M=3, robust_horizon=2, n_d=2, horizon=6)
    A, B = S.mass_spring_matrices(3, 1.0)
    N = len(inst.parent)
    nch = S.num_children(inst.parent)
    for j in range(1, N):
        inst.A[j], inst.B[j] = A, B
    o = oracle.tree_lqr_inst(inst)
    # the chain: stage t carries the number of tree nodes at stage t
    stages = S.stages_of(inst.parent)
    H = stages.max()
    chain = S.tree_parent(H, [], 1)
    cnt = np.array([np.sum(stages == t) for t in range(H + 1)], dtype=float)
    ci = S.LqrInstance(parent=chain, A=np.array([A] * (H + 1)), B=np.array([B] * (H + 1)),
                       c=np.zeros((H + 1, 6)), Q=np.array([np.eye(6) * cnt[t] for t in range(H + 1)]),
                       R=np.array([np.eye(2) * cnt[t] for t in range(H + 1)]), M=np.zeros((H + 1, 2, 6)),
                       q=np.zeros((H + 1, 6)), r=np.zeros((H + 1, 2)), x0=inst.x0)
    ci.R[H] = 0.0
    oc = oracle.tree_lqr_inst(ci)
    for n in range(N):
        np.testing.assert_allclose(o["x"][n], oc["x"][stages[n]], rtol=1e-10, atol=1e-12)
        if nch[n] > 0:
            np.testing.assert_allclose(o["u"][n], oc["u"][stages[n]], rtol=1e-10, atol=1e-12)
