"""Pins of the oracle's branch-MPC pieces and its AL-iLQR loop (CPU only).

Closed-form bicycle motions, finite-difference derivatives, node weights by
hand, a linear-quadratic problem whose AL-iLQR must take exactly one Newton
step, and a box-constrained LQ tree checked against brute-force enumeration
of active sets.
"""
import itertools

import numpy as np
import pytest

import bmpc_synth as S
import oracle

BIKE = oracle.bicycle_model(S.single_bmpc(0))


def test_rk4_straight_line_and_constant_acceleration_exact():
    # delta = 0: psi constant, v linear in t -> positions are polynomials of
    # degree 2 in t, which RK4 integrates exactly
    x = np.array([1.0, -2.0, 0.3, 7.0])
    a = 1.7
    xn, _, _ = oracle.rk4(BIKE, x, [a, 0.0])
    h = BIKE.dt
    dist = x[3] * h + 0.5 * a * h * h
    assert np.allclose(xn, [x[0] + dist * np.cos(x[2]), x[1] + dist * np.sin(x[2]), x[2], x[3] + a * h],
                       atol=1e-14)


def test_rk4_constant_steering_circle_within_rk4_error():
    # a = 0, delta const: exact motion is a circular arc with yaw rate w
    x = np.array([0.0, 0.0, 0.2, 9.0])
    d = 0.3
    xn, _, _ = oracle.rk4(BIKE, x, [0.0, d])
    h, L, v = BIKE.dt, BIKE.wheelbase, x[3]
    w = v * np.tan(d) / L
    psi1 = x[2] + w * h
    exact = [x[0] + v / w * (np.sin(psi1) - np.sin(x[2])),
             x[1] - v / w * (np.cos(psi1) - np.cos(x[2])), psi1, v]
    # local RK4 error ~ v (w h)^5 / 120
    assert np.abs(xn - exact).max() < v * (w * h) ** 5
    assert abs(xn[2] - psi1) < 1e-14 and xn[3] == v


@pytest.mark.parametrize("seed", range(5))
def test_rk4_jacobians_match_finite_differences(seed):
    rng = np.random.default_rng(seed)
    x = np.array([rng.uniform(-5, 5), rng.uniform(-5, 5), rng.uniform(-3, 3), rng.uniform(1, 12)])
    u = np.array([rng.uniform(-3, 3), rng.uniform(-0.5, 0.5)])
    _, A, B = oracle.rk4(BIKE, x, u)
    z = np.concatenate([x, u])

    def f(zz):
        return oracle.rk4(BIKE, zz[:4], zz[4:])[0]

    J = np.zeros((4, 6))
    for i in range(6):
        # Richardson-extrapolated central difference, error O(h^4)
        def cd(h):
            e = np.zeros(6)
            e[i] = h
            return (f(z + e) - f(z - e)) / (2 * h)
        h = 1e-3
        J[:, i] = (4 * cd(h / 2) - cd(h)) / 3
    assert np.allclose(A, J[:, :4], atol=1e-9)
    assert np.allclose(B, J[:, 4:], atol=1e-9)


def test_node_weights_and_refs_by_hand():
    # root -> {1, 2}; 1 -> 3 (leaf); 2 -> {4, 5} leaves
    par = np.array([-1, 0, 0, 1, 2, 2], dtype=np.int32)
    p = np.array([0.5, 0.2, 0.3])          # leaves 3, 4, 5
    y = np.array([1.0, -2.0, 4.0])
    w = oracle.node_weights(par, p)
    assert np.allclose(w, [1.0, 0.5, 0.5, 0.5, 0.2, 0.3])
    ref = oracle.node_refs(par, p, y, 0.1, 10.0)
    assert np.allclose(ref[:, 0], [0, 1, 1, 2, 2, 2])
    assert np.allclose(ref[:, 1], [0.5 * 1 + 0.2 * -2 + 0.3 * 4, 1.0, (0.2 * -2 + 0.3 * 4) / 0.5, 1, -2, 4])
    assert np.allclose(ref[:, 3], 10.0) and np.allclose(ref[:, 2], 0.0)


def _small_problem(seed=0, rho=7.0):
    inst = S.small_bicycle(8, [2], 2, seed)
    pb = oracle.problem_from_instance(inst)
    return inst, pb


@pytest.mark.parametrize("n", [0, 3, 9, 14])
def test_node_terms_gradient_and_gauss_newton_hessian(n):
    inst, pb = _small_problem(1)
    rng = np.random.default_rng(n)
    # place the node near its obstacle (if any) so the obstacle term is active
    x = np.array([0.0, 0.0, 0.1, 8.0])
    if inst.node_obstacle[n] >= 0:
        x[:2] = inst.obstacles[inst.node_obstacle[n]] + rng.uniform(-0.6, 0.6, 2)
    u = np.array([3.4, -0.1])            # upper acceleration bound violated
    ye = np.array([0.5, 0.0, 0.2, 0.1, 0.3])
    rho = 7.0
    v, g, gx, gu, Hxx, Huu = oracle.node_terms(pb, n, x, u, ye, rho)

    def val(xx, uu):
        return oracle.node_terms(pb, n, xx, uu, ye, rho)[0]

    h = 1e-6
    fx = np.array([(val(x + h * e, u) - val(x - h * e, u)) / (2 * h) for e in np.eye(4)])
    fu = np.array([(val(x, u + h * e) - val(x, u - h * e)) / (2 * h) for e in np.eye(2)])
    assert np.allclose(gx, fx, atol=1e-6)
    assert np.allclose(gu, fu, atol=1e-6)
    # Gauss-Newton Hessian: weighted cost Hessian + rho * J^T D J of the
    # active constraints, with J from finite differences of g
    wq = pb.weight[n] * np.array(BIKE.Qd)
    wr = pb.weight[n] * np.array(BIKE.Rd)
    gfun_x = lambda xx: oracle.node_terms(pb, n, xx, u, ye, rho)[1]
    gfun_u = lambda uu: oracle.node_terms(pb, n, x, uu, ye, rho)[1]
    Jx = np.array([(gfun_x(x + h * e) - gfun_x(x - h * e)) / (2 * h) for e in np.eye(4)]).T
    Ju = np.array([(gfun_u(u + h * e) - gfun_u(u - h * e)) / (2 * h) for e in np.eye(2)]).T
    act = np.isfinite(g) & (g + ye / rho > 0)
    Jx = np.where(np.isfinite(Jx), Jx, 0.0)
    Ju = np.where(np.isfinite(Ju), Ju, 0.0)
    Hx_ref = np.diag(wq) + rho * Jx[act].T @ Jx[act]
    is_leaf = S.num_children(inst.parent)[n] == 0
    Hu_ref = (np.zeros((2, 2)) if is_leaf else np.diag(wr)) + rho * Ju[act].T @ Ju[act]
    assert np.allclose(Hxx, Hx_ref, atol=1e-6)
    assert np.allclose(Huu, Hu_ref, atol=1e-6)


def test_kkt_residual_equals_finite_difference_gradient_of_lagrangian():
    inst, pb = _small_problem(2)
    rng = np.random.default_rng(3)
    N = pb.N
    u = rng.uniform(-1, 1, (N, 2)) * [2.0, 0.3]
    x = oracle.rollout(pb, u) + rng.normal(0, 0.05, (N, 4))
    x[0] = pb.x0
    lam = rng.normal(0, 0.1, (N, 4))
    ye = np.abs(rng.normal(0, 0.2, (N, 5)))
    rho = 3.0
    par = inst.parent

    def lagr(xx, uu):
        v = oracle.augmented_lagrangian(pb, xx, uu, ye, rho)
        for j in range(1, N):
            f = oracle.rk4(BIKE, xx[par[j]], uu[par[j]])[0]
            v += lam[j] @ (f - xx[j])
        return v

    h = 1e-6
    gmax = 0.0
    nch = S.num_children(par)
    for n in range(N):
        for a in range(4):
            if n == 0:
                continue
            e = np.zeros_like(x)
            e[n, a] = h
            gmax = max(gmax, abs(lagr(x + e, u) - lagr(x - e, u)) / (2 * h))
        if nch[n] > 0:
            for a in range(2):
                e = np.zeros_like(u)
                e[n, a] = h
                gmax = max(gmax, abs(lagr(x, u + e) - lagr(x, u - e)) / (2 * h))
    dmax = max(np.abs(oracle.rk4(BIKE, x[par[j]], u[par[j]])[0] - x[j]).max() for j in range(1, N))
    r = oracle.kkt(pb, x, u, lam, ye, rho)
    assert r == pytest.approx(max(gmax, dmax), rel=1e-6, abs=1e-7)


def test_adjoint_multipliers_zero_the_state_gradient():
    inst, pb = _small_problem(4)
    N = pb.N
    u = np.tile([0.5, 0.05], (N, 1))
    x = oracle.rollout(pb, u)
    ye = np.zeros((N, 5))
    lam = oracle.adjoint(pb, x, u, ye, 10.0)
    # with d = 0 and grad_x = 0 only the input gradient is left
    r = oracle.kkt(pb, x, u, lam, ye, 10.0)
    lam_bad = lam.copy()
    lam_bad[5] += 0.1
    assert oracle.kkt(pb, x, u, lam_bad, ye, 10.0) >= 0.1 - 1e-12
    # input gradient of the Lagrangian by finite differences of the
    # single-shooting cost (x driven by u), which it must equal here
    h = 1e-6

    def cost(uu):
        return oracle.augmented_lagrangian(pb, oracle.rollout(pb, uu), uu, ye, 10.0)

    nch = S.num_children(inst.parent)
    gu = 0.0
    for n in np.nonzero(nch > 0)[0]:
        for a in range(2):
            e = np.zeros_like(u)
            e[n, a] = h
            gu = max(gu, abs(cost(u + e) - cost(u - e)) / (2 * h))
    assert r == pytest.approx(gu, rel=1e-5)


# ----------------------------------------------------------------------------
# AL-iLQR on linear-quadratic problems
# ----------------------------------------------------------------------------

def _lq_problem(parent, bounds=(1e3, 1e3), seed=0):
    rng = np.random.default_rng(seed)
    Al = np.eye(4) + 0.1 * rng.standard_normal((4, 4))
    Bl = 0.3 * rng.standard_normal((4, 2))
    N = len(parent)
    nl = int((S.num_children(parent) == 0).sum())
    probs = rng.dirichlet(np.ones(nl))
    w = oracle.node_weights(parent, probs)
    ref = rng.standard_normal((N, 4))
    model = oracle.linear_model(Al, Bl, (1.0, 2.0, 0.5, 1.5), (0.3, 0.7), a_max=bounds[0],
                                steer_max=bounds[1])
    x0 = rng.standard_normal(4)
    pb = oracle.BmpcProblem(parent, w, ref, np.zeros((N, 2)), np.zeros(N, np.int32), x0, model)
    return pb, Al, Bl, w, ref, x0


def _lq_dense(parent, Al, Bl, w, ref, x0, qd, rd):
    N = len(parent)
    nch = S.num_children(parent)
    A = np.zeros((N, 4, 4))
    B = np.zeros((N, 4, 2))
    A[1:] = Al
    B[1:] = Bl
    Q = w[:, None, None] * np.diag(qd)[None]
    R = w[:, None, None] * np.diag(rd)[None]
    R[nch == 0] = 0
    q = -np.einsum("nij,nj->ni", Q, ref)
    from qp_dense import dense_tree_qp
    return dense_tree_qp(parent, A, B, np.zeros((N, 4)), Q, R, np.zeros((N, 2, 4)), q,
                         np.zeros((N, 2)), x0)


def test_lq_problem_converges_in_one_newton_step():
    par = S.tree_parent(6, [1, 3], 2)
    pb, Al, Bl, w, ref, x0 = _lq_problem(par)
    st, stats, hist = oracle.solve(pb)
    assert stats["status"] == 0
    assert stats["inner_it"] == 1
    assert hist[0, 2] == 1.0             # alpha = 1 accepted
    assert stats["r_kkt"] < 1e-10
    x, u, _ = _lq_dense(par, Al, Bl, w, ref, x0, (1.0, 2.0, 0.5, 1.5), (0.3, 0.7))
    assert np.allclose(st["x"], x, atol=1e-10) and np.allclose(st["u"], u, atol=1e-10)


def _brute_force_box_qp(par, Al, Bl, w, ref, x0, qd, rd, umax):
    """Minimise the LQ tree cost over inputs with |u| <= umax by enumerating
    every active set (free / lower / upper per input coordinate)."""
    N = len(par)
    nch = S.num_children(par)
    ctrl = list(np.nonzero(nch > 0)[0])
    nv = 2 * len(ctrl)

    def states(uv):
        u = np.zeros((N, 2))
        for k, n in enumerate(ctrl):
            u[n] = uv[2 * k: 2 * k + 2]
        x = np.zeros((N, 4))
        x[0] = x0
        for j in range(1, N):
            x[j] = Al @ x[par[j]] + Bl @ u[par[j]]
        return x, u

    def cost(uv):
        x, u = states(uv)
        e = x - ref
        return 0.5 * np.sum(w[:, None] * e * e * np.array(qd)) + \
            0.5 * np.sum((w * (nch > 0))[:, None] * u * u * np.array(rd))

    # quadratic form of the cost in u by polarisation
    c0 = cost(np.zeros(nv))
    g = np.zeros(nv)
    H = np.zeros((nv, nv))
    E = np.eye(nv)
    for i in range(nv):
        g[i] = (cost(E[i]) - cost(-E[i])) / 2
        H[i, i] = cost(E[i]) + cost(-E[i]) - 2 * c0
    for i in range(nv):
        for j in range(i + 1, nv):
            H[i, j] = H[j, i] = cost(E[i] + E[j]) - cost(E[i]) - cost(E[j]) + c0
    bnd = np.array([umax[0], umax[1]] * len(ctrl))
    best, best_u = np.inf, None
    for pat in itertools.product((0, -1, 1), repeat=nv):
        pat = np.array(pat)
        fixed = pat != 0
        uv = np.where(fixed, pat * bnd, 0.0)
        free = ~fixed
        if free.any():
            rhs = -(g[free] + H[np.ix_(free, fixed)] @ uv[fixed])
            uv[free] = np.linalg.solve(H[np.ix_(free, free)], rhs)
        if np.all(np.abs(uv) <= bnd + 1e-12):
            cv = c0 + g @ uv + 0.5 * uv @ H @ uv
            if cv < best:
                best, best_u = cv, uv
    return states(best_u)


def test_box_constrained_lq_matches_brute_force_active_sets():
    par = S.tree_parent(3, [1], 2)   # 4 control nodes -> 8 inputs, 3^8 active sets
    umax = (0.4, 0.25)
    pb, Al, Bl, w, ref, x0 = _lq_problem(par, bounds=umax, seed=5)
    ref *= 4.0
    pb = oracle.BmpcProblem(par, w, ref, np.zeros((len(par), 2)), np.zeros(len(par), np.int32), x0,
                            pb.model)
    st, stats, hist = oracle.solve(pb)
    assert stats["status"] == 0
    xb, ub = _brute_force_box_qp(par, Al, Bl, w, ref, x0, (1.0, 2.0, 0.5, 1.5), (0.3, 0.7), umax)
    assert np.any(np.isclose(np.abs(ub[S.num_children(par) > 0]), umax))  # bounds are active
    assert np.allclose(st["u"], ub, atol=1e-5)
    assert np.allclose(st["x"], xb, atol=1e-5)


# ----------------------------------------------------------------------------
# AL-iLQR on the bicycle workload
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(40))
def test_single_bmpc_every_seed_converges(seed):
    """Every seed of the single-tree workload reaches max(r_kkt, violation) <
    1e-6 with status OK, at a point that satisfies the KKT conditions of the
    original problem: primal feasibility, dual sign, complementarity, and
    states that are the rollout of the inputs."""
    pb = oracle.problem_from_instance(S.single_bmpc(seed))
    st, stats, hist = oracle.solve(pb)
    assert stats["status"] == 0, stats
    assert stats["r_kkt"] < 1e-6 and stats["viol"] < 1e-6
    # primal feasibility, dual sign and complementarity of the returned
    # multipliers (the residual itself is taken before their update)
    for n in range(pb.N):
        g = oracle.node_terms(pb, n, st["x"][n], st["u"][n], st["ye"][n], stats["rho"])[1]
        act = np.isfinite(g)
        assert np.all(g[act] <= 1e-6)
        assert np.all(st["ye"][n] >= 0)
        assert np.all(np.abs(st["ye"][n][act] * g[act]) <= 1e-5)
    # shared trunk: one input per node, so branches agree by construction;
    # the rollout of the returned inputs reproduces the states
    xr = oracle.rollout(pb, st["u"])
    assert np.abs(xr - st["x"]).max() < 1e-4


# ----------------------------------------------------------------------------
# shifted warm start
# ----------------------------------------------------------------------------

def test_shift_on_a_chain_is_the_one_stage_shift():
    inst = S.small_bicycle(6, [], 1, seed=3)
    pb = oracle.problem_from_instance(inst)
    N = pb.N
    rng = np.random.default_rng(0)
    st = {"u": rng.normal(0, 0.3, (N, 2)), "lam": rng.normal(0, 1, (N, 4)), "ye": np.abs(rng.normal(0, 1, (N, 5)))}
    st["u"][-1] = 0
    st["x"] = oracle.rollout(pb, st["u"])
    new, s = oracle.shift(pb, st)
    x0n = oracle.rk4(pb.model, inst.x0, st["u"][0])[0]
    assert np.allclose(new.x0, x0n)
    # node t takes the values of node t+1; the last control node repeats its input
    assert np.allclose(s["x"][1:N - 1], st["x"][2:N])
    assert np.allclose(s["x"][0], x0n)
    assert np.allclose(s["u"][:N - 2], st["u"][1:N - 1])
    assert np.allclose(s["u"][N - 2], st["u"][N - 2])
    assert np.allclose(s["lam"][:N - 1], st["lam"][1:])
    assert np.allclose(s["ye"][:N - 1], st["ye"][1:])
    # references move one stage ahead
    assert np.allclose(new.ref[:, 0], pb.ref[:, 0] + inst.ref_speed * inst.dt)
    # leaf state rolled out from the shifted parent
    assert np.allclose(s["x"][N - 1], oracle.rk4(pb.model, s["x"][N - 2], s["u"][N - 2])[0])


def test_shift_averages_children_with_probability_weights():
    # root -> {1, 2}; 1 -> 3 -> 5 (leaf), 2 -> 4 -> 6 (leaf)
    par = np.array([-1, 0, 0, 1, 2, 3, 4], dtype=np.int32)
    w = np.array([1.0, 0.25, 0.75, 0.25, 0.75, 0.25, 0.75])
    N = len(par)
    rng = np.random.default_rng(1)
    ref = rng.normal(0, 1, (N, 4))
    model = oracle.bicycle_model(S.single_bmpc(0))
    pb = oracle.BmpcProblem(par, w, ref, np.zeros((N, 2)), np.zeros(N, np.int32), [0, 0, 0, 8.0], model)
    st = {"x": rng.normal(0, 1, (N, 4)), "u": rng.normal(0, 0.2, (N, 2)), "lam": rng.normal(0, 1, (N, 4)),
          "ye": rng.normal(0, 1, (N, 5))}
    new, s = oracle.shift(pb, st)
    assert np.allclose(s["lam"][0], 0.25 * st["lam"][1] + 0.75 * st["lam"][2])
    assert np.allclose(s["u"][0], 0.25 * st["u"][1] + 0.75 * st["u"][2])
    assert np.allclose(new.ref[0], 0.25 * ref[1] + 0.75 * ref[2])
    assert np.allclose(s["x"][1], st["x"][3]) and np.allclose(s["u"][1], st["u"][3])
    assert np.allclose(s["u"][3], st["u"][3])  # children are leaves: input repeated
    assert np.allclose(new.ref[5], 2 * ref[5] - ref[3])


def test_shifted_warm_start_needs_fewer_iterations_than_cold():
    fewer = 0
    for seed in range(6):
        pb = oracle.problem_from_instance(S.single_bmpc(seed))
        st, stats, _ = oracle.solve(pb)
        if stats["status"] != 0:
            continue
        new, ws = oracle.shift(pb, st)
        _, s_warm, _ = oracle.solve(new, warm=ws)
        _, s_cold, _ = oracle.solve(new)
        if s_warm["status"] == 0 and (s_cold["status"] != 0 or s_warm["inner_it"] < s_cold["inner_it"]):
            fewer += 1
    assert fewer >= 4


def test_rollout_start_and_guard():
    """Warm start from inputs alone (states by the exact rollout) and the
    guard that falls back to the cold start when the given start is worse
    by max(KKT residual, violation)."""
    inst = S.single_bmpc(2)
    pb = oracle.problem_from_instance(inst)
    cold, cs, _ = oracle.solve(pb)
    assert cs["status"] == 0 and cs["start"] == 0
    # inputs of the solution: the rollout reproduces its states (the
    # solution's defects are below the tolerance), so the solve is short
    ws, wst, _ = oracle.solve(pb, warm={"u": cold["u"], "ye": cold["ye"]})
    assert wst["status"] == 0 and wst["start"] == 1
    assert wst["inner_it"] < cs["inner_it"] / 2
    assert np.abs(ws["x"] - cold["x"]).max() < 1e-5
    # a useless start is replaced by the cold one: same iterates as cold
    bad_u = np.full_like(cold["u"], 40.0)
    gs, gst, _ = oracle.solve(pb, warm={"u": bad_u, "ye": -cold["ye"]}, guarded=True)
    assert gst["start"] == 0
    assert gst["inner_it"] == cs["inner_it"] and gst["outer_it"] == cs["outer_it"]
    np.testing.assert_array_equal(gs["x"], cold["x"])
    # a good start survives the guard unchanged
    hs, hst, _ = oracle.solve(pb, warm={"u": cold["u"], "ye": cold["ye"]}, guarded=True)
    assert hst["start"] == 1 and hst["inner_it"] == wst["inner_it"]
    np.testing.assert_array_equal(hs["x"], ws["x"])


def test_total_iteration_cap():
    inst = S.single_bmpc(0)
    pb = oracle.problem_from_instance(inst)
    _, full, fh = oracle.solve(pb)
    assert full["inner_it"] > 10
    x, st, h = oracle.solve(pb, oracle.default_settings(max_iter_total=10))
    assert st["status"] == 5 and st["inner_it"] == 10
    np.testing.assert_array_equal(h, fh[:10])
    # a cap above the iterations needed changes nothing
    _, st2, _ = oracle.solve(pb, oracle.default_settings(max_iter_total=full["inner_it"] + 1))
    assert st2["status"] == full["status"] and st2["inner_it"] == full["inner_it"]


def _solve_all(insts):
    """Oracle solves on host threads (the C oracle runs outside the
    interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=8) as ex:
        return list(ex.map(lambda i: oracle.solve(oracle.problem_from_instance(i))[1], insts))


def test_single_tree_workload_all_1000_seeds_converge():
    """The single-tree workload's 1,000 seeds all end with status OK and
    max(r_kkt, violation) < 1e-6."""
    stats = _solve_all([S.single_bmpc(s) for s in range(1000)])
    bad = [(i, s["status"]) for i, s in enumerate(stats) if s["status"] != 0 or s["r_kkt"] >= 1e-6
           or s["viol"] >= 1e-6]
    assert not bad, bad


def test_batched_workload_all_512_instances_converge():
    """All 512 instances of the batched workload (uneven horizons, branch
    counts and branch stages) end with status OK at KKT 1e-6."""
    stats = _solve_all(S.batched_instances(512))
    bad = [(i, s["status"], s["inner_it"]) for i, s in enumerate(stats) if s["status"] != 0]
    assert not bad, bad
    assert max(s["r_kkt"] for s in stats) < 1e-6 and max(s["viol"] for s in stats) < 1e-6


def test_shift_with_a_measured_state_moves_only_the_root_and_its_leaves():
    """A measured next state replaces the predicted one: the shifted tree
    is the same except at the root (the measured state) and at leaves rolled
    out from the root; the new problem's x0 is the measured state."""
    inst = S.single_bmpc(1)
    pb = oracle.problem_from_instance(inst)
    st, stats, _ = oracle.solve(pb)
    new_p, pred = oracle.shift(pb, st)
    meas = new_p.x0 + np.array([0.3, -0.2, 0.05, 0.4])
    new_m, got = oracle.shift(pb, st, x0_meas=meas)
    np.testing.assert_array_equal(new_m.x0, meas)
    np.testing.assert_array_equal(got["x"][0], meas)
    np.testing.assert_array_equal(got["x"][1:], pred["x"][1:])
    for k in ("u", "lam", "ye"):
        np.testing.assert_array_equal(got[k], pred[k])
    np.testing.assert_array_equal(new_m.ref, new_p.ref)
