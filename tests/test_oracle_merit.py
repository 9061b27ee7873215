"""Pins of the oracle's line-search pieces (CPU only).

The merit of eq. merit with J read as the augmented objective L_a of eq. AL,
its slope along the tree-LQR step with the adaptive penalty of Gill et al.
(Sec. IV-A), and the constraint violation c of Sec. IV-B.  Each is checked
against something other than its own formula: a value worked out by hand, a
central difference of the merit, and hand-computed violations.
"""
import numpy as np
import pytest

import bmpc_synth as S
import oracle


def _three_node_linear_problem():
    # chain 0 -> 1 -> 2 (leaf); linear model x+ = x + [u0, u1, 0, 0]
    Al = np.eye(4)
    Bl = np.zeros((4, 2))
    Bl[0, 0] = Bl[1, 1] = 1.0
    model = oracle.linear_model(Al, Bl, q_diag=(2.0, 1.0, 0.0, 0.0), r_diag=(1.0, 0.5),
                                a_max=1.0, steer_max=10.0)
    parent = np.array([-1, 0, 1], dtype=np.int32)
    weight = np.array([1.0, 0.5, 0.25])
    ref = np.zeros((3, 4))
    pb = oracle.BmpcProblem(parent, weight, ref, np.zeros((3, 2)), np.zeros(3, np.int32),
                            np.zeros(4), model)
    return pb


def test_merit_worked_example_three_nodes():
    pb = _three_node_linear_problem()
    x = np.array([[1.0, 0, 0, 0], [2.0, 1.0, 0, 0], [2.0, 3.0, 0, 0]])
    u = np.array([[1.5, 0.5], [-1.25, 2.0], [0.0, 0.0]])
    lam = np.array([[9.0, 9, 9, 9], [1.0, 2, 3, 4], [-2.0, 0, 0, 1]])  # lam_0 is unused
    ye = np.zeros((3, 5))
    ye[1, 1] = 2.0                     # multiplier of node 1's bound -u0 <= 1
    rho, mu = 4.0, 3.0
    # By hand (every number a binary fraction, so the sum is exact):
    # node 0: 1/2*1*(2*1^2 + 1*0^2) = 1;  1/2*1*(1*1.5^2 + 0.5*0.5^2) = 1.1875;
    #         bound u0 <= 1 violated by 0.5: rho/2 * 0.5^2 = 0.5      -> 2.6875
    # node 1: 1/2*0.5*(2*2^2 + 1*1^2) = 2.25; 1/2*0.5*(1.25^2 + 0.5*2^2) = 0.890625;
    #         bound -u0 <= 1: g = 0.25, t = g + y/rho = 0.75: 2*0.75^2 = 1.125
    #                                                                 -> 4.265625
    # leaf 2: 1/2*0.25*(2*2^2 + 1*3^2) = 2.125
    # L_a = 9.078125
    # d_1 = f(x_0, u_0) - x_1 = [2.5, 0.5, 0, 0] - [2, 1, 0, 0] = [0.5, -0.5, 0, 0]
    # d_2 = f(x_1, u_1) - x_2 = [0.75, 3, 0, 0] - [2, 3, 0, 0] = [-1.25, 0, 0, 0]
    # lam^T d = (0.5 - 1) + 2.5 = 2;  mu/2 ||d||^2 = 1.5 * 2.0625 = 3.09375
    assert oracle.augmented_lagrangian(pb, x, u, ye, rho) == 9.078125
    assert oracle.merit(pb, x, u, lam, ye, rho, mu) == 14.171875


def _bicycle_point(seed, rho=30.0):
    """A point of a small bicycle tree with defects, active bounds, an active
    obstacle slot and nonzero multipliers."""
    inst = S.small_bicycle(10, [3], 3, seed)
    pb = oracle.problem_from_instance(inst)
    rng = np.random.default_rng(seed)
    N = pb.N
    u = np.column_stack([rng.uniform(-3.5, 3.5, N), rng.uniform(-0.6, 0.6, N)])
    x = oracle.rollout(pb, u) + 0.05 * rng.standard_normal((N, 4))
    x[0] = pb.x0
    # put one obstacle-bearing node inside its obstacle
    n_obs = int(np.nonzero(pb.has_obs)[0][2])
    x[n_obs, :2] = pb.obs[n_obs] + [0.4, -0.3]
    lam = rng.standard_normal((N, 4))
    ye = np.abs(rng.standard_normal((N, 5))) * (rng.uniform(size=(N, 5)) < 0.5)
    return pb, x, u, lam, ye, rho, n_obs


def test_merit_is_affine_in_lambda_and_mu_with_the_defects_as_slope():
    pb, x, u, lam, ye, rho, _ = _bicycle_point(0)
    mu = 5.0
    phi = oracle.merit(pb, x, u, lam, ye, rho, mu)
    # the defects, from the dynamics directly
    d = np.zeros_like(x)
    for j in range(1, pb.N):
        p = pb.parent[j]
        d[j] = oracle.rk4(pb.model, x[p], u[p])[0] - x[j]
    assert np.abs(d).max() > 1e-3
    # d phi / d lam_j = d_j and d phi / d mu = ||d||^2 / 2
    for j, a in ((1, 0), (7, 2), (pb.N - 1, 3)):
        lp = lam.copy()
        lp[j, a] += 1.0
        assert oracle.merit(pb, x, u, lp, ye, rho, mu) - phi == pytest.approx(d[j, a], abs=1e-9)
    assert (oracle.merit(pb, x, u, lam, ye, rho, mu + 2.0) - phi) == pytest.approx(np.sum(d * d), rel=1e-9)
    # with d = 0 the merit is L_a whatever lam and mu are
    x0 = oracle.rollout(pb, u)
    la = oracle.augmented_lagrangian(pb, x0, u, ye, rho)
    assert oracle.merit(pb, x0, u, lam, ye, rho, 123.0) == pytest.approx(la, rel=1e-14)


@pytest.mark.parametrize("seed", range(4))
def test_merit_slope_matches_central_difference_along_the_lqr_step(seed):
    pb, x, u, lam, ye, rho, n_obs = _bicycle_point(seed)
    dx, du, lh, sl = oracle.direction(pb, x, u, lam, ye, rho, 1.0)
    mu = sl["mu"]
    assert sl["dd"] > 1e-6                      # the point has defects

    def phi(a):
        return oracle.merit(pb, x + a * dx, u + a * du, lam + a * (lh - lam), ye, rho, mu)

    # Richardson-extrapolated central difference; the active sets do not
    # change for |alpha| <= 2h
    def cd(h):
        return (phi(h) - phi(-h)) / (2 * h)
    h = 1e-5
    fd = (4 * cd(h / 2) - cd(h)) / 3
    assert fd == pytest.approx(sl["dphi0"], rel=1e-6, abs=1e-8)
    assert phi(0.0) == pytest.approx(sl["phi0"], rel=1e-15)


def _gn_curvature(pb, x, u, ye, rho, dx, du):
    """dz^T H dz with H the node Hessians of L_a (Gauss-Newton), read node by
    node from the oracle's node terms."""
    nch = S.num_children(pb.parent)
    s = 0.0
    for n in range(pb.N):
        _, _, _, _, Hxx, Huu = oracle.node_terms(pb, n, x[n], u[n], ye[n], rho)
        s += dx[n] @ Hxx @ dx[n]
        if nch[n] > 0:
            s += du[n] @ Huu @ du[n]
    return s


@pytest.mark.parametrize("seed", range(4))
def test_mu_hat_puts_the_slope_at_minus_half_the_curvature(seed):
    pb, x, u, lam, ye, rho, _ = _bicycle_point(seed)
    dx, du, lh, sl = oracle.direction(pb, x, u, lam, ye, rho, 1e-3)
    mu_hat = sl["mu_hat"]
    dhd = _gn_curvature(pb, x, u, ye, rho, dx, du)
    assert dhd == pytest.approx(sl["dhd"], rel=1e-12)

    def slope(mu):
        def phi(a):
            return oracle.merit(pb, x + a * dx, u + a * du, lam + a * (lh - lam), ye, rho, mu)
        h = 1e-5
        c1 = (phi(h) - phi(-h)) / (2 * h)
        c2 = (phi(h / 2) - phi(-h / 2)) / h
        return (4 * c2 - c1) / 3

    # at mu = mu_hat the slope sits exactly on the bound -1/2 dz^T H dz
    assert slope(mu_hat) == pytest.approx(-0.5 * dhd, rel=1e-6, abs=1e-8)
    # the rule raises a small mu to max(mu_hat, 2 mu) and keeps a large one
    if mu_hat > 2e-3:
        assert sl["mu"] == mu_hat
    big = 10.0 * max(mu_hat, 1.0)
    _, _, _, sl2 = oracle.direction(pb, x, u, lam, ye, rho, big)
    assert sl2["mu"] == big
    assert sl2["dphi0"] <= -0.5 * dhd
    small = 0.75 * mu_hat
    if small > 0:
        _, _, _, sl3 = oracle.direction(pb, x, u, lam, ye, rho, small)
        assert sl3["mu"] == max(mu_hat, 2 * small)


def _two_node_bicycle(has_obs_leaf, obs_xy=(0.0, 0.0)):
    model = oracle.bicycle_model(S.single_bmpc(0))   # |a| <= 3, |steer| <= 0.5, r = 1.5
    parent = np.array([-1, 1 - 1], dtype=np.int32)
    obs = np.array([[0.0, 0.0], list(obs_xy)])
    has = np.array([0, 1 if has_obs_leaf else 0], np.int32)
    return oracle.BmpcProblem(parent, np.ones(2), np.zeros((2, 4)), obs, has,
                              np.array([0.0, 0.0, 0.0, 8.0]), model)


def test_violation_worked_examples():
    rho = 10.0
    pb = _two_node_bicycle(True, obs_xy=(10.0, 0.0))
    x = np.array([[0.0, 0.0, 0.0, 8.0], [8.0, 0.0, 0.0, 8.0]])   # leaf 2.0 from the obstacle
    ye = np.zeros((2, 5))
    # root slots: a - 3, -a - 3, steer - 0.5, -steer - 0.5; leaf slot 4: 1.5 - dist
    # (1) u = [2.95, 0.4], ye = 0 except slot 2 with ye/rho = 0.3:
    #     slots: max(-0.05, 0) = 0, max(-5.95, 0) = 0, max(-0.1, -0.3) = -0.1,
    #     max(-0.9, 0) = 0, leaf max(-0.5, 0) = 0  ->  c = |-0.1| = 0.1
    u = np.array([[2.95, 0.4], [0.0, 0.0]])
    ye[0, 2] = 3.0
    assert oracle.violation(pb, x, u, ye, rho) == pytest.approx(0.1, abs=1e-15)
    # (2) an active slot dominates: a = 3.2 -> g = 0.2
    u2 = np.array([[3.2, 0.4], [0.0, 0.0]])
    assert oracle.violation(pb, x, u2, ye, rho) == pytest.approx(0.2, abs=1e-15)
    # (3) the leaf inside the obstacle by 0.3: dist 1.2 -> g = 0.3
    x3 = x.copy()
    x3[1, 0] = 8.8
    assert oracle.violation(pb, x3, u, ye, rho) == pytest.approx(0.3, abs=1e-14)
    # (4) an inactive slot with a large multiplier estimate is bounded by g:
    #     g = -0.1 and ye/rho = 5 -> max(-0.1, -5) = -0.1 -> 0.1
    ye4 = np.zeros((2, 5))
    ye4[0, 2] = 50.0
    assert oracle.violation(pb, x, u, ye4, rho) == pytest.approx(0.1, abs=1e-15)
    # (5) no obstacle slot at the leaf: only the root's slots count
    pb5 = _two_node_bicycle(False)
    assert oracle.violation(pb5, x3, u2, ye, rho) == pytest.approx(0.2, abs=1e-15)


def test_merit_outside_the_bicycle_domain_is_infinite():
    pb, x, u, lam, ye, rho, _ = _bicycle_point(1)
    assert np.isfinite(oracle.merit(pb, x, u, lam, ye, rho, 1.0))
    u2 = u.copy()
    u2[2, 1] = 1.6                       # past the pole of tan at pi/2
    assert oracle.merit(pb, x, u2, lam, ye, rho, 1.0) == np.inf
    u2[2, 1] = -1.5707963267948966
    assert oracle.merit(pb, x, u2, lam, ye, rho, 1.0) == np.inf
