"""Pins of the oracle's exact Hessian with eigenvalue modification (Sec.
IV-A, search direction), CPU only.

Each piece is checked against something other than its own formula:
  - the dynamics curvature (hyper-dual RK4) against central differences of
    the oracle's RK4 Jacobians, which are pinned separately;
  - the Jacobi eigensolver against LAPACK (numpy.linalg.eigh);
  - the modification against its spectral definition rebuilt with LAPACK;
  - the node model against central differences of the node Lagrangian's
    gradient, built from the oracle's (pinned) node terms and Jacobians;
  - the merit slope along the exact-Hessian step against a central
    difference of the merit, and the curvature term against the blocks.
"""
import numpy as np
import pytest

import bmpc_synth as S
import oracle

from test_oracle_merit import _bicycle_point


def _jac_t_mu(model, z, mu):
    """grad_z (mu^T F(z)) = [A B]^T mu from the oracle's RK4 Jacobians."""
    _, A, B = oracle.rk4(model, z[:4], z[4:])
    return np.concatenate([A.T @ mu, B.T @ mu])


def _central(fn, z, h):
    cols = []
    for j in range(len(z)):
        e = np.zeros(len(z))
        e[j] = h
        c1 = (fn(z + e) - fn(z - e)) / (2 * h)
        c2 = (fn(z + e / 2) - fn(z - e / 2)) / h
        cols.append((4 * c2 - c1) / 3)  # Richardson: O(h^4)
    return np.array(cols).T


@pytest.mark.parametrize("seed", range(5))
def test_rk4_hessian_matches_central_differences_of_the_jacobian(seed):
    model = oracle.bicycle_model(S.single_bmpc(0))
    rng = np.random.default_rng(seed)
    x = np.array([rng.uniform(-5, 5), rng.uniform(-2, 2), rng.uniform(-1, 1), rng.uniform(2, 12)])
    u = np.array([rng.uniform(-3, 3), rng.uniform(-0.5, 0.5)])
    mu = rng.standard_normal(4)
    H = oracle.rk4_hessian(model, x, u, mu)
    fd = _central(lambda z: _jac_t_mu(model, z, mu), np.concatenate([x, u]), 1e-4)
    assert np.array_equal(H, H.T)
    assert np.abs(H - fd).max() <= 1e-8 * max(1.0, np.abs(H).max())
    # curvature is nonzero where the model is nonlinear: heading and speed,
    # and speed with steering
    assert abs(H[2, 3]) > 1e-3 and abs(H[3, 5]) > 1e-3
    # the position does not enter the right-hand side: no curvature in it
    # (the acceleration does, through the speed at the later RK4 stages)
    assert np.all(H[0] == 0) and np.all(H[1] == 0) and abs(H[4, 2]) > 0


def test_rk4_hessian_is_linear_in_the_multiplier_and_zero_for_a_linear_model():
    model = oracle.bicycle_model(S.single_bmpc(0))
    x, u = np.array([1.0, 0.5, 0.3, 8.0]), np.array([0.5, 0.1])
    m1, m2 = np.array([1.0, -2.0, 0.5, 3.0]), np.array([0.25, 1.0, -1.0, 0.0])
    H1, H2 = oracle.rk4_hessian(model, x, u, m1), oracle.rk4_hessian(model, x, u, m2)
    H12 = oracle.rk4_hessian(model, x, u, 2.0 * m1 + m2)
    assert np.abs(H12 - (2.0 * H1 + H2)).max() <= 1e-13 * np.abs(H12).max()
    lin = oracle.linear_model(np.eye(4), np.ones((4, 2)), q_diag=(1, 1, 1, 1), r_diag=(1, 1), a_max=1.0,
                              steer_max=1.0)
    assert np.all(oracle.rk4_hessian(lin, x, u, m1) == 0)


@pytest.mark.parametrize("n,seed", [(4, 0), (6, 1), (6, 2), (2, 3)])
def test_jacobi_eigensolver_matches_lapack(n, seed):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n))
    A = G + G.T
    w, V = oracle.sym_eig(A)
    wr = np.linalg.eigvalsh(A)
    assert np.abs(np.sort(w) - wr).max() <= 1e-13 * np.abs(wr).max()
    assert np.abs(V.T @ V - np.eye(n)).max() <= 1e-13
    assert np.abs(A @ V - V * w).max() <= 1e-13 * np.abs(wr).max()


def test_jacobi_eigensolver_repeated_and_diagonal():
    A = np.diag([3.0, 1.0, 3.0, -2.0])
    w, V = oracle.sym_eig(A)
    assert np.array_equal(np.sort(w), [-2.0, 1.0, 3.0, 3.0])
    rng = np.random.default_rng(7)
    Qo, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    A = Qo @ np.diag([2.0, 2.0, 2.0, -1.0, -1.0, 5.0]) @ Qo.T
    w, V = oracle.sym_eig(A)
    assert np.abs(np.sort(w) - [-1, -1, 2, 2, 2, 5]).max() <= 1e-13
    assert np.abs(V @ np.diag(w) @ V.T - A).max() <= 1e-13


@pytest.mark.parametrize("seed", range(4))
def test_eigenvalue_modification_is_the_spectral_clamp(seed):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((6, 6))
    A = G + G.T
    delta = 0.3
    out = oracle.eig_modify(A, delta)
    wr, Vr = np.linalg.eigh(A)
    want = Vr @ np.diag(np.maximum(wr, delta)) @ Vr.T
    assert np.abs(out - want).max() <= 1e-12 * np.abs(A).max()
    assert np.linalg.eigvalsh(out).min() >= delta * (1 - 1e-10)
    # a matrix whose spectrum is above delta is left as it is
    P = G @ G.T + np.eye(6)
    assert np.abs(oracle.eig_modify(P, 0.5) - P).max() <= 1e-12 * np.abs(P).max()


def _node_lagrangian_gradient(pb, nch, n, x, u, lam, ye, rho, z):
    """grad over z = (x_n, u_n) of L_a,n + sum_{j child} lam_j^T F(x_n, u_n),
    from the oracle's node terms and RK4 Jacobians."""
    _, _, gx, gu, _, _ = oracle.node_terms(pb, n, z[:4], z[4:], ye[n], rho)
    g = np.concatenate([gx, gu])
    if nch[n] > 0:
        mu = lam[pb.parent == n].sum(axis=0)
        g = g + _jac_t_mu(pb.model, z, mu)
    return g


@pytest.mark.parametrize("seed", range(3))
def test_exact_node_hessian_matches_central_differences_of_the_gradient(seed):
    """At a point with an active obstacle penalty (the node sits inside the
    obstacle), active and inactive input bounds and nonzero multipliers, the
    unmodified exact node Hessian equals the central difference of the node
    Lagrangian's gradient, at control nodes and at a leaf; the Gauss-Newton
    choice returns the node terms' Hessian with M = 0."""
    pb, x, u, lam, ye, rho, n_obs = _bicycle_point(seed)
    nch = S.num_children(pb.parent)
    leaf = int(np.nonzero(nch == 0)[0][0])
    checked_obs = False
    for n in (0, 1, n_obs, pb.N // 2, leaf):
        q, r, Q, R, M = oracle.node_quadratic(pb, n, x, u, lam, ye, rho, hessian=1, modify=False)
        z = np.concatenate([x[n], u[n]])
        fd = _central(lambda zz: _node_lagrangian_gradient(pb, nch, n, x, u, lam, ye, rho, zz), z, 1e-5)
        scale = max(1.0, np.abs(fd).max())
        assert np.abs(Q - fd[:4, :4]).max() <= 1e-6 * scale, n
        if nch[n] > 0:
            assert np.abs(M - fd[4:, :4]).max() <= 1e-6 * scale, n
            assert np.abs(R - fd[4:, 4:]).max() <= 1e-6 * scale, n
        else:
            assert np.all(M == 0) and np.all(R == 0)
        g = _node_lagrangian_gradient(pb, nch, n, x, u, lam, ye, rho, z)
        _, _, gx, gu, Hxx, Huu = oracle.node_terms(pb, n, x[n], u[n], ye[n], rho)
        assert np.array_equal(q, gx) and (nch[n] == 0 or np.array_equal(r, gu))
        q0, r0, Q0, R0, M0 = oracle.node_quadratic(pb, n, x, u, lam, ye, rho, hessian=0)
        assert np.array_equal(Q0, Hxx) and np.array_equal(R0, Huu) and np.all(M0 == 0)
        if n == n_obs:
            # the obstacle's own curvature: negative along the tangent
            e = x[n, :2] - pb.obs[n]
            t = np.array([-e[1], e[0]]) / np.linalg.norm(e)
            assert t @ Q[:2, :2] @ t < t @ Hxx[:2, :2] @ t
            checked_obs = True
        del g
    assert checked_obs


def test_modified_node_hessian_is_positive_definite_and_unchanged_when_convex():
    """The modified block's spectrum is floored at eig_floor times
    max(1, the block's largest |eigenvalue|); a block already above the
    floor is unchanged.  A large floor exercises both branches."""
    pb, x, u, lam, ye, rho, n_obs = _bicycle_point(1)
    for delta in (1e-9, 1e-2):
        clamped = kept = 0
        for n in range(pb.N):
            q, r, Q, R, M = oracle.node_quadratic(pb, n, x, u, lam, ye, rho, hessian=1, eig_floor=delta)
            _, _, Qe, Re, Me = oracle.node_quadratic(pb, n, x, u, lam, ye, rho, hessian=1, modify=False)
            leaf = not np.any(pb.parent == n)
            H = Q if leaf else np.block([[Q, M.T], [M, R]])
            He = Qe if leaf else np.block([[Qe, Me.T], [Me, Re]])
            we = np.linalg.eigvalsh(He)
            floor = delta * max(1.0, np.abs(we).max())
            assert np.linalg.eigvalsh(H).min() >= floor * (1 - 1e-6)
            if we.min() > floor:
                assert np.abs(H - He).max() <= 1e-12 * np.abs(He).max()
                kept += 1
            else:
                assert np.abs(H - oracle.eig_modify(He, floor)).max() <= 1e-13 * max(1.0, np.abs(He).max())
                clamped += 1
        assert clamped > 0 and kept > 0, (delta, clamped, kept)


@pytest.mark.parametrize("seed", range(3))
def test_merit_slope_along_the_exact_hessian_step(seed):
    """The closed-form slope matches a central difference of the merit along
    the step of the exact-Hessian model, and the curvature term is dz^T H dz
    with the model's Q, R and M blocks."""
    pb, x, u, lam, ye, rho, _ = _bicycle_point(seed)
    dx, du, lh, sl = oracle.direction(pb, x, u, lam, ye, rho, 1.0, hessian=1)
    mu = sl["mu"]

    def phi(a):
        return oracle.merit(pb, x + a * dx, u + a * du, lam + a * (lh - lam), ye, rho, mu)

    h = 1e-5
    c1 = (phi(h) - phi(-h)) / (2 * h)
    c2 = (phi(h / 2) - phi(-h / 2)) / h
    assert (4 * c2 - c1) / 3 == pytest.approx(sl["dphi0"], rel=1e-6, abs=1e-8)
    nch = S.num_children(pb.parent)
    dhd = 0.0
    for n in range(pb.N):
        _, _, Q, R, M = oracle.node_quadratic(pb, n, x, u, lam, ye, rho, hessian=1)
        dhd += dx[n] @ Q @ dx[n]
        if nch[n] > 0:
            dhd += du[n] @ R @ du[n] + 2.0 * du[n] @ M @ dx[n]
    assert dhd == pytest.approx(sl["dhd"], rel=1e-10)
    # the step differs from the Gauss-Newton one
    dxg, _, _, _ = oracle.direction(pb, x, u, lam, ye, rho, 1.0, hessian=0)
    assert np.abs(dxg - dx).max() > 1e-6


def test_exact_hessian_solves_converge_to_kkt_points():
    """Single-tree workload, 8 seeds: the exact-Hessian solver converges
    (KKT residual and violation <= 1e-6), to the same solution as the
    Gauss-Newton solver, in fewer inner iterations in total."""
    it_gn = it_ex = 0
    for seed in range(8):
        inst = S.single_bmpc(seed)
        pb = oracle.problem_from_instance(inst)
        og, sg, _ = oracle.solve(pb)
        oe, se, _ = oracle.solve(pb, oracle.default_settings(hessian=1))
        assert sg["status"] == 0 and se["status"] == 0
        assert se["r_kkt"] <= 1e-6 and se["viol"] <= 1e-6
        assert np.abs(oe["x"] - og["x"]).max() <= 1e-4 * max(1.0, np.abs(og["x"]).max())
        it_gn += sg["inner_it"]
        it_ex += se["inner_it"]
    print(f"inner iterations: Gauss-Newton {it_gn}, exact {it_ex}")
    assert it_ex < it_gn
