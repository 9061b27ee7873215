"""Exact Hessian with eigenvalue modification (Sec. IV-A, search direction)
on the GPU against the oracle, through the C ABI.

Bars: the quadratic model element-wise within 1e-11 of the oracle's
(relative to each array's largest entry; the eigenvalue modification goes
through two different Jacobi eigensolvers, a 6x6 one in the oracle and the
2x2 + 4x4 blocks here); solves as the Gauss-Newton ones: same status,
KKT residual and violation <= 1e-6, solution within 1e-5, iteration path
to 1e-6 over the first iterations.
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
from paper_2506_13624_amd.bicycle import Problem  # noqa: E402

from test_gpu_bmpc import _oracle_solves, dev, gpu_solve, host, relerr, zeros  # noqa: E402

EXACT = dict(hessian=L.HESSIAN_EXACT)


def _point(inst, seed, spread=0.3):
    """A point with defects, active input bounds and obstacle penalties and
    nonzero multipliers."""
    opb = oracle.problem_from_instance(inst)
    N = opb.N
    rng = np.random.default_rng(seed)
    u = np.column_stack([rng.uniform(-3.5, 3.5, N), rng.uniform(-0.6, 0.6, N)])
    x = oracle.rollout(opb, u) + rng.normal(0, spread, (N, 4))
    x[0] = inst.x0
    obs_nodes = np.nonzero(inst.node_obstacle >= 0)[0][::5]
    x[obs_nodes, :2] = inst.obstacles[inst.node_obstacle[obs_nodes]] + rng.uniform(-1, 1, (len(obs_nodes), 2))
    lam = rng.normal(0, 2.0, (N, 4))
    ye = np.abs(rng.normal(0, 0.5, (N, 5)))
    return opb, x, u, lam, ye


def _gpu_model(inst, x, u, lam, ye, rho, floor):
    N = inst.num_nodes
    pb = Problem(inst)
    A, B, c, Q, R, M, q, r = (zeros(N, k) for k in (16, 8, 4, 16, 4, 8, 4, 2))
    kkt, viol = L.bmpc_linearize_exact(pb.handle, floor, dev(x), dev(u), dev(lam), dev(ye), rho,
                                       A, B, c, Q, R, M, q, r)
    pb.close()
    shapes = ((N, 4, 4), (N, 4, 2), (N, 4), (N, 4, 4), (N, 2, 2), (N, 2, 4), (N, 4), (N, 2))
    return [host(t, s) for t, s in zip((A, B, c, Q, R, M, q, r), shapes)], kkt, viol


@pytest.mark.parametrize("seed,floor", [(0, 1e-6), (3, 1e-6), (7, 1e-2)])
def test_exact_model_matches_oracle(seed, floor):
    inst = S.single_bmpc(seed)
    opb, x, u, lam, ye = _point(inst, seed)
    rho = 37.0
    (A, B, c, Q, R, M, q, r), kkt, viol = _gpu_model(inst, x, u, lam, ye, rho, floor)
    N = opb.N
    oQ, oR, oM, oq, orr = np.zeros_like(Q), np.zeros_like(R), np.zeros_like(M), np.zeros_like(q), np.zeros_like(r)
    modified = 0
    for n in range(N):
        oq[n], orr[n], oQ[n], oR[n], oM[n] = oracle.node_quadratic(opb, n, x, u, lam, ye, rho, hessian=1,
                                                                   eig_floor=floor)
        _, _, Qe, _, _ = oracle.node_quadratic(opb, n, x, u, lam, ye, rho, hessian=1, modify=False)
        modified += int(np.abs(Qe - oQ[n]).max() > 0)
    print(f"seed {seed}: {modified} of {N} nodes modified", flush=True)
    assert modified > 0
    for name, g, o in (("Q", Q, oQ), ("R", R, oR), ("M", M, oM), ("q", q, oq), ("r", r, orr)):
        e = relerr(g, o)
        assert e <= 1e-11, f"{name}: {e:.3e}"
    # the dynamics and the KKT residual are those of the Gauss-Newton call
    pb = Problem(inst)
    A0, B0, c0, Q0, R0, q0, r0 = (zeros(N, k) for k in (16, 8, 4, 16, 4, 4, 2))
    kkt0, viol0 = L.bmpc_linearize(pb.handle, dev(x), dev(u), dev(lam), dev(ye), rho, A0, B0, c0, Q0, R0, q0, r0)
    pb.close()
    for g, t, s in ((A, A0, (N, 4, 4)), (B, B0, (N, 4, 2)), (c, c0, (N, 4))):
        np.testing.assert_array_equal(g, host(t, s))
    assert kkt == kkt0 and viol == viol0


@pytest.mark.parametrize("seed", range(8))
def test_exact_solve_matches_oracle(seed):
    inst = S.single_bmpc(seed)
    g, gs = gpu_solve(inst, L.bmpc_settings_default(**EXACT))
    o, os_, _ = oracle.solve(oracle.problem_from_instance(inst), oracle.default_settings(hessian=1))
    print(f"seed {seed}: gpu status {gs['status']} inner {gs['inner_it']}; oracle {os_['status']} "
          f"inner {os_['inner_it']}", flush=True)
    assert gs["status"] == os_["status"] == 0
    assert gs["r_kkt"] <= 1e-6 and gs["viol"] <= 1e-6
    assert np.abs(g["x"] - o["x"]).max() <= 1e-5 * max(1.0, np.abs(o["x"]).max())
    assert np.abs(g["u"] - o["u"]).max() <= 1e-5 * max(1.0, np.abs(o["u"]).max())
    assert abs(gs["inner_it"] - os_["inner_it"]) <= 2


def test_exact_iteration_path_follows_oracle():
    inst = S.single_bmpc(2)
    pb = Problem(inst)
    cap = 64
    b = L.bmpc_batch_create([pb.handle], hist_cap=cap)
    L.bmpc_batch_launch(b, L.bmpc_settings_default(**EXACT))
    st = L.bmpc_batch_stats(b, 1)[0]
    h = L.bmpc_batch_history(b, 0, cap)
    L.bmpc_batch_destroy(b)
    pb.close()
    _, os_, oh = oracle.solve(oracle.problem_from_instance(inst), oracle.default_settings(hessian=1))
    k = min(8, len(oh), st["inner_it"])
    assert k >= 3
    np.testing.assert_allclose(h[:k, :5], oh[:k, :5], rtol=1e-6)


@pytest.mark.parametrize("variant,block", [(L.RICCATI_LEVEL, 256), (L.RICCATI_SEGSCAN, 128),
                                           (L.RICCATI_LEVEL, 64)])
def test_exact_batch_matches_oracle(variant, block):
    """24 instances of the 512-instance workload in one launch, for the level
    and segment-scan backward passes (the cross block M enters both)."""
    insts = S.batched_instances(512)[:24]
    pbs = [Problem(i) for i in insts]
    b = L.bmpc_batch_create([p.handle for p in pbs])
    L.bmpc_batch_launch(b, L.bmpc_settings_default(riccati_variant=variant, block_size=block, **EXACT))
    stats = L.bmpc_batch_stats(b, len(insts))
    ores = _oracle_solves(insts, hessian=1)
    for i, inst in enumerate(insts):
        N = inst.num_nodes
        x, u = zeros(N, 4), zeros(N, 2)
        L.bmpc_batch_state(b, i, x=x, u=u)
        torch.cuda.synchronize()
        o, os_, _ = ores[i]
        print(f"instance {i} N={N}: gpu {stats[i]['status']} inner {stats[i]['inner_it']}; oracle "
              f"{os_['status']} inner {os_['inner_it']}", flush=True)
        assert stats[i]["status"] == os_["status"] == 0
        assert stats[i]["r_kkt"] <= 1e-6 and stats[i]["viol"] <= 1e-6
        assert np.abs(host(x, (N, 4)) - o["x"]).max() <= 1e-5 * max(1.0, np.abs(o["x"]).max())
        assert np.abs(host(u, (N, 2)) - o["u"]).max() <= 1e-5 * max(1.0, np.abs(o["u"]).max())
    L.bmpc_batch_destroy(b)
    for p in pbs:
        p.close()


def test_hessian_settings_validated():
    inst = S.single_bmpc(0)
    for kw in (dict(hessian=2), dict(hessian=1, eig_floor=0.0), dict(hessian=1, eig_floor=float("nan"))):
        pb = Problem(inst)
        N = pb.N
        with pytest.raises(L.BmpcError) as e:
            L.bmpc_solve(pb.handle, L.bmpc_settings_default(**kw), 0, zeros(N, 4), zeros(N, 2), zeros(N, 4),
                         zeros(N, 5))
        assert e.value.status == 1
        pb.close()
