"""The linearisation entry point that allocates nothing
(bmpc_linearize_noalloc, workspace in the library's fixed device array)
against bmpc_linearize, through the C ABI: two calls in a row, the second on
a smaller problem, each equal to the allocating entry point's result within
the linearisation bar (1e-12 relative per array)."""
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

PARTS = (("A", 16), ("B", 8), ("c", 4), ("Q", 16), ("R", 4), ("q", 4), ("r", 2))


def _point(inst, seed):
    opb = oracle.problem_from_instance(inst)
    N = opb.N
    rng = np.random.default_rng(seed)
    u = np.column_stack([rng.uniform(-3.5, 3.5, N), rng.uniform(-0.6, 0.6, N)])
    x = oracle.rollout(opb, u) + rng.normal(0, 0.3, (N, 4))
    x[0] = inst.x0
    obs = np.nonzero(inst.node_obstacle >= 0)[0][::5]
    x[obs, :2] = inst.obstacles[inst.node_obstacle[obs]] + rng.uniform(-1, 1, (len(obs), 2))
    lam = rng.normal(0, 0.2, (N, 4))
    ye = np.abs(rng.normal(0, 0.5, (N, 5)))
    return [torch.from_numpy(np.ascontiguousarray(a).ravel().copy()).cuda() for a in (x, u, lam, ye)]


def _outs(N):
    return [torch.full((N * w,), np.nan, dtype=torch.float64, device="cuda") for _, w in PARTS]


def test_noalloc_linearize_equals_allocating_entry_point_twice():
    big = next(i for i in S.batched_instances(64) if i.num_nodes > 400)
    small = S.single_bmpc(3)
    assert small.num_nodes < big.num_nodes <= L.NOALLOC_MAX_NODES
    for call, (inst, rho) in enumerate(((big, 37.0), (small, 5.0))):
        N = inst.num_nodes
        print(f"no-alloc linearise call {call}: N={N}", flush=True)
        pb = Problem(inst)
        pt = _point(inst, 11 + call)
        ref = _outs(N)
        kkt, viol = L.bmpc_linearize(pb.handle, *pt, rho, *ref)
        got = _outs(N)
        kv = torch.full((2,), np.nan, dtype=torch.float64, device="cuda")
        L.bmpc_linearize_noalloc(pb.handle, *pt, rho, *got, kkt_viol=kv)
        torch.cuda.synchronize()
        for (name, _), a, b in zip(PARTS, got, ref):
            a, b = a.cpu().numpy(), b.cpu().numpy()
            assert np.all(np.isfinite(a)), name
            err = np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)
            assert err <= 1e-12, f"call {call}, {name}: {err:.3e}"
        k = kv.cpu().numpy()
        assert k[0] == pytest.approx(kkt, rel=1e-12) and k[1] == pytest.approx(viol, rel=1e-12)
        pb.close()


def test_noalloc_linearize_rejects_problems_beyond_the_workspace():
    inst = S.small_bicycle(40, [0, 4, 8, 12, 16, 20, 24], 2, seed=1)
    assert inst.num_nodes > L.NOALLOC_MAX_NODES
    pb = Problem(inst)
    N = inst.num_nodes
    pt = [torch.zeros(N * w, dtype=torch.float64, device="cuda") for w in (4, 2, 4, 5)]
    with pytest.raises(L.BmpcError) as e:
        L.bmpc_linearize_noalloc(pb.handle, *pt, 1.0, *_outs(N))
    assert e.value.status == 1
    pb.close()
