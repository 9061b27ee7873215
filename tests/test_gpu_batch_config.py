"""Batched-solve launch configuration: every (backward variant, threads per
problem) instantiation against the default one and the oracle, the
autotuner, and graph replay of a receding-horizon loop against the same
calls made eagerly."""
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


def _batch(insts):
    pbs = [Problem(i) for i in insts]
    return pbs, L.bmpc_batch_create([p.handle for p in pbs])


def _states(b, insts):
    out = []
    for i, inst in enumerate(insts):
        N = inst.num_nodes
        x = torch.zeros(N * 4, dtype=torch.float64, device="cuda")
        u = torch.zeros(N * 2, dtype=torch.float64, device="cuda")
        L.bmpc_batch_state(b, i, x=x, u=u)
        out.append((x, u))
    torch.cuda.synchronize()
    return [(x.cpu().numpy().reshape(-1, 4), u.cpu().numpy().reshape(-1, 2)) for x, u in out]


@pytest.mark.parametrize("variant,block", L.bmpc_batch_tune_candidates())
def test_every_instantiation_agrees(variant, block):
    insts = S.batched_instances(512)[:12]
    print(f"variant {variant} block {block}", flush=True)
    pbs, b = _batch(insts)
    L.bmpc_batch_launch(b, L.bmpc_settings_default(riccati_variant=L.RICCATI_LEVEL, block_size=256))
    ref = L.bmpc_batch_stats(b, len(insts))
    ref_x = _states(b, insts)
    L.bmpc_batch_launch(b, L.bmpc_settings_default(riccati_variant=variant, block_size=block))
    got = L.bmpc_batch_stats(b, len(insts))
    got_x = _states(b, insts)
    L.bmpc_batch_destroy(b)
    for p in pbs:
        p.close()
    same = 0
    for i, inst in enumerate(insts):
        if ref[i]["status"] == 0 and got[i]["status"] == 0:
            scale = max(1.0, np.abs(ref_x[i][0]).max())
            assert np.abs(got_x[i][0] - ref_x[i][0]).max() <= 2e-5 * scale
        same += ref[i]["status"] == got[i]["status"]
    assert same >= len(insts) - 1
    # converged instances are KKT points of the oracle's problem
    for i in (0, 1):
        if got[i]["status"] == 0:
            o, os_, _ = oracle.solve(oracle.problem_from_instance(insts[i]))
            if os_["status"] == 0:
                assert np.abs(got_x[i][0] - o["x"]).max() <= 2e-5 * max(1.0, np.abs(o["x"]).max())


def test_block_size_validated():
    insts = S.batched_instances(512)[:1]
    pbs, b = _batch(insts)
    with pytest.raises(L.BmpcError) as e:
        L.bmpc_batch_launch(b, L.bmpc_settings_default(block_size=96))
    assert e.value.status == 1
    L.bmpc_batch_destroy(b)
    pbs[0].close()


def test_tuner_restores_state_and_sets_auto():
    insts = S.batched_instances(512)[:64]
    pbs, b = _batch(insts)
    st = L.bmpc_settings_default()
    L.bmpc_batch_launch(b, st)
    L.bmpc_batch_stats(b, len(insts))
    before = _states(b, insts)
    variant, block, ms = L.bmpc_batch_tune(b, st, warm=0, reps=1)
    print(f"tuned: variant {variant} block {block}; candidates {ms}", flush=True)
    assert (variant, block) in ms and all(v > 0 for v in ms.values())
    assert ms[(variant, block)] == min(ms.values())
    after = _states(b, insts)
    for (x0, u0), (x1, u1) in zip(before, after):
        np.testing.assert_array_equal(x0, x1)
        np.testing.assert_array_equal(u0, u1)
    # AUTO launches now use the tuned pair: identical results to asking for it
    L.bmpc_batch_launch(b, st)
    auto = L.bmpc_batch_stats(b, len(insts))
    auto_x = _states(b, insts)
    L.bmpc_batch_launch(b, L.bmpc_settings_default(riccati_variant=variant, block_size=block))
    expl = L.bmpc_batch_stats(b, len(insts))
    expl_x = _states(b, insts)
    L.bmpc_batch_destroy(b)
    for p in pbs:
        p.close()
    assert [a["inner_it"] for a in auto] == [e["inner_it"] for e in expl]
    for (x0, _), (x1, _) in zip(auto_x, expl_x):
        np.testing.assert_array_equal(x0, x1)


def test_graph_replay_of_receding_horizon_loop_matches_eager():
    """Capture [shift, warm solve] once; replay it step by step, with eager
    work and synchronisation between replays, and compare every step with
    the same two calls made eagerly on a twin batch."""
    insts = S.batched_instances(512)[:16]
    pa, ba = _batch(insts)
    pb, bb = _batch(insts)
    st = L.bmpc_settings_default()
    s = torch.cuda.Stream()
    for b in (ba, bb):
        L.bmpc_batch_launch(b, st, stream=s)
    s.synchronize()
    L.bmpc_graph_begin(s)
    L.bmpc_batch_shift(ba, stream=s)
    L.bmpc_batch_launch(ba, st, warm=7, stream=s)
    g = L.bmpc_graph_end(s)
    for step in range(3):
        L.bmpc_graph_launch(g, s)
        L.bmpc_batch_shift(bb, stream=s)
        L.bmpc_batch_launch(bb, st, warm=7, stream=s)
        sa = L.bmpc_batch_stats(ba, len(insts), stream=s)
        sb = L.bmpc_batch_stats(bb, len(insts), stream=s)
        xa, xb = _states(ba, insts), _states(bb, insts)
        print(f"step {step}: inner {[x['inner_it'] for x in sa]}", flush=True)
        assert [x["status"] for x in sa] == [x["status"] for x in sb]
        assert [x["inner_it"] for x in sa] == [x["inner_it"] for x in sb]
        for (x0, u0), (x1, u1) in zip(xa, xb):
            np.testing.assert_array_equal(x0, x1)
            np.testing.assert_array_equal(u0, u1)
    L.bmpc_graph_destroy(g)
    for b in (ba, bb):
        L.bmpc_batch_destroy(b)
    for p in pa + pb:
        p.close()
