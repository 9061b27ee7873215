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


def test_autotune_budget_and_shape_keyed_cache(tmp_path):
    """The budgeted autotuner times the candidates, keeps the one with the
    shortest time per inner iteration and appends it to the cache; a second
    batch of the same shape takes the cached choice without timing runs,
    and a batch of another shape is tuned afresh."""
    cache = str(tmp_path / "tune.txt")
    insts = S.batched_instances(512)[:32]
    st = L.bmpc_settings_default()
    pbs, b = _batch(insts)
    v1, b1, t1, cached = L.bmpc_batch_autotune(b, st, budget_ms=200, cache_path=cache)
    print(f"autotuned: variant {v1} block {b1}, {t1:.4f} ms per inner iteration", flush=True)
    assert not cached and t1 > 0 and (v1, b1) in L.bmpc_batch_tune_candidates()
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and lines[0].startswith("bmpc-autotune ")
    L.bmpc_batch_destroy(b)
    pbs2, b2 = _batch(insts)
    v2, bb2, t2, cached2 = L.bmpc_batch_autotune(b2, st, budget_ms=200, cache_path=cache)
    assert cached2 and (v2, bb2) == (v1, b1) and t2 == pytest.approx(t1, rel=1e-8)
    L.bmpc_batch_destroy(b2)
    pbs3, b3 = _batch(insts[:16])
    _, _, _, cached3 = L.bmpc_batch_autotune(b3, st, budget_ms=0, cache_path=cache)
    assert not cached3 and len(open(cache).read().splitlines()) == 2
    L.bmpc_batch_destroy(b3)
    for p in pbs + pbs2 + pbs3:
        p.close()


def test_phase_times_cover_the_solve():
    """Per-phase device times of a solve are positive and their sum is at
    most the launch time measured around it (the start point is not
    counted), and at least half of it."""
    insts = S.batched_instances(512)[:1]
    pbs, b = _batch(insts)
    st = L.bmpc_settings_default()
    L.bmpc_batch_launch(b, st)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    L.bmpc_batch_launch(b, st)
    e1.record()
    torch.cuda.synchronize()
    launch = e0.elapsed_time(e1)
    s = L.bmpc_batch_stats(b, 1)[0]
    L.bmpc_batch_destroy(b)
    pbs[0].close()
    ph = s["time_ms"]
    print(f"launch {launch:.3f} ms, {s['inner_it']} inner iterations, phases {ph}", flush=True)
    assert all(v > 0 for v in ph.values())
    assert 0.5 * launch <= sum(ph.values()) <= launch * 1.02


def test_warm_shift_with_measured_state_matches_oracle():
    """bmpc_warm_shift of one problem's solution with a measured next state
    equals the oracle's shift with that state; a warm solve from it reaches
    the oracle's solution of the shifted problem."""
    inst = S.single_bmpc(4)
    opb = oracle.problem_from_instance(inst)
    o, os_, _ = oracle.solve(opb)
    assert os_["status"] == 0
    N = inst.num_nodes
    pb = Problem(inst)
    dev = {k: torch.from_numpy(np.ascontiguousarray(o[k]).ravel().copy()).cuda() for k in ("x", "u", "lam", "ye")}
    onew0, _ = oracle.shift(opb, o)
    meas = onew0.x0 + np.array([0.2, -0.1, 0.03, -0.3])
    L.bmpc_warm_shift(pb.handle, dev["x"], dev["u"], dev["lam"], dev["ye"], x0_new=meas)
    torch.cuda.synchronize()
    onew, osh = oracle.shift(opb, o, x0_meas=meas)
    np.testing.assert_array_equal(L.bmpc_problem_get_x0(pb.handle), meas)
    shapes = {"x": (N, 4), "u": (N, 2), "lam": (N, 4), "ye": (N, 5)}
    for k, shp in shapes.items():
        g = dev[k].cpu().numpy().reshape(shp)
        assert np.abs(g - osh[k]).max() <= 1e-12 * max(1.0, np.abs(osh[k]).max()), k
    gs = L.bmpc_solve(pb.handle, L.bmpc_settings_default(), 7, dev["x"], dev["u"], dev["lam"], dev["ye"])
    pb.close()
    o2, os2, _ = oracle.solve(onew, warm=osh)
    print(f"warm after measured shift: gpu {gs['status']} inner {gs['inner_it']}; oracle {os2['status']} "
          f"inner {os2['inner_it']}", flush=True)
    assert gs["status"] == os2["status"] == 0
    g = dev["x"].cpu().numpy().reshape(N, 4)
    assert np.abs(g - o2["x"]).max() <= 1e-5 * max(1.0, np.abs(o2["x"]).max())
