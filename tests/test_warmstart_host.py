"""Host-side encoding of the learned warm start (no GPU needed)."""
import numpy as np

import bmpc_synth as S
from paper_2506_13624_amd import warmstart as W


def test_learned_topology_sizes():
    inst = S.learned_topology_instance(0)
    assert inst.num_nodes == 109
    ctl, pairs = W.output_layout(inst)
    # 105 control nodes x 2 inputs; trunk 5 x 4 bounds, branch nodes
    # 100 x (4 bounds + obstacle), leaves 4 x obstacle
    assert len(ctl) == 105
    assert len(pairs) == 5 * 4 + 100 * 5 + 4
    assert 2 * len(ctl) + len(pairs) == 734


def test_features_encode_scenarios():
    inst = S.learned_topology_instance(3)
    f = W.features(inst)
    assert f.shape == (W.NUM_FEATURES,) == (44,)
    np.testing.assert_array_equal(f[:4], inst.x0)
    S8 = W.SCENARIO_SLOTS
    np.testing.assert_array_equal(f[4:8], inst.leaf_offset)
    assert np.all(f[8:12] == 0)
    probs, mask = f[4 + 3 * S8: 4 + 4 * S8], f[4 + 4 * S8:]
    assert probs.sum() == np.float64(inst.leaf_prob.sum())
    np.testing.assert_array_equal(mask, [1, 1, 1, 1, 0, 0, 0, 0])
    # each scenario carries the obstacle of its own branch
    leaves = np.nonzero(S.num_children(inst.parent) == 0)[0]
    for k, leaf in enumerate(leaves):
        np.testing.assert_array_equal(f[4 + S8 + 2 * k: 6 + S8 + 2 * k], inst.obstacles[inst.node_obstacle[leaf]])


def test_targets_roundtrip_layout():
    inst = S.learned_topology_instance(1)
    rng = np.random.default_rng(0)
    u, ye = rng.normal(size=(109, 2)), rng.normal(size=(109, 5))
    t = W.targets(inst, u, ye)
    ctl, pairs = W.output_layout(inst)
    np.testing.assert_array_equal(t[:210].reshape(-1, 2), u[ctl])
    # (node, slot) order: node-major, slots increasing
    assert np.all(np.diff(pairs[:, 0] * 5 + pairs[:, 1]) > 0)
    np.testing.assert_array_equal(t[210:], ye[pairs[:, 0], pairs[:, 1]])
