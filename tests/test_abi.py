"""The C ABI library loads on a machine without a GPU, exports every symbol
that include/*.h declares, and its host-only logic (topology analysis,
probability weights, argument checks) behaves as documented."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

import bmpc_synth as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    lib_path = os.path.join(ROOT, "paper_2506_13624_amd", "libbmpc.so")
    if not os.path.exists(lib_path):
        from paper_2506_13624_amd import build
        build.build()
    from paper_2506_13624_amd import _lib
    return _lib


def declared_symbols():
    names = []
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        names += re.findall(r"BMPC_API\s+[\w\s\*]+?\b(bmpc_\w+)\s*\(", txt)
    return sorted(set(names))


def test_every_declared_symbol_is_exported(L):
    names = declared_symbols()
    assert len(names) >= 10
    missing = [n for n in names if not hasattr(L.lib, n)]
    assert not missing, missing


def test_python_binding_covers_every_symbol(L):
    missing = [n for n in declared_symbols() if not hasattr(L, n) and n != "bmpc_last_error"]
    assert not missing, missing


def test_tree_analysis_on_host(L):
    par = S.large_tree(0).parent
    t = L.bmpc_tree_create(par)
    try:
        info = L.bmpc_tree_info(t)
        assert info == {"num_nodes": 122871, "num_leaves": 4096, "depth": 80, "num_segments": 8191}
        seg = L.bmpc_tree_segments(t, len(par))
        ref, _ = S.segments_of(par)
        assert np.array_equal(seg, ref)
    finally:
        L.bmpc_tree_destroy(t)


def test_weights_from_probs_sum_subtrees(L):
    par = np.array([-1, 0, 0, 1, 2, 2], dtype=np.int32)
    t = L.bmpc_tree_create(par)
    try:
        w = L.bmpc_weights_from_probs(t, [0.5, 0.2, 0.3], len(par))
        assert np.allclose(w, [1.0, 0.5, 0.5, 0.5, 0.2, 0.3])
        with pytest.raises(L.BmpcError):
            L.bmpc_weights_from_probs(t, [0.5, np.nan, 0.3], len(par))
    finally:
        L.bmpc_tree_destroy(t)


@pytest.mark.parametrize("parent,msg", [([-1, 0, 2], "parent"), ([-1, 0, 0, 1, 0], "non-decreasing"),
                                        ([0, 0], "-1")])
def test_bad_topologies_rejected(L, parent, msg):
    with pytest.raises(L.BmpcError) as e:
        L.bmpc_tree_create(parent)
    assert e.value.status == 2 and msg in str(e.value)


def test_supported_dimensions_reported(L):
    assert L.bmpc_lqr_supported(4, 2)
    assert L.bmpc_lqr_supported(12, 4)
    assert not L.bmpc_lqr_supported(5, 5)


def test_binding_rejects_mistyped_or_short_arrays_before_the_call(L):
    """Every device array passed through the binding is checked against the
    sizes behind its handle (element type, element count) before the C call,
    so no kernel can read past a short or mistyped buffer.  Host tensors are
    enough here: the checks come first."""
    import torch
    N, n, m = 10, 3, 2
    fake = ctypes.c_void_p(0x1000)
    L._dims[L._key(fake)] = (N, n, m)
    try:
        good = {k: torch.zeros(N * w, dtype=torch.float64) for k, w in
                (("A", n * n), ("B", n * m), ("c", n), ("Q", n * n), ("R", m * m), ("M", m * n), ("q", n),
                 ("r", m), ("x", n), ("u", m), ("lam", n))}
        x0 = torch.zeros(n, dtype=torch.float64)
        args = lambda d: (d["A"], d["B"], d["c"], d["Q"], d["R"], d["M"], d["q"], d["r"], x0, d["x"],
                          d["u"], d["lam"])
        bad = dict(good, B=torch.zeros(N * n * m, dtype=torch.float32))
        with pytest.raises(ValueError, match="element type"):
            L.bmpc_lqr_solve(fake, *args(bad))
        bad = dict(good, Q=torch.zeros(N * n * n - 1, dtype=torch.float64))
        with pytest.raises(ValueError, match="at least"):
            L.bmpc_lqr_solve(fake, *args(bad))
        # right types and sizes: only the device check is left
        with pytest.raises(ValueError, match="device array expected"):
            L.bmpc_lqr_solve(fake, *args(good))
        # a problem of N nodes: state arrays N x 4, N x 2, N x 4, N x 5
        L._dims[L._key(fake)] = N
        st = L.bmpc_settings_default()
        with pytest.raises(ValueError, match="ye"):
            L.bmpc_solve(fake, st, 0, torch.zeros(N * 4, dtype=torch.float64),
                         torch.zeros(N * 2, dtype=torch.float64), torch.zeros(N * 4, dtype=torch.float64),
                         torch.zeros(N * 4, dtype=torch.float64))
        # a network with 4 inputs and 2 outputs
        L._dims[L._key(fake)] = (4, 2)
        with pytest.raises(ValueError, match="element type"):
            L.bmpc_mlp_forward(fake, torch.zeros((3, 4), dtype=torch.float64),
                               torch.zeros(6, dtype=torch.float32))
        with pytest.raises(ValueError, match="at least"):
            L.bmpc_mlp_forward(fake, torch.zeros((3, 4), dtype=torch.float32),
                               torch.zeros(5, dtype=torch.float32))
    finally:
        L._dims.pop(L._key(fake), None)


def _shuffled(parent, seed):
    """The same tree with node i renamed sigma[i] (root anywhere)."""
    rng = np.random.default_rng(seed)
    sigma = rng.permutation(len(parent)).astype(np.int32)
    cpar = np.full(len(parent), -1, dtype=np.int32)
    for i, p in enumerate(parent):
        cpar[sigma[i]] = -1 if p < 0 else sigma[p]
    return cpar, sigma


@pytest.mark.parametrize("seed", range(6))
def test_tree_order_of_a_shuffled_tree(L, seed):
    """Library order of a tree in any node order: a permutation that keeps
    every parent link, gives a parent array the library accepts, and lists
    each node's children in increasing caller index (which fixes it)."""
    base = [S.tree_parent(9, [1, 3, 6], 3), S.tree_parent(12, [0, 4, 8], 2),
            np.array([-1, 0, 1, 1, 2, 3, 4, 5, 5, 6, 7, 8], dtype=np.int32)][seed % 3]
    cpar, _ = _shuffled(base, seed)
    order, lpar = L.bmpc_tree_order(cpar)
    N = len(cpar)
    assert sorted(order.tolist()) == list(range(N))
    assert cpar[order[0]] == -1
    inv = np.empty(N, dtype=np.int64)
    inv[order] = np.arange(N)
    for k in range(1, N):
        assert lpar[k] == inv[cpar[order[k]]]
    for k in range(2, N):
        if lpar[k] == lpar[k - 1]:
            assert order[k] > order[k - 1]
    t = L.bmpc_tree_create(lpar)
    t2, order2 = L.bmpc_tree_create_any(cpar)
    try:
        assert L.bmpc_tree_info(t) == L.bmpc_tree_info(t2)
        np.testing.assert_array_equal(order, order2)
    finally:
        L.bmpc_tree_destroy(t)
        L.bmpc_tree_destroy(t2)


def test_tree_order_is_identity_on_library_order(L):
    par = S.tree_parent(12, [0, 4, 8], 2)
    order, lpar = L.bmpc_tree_order(par)
    np.testing.assert_array_equal(order, np.arange(len(par)))
    np.testing.assert_array_equal(lpar, par)


@pytest.mark.parametrize("parent", [[-1, -1], [1, 0], [-1, 2, 1], [-1, 5], [-1, 1], [0]])
def test_tree_order_rejects_non_trees(L, parent):
    with pytest.raises(L.BmpcError) as e:
        L.bmpc_tree_order(parent)
    assert e.value.status == 2
    with pytest.raises(L.BmpcError):
        L.bmpc_tree_create_any(parent)


def test_host_lqr_binding_rejects_short_arrays_before_the_call(L):
    t = L.bmpc_tree_create(S.tree_parent(3, [0], 2))
    try:
        plan_dims = (7, 4, 2)
        fake = ctypes.c_void_p(12345)
        L._dims[L._key(fake)] = plan_dims
        N, n, m = plan_dims
        arrs = [np.zeros(N * n * n), np.zeros(N * n * m), np.zeros(N * n), np.zeros(N * n * n),
                np.zeros(N * m * m), np.zeros(N * m * n), np.zeros(N * n), np.zeros(N * m - 1),
                np.zeros(n)]
        with pytest.raises(ValueError, match="r:"):
            L.bmpc_lqr_solve_host(fake, *arrs)
    finally:
        L._dims.pop(12345, None)
        L.bmpc_tree_destroy(t)
