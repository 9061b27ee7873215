"""Build library problem handles for the kinematic-bicycle lane workload.

Only marshalling: the node weights and references come from the library's
own helpers (bmpc_weights_from_probs, bmpc_node_refs).
"""
from __future__ import annotations

import numpy as np

from . import _lib as L


def problem_arrays(inst, tree, x0=None):
    """Host arrays of bmpc_problem_create for one instance on `tree`:
    (params, node_weight, node_ref, node_obs, has_obs, x0)."""
    N = inst.num_nodes
    w = L.bmpc_weights_from_probs(tree, inst.leaf_prob, N)
    ref = L.bmpc_node_refs(tree, inst.leaf_prob, inst.leaf_offset, inst.dt, inst.ref_speed, N)
    has = (inst.node_obstacle >= 0).astype(np.int32)
    xy = np.zeros((N, 2))
    if len(inst.obstacles):
        xy[has == 1] = inst.obstacles[inst.node_obstacle[has == 1]]
    prm = L.bmpc_bicycle_default(wheelbase=inst.wheelbase, dt=inst.dt, a_max=inst.a_max,
                                 steer_max=inst.steer_max, obs_radius=inst.obs_radius)
    for i in range(4):
        prm.Qd[i] = inst.q_diag[i]
    for i in range(2):
        prm.Rd[i] = inst.r_diag[i]
    return prm, w, ref, xy, has, (inst.x0 if x0 is None else x0)


class Problem:
    """Owns a tree handle and a problem handle for one bicycle instance."""

    def __init__(self, inst, x0=None):
        self.N = inst.num_nodes
        self.tree = L.bmpc_tree_create(inst.parent)
        self.handle = L.bmpc_problem_create(self.tree, *problem_arrays(inst, self.tree, x0))

    def close(self):
        if self.handle is not None:
            L.bmpc_problem_destroy(self.handle)
            L.bmpc_tree_destroy(self.tree)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ProblemPool:
    """`size` problems on one shared tree and one batch over them; load()
    replaces the problems' data (same topology) for the next launch."""

    def __init__(self, parent, size, first_inst=None, hist_cap=0):
        self.parent = np.asarray(parent, dtype=np.int32)
        self.N = len(self.parent)
        self.size = size
        self.tree = L.bmpc_tree_create(self.parent)
        self.handles = []
        if first_inst is None:
            raise ValueError("an instance of the topology is needed to create the problems")
        arrays = problem_arrays(first_inst, self.tree)
        for _ in range(size):
            self.handles.append(L.bmpc_problem_create(self.tree, *arrays))
        self.batch = L.bmpc_batch_create(self.handles, hist_cap=hist_cap)

    def load(self, insts):
        if len(insts) > self.size:
            raise ValueError("more instances than problems in the pool")
        for h, inst in zip(self.handles, insts):
            if len(inst.parent) != self.N or not np.array_equal(inst.parent, self.parent):
                raise ValueError("instance topology differs from the pool's tree")
            _, w, ref, xy, has, x0 = problem_arrays(inst, self.tree)
            L.bmpc_problem_update(h, w, ref, xy, has, x0)

    def close(self):
        if self.batch is not None:
            L.bmpc_batch_destroy(self.batch)
            for h in self.handles:
                L.bmpc_problem_destroy(h)
            L.bmpc_tree_destroy(self.tree)
            self.batch = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
