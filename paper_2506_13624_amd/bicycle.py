"""Build library problem handles for the kinematic-bicycle lane workload.

Only marshalling: the node weights and references come from the library's
own helpers (bmpc_weights_from_probs, bmpc_node_refs).
"""
from __future__ import annotations

import numpy as np

from . import _lib as L


class Problem:
    """Owns a tree handle and a problem handle for one bicycle instance."""

    def __init__(self, inst, x0=None):
        self.N = inst.num_nodes
        self.tree = L.bmpc_tree_create(inst.parent)
        w = L.bmpc_weights_from_probs(self.tree, inst.leaf_prob, self.N)
        ref = L.bmpc_node_refs(self.tree, inst.leaf_prob, inst.leaf_offset, inst.dt, inst.ref_speed,
                               self.N)
        has = (inst.node_obstacle >= 0).astype(np.int32)
        xy = np.zeros((self.N, 2))
        if len(inst.obstacles):
            xy[has == 1] = inst.obstacles[inst.node_obstacle[has == 1]]
        prm = L.bmpc_bicycle_default(wheelbase=inst.wheelbase, dt=inst.dt, a_max=inst.a_max,
                                     steer_max=inst.steer_max, obs_radius=inst.obs_radius)
        for i in range(4):
            prm.Qd[i] = inst.q_diag[i]
        for i in range(2):
            prm.Rd[i] = inst.r_diag[i]
        self.handle = L.bmpc_problem_create(self.tree, prm, w, ref, xy, has,
                                            inst.x0 if x0 is None else x0)

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
