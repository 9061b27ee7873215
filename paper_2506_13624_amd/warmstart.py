"""Learned warm start for the branch-MPC solver.

The augmented-Lagrangian solver can start from any point (x, u, lam, ye);
the paper chooses the AL method partly because of this.  Here a multilayer
perceptron maps a problem description to a start point:

  input (44): x0 (4), then for up to 8 scenarios (leaves, increasing node
      order; unused slots zero): lateral offset (8), obstacle centre of the
      scenario's branch (8 x 2), probability (8), presence mask (8);
  output: u of every control node (node order, 2 each), then the PHR
      multiplier estimate of every active constraint slot in (node, slot)
      order (input bounds of control nodes, obstacle of nodes carrying one).
      For the horizon-30 tree with 4 branches at stage 4: 105 x 2 + 524 = 734.

The start is completed on the GPU: bmpc_batch_start_from_network scatters
the outputs, the solver rolls the states out from x0 and takes lam from the
adjoint sweep (warm bits 8 | 4), and the guard (bit 16) keeps the cold start
when the predicted one is worse by max(KKT residual, violation).

Network training and inference run in the library's BF16 matrix-core
kernels (bmpc_mlp_*).  The inference network takes raw features: input
standardisation is its FP32 input map and target de-standardisation is
folded into its last layer.  This module is data handling around those
calls.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import _lib as L
from .bicycle import ProblemPool

SCENARIO_SLOTS = 8
NUM_FEATURES = 4 + SCENARIO_SLOTS * 5
HIDDEN = (256, 256, 256)
WARM_BITS = 8 | 4
GUARD_BIT = 16


def num_children(parent):
    n = np.zeros(len(parent), dtype=np.int64)
    np.add.at(n, np.asarray(parent)[1:], 1)
    return n


def features(inst) -> np.ndarray:
    """Network input of one instance (float64, NUM_FEATURES)."""
    leaves = np.nonzero(num_children(inst.parent) == 0)[0]
    if len(leaves) > SCENARIO_SLOTS:
        raise ValueError(f"at most {SCENARIO_SLOTS} scenarios are encoded")
    f = np.zeros(NUM_FEATURES)
    f[:4] = inst.x0
    S = SCENARIO_SLOTS
    for k, leaf in enumerate(leaves):
        f[4 + k] = inst.leaf_offset[k]
        o = inst.node_obstacle[leaf]
        if o >= 0:
            f[4 + S + 2 * k: 4 + S + 2 * k + 2] = inst.obstacles[o]
        f[4 + 3 * S + k] = inst.leaf_prob[k]
        f[4 + 4 * S + k] = 1.0
    return f


def output_layout(inst):
    """(control nodes, active (node, slot) pairs) in the output order."""
    ctl = np.nonzero(num_children(inst.parent) > 0)[0]
    has = inst.node_obstacle >= 0
    isctl = num_children(inst.parent) > 0
    pairs = [(n, s) for n in range(len(inst.parent)) for s in range(5)
             if (s < 4 and isctl[n]) or (s == 4 and has[n])]
    return ctl, np.array(pairs, dtype=np.int64).reshape(-1, 2)


def targets(inst, u, ye) -> np.ndarray:
    """Network output that reproduces (u, ye) of a solution."""
    ctl, pairs = output_layout(inst)
    return np.concatenate([np.asarray(u)[ctl].ravel(), np.asarray(ye)[pairs[:, 0], pairs[:, 1]]])


def read_states(pool, count, parts=("u", "ye")):
    """Copy the batch state of problems 0 .. count-1 to host arrays (one
    device copy per part for the whole pool)."""
    import torch
    N = pool.N
    dims = {"x": 4, "u": 2, "lam": 4, "ye": 5}
    T = L.bmpc_batch_total_nodes(pool.batch)
    dev = {k: torch.empty(T * dims[k], dtype=torch.float64, device="cuda") for k in parts}
    L.bmpc_batch_state_all(pool.batch, **dev)
    torch.cuda.synchronize()
    return {k: dev[k].cpu().numpy().reshape(pool.size, N, dims[k])[:count] for k in parts}


def generate(instances, pool_size=512, settings=None, progress=None):
    """Solve `instances` (one topology) cold on the GPU, pool_size at a time.
    Returns (features, targets, converged mask, inner iterations)."""
    insts = list(instances)
    st = settings or L.bmpc_settings_default()
    pool = ProblemPool(insts[0].parent, min(pool_size, len(insts)), first_inst=insts[0])
    ctl, pairs = output_layout(insts[0])
    X, T, ok, its = [], [], [], []
    try:
        for c0 in range(0, len(insts), pool.size):
            chunk = insts[c0:c0 + pool.size]
            pool.load(chunk)
            L.bmpc_batch_launch(pool.batch, st)
            stats = L.bmpc_batch_stats(pool.batch, pool.size)[:len(chunk)]
            s = read_states(pool, len(chunk))
            X.append(np.array([features(inst) for inst in chunk]))
            T.append(np.concatenate([s["u"][:, ctl].reshape(len(chunk), -1),
                                     s["ye"][:, pairs[:, 0], pairs[:, 1]]], axis=1))
            ok.extend(x["status"] == 0 for x in stats)
            its.extend(x["inner_it"] for x in stats)
            if progress:
                progress(c0 + len(chunk), len(insts))
    finally:
        pool.close()
    return np.concatenate(X), np.concatenate(T), np.array(ok), np.array(its)


def init_params(widths, seed=0):
    """He-normal weights, zero biases (float32 parameter vector)."""
    rng = np.random.default_rng(seed)
    ws = [rng.normal(0.0, math.sqrt(2.0 / widths[l]), widths[l] * widths[l + 1]) for l in range(len(widths) - 1)]
    bs = [np.zeros(widths[l + 1]) for l in range(len(widths) - 1)]
    return np.concatenate(ws + bs).astype(np.float32)


def split_params(widths, p):
    Ws, bs, off = [], [], 0
    for l in range(len(widths) - 1):
        n = widths[l] * widths[l + 1]
        Ws.append(p[off:off + n].reshape(widths[l], widths[l + 1]))
        off += n
    for l in range(len(widths) - 1):
        bs.append(p[off:off + widths[l + 1]])
        off += widths[l + 1]
    return Ws, bs


def join_params(Ws, bs):
    return np.concatenate([W.ravel() for W in Ws] + [b.ravel() for b in bs]).astype(np.float32)


class WarmStarter:
    """Trains the network on standardised data and serves raw-unit
    predictions through an inference network that standardises its input
    and de-standardises its output itself."""

    def __init__(self, out_width, hidden=HIDDEN, max_batch=1024, seed=0):
        self.widths = [NUM_FEATURES, *hidden, out_width]
        self.max_batch = max_batch
        self.seed = seed
        self.train_net = L.bmpc_mlp_create(self.widths, max_batch)
        L.bmpc_mlp_set_params(self.train_net, init_params(self.widths, seed))
        self.infer_net = None
        self.x_mean = self.x_std = self.t_mean = self.t_std = None

    def close(self):
        for h in (self.train_net, self.infer_net):
            if h is not None:
                L.bmpc_mlp_destroy(h)
        self.train_net = self.infer_net = None

    def fit(self, X, T, steps, batch=1024, lr=1e-3, lr_final=1e-5, log_every=0):
        """Adam on the mean squared error of standardised targets; the step
        size decays geometrically from lr to lr_final.  Returns (loss log,
        seconds spent in training steps, samples per second)."""
        import torch
        X = np.asarray(X, dtype=np.float64)
        T = np.asarray(T, dtype=np.float64)
        self.x_mean, self.x_std = X.mean(0), X.std(0)
        self.x_std[self.x_std < 1e-6] = 1.0
        self.t_mean, self.t_std = T.mean(0), T.std(0)
        self.t_std = np.maximum(self.t_std, 1e-3 * max(self.t_std.max(), 1e-12))
        Xn = torch.from_numpy(((X - self.x_mean) / self.x_std).astype(np.float32)).cuda()
        Tn = torch.from_numpy(((T - self.t_mean) / self.t_std).astype(np.float32)).cuda()
        n = Xn.shape[0]
        batch = min(batch, n, self.max_batch)
        gen = torch.Generator(device="cuda")
        gen.manual_seed(self.seed)
        per_epoch = n // batch
        log = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        perm = None
        for step in range(steps):
            if step % per_epoch == 0:
                perm = torch.randperm(n, device="cuda", generator=gen)
                Xe, Te = Xn[perm].contiguous(), Tn[perm].contiguous()
            j = (step % per_epoch) * batch
            rate = lr * (lr_final / lr) ** (step / max(steps - 1, 1))
            want = bool(log_every) and (step % log_every == 0 or step == steps - 1)
            loss = L.bmpc_mlp_train_step(self.train_net, Xe[j:j + batch], Te[j:j + batch], rate, want_loss=want)
            if want:
                log.append((step, loss))
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        self._fold()
        return log, secs, steps * batch / secs

    def _fold(self):
        """Inference network: input standardisation as the network's FP32
        input map, target de-standardisation folded into the last layer
        (t = t_n s + m  =>  W_L s[None, :], b_L s + m)."""
        Ws, bs = split_params(self.widths, L.bmpc_mlp_get_params(self.train_net).astype(np.float64))
        Ws[-1] = Ws[-1] * self.t_std[None, :]
        bs[-1] = bs[-1] * self.t_std + self.t_mean
        if self.infer_net is None:
            self.infer_net = L.bmpc_mlp_create(self.widths, self.max_batch)
        L.bmpc_mlp_set_params(self.infer_net, join_params(Ws, bs))
        L.bmpc_mlp_set_input_map(self.infer_net, self.x_mean, 1.0 / self.x_std)

    def predict(self, X_dev, Y_dev, stream=None):
        """Raw-unit outputs for raw features (float32 device tensors)."""
        L.bmpc_mlp_forward(self.infer_net, X_dev, Y_dev, stream)

    def loss(self, X, T):
        """Mean squared error of standardised targets on host data (X, T)."""
        import torch
        Xn = torch.from_numpy(((X - self.x_mean) / self.x_std).astype(np.float32)).cuda()
        Tn = torch.from_numpy(((T - self.t_mean) / self.t_std).astype(np.float32)).cuda()
        tot, cnt = 0.0, 0
        for j in range(0, Xn.shape[0], self.max_batch):
            xb, tb = Xn[j:j + self.max_batch].contiguous(), Tn[j:j + self.max_batch].contiguous()
            l, _ = L.bmpc_mlp_gradients(self.train_net, xb, tb)
            tot += l * xb.shape[0]
            cnt += xb.shape[0]
        return tot / cnt


def solve_with_network(pool, insts, starter, settings=None, guarded=True, feats=None, with_multipliers=True):
    """Predict start points for the problems loaded in the pool (instances
    `insts`, or raw feature rows `feats`) and solve them.  With `insts` the
    pool is loaded first.  The network runs in chunks of its batch limit.
    with_multipliers=False keeps only the predicted inputs (multipliers
    start at zero).  Returns (stats list, timing dict in ms: network
    inference, scatter + solve)."""
    import torch
    st = settings or L.bmpc_settings_default()
    if feats is None:
        pool.load(insts)
        feats = np.array([features(i) for i in insts])
    rows = len(feats)
    X = torch.from_numpy(np.asarray(feats, dtype=np.float32)).cuda()
    width = L.bmpc_problem_output_width(pool.handles[0])
    Y = torch.empty((rows, width), dtype=torch.float32, device="cuda")
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    torch.cuda.synchronize()
    e[0].record()
    for j in range(0, rows, starter.max_batch):
        starter.predict(X[j:j + starter.max_batch], Y[j:j + starter.max_batch])
    e[1].record()
    L.bmpc_batch_start_from_network(pool.batch, Y, rows, width)
    warm = 8 | (4 if with_multipliers else 0) | (GUARD_BIT if guarded else 0)
    L.bmpc_batch_launch(pool.batch, st, warm=warm)
    e[2].record()
    stats = L.bmpc_batch_stats(pool.batch, pool.size)[:rows]
    torch.cuda.synchronize()
    return stats, {"network_ms": e[0].elapsed_time(e[1]), "solve_ms": e[1].elapsed_time(e[2])}


def shifted_features(pool, insts):
    """Features of the pool's problems after bmpc_batch_shift: the advanced
    measured state with the instances' scenarios."""
    F = np.array([features(i) for i in insts])
    for k, h in enumerate(pool.handles[:len(insts)]):
        F[k, :4] = L.bmpc_problem_get_x0(h)
    return F
