"""Dense reference solvers used to pin the oracle (test helpers).

Nothing here uses a Riccati recursion: the tree QP is assembled as one dense
KKT system and solved by LU, and the scenario form duplicates every path
with explicit nonanticipativity rows.
"""
from __future__ import annotations

import numpy as np


def children_counts(parent):
    nch = np.zeros(len(parent), dtype=int)
    for i in range(1, len(parent)):
        nch[parent[i]] += 1
    return nch


def dense_tree_qp(parent, A, B, c, Q, R, M, q, r, x0):
    """Solve the equality-constrained tree QP by one dense KKT solve.

    Returns x (N, nx), u (N, nu; zero at leaves) and lam (N, nx), the
    multipliers of x_j = A_j x_p + B_j u_p + c_j in the convention
    L = cost + lam^T (A x + B u + c - x)."""
    N = len(parent)
    nx = A.shape[1]
    nu = B.shape[2]
    nch = children_counts(parent)
    ctrl = np.nonzero(nch > 0)[0]
    uidx = {int(n): i for i, n in enumerate(ctrl)}
    nv = N * nx + len(ctrl) * nu
    ne = N * nx

    def X(i):
        return slice(i * nx, (i + 1) * nx)

    def U(n):
        k = uidx[int(n)]
        return slice(N * nx + k * nu, N * nx + (k + 1) * nu)

    H = np.zeros((nv, nv))
    g = np.zeros(nv)
    for i in range(N):
        H[X(i), X(i)] += Q[i]
        g[X(i)] += q[i]
        if nch[i] > 0:
            H[U(i), U(i)] += R[i]
            H[U(i), X(i)] += M[i]
            H[X(i), U(i)] += M[i].T
            g[U(i)] += r[i]
    Aeq = np.zeros((ne, nv))
    b = np.zeros(ne)
    Aeq[X(0), X(0)] = np.eye(nx)
    b[X(0)] = x0
    for j in range(1, N):
        p = parent[j]
        Aeq[X(j), X(j)] = np.eye(nx)
        Aeq[X(j), X(p)] = -A[j]
        Aeq[X(j), U(p)] = -B[j]
        b[X(j)] = c[j]
    K = np.block([[H, Aeq.T], [Aeq, np.zeros((ne, ne))]])
    sol = np.linalg.solve(K, np.concatenate([-g, b]))
    z = sol[:nv]
    nu_ = sol[nv:]
    x = z[: N * nx].reshape(N, nx)
    u = np.zeros((N, nu))
    for n in ctrl:
        u[n] = z[U(n)]
    # KKT row of x_j: grad + nu_j - ... ; lam = -nu in the (f - x) convention
    lam = -nu_.reshape(N, nx)
    return x, u, lam


def scenario_qp(parent, A, B, c, Q, R, M, q, r, x0, leaf_weight):
    """Scenario form: one full copy of every root-to-leaf path, node costs
    split between the copies of a node in proportion to ``leaf_weight``, and
    explicit nonanticipativity rows u^s_n = u^{s'}_n for copies of one node.

    Returns per-scenario inputs as a dict {(leaf, node): u}."""
    N = len(parent)
    nx = A.shape[1]
    nu = B.shape[2]
    nch = children_counts(parent)
    leaves = [i for i in range(N) if nch[i] == 0]
    paths = []
    for l in leaves:
        p = [l]
        while parent[p[-1]] >= 0:
            p.append(parent[p[-1]])
        paths.append(p[::-1])
    # node weight = sum of leaf weights through the node
    below = {}
    for s, path in enumerate(paths):
        for n in path:
            below.setdefault(n, []).append(s)
    wsum = {n: sum(leaf_weight[s] for s in ss) for n, ss in below.items()}
    # variable layout per scenario: x for every path node, u for every control node
    off = []
    nv = 0
    for path in paths:
        off.append(nv)
        nv += len(path) * nx + (len(path) - 1) * nu

    def xs(s, t):
        return slice(off[s] + t * nx, off[s] + (t + 1) * nx)

    def us(s, t):
        L = len(paths[s])
        base = off[s] + L * nx
        return slice(base + t * nu, base + (t + 1) * nu)

    H = np.zeros((nv, nv))
    g = np.zeros(nv)
    rows = []
    rhs = []
    for s, path in enumerate(paths):
        for t, n in enumerate(path):
            f = leaf_weight[s] / wsum[n]
            H[xs(s, t), xs(s, t)] += f * Q[n]
            g[xs(s, t)] += f * q[n]
            if t < len(path) - 1:
                H[us(s, t), us(s, t)] += f * R[n]
                H[us(s, t), xs(s, t)] += f * M[n]
                H[xs(s, t), us(s, t)] += f * M[n].T
                g[us(s, t)] += f * r[n]
        # x_0 = x0
        row = np.zeros((nx, nv))
        row[:, xs(s, 0)] = np.eye(nx)
        rows.append(row)
        rhs.append(np.asarray(x0, float))
        for t in range(1, len(path)):
            j = path[t]
            row = np.zeros((nx, nv))
            row[:, xs(s, t)] = np.eye(nx)
            row[:, xs(s, t - 1)] = -A[j]
            row[:, us(s, t - 1)] = -B[j]
            rows.append(row)
            rhs.append(c[j])
    # nonanticipativity on inputs of shared control nodes
    for n, ss in below.items():
        if nch[n] == 0 or len(ss) < 2:
            continue
        t = paths[ss[0]].index(n)
        for s2 in ss[1:]:
            row = np.zeros((nu, nv))
            row[:, us(ss[0], t)] = np.eye(nu)
            row[:, us(s2, t)] = -np.eye(nu)
            rows.append(row)
            rhs.append(np.zeros(nu))
    Aeq = np.vstack(rows)
    b = np.concatenate(rhs)
    ne = Aeq.shape[0]
    K = np.block([[H, Aeq.T], [Aeq, np.zeros((ne, ne))]])
    sol = np.linalg.lstsq(K, np.concatenate([-g, b]), rcond=None)[0]
    z = sol[:nv]
    out = {}
    for s, path in enumerate(paths):
        for t, n in enumerate(path[:-1]):
            out[(leaves[s], n)] = z[us(s, t)]
    return out
