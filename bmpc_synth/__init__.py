"""Seeded synthetic inputs for branch-MPC trees.

This module only *draws* problem data: tree topologies, scenario
probabilities, lane offsets, obstacle positions, random LQR matrices and
initial states.  It holds none of the solver's arithmetic (no weights
derived from probabilities, no references averaged over scenarios, no
Riccati, no dynamics).  Both the CPU oracle and the HIP path read the same
arrays from here.

Seeds: every instance uses NumPy PCG64 with seed ``1_000_003 * config +
instance``.  Per instance the draws happen in a fixed order: topology
parameters (batched workload only), lateral offset per scenario in leaf
order, Dirichlet(1) scenario probabilities, then one (ox, oy) per
obstacle-bearing segment in segment order.

Trees are produced in stage-major breadth-first order: ``parent[0] = -1``,
``parent[i] < i`` and ``parent`` is non-decreasing, so the nodes of one
stage are contiguous and the children of a node are contiguous.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_MUL = 1_000_003

# Bicycle-workload constants (kinematic bicycle, lane following, round obstacles).
WHEELBASE = 2.7
DT = 0.1
Q_DIAG = (1.0, 1.0, 0.1, 0.1)
R_DIAG = (0.1, 1.0)
A_MAX = 3.0
STEER_MAX = 0.5
OBS_RADIUS = 1.5
REF_SPEED = 10.0
X0_DEFAULT = (0.0, 0.0, 0.0, 8.0)


def rng_for(config: int, instance: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_MUL * int(config) + int(instance)))


# ----------------------------------------------------------------------------
# topology
# ----------------------------------------------------------------------------

def tree_parent(horizon: int, branch_stages, branch_factor: int) -> np.ndarray:
    """Parent array of a tree with control stages 0..horizon-1 and leaves at
    stage ``horizon``.  A node at a stage listed in ``branch_stages`` has
    ``branch_factor`` children, every other control node has one child."""
    bset = set(int(s) for s in branch_stages)
    parent = [-1]
    level = [0]
    for t in range(horizon):
        nxt = []
        nch = branch_factor if t in bset else 1
        for p in level:
            for _ in range(nch):
                parent.append(p)
                nxt.append(len(parent) - 1)
        level = nxt
    return np.asarray(parent, dtype=np.int32)


def stages_of(parent: np.ndarray) -> np.ndarray:
    st = np.zeros(len(parent), dtype=np.int32)
    for i in range(1, len(parent)):
        st[i] = st[parent[i]] + 1
    return st


def num_children(parent: np.ndarray) -> np.ndarray:
    nch = np.zeros(len(parent), dtype=np.int32)
    for i in range(1, len(parent)):
        nch[parent[i]] += 1
    return nch


def segments_of(parent: np.ndarray):
    """Maximal unbranched segments.  A segment starts at the root or at a child
    of a node with two or more children, follows single-child nodes and ends at
    a leaf or at a node with two or more children.  Returns
    ``seg_of_node`` (int32, N) and the list of segment start nodes in
    increasing node order (the segment order used for obstacle draws)."""
    n = len(parent)
    nch = num_children(parent)
    seg = np.full(n, -1, dtype=np.int32)
    starts = []
    for i in range(n):
        p = parent[i]
        if p < 0 or nch[p] != 1:
            seg[i] = len(starts)
            starts.append(i)
        else:
            seg[i] = seg[p]
    return seg, starts


# ----------------------------------------------------------------------------
# bicycle branch-MPC instances
# ----------------------------------------------------------------------------

@dataclass
class BicycleInstance:
    parent: np.ndarray            # int32 (N,)
    leaf_prob: np.ndarray         # float64 (Z,) scenario probabilities, leaf order
    leaf_offset: np.ndarray       # float64 (Z,) lateral lane offset per scenario
    obstacles: np.ndarray         # float64 (n_obs, 2) obstacle centres (ox, oy)
    node_obstacle: np.ndarray     # int32 (N,) obstacle index per node, -1 = none
    x0: np.ndarray                # float64 (4,)
    horizon: int
    dt: float = DT
    wheelbase: float = WHEELBASE
    q_diag: tuple = Q_DIAG
    r_diag: tuple = R_DIAG
    a_max: float = A_MAX
    steer_max: float = STEER_MAX
    obs_radius: float = OBS_RADIUS
    ref_speed: float = REF_SPEED
    meta: dict = field(default_factory=dict)

    @property
    def num_nodes(self) -> int:
        return int(len(self.parent))

    @property
    def leaves(self) -> np.ndarray:
        return np.nonzero(num_children(self.parent) == 0)[0].astype(np.int32)


def _bicycle_from_topology(rng, parent, horizon, x0, meta) -> BicycleInstance:
    nch = num_children(parent)
    leaves = np.nonzero(nch == 0)[0]
    z = len(leaves)
    offsets = rng.uniform(-2.0, 2.0, size=z)
    probs = rng.dirichlet(np.ones(z))
    seg, starts = segments_of(parent)
    # every segment except the one holding the root carries one obstacle
    obs_segments = [s for s in range(len(starts)) if starts[s] != 0]
    obstacles = np.empty((len(obs_segments), 2))
    seg_to_obs = np.full(len(starts), -1, dtype=np.int32)
    for k, s in enumerate(obs_segments):
        obstacles[k, 0] = rng.uniform(15.0, 40.0)
        obstacles[k, 1] = rng.uniform(-2.0, 2.0)
        seg_to_obs[s] = k
    node_obstacle = seg_to_obs[seg].astype(np.int32)
    return BicycleInstance(parent=parent, leaf_prob=probs, leaf_offset=offsets,
                           obstacles=obstacles, node_obstacle=node_obstacle,
                           x0=np.asarray(x0, dtype=np.float64), horizon=horizon,
                           meta=meta)


def single_bmpc(instance: int = 0, x0=X0_DEFAULT) -> BicycleInstance:
    """Single branch-MPC tree: horizon 20, trunk stages 0-4, node at stage 4
    branches into 3 (53 nodes: 50 control + 3 leaves)."""
    rng = rng_for(0, instance)
    parent = tree_parent(20, [4], 3)
    return _bicycle_from_topology(rng, parent, 20, x0, {"config": 0, "instance": instance})


def large_tree(instance: int = 0, x0=X0_DEFAULT) -> BicycleInstance:
    """Large tree: horizon 80, binary branching at stages 0, 5, ..., 55
    (4096 scenarios, 122,871 nodes, 8,191 segments)."""
    rng = rng_for(4, instance)
    parent = tree_parent(80, list(range(0, 60, 5)), 2)
    return _bicycle_from_topology(rng, parent, 80, x0, {"config": 4, "instance": instance})


def learned_topology_instance(instance: int, x0=None) -> BicycleInstance:
    """Warm-starter workload: horizon 30, 4 branches at stage 4 (109 nodes).
    ``x0`` defaults to a draw [0, U(-1,1), U(-0.2,0.2), U(6,10)]."""
    rng = rng_for(3, instance)
    if x0 is None:
        x0 = np.array([0.0, rng.uniform(-1, 1), rng.uniform(-0.2, 0.2), rng.uniform(6, 10)])
    parent = tree_parent(30, [4], 4)
    return _bicycle_from_topology(rng, parent, 30, x0, {"config": 3, "instance": instance})


def batched_instances(count: int = 512, x0=X0_DEFAULT):
    """Batched workload: per instance branches ~U{2..8} at a branch stage
    ~U{0..5}, horizon ~U{20..60}."""
    out = []
    for i in range(count):
        rng = rng_for(2, i)
        b = int(rng.integers(2, 9))
        s = int(rng.integers(0, 6))
        h = int(rng.integers(20, 61))
        parent = tree_parent(h, [s], b)
        out.append(_bicycle_from_topology(rng, parent, h, x0,
                                          {"config": 2, "instance": i, "b": b, "s": s, "H": h}))
    return out


def small_bicycle(horizon: int, branch_stages, branch_factor: int, seed: int,
                  x0=X0_DEFAULT) -> BicycleInstance:
    """Arbitrary small bicycle tree for tests (seed space of its own)."""
    rng = np.random.Generator(np.random.PCG64(7_000_001 + seed))
    parent = tree_parent(horizon, branch_stages, branch_factor)
    return _bicycle_from_topology(rng, parent, horizon, x0, {"seed": seed})


# ----------------------------------------------------------------------------
# random tree-LQR instances
# ----------------------------------------------------------------------------

@dataclass
class LqrInstance:
    parent: np.ndarray   # (N,)
    A: np.ndarray        # (N, nx, nx) dynamics of the edge into node i (row 0 unused)
    B: np.ndarray        # (N, nx, nu)
    c: np.ndarray        # (N, nx)
    Q: np.ndarray        # (N, nx, nx) stage cost (terminal cost at leaves)
    R: np.ndarray        # (N, nu, nu) (unused at leaves)
    M: np.ndarray        # (N, nu, nx) (unused at leaves)
    q: np.ndarray        # (N, nx)
    r: np.ndarray        # (N, nu)
    x0: np.ndarray       # (nx,)

    @property
    def nx(self):
        return self.A.shape[1]

    @property
    def nu(self):
        return self.B.shape[2]


def random_lqr(parent: np.ndarray, nx: int, nu: int, rng: np.random.Generator,
               a_scale: float = 0.1, r_scale: float = 0.1, random_cost: bool = False) -> LqrInstance:
    """Random tree LQR data.  Per edge: A = I + a_scale*N(0,1), B = N(0,1),
    c ~ N(0,1).  Per control node Q = I, R = r_scale*I, M = 0 (or, with
    ``random_cost``, random SPD Q, R and a random cross term M keeping the
    stage Hessian positive definite); q, r ~ N(0,1).  Leaves: Q_f = I
    (or random SPD), q_f ~ N(0,1).  x0 ~ N(0,1)."""
    n = len(parent)
    A = np.eye(nx)[None] + a_scale * rng.standard_normal((n, nx, nx))
    B = rng.standard_normal((n, nx, nu))
    c = rng.standard_normal((n, nx))
    A[0] = 0.0
    B[0] = 0.0
    c[0] = 0.0
    if random_cost:
        Q = np.empty((n, nx, nx))
        R = np.empty((n, nu, nu))
        M = np.empty((n, nu, nx))
        for i in range(n):
            G = rng.standard_normal((nx + nu, nx + nu))
            H = G @ G.T / (nx + nu) + 0.5 * np.eye(nx + nu)
            Q[i] = H[:nx, :nx]
            R[i] = H[nx:, nx:]
            M[i] = H[nx:, :nx]
    else:
        Q = np.broadcast_to(np.eye(nx), (n, nx, nx)).copy()
        R = np.broadcast_to(r_scale * np.eye(nu), (n, nu, nu)).copy()
        M = np.zeros((n, nu, nx))
    q = rng.standard_normal((n, nx))
    r = rng.standard_normal((n, nu))
    x0 = rng.standard_normal(nx)
    leaves = num_children(parent) == 0
    R[leaves] = 0.0
    M[leaves] = 0.0
    r[leaves] = 0.0
    return LqrInstance(parent=np.asarray(parent, np.int32), A=A, B=B, c=c, Q=Q, R=R, M=M,
                       q=q, r=r, x0=x0)


def lqr_microbench(instance: int = 0) -> LqrInstance:
    """Tree-Riccati microbenchmark: nx=12, nu=4, horizon 40, binary branching
    at stages 0, 4, ..., 36 (1024 scenarios, 8,185 nodes)."""
    rng = rng_for(1, instance)
    parent = tree_parent(40, list(range(0, 40, 4)), 2)
    return random_lqr(parent, 12, 4, rng)


def lqr_on(parent, nx, nu, seed, **kw) -> LqrInstance:
    rng = np.random.Generator(np.random.PCG64(9_000_011 + seed))
    return random_lqr(np.asarray(parent, np.int32), nx, nu, rng, **kw)


# ----------------------------------------------------------------------------
# chain of masses and springs (tree LQR with per-scenario dynamics)
# ----------------------------------------------------------------------------

MS_DT = 0.5          # sampling time of the discretised chain
MS_K_RANGE = (0.5, 1.5)   # sampled spring constants (nominal 1)


def mass_spring_matrices(M: int, k: float, dt: float = MS_DT, mass: float = 1.0):
    """Discrete-time matrices of a chain of M equal masses joined by springs
    of constant k, with walls at both ends (M + 1 springs) and M - 1
    actuators, actuator i pushing mass i and mass i + 1 apart.  State
    [positions (M), velocities (M)], input the M - 1 actuator forces.  The
    continuous model  p' = v,  v' = (k/m) L p + (1/m) E u  (L tridiagonal
    1, -2, 1) is held over dt (zero-order hold, matrix exponential of the
    augmented system).  These matrices are data of the tree LQR, the model
    a user would pass."""
    from scipy.linalg import expm
    nx, nu = 2 * M, M - 1
    Lm = -2.0 * np.eye(M) + np.eye(M, k=1) + np.eye(M, k=-1)
    E = np.zeros((M, nu))
    for i in range(nu):
        E[i, i] = -1.0
        E[i + 1, i] = 1.0
    Ac = np.zeros((nx, nx))
    Ac[:M, M:] = np.eye(M)
    Ac[M:, :M] = (k / mass) * Lm
    Bc = np.zeros((nx, nu))
    Bc[M:, :] = E / mass
    aug = np.zeros((nx + nu, nx + nu))
    aug[:nx, :nx] = Ac
    aug[:nx, nx:] = Bc
    ex = expm(aug * dt)
    return ex[:nx, :nx], ex[:nx, nx:]


def mass_spring_tree(M: int = 15, robust_horizon: int = 10, n_d: int = 2, horizon: int = 40,
                     instance: int = 0, random_terms: bool = False) -> LqrInstance:
    """Tree LQR of the mass-spring chain under spring-constant uncertainty:
    n_d spring constants are drawn from U[0.5, 1.5]; every node of the first
    ``robust_horizon`` stages branches into n_d children, child d taking
    constant k_d for its incoming edge and every edge below it (so there are
    Z = n_d ** robust_horizon scenarios); ``horizon`` control stages and
    leaves at stage ``horizon``.  Costs Q = I, R = I, M = 0 at every control
    node and Q_f = I at the leaves; the initial state draws positions and
    velocities from U[-1, 1].  Linear terms and defects are zero, or with
    ``random_terms`` N(0, 1) (q, r per control node, q_f per leaf, c per
    edge).  Draw order: the n_d constants, then x0, then the linear terms."""
    rng = rng_for(5, instance)
    ks = rng.uniform(MS_K_RANGE[0], MS_K_RANGE[1], size=n_d)
    parent = tree_parent(horizon, list(range(robust_horizon)), n_d)
    N = len(parent)
    nx, nu = 2 * M, M - 1
    mats = [mass_spring_matrices(M, k) for k in ks]
    # branch index of each node: its rank among its siblings where its
    # parent branches, else its parent's
    nch = num_children(parent)
    branch = np.zeros(N, dtype=np.int64)
    first = {}
    for j in range(1, N):
        p = parent[j]
        if nch[p] > 1:
            first.setdefault(p, j)
            branch[j] = j - first[p]
        else:
            branch[j] = branch[p]
    A = np.empty((N, nx, nx))
    B = np.empty((N, nx, nu))
    for d in range(n_d):
        sel = branch == d
        A[sel] = mats[d][0]
        B[sel] = mats[d][1]
    A[0] = 0.0
    B[0] = 0.0
    Q = np.broadcast_to(np.eye(nx), (N, nx, nx)).copy()
    R = np.broadcast_to(np.eye(nu), (N, nu, nu)).copy()
    Mx = np.zeros((N, nu, nx))
    x0 = rng.uniform(-1.0, 1.0, size=nx)
    if random_terms:
        q = rng.standard_normal((N, nx))
        r = rng.standard_normal((N, nu))
        c = rng.standard_normal((N, nx))
        c[0] = 0.0
    else:
        q, r, c = np.zeros((N, nx)), np.zeros((N, nu)), np.zeros((N, nx))
    leaves = nch == 0
    R[leaves] = 0.0
    r[leaves] = 0.0
    return LqrInstance(parent=parent, A=A, B=B, c=c, Q=Q, R=R, M=Mx, q=q, r=r, x0=x0)
