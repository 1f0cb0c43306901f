"""Seeded synthetic workloads for DLMPC (networks, plant parameters, cost, bounds, x0).

This module holds no part of the DLMPC method's arithmetic: it only draws the networked
linear plant ``x_{t+1} = A x_t + B u_t`` (Section II-A, eq. (MPC)), its interconnection
graph G_(A,B), the quadratic cost and box constraints, and initial conditions. Both the
HIP path (through the C ABI) and the CPU oracle consume what it returns, so it depends on
nothing but NumPy and imports neither of them.

Plant ("swing" network of 2-state nodes, one input each; theta = angle, omega = frequency):

    A_ii = [[1, dt], [-(k_i/m_i) dt, 1 - (d_i/m_i) dt]],   A_ij = [[0, 0], [(k_ij/m_i) dt, 0]]
    B_i  = [0, dt]^T,   dt = 0.2,   1/m_i ~ U[0, 2],   d_i ~ U[0.5, 1],   k_ij = k_ji ~ U[0.5, 1]

with k_i the sum of k_ij over the neighbours of i (Laplacian coupling). The paper's
evaluation uses synthetic chain networks of 2-state nodes (Section IV-A); the grid and
irregular-mesh topologies and the swing parameters follow the workload definitions this
project is measured on.

The paper's own evaluation plant (Section IV-A) is ``paper_chain``: a chain of 2-state nodes
with A_ii = [[1, 0.1], [-0.3, 0.7]], A_ij = [[0, 0], [0.1, 0.1]] for the chain neighbours,
B_ii = I (two inputs per node, as the printed matrix says; the text's count of one input per
node would need a 2x1 block the paper does not give), Q = I, R = I and
-0.2 <= x_{i,1} <= 1.2 on the first state of every node for t >= 1.

Every random draw goes through ``numpy.random.default_rng(seed)`` in a fixed order, so a
(topology, seed) pair always yields the same plant.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

DT = 0.2
NX = 2  # states per subsystem: (theta, omega)
NU = 1  # inputs per subsystem


@dataclass
class Network:
    """A networked LTI plant in subsystem-block form.

    ``edges`` is the sorted list of undirected edges (i < j). ``a_rowptr``/``a_colidx``/
    ``a_blocks`` are block-CSR over subsystems (diagonal included, columns ascending),
    ``b_blocks`` the diagonal input blocks, shape ``[N, nx, nu]``.
    """

    name: str
    n_sub: int
    nx: int
    nu: int
    edges: np.ndarray  # [E, 2] int64, i < j
    a_rowptr: np.ndarray  # [N+1] int64
    a_colidx: np.ndarray  # [nnzb] int32
    a_blocks: np.ndarray  # [nnzb, nx, nx] float64
    b_blocks: np.ndarray  # [N, nx, nu] float64
    meta: dict = field(default_factory=dict)

    def dense_A(self) -> np.ndarray:
        n, nx = self.n_sub, self.nx
        A = np.zeros((n * nx, n * nx))
        for i in range(n):
            for p in range(self.a_rowptr[i], self.a_rowptr[i + 1]):
                j = int(self.a_colidx[p])
                A[i * nx:(i + 1) * nx, j * nx:(j + 1) * nx] = self.a_blocks[p]
        return A

    def dense_B(self) -> np.ndarray:
        n, nx, nu = self.n_sub, self.nx, self.nu
        B = np.zeros((n * nx, n * nu))
        for i in range(n):
            B[i * nx:(i + 1) * nx, i * nu:(i + 1) * nu] = self.b_blocks[i]
        return B


@dataclass
class Cost:
    """Diagonal stage weights and box bounds (``None`` = unbounded).

    ``q_diag`` weights every state row x_0..x_{T-1}; ``r_diag`` every input row
    u_0..u_{T-2}. State bounds apply at t = 1..T-1 and input bounds at t = 0..T-2.
    """

    q_diag: np.ndarray
    r_diag: np.ndarray
    x_lo: np.ndarray | None = None
    x_hi: np.ndarray | None = None
    u_lo: np.ndarray | None = None
    u_hi: np.ndarray | None = None

    @property
    def constrained(self) -> bool:
        return any(v is not None for v in (self.x_lo, self.x_hi, self.u_lo, self.u_hi))


# ----------------------------------------------------------------------------- topologies

def chain_edges(n: int) -> np.ndarray:
    return np.array([(i, i + 1) for i in range(n - 1)], dtype=np.int64).reshape(-1, 2)


def grid_edges(rows: int, cols: int) -> np.ndarray:
    e = []
    for r in range(rows):
        for c in range(cols):
            v = r * cols + c
            if c + 1 < cols:
                e.append((v, v + 1))
            if r + 1 < rows:
                e.append((v, v + cols))
    return np.array(sorted(e), dtype=np.int64)


def irregular_mesh_edges(rows: int, cols: int, seed: int, drop_frac: float = 0.30,
                         chord_frac: float = 0.05) -> np.ndarray:
    """Grid with a share of edges dropped (never disconnecting it) plus random chords.

    A random spanning tree of the grid (Kruskal over a random edge order) is kept intact;
    ``round(drop_frac * E)`` of the remaining grid edges are removed uniformly at random, then
    ``round(chord_frac * N)`` chords are added between uniformly drawn non-adjacent pairs.
    """
    rng = np.random.default_rng(seed)
    n = rows * cols
    grid = grid_edges(rows, cols)
    order = rng.permutation(len(grid))
    parent = list(range(n))

    def find(a: int) -> int:
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    tree = np.zeros(len(grid), dtype=bool)
    for idx in order:
        a, b = (int(v) for v in grid[idx])
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[ra] = rb
            tree[idx] = True
    non_tree = np.flatnonzero(~tree)
    n_drop = int(round(drop_frac * len(grid)))
    if n_drop > len(non_tree):
        raise ValueError("cannot drop that many edges and stay connected")
    drop = set(int(v) for v in rng.choice(non_tree, size=n_drop, replace=False))
    kept = {(int(a), int(b)) for k, (a, b) in enumerate(grid) if k not in drop}
    n_chord = int(round(chord_frac * n))
    while n_chord > 0:
        a, b = (int(v) for v in rng.integers(0, n, size=2))
        if a == b:
            continue
        key = (min(a, b), max(a, b))
        if key in kept:
            continue
        kept.add(key)
        n_chord -= 1
    return np.array(sorted(kept), dtype=np.int64)


# ----------------------------------------------------------------------------- plants

def swing_network(name: str, n: int, edges: np.ndarray, seed: int, dt: float = DT) -> Network:
    """Swing-equation network on a given undirected edge list (see module docstring)."""
    rng = np.random.default_rng(seed)
    inv_m = rng.uniform(0.0, 2.0, size=n)
    damp = rng.uniform(0.5, 1.0, size=n)
    k_edge = rng.uniform(0.5, 1.0, size=len(edges))
    nbr: list[dict[int, float]] = [dict() for _ in range(n)]
    for (a, b), k in zip(edges, k_edge):
        nbr[int(a)][int(b)] = float(k)
        nbr[int(b)][int(a)] = float(k)
    rowptr = [0]
    colidx: list[int] = []
    blocks: list[np.ndarray] = []
    for i in range(n):
        k_i = sum(nbr[i].values())
        for j in sorted(set(nbr[i]) | {i}):
            if j == i:
                blk = np.array([[1.0, dt], [-(k_i * inv_m[i]) * dt, 1.0 - damp[i] * inv_m[i] * dt]])
            else:
                blk = np.array([[0.0, 0.0], [nbr[i][j] * inv_m[i] * dt, 0.0]])
            colidx.append(j)
            blocks.append(blk)
        rowptr.append(len(colidx))
    b = np.zeros((n, NX, NU))
    b[:, 1, 0] = dt
    return Network(name=name, n_sub=n, nx=NX, nu=NU, edges=np.asarray(edges, dtype=np.int64),
                   a_rowptr=np.array(rowptr, dtype=np.int64),
                   a_colidx=np.array(colidx, dtype=np.int32),
                   a_blocks=np.array(blocks, dtype=np.float64).reshape(-1, NX, NX), b_blocks=b,
                   meta={"seed": seed, "dt": dt})


def paper_chain(n: int) -> Network:
    """The paper's chain plant (Section IV-A; see the module docstring): no random draw."""
    edges = chain_edges(n)
    a_ii = np.array([[1.0, 0.1], [-0.3, 0.7]])
    a_ij = np.array([[0.0, 0.0], [0.1, 0.1]])
    rowptr, colidx, blocks = [0], [], []
    for i in range(n):
        for j in sorted({i, i - 1, i + 1} & set(range(n))):
            colidx.append(j)
            blocks.append(a_ii if j == i else a_ij)
        rowptr.append(len(colidx))
    b = np.broadcast_to(np.eye(2), (n, 2, 2)).copy()
    return Network(name=f"paper_chain{n}", n_sub=n, nx=2, nu=2, edges=np.asarray(edges, dtype=np.int64),
                   a_rowptr=np.array(rowptr, dtype=np.int64), a_colidx=np.array(colidx, dtype=np.int32),
                   a_blocks=np.array(blocks, dtype=np.float64).reshape(-1, 2, 2), b_blocks=b, meta={})


def paper_cost(net: Network, lo: float = -0.2, hi: float = 1.2) -> Cost:
    """Q = I, R = I, lo <= x_{i,1} <= hi (the first state of every node), inputs unbounded."""
    c = unit_cost(net)
    nxs = net.n_sub * net.nx
    x_lo, x_hi = np.full(nxs, -np.inf), np.full(nxs, np.inf)
    x_lo[0::net.nx], x_hi[0::net.nx] = lo, hi
    c.x_lo, c.x_hi = x_lo, x_hi
    return c


def line_limits(net: Network, T: int, limit: float, t0: int = 2) -> tuple:
    """Couplings lo <= x_{i,1}(t) - x_{j,1}(t) <= hi with lo = -limit, hi = limit for every edge
    (i < j) and t = t0..T-1 (first state of each node; on the swing network the angle difference
    of a line, whose flow it sets). Returns (ra, rb, lo, hi) in the canonical row order (state
    rows x_t subsystem-major). On the swing plant the angles at t = 1 follow from x0 alone, so
    the default starts at t = 2."""
    Nx = net.n_sub * net.nx
    ra, rb = [], []
    for t in range(t0, T):
        for i, j in net.edges:
            ra.append(t * Nx + int(i) * net.nx)
            rb.append(t * Nx + int(j) * net.nx)
    n = len(ra)
    return (np.array(ra, dtype=np.int64), np.array(rb, dtype=np.int64), np.full(n, -float(limit)),
            np.full(n, float(limit)))


def chain(n: int, seed: int = 0) -> Network:
    return swing_network(f"chain{n}", n, chain_edges(n), seed)


def grid(rows: int, cols: int | None = None, seed: int = 0) -> Network:
    cols = rows if cols is None else cols
    return swing_network(f"grid{rows}x{cols}", rows * cols, grid_edges(rows, cols), seed)


def irregular_mesh(rows: int = 32, cols: int = 32, seed: int = 0) -> Network:
    e = irregular_mesh_edges(rows, cols, seed)
    return swing_network(f"irregular{rows}x{cols}", rows * cols, e, seed)


def generic_network(n: int, edges: np.ndarray, nx: int, nu: int, seed: int,
                    scale: float = 0.3) -> Network:
    """Random dense-block plant on a given graph (for shape and edge-case tests).

    Every nonzero block is drawn i.i.d. normal; ``A_ii`` is shifted by the identity so
    the plant is not trivially nilpotent. B blocks are i.i.d. normal ``nx x nu``.
    """
    rng = np.random.default_rng(seed)
    nbr: list[set[int]] = [set() for _ in range(n)]
    for a, b in edges:
        nbr[int(a)].add(int(b))
        nbr[int(b)].add(int(a))
    rowptr = [0]
    colidx: list[int] = []
    blocks = []
    for i in range(n):
        for j in sorted(nbr[i] | {i}):
            blk = scale * rng.standard_normal((nx, nx))
            if j == i:
                blk += np.eye(nx)
            colidx.append(j)
            blocks.append(blk)
        rowptr.append(len(colidx))
    b = rng.standard_normal((n, nx, nu))
    return Network(name=f"generic{n}", n_sub=n, nx=nx, nu=nu, edges=np.asarray(edges, np.int64),
                   a_rowptr=np.array(rowptr, dtype=np.int64), a_colidx=np.array(colidx, np.int32),
                   a_blocks=np.array(blocks, dtype=np.float64).reshape(-1, nx, nx), b_blocks=b,
                   meta={"seed": seed})


# ----------------------------------------------------------------------------- cost, x0

def unit_cost(net: Network) -> Cost:
    return Cost(q_diag=np.ones(net.n_sub * net.nx), r_diag=np.ones(net.n_sub * net.nu))


def box_cost(net: Network, theta_max: float = 0.8, u_max: float = 2.0) -> Cost:
    """Q = I, R = I, |theta_i| <= theta_max (state 0 of every node), |u_i| <= u_max."""
    c = unit_cost(net)
    nxs = net.n_sub * net.nx
    x_hi = np.full(nxs, np.inf)
    x_hi[0::net.nx] = theta_max
    c.x_lo, c.x_hi = -x_hi, x_hi
    c.u_hi = np.full(net.n_sub * net.nu, u_max)
    c.u_lo = -c.u_hi
    return c


def x0(net: Network, seed: int, sigma: float = 1.0) -> np.ndarray:
    """x0 = sigma * z, z ~ N(0, I), drawn from ``default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    return sigma * rng.standard_normal(net.n_sub * net.nx)


# ----------------------------------------------------------------------------- configs

@dataclass
class Workload:
    name: str
    net: Network
    d: int
    T: int
    cost: Cost
    sigma: float
    rho: float = 5.0
    eps: float = 1e-4
    max_iter: int = 500

    def x0(self, seed: int) -> np.ndarray:
        """sigma * z with z ~ N(0, I) from ``default_rng(seed)``; on a constrained workload a
        draw whose uncontrollable first step leaves the box (see ``first_step_outside_box``)
        is replaced by the next draw of the same generator, so every returned x0 passes that
        check and a draw that passes is returned unchanged."""
        if not self.cost.constrained:
            return x0(self.net, seed, self.sigma)
        rng = np.random.default_rng(seed)
        for _ in range(1000):
            v = self.sigma * rng.standard_normal(self.net.n_sub * self.net.nx)
            if not first_step_outside_box(self.net, self.cost, v):
                return v
        raise RuntimeError(f"no x0 within the box after 1000 draws (seed {seed})")


def first_step_outside_box(net: Network, cost: Cost, x: np.ndarray) -> bool:
    """True if some state that no input reaches in one step (a zero row of B) leaves its bound
    at t = 1: x_s(1) = (A x)_s for such a state whatever u(0) is, so the instance of eq. (MPC)
    is infeasible. (On the swing plant this is theta_i(1) = theta_i(0) + dt omega_i(0).)"""
    if cost.x_lo is None and cost.x_hi is None:
        return False
    free, A = _free_rows(net)
    if not free.any():
        return False
    ax = A[free] @ x
    lo = -np.inf if cost.x_lo is None else np.asarray(cost.x_lo)[free]
    hi = np.inf if cost.x_hi is None else np.asarray(cost.x_hi)[free]
    return bool(np.any((ax < lo) | (ax > hi)))


def _free_rows(net: Network):
    """(mask of the state rows with a zero row of B, A as a sparse matrix), cached per network."""
    cached = net.meta.get("_free_rows")
    if cached is None:
        from scipy.sparse import csr_matrix
        n, nx = net.n_sub, net.nx
        rows, cols, vals = [], [], []
        for i in range(n):
            for p in range(net.a_rowptr[i], net.a_rowptr[i + 1]):
                j = int(net.a_colidx[p])
                for r in range(nx):
                    for c in range(nx):
                        rows.append(i * nx + r)
                        cols.append(j * nx + c)
                        vals.append(net.a_blocks[p][r, c])
        A = csr_matrix((vals, (rows, cols)), shape=(n * nx, n * nx))
        free = ~np.any(net.b_blocks != 0, axis=2).reshape(-1)
        cached = (free, A)
        net.meta["_free_rows"] = cached
    return cached


# Scale of x0 for the box-constrained workloads. With |theta| <= 0.8 and x0 ~ N(0, 1) the
# first-step angle theta_i(1) = theta_i(0) + dt * omega_i(0) cannot be influenced by any
# input and violates the bound at roughly 43% of nodes, so such instances are infeasible;
# x0 is therefore drawn as sigma * N(0, I) for these workloads.
CONSTRAINED_SIGMA = {"grid16": 0.2, "irregular32": 0.15}


def paper_workload(n: int, d: int = 1, T: int = 5, sigma: float = 1.0) -> Workload:
    """The paper's chain plant and cost (Section IV-A) with N = n, locality d and horizon T;
    x0 = sigma * N(0, I) (the paper does not state its initial conditions)."""
    net = paper_chain(n)
    return Workload(f"paper_chain{n}_d{d}_T{T}", net, d=d, T=T, cost=paper_cost(net), sigma=sigma)


def workload(name: str) -> Workload:
    """Named workloads (parameter seed 0 for every network)."""
    if name == "chain10":
        net = chain(10)
        return Workload(name, net, d=1, T=5, cost=unit_cost(net), sigma=1.0)
    if name == "grid16_box":
        net = grid(16)
        return Workload(name, net, d=2, T=10, cost=box_cost(net), sigma=CONSTRAINED_SIGMA["grid16"])
    if name == "grid16":
        net = grid(16)
        return Workload(name, net, d=2, T=10, cost=unit_cost(net), sigma=1.0)
    if name == "irregular1024_box":
        net = irregular_mesh(32, 32, 0)
        return Workload(name, net, d=3, T=15, cost=box_cost(net),
                        sigma=CONSTRAINED_SIGMA["irregular32"])
    if name == "irregular1024":
        net = irregular_mesh(32, 32, 0)
        return Workload(name, net, d=3, T=15, cost=unit_cost(net), sigma=1.0)
    if name.startswith("paper_chain"):  # paper_chain<N>[_d<d>_T<T>]
        parts = name[len("paper_chain"):].split("_")
        kw = {p[0]: int(p[1:]) for p in parts[1:]}
        return paper_workload(int(parts[0]), d=kw.get("d", 1), T=kw.get("T", 5))
    if name in ("grid8", "grid32"):
        side = int(name[4:])
        net = grid(side)
        return Workload(name, net, d=2, T=10, cost=unit_cost(net), sigma=1.0)
    raise KeyError(name)
