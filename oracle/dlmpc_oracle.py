"""Plain FP64 CPU oracle of DLMPC-ADMM — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import this module. The product path (the HIP library and its Python binding) never calls it
and shares no code with it; the two meet only in the seeded inputs.

What it computes (Amo Alonso & Tseng, "Effective GPU Parallelization of Distributed and
Localized MPC", Section II-A):

* eq. (MPC): minimise sum_t x_t' Q x_t + u_t' R u_t over a horizon, with the dynamics
  x_{t+1} = A x_t + B u_t, box bounds, and d-locality according to the graph G_(A,B);
* the SLS parametrisation (Section II-A): the decision variable is a matrix Phi with
  N_x*T + N_u*(T-1) rows (every state has T rows, every input T-1) and N_x columns, and
  locality becomes a sparsity pattern on Phi;
* Algorithm 2 (ADMM sketch): Phi-comp row by row, Psi-comp column by column,
  Lambda <- Lambda + Phi - Psi, then the convergence check, repeated until it passes.

The paper defers the formulas of each step to its references. This module uses the
following readings (each is listed with its reason in the design notes):

* horizon: state rows x_0..x_{T-1}, input rows u_0..u_{T-2} (the row counts of Phi);
* locality: Phi[r, c] may be nonzero iff hop(sub(r), sub(c)) <= d (Lemma 1 counts nodes
  within d hops);
* achievability: Z_AB Phi = I with Z_AB the block-bidiagonal SLS operator,
  block row 0: Phi_x[0] = I; block row t >= 1: Phi_x[t] - A Phi_x[t-1] - B Phi_u[t-1] = 0;
* cost per row r: w_r (phi_r . x0)^2 with w = diag(Q) / diag(R) on every row;
* scaled-form ADMM with penalty (rho/2)||Phi - Psi + Lambda||_F^2, matching the dual update
  of Algorithm 2; Phi-comp minimises w (phi.x)^2 + (rho/2)||phi - v||^2 with v = Psi - Lambda
  on the row's support, subject to lb <= phi.x <= ub on bounded rows (an exact per-row clip,
  since the problem is a one-dimensional convex quadratic in s = phi.x);
* Psi-comp: the Euclidean projection of (Phi + Lambda)[:, c] onto {psi : Z_AB psi = e_c,
  psi supported on the d-hop rows of column c}, i.e. psi = P_j v + o_c with
  P_j = I - H_j^+ H_j and o_c = H_j^+ e_c, H_j the block of Z_AB on that support;
* convergence: for every column c, ||Phi[:,c] - Psi[:,c]|| <= eps and
  ||Psi^{k+1}[:,c] - Psi^k[:,c]|| <= eps (absolute, 2-norm over the column);
* cold start Psi^0 = Lambda^0 = 0; u(0) and the objective are read from Phi at the stopping
  iterate.

Everything is dense FP64 NumPy on R x N_x matrices whose entries outside the locality
pattern are kept at zero; that is slow and obviously equivalent to the sparse definition.
"""
from __future__ import annotations

from collections import deque
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

FEASIBILITY_TOL = 1e-10


# --------------------------------------------------------------------- graph and locality

def interconnection_graph(A: np.ndarray, n_sub: int, nx: int) -> list[set[int]]:
    """Undirected G_(A,B): subsystems i != j are adjacent iff block A_ij or A_ji is nonzero."""
    adj: list[set[int]] = [set() for _ in range(n_sub)]
    for i in range(n_sub):
        for j in range(n_sub):
            if i != j and np.any(A[i * nx:(i + 1) * nx, j * nx:(j + 1) * nx] != 0):
                adj[i].add(j)
                adj[j].add(i)
    return adj


def hop_distances(adj: list[set[int]]) -> np.ndarray:
    """All-pairs hop counts by breadth-first search (-1 = unreachable)."""
    n = len(adj)
    dist = -np.ones((n, n), dtype=np.int64)
    for s in range(n):
        dist[s, s] = 0
        q = deque([s])
        while q:
            u = q.popleft()
            for v in adj[u]:
                if dist[s, v] < 0:
                    dist[s, v] = dist[s, u] + 1
                    q.append(v)
    return dist


@dataclass
class Layout:
    """Canonical row order of Phi: x_t blocks t = 0..T-1, then u_t blocks t = 0..T-2,
    subsystem-major inside a block. Columns are the N_x components of x0."""

    n_sub: int
    nx: int
    nu: int
    T: int

    @property
    def Nx(self) -> int:
        return self.n_sub * self.nx

    @property
    def Nu(self) -> int:
        return self.n_sub * self.nu

    @property
    def R(self) -> int:
        return self.Nx * self.T + self.Nu * (self.T - 1)

    def sub_of_row(self) -> np.ndarray:
        x_part = np.tile(np.repeat(np.arange(self.n_sub), self.nx), self.T)
        u_part = np.tile(np.repeat(np.arange(self.n_sub), self.nu), self.T - 1)
        return np.concatenate([x_part, u_part])

    def sub_of_col(self) -> np.ndarray:
        return np.repeat(np.arange(self.n_sub), self.nx)

    def u0_rows(self) -> np.ndarray:
        return self.Nx * self.T + np.arange(self.Nu)


def locality_mask(dist: np.ndarray, d: int, lay: Layout) -> np.ndarray:
    """Boolean R x N_x pattern L_d: entry allowed iff hop(sub(r), sub(c)) in [0, d]."""
    dr = dist[np.ix_(lay.sub_of_row(), lay.sub_of_col())]
    return (dr >= 0) & (dr <= d)


# --------------------------------------------------------------------- achievability

def build_zab(A: np.ndarray, B: np.ndarray, T: int) -> sp.csr_matrix:
    """SLS achievability operator Z_AB (N_x*T x R) so that Z_AB Phi = [I; 0; ...; 0]."""
    Nx, Nu = B.shape
    R = Nx * T + Nu * (T - 1)
    As, Bs, I = sp.csr_matrix(A), sp.csr_matrix(B), sp.identity(Nx, format="csr")
    blocks = [[None] * (T + (T - 1)) for _ in range(T)]
    blocks[0][0] = I
    for t in range(1, T):
        blocks[t][t] = I
        blocks[t][t - 1] = -As
        blocks[t][T + t - 1] = -Bs
    Z = sp.bmat(blocks, format="csr")  # every block row and column holds a block
    assert Z.shape == (Nx * T, R)
    return Z


@dataclass
class ColumnBlock:
    """Psi-comp data of one subsystem j (shared by its nx columns)."""

    j: int  # the subsystem whose columns this block serves
    rows: np.ndarray  # canonical row indices of the support (sorted)
    P: np.ndarray  # D x D projector onto null(H_j)
    O: np.ndarray  # D x nx offsets o_c = H_j^+ e_c
    rank: int
    feas_resid: float


def column_block(Z: sp.csr_matrix, mask: np.ndarray, lay: Layout, j: int) -> ColumnBlock:
    """H_j = Z_AB restricted to the support rows of subsystem j's columns (zero rows dropped),
    projector P_j = I - H_j^+ H_j and offsets o_c = H_j^+ e_c from an FP64 SVD."""
    Zc = Z.tocsc()
    cols = np.arange(j * lay.nx, (j + 1) * lay.nx)
    rows = np.flatnonzero(mask[:, cols[0]])
    H = Zc[:, rows].toarray()
    keep = np.any(H != 0, axis=1)
    rhs = np.zeros((Z.shape[0], lay.nx))
    rhs[cols, np.arange(lay.nx)] = 1.0  # e_c: the x_0 row of state c (block row 0 of Z_AB)
    H, E = H[keep], rhs[keep]
    U, s, Vt = np.linalg.svd(H, full_matrices=False)
    tol = max(H.shape) * np.finfo(np.float64).eps * (s[0] if s.size else 0.0)
    r = int(np.sum(s > tol))
    Ur, sr, Vr = U[:, :r], s[:r], Vt[:r].T
    Hpinv_E = Vr @ ((Ur.T @ E) / sr[:, None])
    P = np.eye(len(rows)) - Vr @ Vr.T
    feas = float(np.abs(H @ Hpinv_E - E).max())
    return ColumnBlock(j=j, rows=rows, P=P, O=Hpinv_E, rank=r, feas_resid=feas)


def column_blocks(Z: sp.csr_matrix, mask: np.ndarray, lay: Layout) -> list[ColumnBlock]:
    """Psi-comp data of every subsystem (see column_block)."""
    return [column_block(Z, mask, lay, j) for j in range(lay.n_sub)]


# --------------------------------------------------------------------- problem

@dataclass
class Problem:
    lay: Layout
    d: int
    A: np.ndarray
    B: np.ndarray
    dist: np.ndarray
    mask: np.ndarray  # R x N_x
    w: np.ndarray  # [R] row weights
    lb: np.ndarray  # [R]
    ub: np.ndarray  # [R]
    blocks: list[ColumnBlock]

    @property
    def feasible(self) -> bool:
        return all(b.feas_resid <= FEASIBILITY_TOL for b in self.blocks)


def row_weights_and_bounds(lay: Layout, q_diag, r_diag, x_lo=None, x_hi=None, u_lo=None,
                           u_hi=None):
    """w_r from diag(Q)/diag(R) on every row; bounds on x rows t >= 1 and u rows t <= T-2."""
    T, Nx, Nu = lay.T, lay.Nx, lay.Nu
    w = np.concatenate([np.tile(np.asarray(q_diag, float), T), np.tile(np.asarray(r_diag, float), T - 1)])
    lb = np.full(lay.R, -np.inf)
    ub = np.full(lay.R, np.inf)
    for t in range(1, T):
        if x_lo is not None:
            lb[t * Nx:(t + 1) * Nx] = x_lo
        if x_hi is not None:
            ub[t * Nx:(t + 1) * Nx] = x_hi
    for t in range(T - 1):
        s = Nx * T + t * Nu
        if u_lo is not None:
            lb[s:s + Nu] = u_lo
        if u_hi is not None:
            ub[s:s + Nu] = u_hi
    return w, lb, ub


def setup(A: np.ndarray, B: np.ndarray, n_sub: int, nx: int, nu: int, d: int, T: int,
          q_diag, r_diag, x_lo=None, x_hi=None, u_lo=None, u_hi=None,
          blocks: bool = True) -> Problem:
    """Offline precomputation (Algorithm 1, first step): graph, pattern, per-column projectors."""
    lay = Layout(n_sub, nx, nu, T)
    dist = hop_distances(interconnection_graph(A, n_sub, nx))
    mask = locality_mask(dist, d, lay)
    w, lb, ub = row_weights_and_bounds(lay, q_diag, r_diag, x_lo, x_hi, u_lo, u_hi)
    cb = column_blocks(build_zab(A, B, T), mask, lay) if blocks else []
    return Problem(lay=lay, d=d, A=A, B=B, dist=dist, mask=mask, w=w, lb=lb, ub=ub, blocks=cb)


def setup_from_network(net, d: int, T: int, cost, blocks: bool = True) -> Problem:
    return setup(net.dense_A(), net.dense_B(), net.n_sub, net.nx, net.nu, d, T, cost.q_diag,
                 cost.r_diag, cost.x_lo, cost.x_hi, cost.u_lo, cost.u_hi, blocks=blocks)


# --------------------------------------------------------------------- ADMM steps

def phi_comp(pb: Problem, Psi, Lam, x0, rho):
    """Row-wise explicit solve (Algorithm 2, Phi-comp).

    For every row r with support S_r and x_r = x0[S_r], v = (Psi - Lam)[r, S_r]:
    minimise w_r (phi.x_r)^2 + (rho/2)||phi - v||^2 s.t. lb_r <= phi.x_r <= ub_r.
    The minimiser is phi = v + alpha x_r with s = phi.x_r the clip of
    rho a / (rho + 2 w_r ||x_r||^2), a = v.x_r, alpha = (s - a)/||x_r||^2; when x_r = 0 the
    row cost vanishes and phi = v. Returns (Phi, s) where s = Phi x0 row by row.
    """
    Xr = pb.mask * x0[None, :]  # row r holds x_r on its support, zeros elsewhere
    V = Psi - Lam
    a = V @ x0  # V is zero off the pattern, so this is v . x_r
    n = np.sum(Xr * Xr, axis=1)
    s = np.clip(rho * a / (rho + 2.0 * pb.w * np.where(n > 0, n, 1.0)), pb.lb, pb.ub)
    s = np.where(n > 0, s, a)
    alpha = np.where(n > 0, (s - a) / np.where(n > 0, n, 1.0), 0.0)
    Phi = V + alpha[:, None] * Xr
    return Phi, s


def psi_comp(pb: Problem, Phi, Lam):
    """Column-wise projection (Algorithm 2, Psi-comp): Psi[S_j, c] = P_j (Phi + Lam)[S_j, c] + o_c."""
    Psi = np.zeros_like(Phi)
    nx = pb.lay.nx
    for blk in pb.blocks:
        cols = slice(blk.j * nx, (blk.j + 1) * nx)
        Vv = Phi[blk.rows, cols] + Lam[blk.rows, cols]
        Psi[blk.rows, cols] = blk.P @ Vv + blk.O
    return Psi


def lambda_comp(Lam, Phi, Psi):
    """Dual update (Algorithm 2, Lambda-comp): Lambda + Phi - Psi."""
    return Lam + Phi - Psi


def conv_residuals(Phi, Psi, Psi_prev):
    """Per-column primal ||Phi - Psi|| and dual ||Psi^{k+1} - Psi^k|| (Algorithm 2, Conv)."""
    return np.linalg.norm(Phi - Psi, axis=0), np.linalg.norm(Psi - Psi_prev, axis=0)


@dataclass
class Result:
    u0: np.ndarray
    y: np.ndarray  # Phi x0 (all R rows)
    J: float
    Phi: np.ndarray
    Psi: np.ndarray
    Lam: np.ndarray
    iters: int
    converged: bool
    r_primal: float
    r_dual: float


def solve(pb: Problem, x0: np.ndarray, rho: float = 5.0, eps: float = 1e-4, max_iter: int = 500,
          psi0: np.ndarray | None = None, lam0: np.ndarray | None = None,
          progress=None) -> Result:
    """Algorithm 2 from Psi^0 = psi0 (default 0) and Lambda^0 = lam0 (default 0).

    ``progress``, if given, is called as progress(k, r_primal, r_dual) after every iteration
    (reporting only; it cannot change the iteration)."""
    R, Nx = pb.lay.R, pb.lay.Nx
    Psi = np.zeros((R, Nx)) if psi0 is None else np.array(psi0, dtype=np.float64)
    Lam = np.zeros((R, Nx)) if lam0 is None else np.array(lam0, dtype=np.float64)
    x0 = np.asarray(x0, dtype=np.float64)
    it, conv, rp, rd = 0, False, np.inf, np.inf
    Phi, s = np.zeros((R, Nx)), np.zeros(R)
    while it < max_iter:
        Phi, s = phi_comp(pb, Psi, Lam, x0, rho)
        Psi_new = psi_comp(pb, Phi, Lam)
        Lam = lambda_comp(Lam, Phi, Psi_new)
        rpc, rdc = conv_residuals(Phi, Psi_new, Psi)
        Psi = Psi_new
        it += 1
        rp, rd = float(rpc.max()), float(rdc.max())
        if progress is not None:
            progress(it, rp, rd)
        if rp <= eps and rd <= eps:
            conv = True
            break
    y = Phi @ x0
    return Result(u0=y[pb.lay.u0_rows()], y=y, J=float(np.sum(pb.w * y * y)), Phi=Phi, Psi=Psi,
                  Lam=Lam, iters=it, converged=conv, r_primal=rp, r_dual=rd)


# --------------------------------------------------------------------- certificates

def kkt_residuals(pb: Problem, res: Result, x0: np.ndarray, rho: float) -> dict:
    """Residuals that certify an ADMM fixed point without reference to the iteration.

    eq: max_c ||H_j Psi[:,c] - e_c|| via Z_AB; pf: max|Phi - Psi|; box: bound violation of
    Phi x0; stat: max_c ||P_j rho Lam[S_j, c]|| (Psi-step optimality puts -rho Lam_c in the
    row space of H_j); pattern: largest entry of Phi, Psi or Lam outside L_d.
    """
    Z = build_zab(pb.A, pb.B, pb.lay.T)
    rhs = np.zeros((Z.shape[0], pb.lay.Nx))
    rhs[:pb.lay.Nx] = np.eye(pb.lay.Nx)
    eq = float(np.abs(Z @ res.Psi - rhs).max())
    stat = 0.0
    nx = pb.lay.nx
    for blk in pb.blocks:
        L = rho * res.Lam[blk.rows, blk.j * nx:(blk.j + 1) * nx]
        stat = max(stat, float(np.abs(blk.P @ L).max()))
    y = res.Phi @ x0
    box = float(max(np.max(pb.lb - y), np.max(y - pb.ub), 0.0))
    off = ~pb.mask
    pattern = float(max(np.abs(res.Phi[off]).max(initial=0), np.abs(res.Psi[off]).max(initial=0),
                        np.abs(res.Lam[off]).max(initial=0)))
    return {"eq": eq, "pf": float(np.abs(res.Phi - res.Psi).max()), "box": box, "stat": stat,
            "pattern": pattern}


def lemma1_bounds(adj: list[set[int]], d: int, T: int, s: int) -> tuple[float, float]:
    """Lemma 1: D_row <= s (l^{d+1}-1)/(l-1), D_col <= (2T-1) s (l^{d+1}-1)/(l-1), l = max degree."""
    l = max(len(a) for a in adj)
    nodes = (d + 1) if l == 1 else (l ** (d + 1) - 1) / (l - 1)
    return s * nodes, (2 * T - 1) * s * nodes
