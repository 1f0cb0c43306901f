"""FP64 reference of the trajectory warm start — TEST INFRASTRUCTURE ONLY.

Only ``tests/`` use this module; the library's HIP kernels are checked against it.

Section V names a better initial point than the zero start of Algorithm 2 as future work.
The construction here starts ADMM from a predicted input trajectory u_hat (what the learned
network outputs):

1. y_hat: the trajectory that u_hat drives from x0 (state rows simulated with A, B; these are
   the dynamics that Z_AB Phi = I encodes, applied to the vector Phi x0).
2. beta: fixed number of conjugate-gradient steps from zero on M beta = y_hat - b, where
   M = sum_j ||x0_j||^2 P_j (each term lifted from the support rows of subsystem j to all R
   rows) and b = sum_c x0_c o_c. For Psi[:,c] = o_c + x0_c P_j beta (on the support of c),
   Psi x0 = b + M beta, so beta picks a feasible, local Psi whose trajectory is y_hat.
3. alpha = -2 w y_hat / rho (the Phi-comp row multiplier of an unconstrained row at a fixed
   point with trajectory y_hat).
4. Psi^0[:,c] = o_c + x0_c P_j beta and Lambda^0[:,c] = x0_c (I - P_j) alpha on the support of
   column c (zero elsewhere): Psi^0 satisfies Z_AB Psi^0 = I and the locality pattern, and for
   y_hat = y* (the optimum) with converged CG the pair is an ADMM fixed point.
"""
from __future__ import annotations

import numpy as np

from oracle import dlmpc_oracle as O


def simulate_states(pb: O.Problem, x0: np.ndarray, y: np.ndarray) -> np.ndarray:
    """y with its state rows replaced by x_0 = x0, x_{t+1} = A x_t + B u_t (u rows kept)."""
    lay = pb.lay
    Nx, Nu, T = lay.Nx, lay.Nu, lay.T
    out = np.array(y, dtype=np.float64)
    x = np.asarray(x0, dtype=np.float64).copy()
    out[:Nx] = x
    for t in range(T - 1):
        u = out[Nx * T + t * Nu:Nx * T + (t + 1) * Nu]
        x = pb.A @ x + pb.B @ u
        out[(t + 1) * Nx:(t + 2) * Nx] = x
    return out


def offset_rows(pb: O.Problem, x0: np.ndarray) -> np.ndarray:
    """b = sum_c x0_c o_c (each o_c on the support rows of its column)."""
    nx = pb.lay.nx
    b = np.zeros(pb.lay.R)
    for blk in pb.blocks:
        b[blk.rows] += blk.O @ x0[blk.j * nx:(blk.j + 1) * nx]
    return b


def apply_m(pb: O.Problem, x0: np.ndarray, v: np.ndarray) -> np.ndarray:
    """M v = sum_j ||x0_j||^2 P_j v (restricted to and lifted from j's support rows)."""
    nx = pb.lay.nx
    out = np.zeros(pb.lay.R)
    for blk in pb.blocks:
        xj = x0[blk.j * nx:(blk.j + 1) * nx]
        out[blk.rows] += float(xj @ xj) * (blk.P @ v[blk.rows])
    return out


def conjugate_gradient(apply, rhs: np.ndarray, iters: int) -> np.ndarray:
    """Hestenes-Stiefel conjugate gradients from zero, exactly `iters` steps (fewer only if
    the residual vanishes)."""
    x = np.zeros_like(rhs)
    r = rhs.copy()
    p = r.copy()
    rr = float(r @ r)
    for _ in range(iters):
        if rr == 0.0:
            break
        q = apply(p)
        pq = float(p @ q)
        if pq <= 0.0:
            break
        a = rr / pq
        x = x + a * p
        r = r - a * q
        rr_new = float(r @ r)
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x


def trajectory_start(pb: O.Problem, x0: np.ndarray, u_hat: np.ndarray, rho: float, cg_iters: int):
    """(Psi^0, Lambda^0, y_hat, beta) of the warm start from the input rows u_hat
    [Nu*(T-1)] (canonical order: u_0 of all subsystems, then u_1, ...)."""
    lay = pb.lay
    x0 = np.asarray(x0, dtype=np.float64)
    y = np.zeros(lay.R)
    y[lay.Nx * lay.T:] = u_hat
    y_hat = simulate_states(pb, x0, y)
    b = offset_rows(pb, x0)
    beta = conjugate_gradient(lambda v: apply_m(pb, x0, v), y_hat - b, cg_iters)
    alpha = -2.0 * pb.w * y_hat / rho
    nx = lay.nx
    psi0, lam0 = np.zeros((lay.R, lay.Nx)), np.zeros((lay.R, lay.Nx))
    for blk in pb.blocks:
        pb_ = blk.P @ beta[blk.rows]
        qa = alpha[blk.rows] - blk.P @ alpha[blk.rows]
        for ci in range(nx):
            c = blk.j * nx + ci
            psi0[blk.rows, c] = blk.O[:, ci] + x0[c] * pb_
            lam0[blk.rows, c] = x0[c] * qa
    return psi0, lam0, y_hat, beta
