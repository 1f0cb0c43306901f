"""Brute-force certifiers that pin the DLMPC oracle — TEST INFRASTRUCTURE ONLY.

Only ``tests/`` (and the oracle's own checks) use this module. None of it shares code with
the ADMM oracle in ``dlmpc_oracle.py``: it rebuilds the problem of eq. (MPC) under the SLS
parametrisation (Section II-A) from A and B directly, and solves it as one dense program.

* ``lqr_riccati``: centralised finite-horizon LQR by the backward Riccati recursion (no
  locality, no bounds). With generic x0 and a dedicated actuator at every node, the
  localised optimum has the same trajectory, so u(0) and the objective must match.
* ``localized_qp``: the d-localised SLS program written out as one dense quadratic program
  in the supported entries of Phi: each column of Phi must be a trajectory of the plant from
  the unit initial state e_c (simulated row by row from A and B), entries outside the d-hop
  pattern are absent, and bounds act on Phi x0. Solved by the null-space method (no bounds)
  or by a dual active-set loop for the convex QP in trajectory space (with bounds), and in
  both cases returned together with a KKT certificate.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla
from scipy.sparse.csgraph import shortest_path


def lqr_riccati(A: np.ndarray, B: np.ndarray, q_diag, r_diag, T: int, x0: np.ndarray):
    """Finite-horizon LQR over states x_0..x_{T-1} and inputs u_0..u_{T-2}.

    Cost sum_{t<T} x_t'Qx_t + sum_{t<T-1} u_t'Ru_t (terminal weight Q on x_{T-1}).
    P_{T-1} = Q; K_t = (R + B'P_{t+1}B)^{-1} B'P_{t+1}A; P_t = Q + A'P_{t+1}(A - BK_t).
    Returns (u0, J, y) with y the trajectory in the canonical Phi row order.
    """
    Q, R = np.diag(np.asarray(q_diag, float)), np.diag(np.asarray(r_diag, float))
    P = Q.copy()
    Ks = [None] * (T - 1)
    for t in range(T - 2, -1, -1):
        K = np.linalg.solve(R + B.T @ P @ B, B.T @ P @ A)
        P = Q + A.T @ P @ (A - B @ K)
        Ks[t] = K
    xs, us = [np.asarray(x0, float)], []
    for t in range(T - 1):
        us.append(-Ks[t] @ xs[-1])
        xs.append(A @ xs[-1] + B @ us[-1])
    y = np.concatenate(xs + us)
    J = float(np.asarray(x0) @ P @ np.asarray(x0))
    return us[0], J, y


@dataclass
class DenseSLS:
    """The localised program as dense algebra: E z = f (achievability), y = G z (= Phi x0)."""

    E: np.ndarray
    f: np.ndarray
    G: np.ndarray
    var_rc: np.ndarray  # [nvar, 2] (row, col) of each variable in canonical Phi order
    R: int


def dense_sls(A: np.ndarray, B: np.ndarray, n_sub: int, nx: int, nu: int, d: int, T: int,
              x0: np.ndarray) -> DenseSLS:
    Nx, Nu = n_sub * nx, n_sub * nu
    R = Nx * T + Nu * (T - 1)
    adj = np.zeros((n_sub, n_sub))
    for i in range(n_sub):
        for j in range(n_sub):
            if i != j and (np.any(A[i * nx:(i + 1) * nx, j * nx:(j + 1) * nx])
                           or np.any(A[j * nx:(j + 1) * nx, i * nx:(i + 1) * nx])):
                adj[i, j] = 1
    hops = shortest_path(adj, unweighted=True, directed=False)

    def xrow(t, s):  # canonical row of state s at time t
        return t * Nx + s

    def urow(t, k):
        return Nx * T + t * Nu + k

    owner = np.concatenate([np.repeat(np.arange(n_sub), nx)] * T + [np.repeat(np.arange(n_sub), nu)] * (T - 1))
    var_index = {}
    var_rc = []
    for c in range(Nx):
        jc = c // nx
        for r in range(R):
            if hops[owner[r], jc] <= d:
                var_index[(r, c)] = len(var_rc)
                var_rc.append((r, c))
    nvar = len(var_rc)
    eq_rows, f = [], []
    for c in range(Nx):
        for t in range(T):
            for s in range(Nx):
                row = {}
                if t == 0:
                    if (xrow(0, s), c) in var_index:
                        row[var_index[(xrow(0, s), c)]] = 1.0
                    rhs = 1.0 if s == c else 0.0
                else:
                    if (xrow(t, s), c) in var_index:
                        row[var_index[(xrow(t, s), c)]] = 1.0
                    for s2 in np.flatnonzero(A[s]):
                        key = (xrow(t - 1, s2), c)
                        if key in var_index:
                            row[var_index[key]] = row.get(var_index[key], 0.0) - A[s, s2]
                    for k in np.flatnonzero(B[s]):
                        key = (urow(t - 1, k), c)
                        if key in var_index:
                            row[var_index[key]] = row.get(var_index[key], 0.0) - B[s, k]
                    rhs = 0.0
                if row or rhs != 0.0:
                    eq_rows.append(row)
                    f.append(rhs)
    E = np.zeros((len(eq_rows), nvar))
    for i, row in enumerate(eq_rows):
        for k, v in row.items():
            E[i, k] = v
    G = np.zeros((R, nvar))
    for k, (r, c) in enumerate(var_rc):
        G[r, k] = x0[c]
    return DenseSLS(E=E, f=np.array(f), G=G, var_rc=np.array(var_rc), R=R)


@dataclass
class QPSolution:
    y: np.ndarray
    J: float
    active_lower: np.ndarray
    active_upper: np.ndarray
    kkt: dict
    feasible_resid: float
    active_pairs: np.ndarray | None = None  # indices into 2 * n_pairs rows: e (upper), n_pairs + e (lower)


def separable_qp(c, m, lb, ub, ra, rb, lo, hi, max_active_iter=500, tol=1e-10):
    """min sum_r c_r (y_r - m_r)^2 s.t. lb <= y <= ub, lo_e <= y[ra_e] - y[rb_e] <= hi_e, by the
    same dual active-set loop on the dense KKT system (a direct solve of the Phi-step problem that
    the nested ADMM iterates on). Returns (y, kkt residuals)."""
    c, m = np.asarray(c, float), np.asarray(m, float)
    n = len(c)
    rows, rhs = [], []
    for r in range(n):
        if np.isfinite(ub[r]):
            e = np.zeros(n)
            e[r] = 1.0
            rows.append(e)
            rhs.append(ub[r])
        if np.isfinite(lb[r]):
            e = np.zeros(n)
            e[r] = -1.0
            rows.append(e)
            rhs.append(-lb[r])
    for a_, b_, l_, h_ in zip(ra, rb, lo, hi):
        e = np.zeros(n)
        e[a_], e[b_] = 1.0, -1.0
        rows += [e, -e]
        rhs += [h_, -l_]
    Ain, bin_ = np.array(rows).reshape(-1, n), np.array(rhs)
    H, g = np.diag(2.0 * c), -2.0 * c * m
    active: list[int] = []
    for _ in range(max_active_iter):
        k = len(active)
        Aa = Ain[active]
        KKT = np.block([[H, Aa.T], [Aa, np.zeros((k, k))]])
        sol = np.linalg.lstsq(KKT, np.concatenate([-g, bin_[active]]), rcond=None)[0]
        y, lam = sol[:n], sol[n:]
        if k and lam.min() < -tol:
            active.pop(int(np.argmin(lam)))
            continue
        viol = Ain @ y - bin_
        if len(viol) and viol.max() > tol:
            cand = int(np.argmax(viol))
            if cand in active:
                raise RuntimeError("active-set loop stalled")
            active.append(cand)
            continue
        break
    else:
        raise RuntimeError("active-set loop did not converge")
    mult = np.zeros(len(bin_))
    mult[active] = lam
    viol = Ain @ y - bin_
    kkt = {"stationarity": float(np.abs(H @ y + g + Ain.T @ mult).max()),
           "primal": float(max(viol.max(initial=0.0), 0.0)),
           "dual_sign": float(max(-mult.min(initial=0.0), 0.0)),
           "complementarity": float(np.abs(mult * viol).max(initial=0.0))}
    return y, kkt


def _affine_trajectory_set(sls: DenseSLS, tol: float = 1e-10):
    """Y = {G z : E z = f} as y_p + range(U) with U orthonormal. Returns (y_p, U, eq_resid)."""
    z_p, *_ = np.linalg.lstsq(sls.E, sls.f, rcond=None)
    eq_resid = float(np.abs(sls.E @ z_p - sls.f).max())
    K = sla.null_space(sls.E, rcond=tol)
    M = sls.G @ K
    Um, sm, _ = np.linalg.svd(M, full_matrices=False)
    r = int(np.sum(sm > tol * (sm[0] if sm.size else 0.0)))
    return sls.G @ z_p, Um[:, :r], eq_resid


def localized_qp(A, B, n_sub, nx, nu, d, T, w, x0, lb=None, ub=None, max_active_iter=500,
                 tol=1e-10, pairs=None) -> QPSolution:
    """Optimum of min sum_r w_r y_r^2 over y in the localised achievable set, lb <= y <= ub,
    and, with pairs = (ra, rb, lo, hi), lo_e <= y[ra_e] - y[rb_e] <= hi_e.

    Dual active-set loop on the strictly convex QP in coordinates s (y = y_p + U s): start
    from the unconstrained minimiser, add the most violated bound, solve the equality-
    constrained subproblem, drop the most negative multiplier, until the KKT conditions hold.
    """
    sls = dense_sls(A, B, n_sub, nx, nu, d, T, np.asarray(x0, float))
    y_p, U, eq_resid = _affine_trajectory_set(sls)
    w = np.asarray(w, float)
    R = sls.R
    lb = np.full(R, -np.inf) if lb is None else np.asarray(lb, float)
    ub = np.full(R, np.inf) if ub is None else np.asarray(ub, float)
    Hs = 2.0 * U.T @ (w[:, None] * U)
    gs = 2.0 * U.T @ (w * y_p)
    # inequality rows: a_i . s <= b_i ; upper: U_r s <= ub_r - y_p_r ; lower: -U_r s <= y_p_r - lb_r
    ups = np.flatnonzero(np.isfinite(ub))
    los = np.flatnonzero(np.isfinite(lb))
    Ain = np.vstack([U[ups], -U[los]]) if (len(ups) + len(los)) else np.zeros((0, U.shape[1]))
    bin_ = np.concatenate([ub[ups] - y_p[ups], y_p[los] - lb[los]])
    n_box = len(bin_)
    if pairs is not None:
        ra, rb, plo, phi_ = (np.asarray(v) for v in pairs)
        Dm, dp = U[ra] - U[rb], y_p[ra] - y_p[rb]
        Ain = np.vstack([Ain, Dm, -Dm])
        bin_ = np.concatenate([bin_, phi_ - dp, dp - plo])
    active: list[int] = []
    s = lam = None
    for _ in range(max_active_iter):
        k = len(active)
        Aa = Ain[active]
        KKT = np.block([[Hs, Aa.T], [Aa, np.zeros((k, k))]])
        rhs = np.concatenate([-gs, bin_[active]])
        sol = np.linalg.lstsq(KKT, rhs, rcond=None)[0]
        s, lam = sol[:U.shape[1]], sol[U.shape[1]:]
        if k and lam.min() < -tol:
            active.pop(int(np.argmin(lam)))
            continue
        viol = Ain @ s - bin_ if len(bin_) else np.zeros(0)
        if len(viol) and viol.max() > tol:
            cand = int(np.argmax(viol))
            if cand in active:
                raise RuntimeError("active-set loop stalled")
            active.append(cand)
            continue
        break
    else:
        raise RuntimeError("active-set loop did not converge")
    y = y_p + U @ s
    mult = np.zeros(len(bin_))
    mult[active] = lam
    viol = Ain @ s - bin_ if len(bin_) else np.zeros(0)
    kkt = {
        "stationarity": float(np.abs(Hs @ s + gs + Ain.T @ mult).max()) if len(bin_) else float(np.abs(Hs @ s + gs).max()),
        "primal": float(max(viol.max(initial=0.0), 0.0)),
        "dual_sign": float(max(-mult.min(initial=0.0), 0.0)),
        "complementarity": float(np.abs(mult * viol).max(initial=0.0)),
    }
    act = set(active)
    nu_ = len(ups)
    return QPSolution(y=y, J=float(np.sum(w * y * y)),
                      active_lower=np.array([los[i - nu_] for i in sorted(act) if nu_ <= i < n_box], dtype=int),
                      active_upper=np.array([ups[i] for i in sorted(act) if i < nu_], dtype=int),
                      kkt=kkt, feasible_resid=eq_resid,
                      active_pairs=np.array(sorted(i - n_box for i in act if i >= n_box), dtype=int))


def projection_by_kkt(H: np.ndarray, v: np.ndarray, e: np.ndarray) -> np.ndarray:
    """argmin ||psi - v|| s.t. H psi = e, from the (minimum-norm) solution of the KKT system
    [[I, H'], [H, 0]] [psi; mu] = [v; e] — an independent route to the Psi-comp projection."""
    m, n = H.shape
    K = np.block([[np.eye(n), H.T], [H, np.zeros((m, m))]])
    sol = np.linalg.lstsq(K, np.concatenate([v, e]), rcond=None)[0]
    return sol[:n]


def admm_entry_space(A, B, n_sub, nx, nu, d, T, w, x0, rho, n_iter, lb=None, ub=None):
    """Algorithm 2 run a second way, to pin the oracle's iteration and its stopping rule.

    The unknowns are the supported entries z of Phi (one vector over all columns, as in
    ``dense_sls``); achievability is E z = f built by simulating the plant. Phi-comp solves
    each row's problem min w (phi.x)^2 + (rho/2)||phi - v||^2 (lb <= phi.x <= ub) as linear
    systems: the unconstrained stationarity system, and when its phi.x leaves the box the
    equality-constrained KKT system with phi.x on the violated bound. Psi-comp is the
    minimum-norm correction onto {E z = f} for all columns at once (pseudo-inverse of E),
    not a per-column projector. Residuals are summed per column with ``np.bincount``.

    Runs exactly ``n_iter`` iterations from Psi^0 = Lambda^0 = 0 and returns the per-iteration
    per-column residuals (primal ||Phi - Psi||, dual ||Psi^{k+1} - Psi^k||), each
    [n_iter, N_x], and the final (Phi, Psi, Lambda) entry vectors with ``var_rc``.
    """
    x0 = np.asarray(x0, float)
    sls = dense_sls(A, B, n_sub, nx, nu, d, T, x0)
    R, Nx = sls.R, n_sub * nx
    rows, cols = sls.var_rc[:, 0], sls.var_rc[:, 1]
    lb = np.full(R, -np.inf) if lb is None else np.asarray(lb, float)
    ub = np.full(R, np.inf) if ub is None else np.asarray(ub, float)
    w = np.asarray(w, float)
    E_pinv = np.linalg.pinv(sls.E, rcond=1e-12)
    by_row = [np.flatnonzero(rows == r) for r in range(R)]
    nvar = len(rows)
    psi, lam = np.zeros(nvar), np.zeros(nvar)
    rp_hist, rd_hist = np.zeros((n_iter, Nx)), np.zeros((n_iter, Nx))
    phi = np.zeros(nvar)
    for k in range(n_iter):
        v = psi - lam
        phi = v.copy()
        for r, idx in enumerate(by_row):
            if idx.size == 0:
                continue
            x = x0[cols[idx]]
            if not np.any(x):
                continue  # the row cost vanishes: phi = v
            n = idx.size
            H = 2.0 * w[r] * np.outer(x, x) + rho * np.eye(n)
            p = np.linalg.solve(H, rho * v[idx])
            s = x @ p
            bound = lb[r] if s < lb[r] else (ub[r] if s > ub[r] else None)
            if bound is not None:  # min (rho/2)||phi - v||^2 + w bound^2 s.t. x.phi = bound
                K = np.block([[rho * np.eye(n), x[:, None]], [x[None, :], np.zeros((1, 1))]])
                p = np.linalg.solve(K, np.concatenate([rho * v[idx], [bound]]))[:n]
            phi[idx] = p
        u = phi + lam
        psi_new = u - E_pinv @ (sls.E @ u - sls.f)
        lam = lam + phi - psi_new
        rp_hist[k] = np.sqrt(np.bincount(cols, weights=(phi - psi_new) ** 2, minlength=Nx))
        rd_hist[k] = np.sqrt(np.bincount(cols, weights=(psi_new - psi) ** 2, minlength=Nx))
        psi = psi_new
    return rp_hist, rd_hist, (phi, psi, lam, sls.var_rc)
