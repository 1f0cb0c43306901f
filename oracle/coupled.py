"""FP64 reference of DLMPC with neighbour-coupled constraints — TEST INFRASTRUCTURE ONLY.

Only ``tests/`` use this module; the library's coupled Phi-step is checked against it.

Constraints that couple rows of different subsystems (e.g. lo <= theta_i(t) - theta_j(t) <= hi
on the rows of neighbours i and j: a line-flow limit of the swing network) make the Phi-step of
Algorithm 2 non-separable by rows. The paper's Phi-comp defers to the explicit solution of its
reference work, which handles such constraints with an inner (nested) ADMM whose iterations
exchange values between the coupled subsystems. Written out here:

Phi-step. With a = v . x_r, n = ||x_r||^2 and y_r = phi . x_r, the row minimiser for given y_r is
phi = v + ((y_r - a)/n) x_r (the smallest change of v that gives y_r), at cost
w_r y_r^2 + (rho / (2 n)) (y_r - a)^2 = c_r (y_r - m_r)^2 + const, c_r = w_r + rho / (2 n),
m_r = rho a / (rho + 2 w_r n). So the Phi-step is

    min_y  sum_r c_r (y_r - m_r)^2   s.t.  lb <= y <= ub,  lo_e <= y[ra_e] - y[rb_e] <= hi_e.

Rows with n = 0 keep phi = v (their y is v . x_r = 0 and they take part in no update). Without
couplings the problem separates into the per-row clip of the uncoupled Phi-comp.

Nested ADMM (penalty sigma, scaled form). Every coupling e holds copies (z_e^a, z_e^b) of its two
rows' values and a scaled dual (l_e^a, l_e^b); with A the copy operator y -> (y[ra], y[rb]):
  y-update (per row, its own couplings only): y_r = clip((2 c_r m_r + sigma sum_{e at r}
      (z_e^r - l_e^r)) / (2 c_r + sigma deg_r), lb_r, ub_r)   (1-D quadratic over a box);
  z-update (per coupling): (z^a, z^b) = Euclidean projection of (y_a + l^a, y_b + l^b) onto
      {lo_e <= z^a - z^b <= hi_e}: both move by half the clip of their difference, opposite ways;
  dual update: l += A y - z;
  stop when max |A y - z| <= inner_eps and sigma max |z - z_prev| <= inner_eps, or after
  inner_max iterations.
The copies and duals are kept from one outer iteration to the next (warm start of the inner
problem); the first outer iteration starts them at zero.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from oracle import dlmpc_oracle as O


@dataclass
class Coupling:
    ra: np.ndarray  # canonical row indices of the first row of each coupling
    rb: np.ndarray  # and of the second
    lo: np.ndarray
    hi: np.ndarray
    sigma: float = 1.0
    inner_max: int = 50
    inner_eps: float = 1e-9


@dataclass
class InnerState:
    za: np.ndarray
    zb: np.ndarray
    la: np.ndarray
    lb: np.ndarray
    iters: list = field(default_factory=list)  # inner iterations of every outer iteration


def new_state(cp: Coupling) -> InnerState:
    z = np.zeros(len(cp.ra))
    return InnerState(za=z.copy(), zb=z.copy(), la=z.copy(), lb=z.copy())


def phi_step_qp(pb: O.Problem, Psi, Lam, x0, rho):
    """(V, Xr, a, n, c, m): the data of the Phi-step's problem in y (module docstring)."""
    Xr = pb.mask * x0[None, :]
    V = Psi - Lam
    a = V @ x0
    n = np.sum(Xr * Xr, axis=1)
    nn = np.where(n > 0, n, 1.0)
    c = pb.w + rho / (2.0 * nn)
    m = rho * a / (rho + 2.0 * pb.w * nn)
    return V, Xr, a, n, c, m


def project_pairs(pa, pb, lo, hi):
    """Euclidean projection of (pa, pb) onto {lo <= za - zb <= hi}, coupling by coupling."""
    d = pa - pb
    shift = 0.5 * (np.clip(d, lo, hi) - d)
    return pa + shift, pb - shift


def nested_admm(c, m, lb, ub, free, cp: Coupling, st: InnerState) -> np.ndarray:
    """The inner ADMM on min sum c (y - m)^2 s.t. boxes and couplings; rows with free == False
    keep y = m (the rows with n = 0). Updates st in place, returns y."""
    y = np.where(free, np.clip(m, lb, ub), m)
    ra, rb, sig = cp.ra, cp.rb, cp.sigma
    R = len(c)
    deg = np.bincount(ra, minlength=R) + np.bincount(rb, minlength=R)
    coupled = (deg > 0) & free
    k = 0
    for k in range(1, cp.inner_max + 1):
        acc = (np.bincount(ra, weights=st.za - st.la, minlength=R)
               + np.bincount(rb, weights=st.zb - st.lb, minlength=R))
        yc = np.clip((2.0 * c * m + sig * acc) / (2.0 * c + sig * deg), lb, ub)
        y = np.where(coupled, yc, y)
        za, zb = project_pairs(y[ra] + st.la, y[rb] + st.lb, cp.lo, cp.hi)
        dz = max(np.abs(za - st.za).max(initial=0.0), np.abs(zb - st.zb).max(initial=0.0))
        st.la = st.la + y[ra] - za
        st.lb = st.lb + y[rb] - zb
        st.za, st.zb = za, zb
        rp = max(np.abs(y[ra] - za).max(initial=0.0), np.abs(y[rb] - zb).max(initial=0.0))
        if rp <= cp.inner_eps and sig * dz <= cp.inner_eps:
            break
    st.iters.append(k)
    return y


def phi_comp_coupled(pb: O.Problem, Psi, Lam, x0, rho, cp: Coupling, st: InnerState):
    """Phi-comp with the couplings: nested ADMM for y, then phi = v + ((y - a)/n) x_r."""
    V, Xr, a, n, c, m = phi_step_qp(pb, Psi, Lam, x0, rho)
    free = n > 0
    y = nested_admm(c, np.where(free, m, a), pb.lb, pb.ub, free, cp, st)
    alpha = np.where(free, (y - a) / np.where(free, n, 1.0), 0.0)
    return V + alpha[:, None] * Xr, np.where(free, y, a)


def solve(pb: O.Problem, x0: np.ndarray, cp: Coupling, rho: float = 5.0, eps: float = 1e-4,
          max_iter: int = 500) -> tuple[O.Result, InnerState]:
    """Algorithm 2 (cold start) with the coupled Phi-comp; Psi-comp, Lambda-comp and Conv as in
    the uncoupled oracle."""
    R, Nx = pb.lay.R, pb.lay.Nx
    x0 = np.asarray(x0, dtype=np.float64)
    Psi, Lam = np.zeros((R, Nx)), np.zeros((R, Nx))
    st = new_state(cp)
    it, conv, rp, rd = 0, False, np.inf, np.inf
    Phi = np.zeros((R, Nx))
    while it < max_iter:
        Phi, _ = phi_comp_coupled(pb, Psi, Lam, x0, rho, cp, st)
        Psi_new = O.psi_comp(pb, Phi, Lam)
        Lam = O.lambda_comp(Lam, Phi, Psi_new)
        rpc, rdc = O.conv_residuals(Phi, Psi_new, Psi)
        Psi = Psi_new
        it += 1
        rp, rd = float(rpc.max()), float(rdc.max())
        if rp <= eps and rd <= eps:
            conv = True
            break
    y = Phi @ x0
    res = O.Result(u0=y[pb.lay.u0_rows()], y=y, J=float(np.sum(pb.w * y * y)), Phi=Phi, Psi=Psi, Lam=Lam,
                   iters=it, converged=conv, r_primal=rp, r_dual=rd)
    return res, st
