"""FP64 reference of closed-loop DLMPC (Algorithm 1) — TEST INFRASTRUCTURE ONLY.

Only ``tests/`` use this module; the library's closed-loop entry point is checked against it.

Algorithm 1 of the paper runs the MPC loop: at every time step the subsystems measure the state
x(t), the controller precomputes what depends on it, runs the ADMM of Algorithm 2, reads u(t)
from Phi, and the plant moves to x(t+1) = A x(t) + B u(t). Here every solve is the oracle's own
Algorithm 2 (``dlmpc_oracle.solve``), and the plant step is the dynamics of eq. (MPC).

Two initial iterates per step:

* cold: Psi^0 = Lambda^0 = 0 at every step;
* shifted (a warm start across steps, the receding-horizon reading of a better initial point):
  the previous step's input trajectory moved one step ahead (u_1..u_{T-2} of the previous
  solution become u_0..u_{T-3}; the last input is held), turned into a start by
  ``warm_start.trajectory_start`` (state rows simulated from x(t), CG on M beta = y - b, the
  multiplier guess), then Algorithm 2 with eps_warm; an unconverged warm-started step is solved
  again from the cold start with eps.

Penalty per step: rho (the paper's fixed penalty), or, with scale_rho, rho times
||x(t)||^2 / ||x(0)||^2 (at least 1e-20). The Phi-step minimises w (phi . x_r)^2 +
(rho/2) ||phi - v||^2; with x(t) = s z this is s^2 [w (phi . z_r)^2 + (rho/(2 s^2)) ||phi - v||^2],
so a penalty of rho s^2 at x(t) runs the Phi iterates of rho at z with the bounds divided by s:
the iteration no longer slows down as the loop drives the state to zero.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from oracle import dlmpc_oracle as O
from oracle import warm_start as WS


def shift_inputs(lay: O.Layout, y: np.ndarray) -> np.ndarray:
    """Input rows [N_u (T-1)] (canonical order) of y moved one step ahead, last step held."""
    Nx, Nu, T = lay.Nx, lay.Nu, lay.T
    u = np.asarray(y[Nx * T:], dtype=np.float64).reshape(T - 1, Nu)
    out = np.empty_like(u)
    out[:-1] = u[1:]
    out[-1] = u[-1]
    return out.reshape(-1)


@dataclass
class ClosedLoop:
    x: np.ndarray  # [T_sim + 1, N_x] states x(0) .. x(T_sim)
    u: np.ndarray  # [T_sim, N_u] applied inputs u(0) .. u(T_sim - 1)
    iters: list  # ADMM iterations per step (a cold fallback adds its own)
    converged: list
    fell_back: list
    J: list  # objective of every step's solve


def step_rho(rho: float, x: np.ndarray, x0: np.ndarray) -> float:
    """rho ||x||^2 / ||x0||^2, at least rho * 1e-20 (rho when x0 = 0)."""
    n0 = float(np.dot(x0, x0))
    return rho if n0 == 0.0 else rho * max(float(np.dot(x, x)) / n0, 1e-20)


def closed_loop(pb: O.Problem, x0: np.ndarray, T_sim: int, rho0: float, eps: float, max_iter: int,
                warm: bool = False, eps_warm: float | None = None, cg_iters: int = 12,
                scale_rho: bool = False) -> ClosedLoop:
    """Algorithm 1 over T_sim steps from x(0) = x0 (penalty rho0, or step_rho with scale_rho)."""
    eps_warm = eps if eps_warm is None else eps_warm
    x = np.asarray(x0, dtype=np.float64)
    xs, us, iters, conv, fb, Js = [x], [], [], [], [], []
    prev_y = None
    for _ in range(T_sim):
        rho = step_rho(rho0, x, xs[0]) if scale_rho else rho0
        fell = False
        if warm and prev_y is not None:
            psi0, lam0, _, _ = WS.trajectory_start(pb, x, shift_inputs(pb.lay, prev_y), rho, cg_iters)
            res = O.solve(pb, x, rho, eps_warm, max_iter, psi0=psi0, lam0=lam0)
            if not res.converged:
                first = res.iters
                res = O.solve(pb, x, rho, eps, max_iter)
                res.iters += first
                fell = True
        else:
            res = O.solve(pb, x, rho, eps, max_iter)
        us.append(res.u0)
        iters.append(res.iters)
        conv.append(res.converged)
        fb.append(fell)
        Js.append(res.J)
        x = pb.A @ x + pb.B @ res.u0
        xs.append(x)
        prev_y = res.y
    return ClosedLoop(x=np.array(xs), u=np.array(us), iters=iters, converged=conv, fell_back=fb, J=Js)
