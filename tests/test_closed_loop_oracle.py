"""Pins of the closed-loop oracle (Algorithm 1) (no GPU).

* Unconstrained, generic x0, an actuator at every node: each step's localised optimum has the
  centralised finite-horizon LQR trajectory (the pin of the single solve), so the closed loop run
  to a tight eps must follow the receding-horizon LQR loop x(t+1) = A x(t) + B u_LQR(x(t)), with
  u_LQR from the backward Riccati recursion of the same horizon (certify.lqr_riccati), from the
  cold and from the shifted start alike.
* The shift moves the input rows one step ahead and holds the last one (checked by hand).
* A planted mistake (the loop applying the second input of the horizon instead of the first)
  breaks the LQR pin.
* At eps = 1e-4 the shifted start needs fewer iterations than the cold start over the loop.
* Penalty scaled with the state (scale_rho): the equivalence it rests on holds to rounding
  (ADMM from s x with penalty rho s^2 takes the iterates of ADMM from x with rho and the bounds
  divided by s: same iteration count, u(0) scaled by s), unconstrained and with active bounds;
  the scaled loop follows the same LQR loop, and over a loop whose state decays it needs far
  fewer iterations than the fixed penalty.
"""
import numpy as np
import pytest

from oracle import certify as C
from oracle import closed_loop as CL
from oracle import dlmpc_oracle as O
from paper_2103_14990_amd import workloads as W

RHO = 5.0
T_SIM = 20


@pytest.fixture(scope="module")
def chain():
    wl = W.workload("chain10")
    return wl, O.setup_from_network(wl.net, wl.d, wl.T, wl.cost)


def _lqr_loop(wl, x0, T_sim):
    A, B = wl.net.dense_A(), wl.net.dense_B()
    xs, us = [np.asarray(x0, float)], []
    for _ in range(T_sim):
        u, _, _ = C.lqr_riccati(A, B, wl.cost.q_diag, wl.cost.r_diag, wl.T, xs[-1])
        us.append(u)
        xs.append(A @ xs[-1] + B @ u)
    return np.array(xs), np.array(us)


@pytest.mark.parametrize("warm,scale", [(False, False), (True, False), (False, True), (True, True)])
def test_closed_loop_follows_receding_horizon_lqr(chain, warm, scale):
    wl, pb = chain
    x0 = wl.x0(1)
    cl = CL.closed_loop(pb, x0, T_SIM, RHO, 1e-10, 40000, warm=warm, scale_rho=scale)
    xl, ul = _lqr_loop(wl, x0, T_SIM)
    assert all(cl.converged)
    assert np.abs(cl.x - xl).max() <= 1e-7 * np.abs(xl).max()
    assert np.abs(cl.u - ul).max() <= 1e-7 * np.abs(ul).max()


def test_shift_inputs_by_hand():
    lay = O.Layout(n_sub=2, nx=2, nu=1, T=4)
    y = np.zeros(lay.R)
    y[lay.Nx * lay.T:] = [1, 2, 3, 4, 5, 6]  # u_0 = (1, 2), u_1 = (3, 4), u_2 = (5, 6)
    assert CL.shift_inputs(lay, y).tolist() == [3, 4, 5, 6, 5, 6]


def test_planted_wrong_input_row_fails_pin(chain, monkeypatch):
    wl, pb = chain
    x0 = wl.x0(1)
    good = CL.closed_loop(pb, x0, 5, RHO, 1e-10, 40000)
    xl, _ = _lqr_loop(wl, x0, 5)
    assert np.abs(good.x - xl).max() <= 1e-7 * np.abs(xl).max()
    lay = pb.lay
    monkeypatch.setattr(O.Layout, "u0_rows", lambda self: self.Nx * self.T + self.Nu + np.arange(self.Nu))
    bad = CL.closed_loop(pb, x0, 5, RHO, 1e-10, 40000)
    assert lay.Nu == 10
    assert np.abs(bad.x - xl).max() > 1e-3 * np.abs(xl).max()


def test_shifted_start_saves_iterations():
    """8x8 grid (the 10-node chain's loop slows down badly once its state is small: steps of
    several thousand iterations from either start)."""
    wl = W.workload("grid8")
    pb = O.setup_from_network(wl.net, wl.d, wl.T, wl.cost)
    x0 = wl.x0(9)
    cold = CL.closed_loop(pb, x0, 10, RHO, 1e-4, 1000)
    warm = CL.closed_loop(pb, x0, 10, RHO, 1e-4, 1000, warm=True, eps_warm=0.5e-4)
    assert all(cold.converged) and all(warm.converged) and not any(warm.fell_back)
    assert sum(warm.iters[1:]) < 0.8 * sum(cold.iters[1:])
    # both loops stay near each other (each step eps-converged from a different start)
    assert np.abs(warm.x - cold.x).max() <= 1e-2 * np.abs(cold.x).max()


def test_step_rho():
    x0 = np.array([3.0, 4.0])
    assert CL.step_rho(5.0, x0, x0) == 5.0
    assert CL.step_rho(5.0, 0.1 * x0, x0) == pytest.approx(5.0 * 0.01, rel=1e-15)
    assert CL.step_rho(5.0, np.zeros(2), x0) == 5.0 * 1e-20
    assert CL.step_rho(5.0, x0, np.zeros(2)) == 5.0


def test_penalty_scaling_equivalence_unconstrained(chain):
    wl, pb = chain
    x = wl.x0(3)
    s = 0.01
    a = O.solve(pb, x, RHO, 1e-4, 5000)
    b = O.solve(pb, s * x, RHO * s * s, 1e-4, 5000)
    assert a.converged and b.iters == a.iters
    assert np.abs(b.u0 - s * a.u0).max() <= 1e-12 * np.abs(s * a.u0).max()
    # the fixed penalty at the small state is a different (slower) iteration
    c = O.solve(pb, s * x, RHO, 1e-4, 50000)
    assert c.iters > 2 * a.iters


def test_penalty_scaling_equivalence_with_active_bounds():
    """s x with penalty rho s^2 and bounds B = x with rho and bounds B / s (|theta| <= 0.8,
    |u| <= 0.3 against 1.6 and 0.6 at s = 1/2), with bounds active at the stopping iterate."""
    net = W.chain(10)
    s = 0.5
    pa = O.setup_from_network(net, 1, 5, W.box_cost(net, theta_max=0.8, u_max=0.3))
    pb_ = O.setup_from_network(net, 1, 5, W.box_cost(net, theta_max=0.8 / s, u_max=0.3 / s))
    x = W.Workload("t", net, 1, 5, W.box_cost(net, theta_max=0.8 / s, u_max=0.3 / s), sigma=0.8).x0(4)
    a = O.solve(pa, s * x, RHO * s * s, 1e-4, 5000)
    b = O.solve(pb_, x, RHO, 1e-4, 5000)
    assert a.converged and b.converged and a.iters == b.iters
    assert np.abs(a.u0 - s * b.u0).max() <= 1e-12 * np.abs(s * b.u0).max()
    active = np.sum(np.isclose(np.abs(a.y[pa.lay.Nx * pa.lay.T:]), 0.3, rtol=0, atol=1e-6))
    assert active >= 1


def test_scaled_penalty_keeps_loop_iterations_down(chain):
    """The chain's loop at a fixed penalty slows down as the state shrinks (thousands of
    iterations in late steps); the scaled penalty needs well under half of its iterations."""
    wl, pb = chain
    x0 = wl.x0(1)
    fixed = CL.closed_loop(pb, x0, T_SIM, RHO, 1e-4, 20000)
    scaled = CL.closed_loop(pb, x0, T_SIM, RHO, 1e-4, 20000, scale_rho=True)
    assert all(fixed.converged) and all(scaled.converged)
    assert fixed.iters[0] == scaled.iters[0]  # step 0 runs with rho itself
    assert sum(scaled.iters) < 0.5 * sum(fixed.iters)
    assert np.abs(scaled.x - fixed.x).max() <= 1e-2 * np.abs(fixed.x).max()
