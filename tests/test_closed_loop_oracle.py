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


@pytest.mark.parametrize("warm", [False, True])
def test_closed_loop_follows_receding_horizon_lqr(chain, warm):
    wl, pb = chain
    x0 = wl.x0(1)
    cl = CL.closed_loop(pb, x0, T_SIM, RHO, 1e-10, 40000, warm=warm)
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
