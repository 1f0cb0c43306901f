"""Pins of the FP64 trajectory warm start (no GPU).

* simulated trajectories satisfy the achievability equations Z_AB y = [x0; 0; ...];
* conjugate gradients reach the exact solution of an SPD system in n steps (textbook), checked
  against a direct solve;
* the start is feasible and local (Z_AB Psi^0 = I on every column, pattern L_d), and its
  trajectory is b + M beta (the identity the construction relies on);
* from the optimal input trajectory (oracle run to 1e-10) the start is a fixed point when no
  bound is active (ADMM stops within two iterations at the same u(0)); with active bounds the
  multiplier guess -2 w y / rho misses the bound multipliers, so the start only needs fewer
  iterations than the zero start; from a perturbed trajectory it still meets eps and needs
  fewer iterations than the zero start.
"""
import numpy as np
import pytest

from oracle import dlmpc_oracle as O
from oracle import warm_start as WS
from paper_2103_14990_amd import workloads as W

RHO, EPS = 5.0, 1e-4


@pytest.fixture(scope="module")
def chain():
    wl = W.workload("chain10")
    return wl, O.setup_from_network(wl.net, wl.d, wl.T, wl.cost)


@pytest.fixture(scope="module")
def chain_box():
    net = W.chain(10)
    cost = W.box_cost(net, theta_max=0.8, u_max=0.3)
    return W.Workload("chain10_box", net, 1, 5, cost, sigma=0.4), O.setup_from_network(net, 1, 5, cost)


def test_simulation_satisfies_achievability(chain):
    wl, pb = chain
    rng = np.random.default_rng(0)
    x0 = rng.standard_normal(pb.lay.Nx)
    y = WS.simulate_states(pb, x0, rng.standard_normal(pb.lay.R))
    Z = O.build_zab(pb.A, pb.B, pb.lay.T)
    rhs = np.zeros(Z.shape[0])
    rhs[:pb.lay.Nx] = x0
    assert np.abs(Z @ y - rhs).max() < 1e-12


def test_conjugate_gradient_solves_spd_system_in_n_steps():
    rng = np.random.default_rng(1)
    n = 12
    G = rng.standard_normal((n, n))
    A = G @ G.T + 0.1 * np.eye(n)
    b = rng.standard_normal(n)
    x = WS.conjugate_gradient(lambda v: A @ v, b, n)
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-8, atol=1e-10)
    # one step is the steepest-descent step along b
    x1 = WS.conjugate_gradient(lambda v: A @ v, b, 1)
    assert np.allclose(x1, (b @ b) / (b @ A @ b) * b, rtol=1e-14)


def test_start_is_feasible_local_and_tracks_b_plus_m_beta(chain):
    wl, pb = chain
    x0 = wl.x0(3)
    rng = np.random.default_rng(2)
    u_hat = rng.standard_normal(pb.lay.Nu * (pb.lay.T - 1))
    psi0, lam0, y_hat, beta = WS.trajectory_start(pb, x0, u_hat, RHO, 30)
    Z = O.build_zab(pb.A, pb.B, pb.lay.T)
    rhs = np.zeros((Z.shape[0], pb.lay.Nx))
    rhs[:pb.lay.Nx] = np.eye(pb.lay.Nx)
    assert np.abs(Z @ psi0 - rhs).max() < 1e-10
    assert np.all(psi0[~pb.mask] == 0) and np.all(lam0[~pb.mask] == 0)
    b = WS.offset_rows(pb, x0)
    assert np.allclose(psi0 @ x0, b + WS.apply_m(pb, x0, beta), rtol=1e-12, atol=1e-12)
    assert np.allclose(y_hat[pb.lay.Nx * pb.lay.T:], u_hat)


@pytest.mark.parametrize("case", ["chain", "chain_box"])
def test_optimal_trajectory_start_is_a_fixed_point(case, request):
    wl, pb = request.getfixturevalue(case)
    seeds = (3, 4) if case == "chain" else (9, 10)
    for seed in seeds:
        x0 = wl.x0(seed)
        exact = O.solve(pb, x0, RHO, 1e-10, 20000)
        cold = O.solve(pb, x0, RHO, EPS, 500)
        u_star = exact.y[pb.lay.Nx * pb.lay.T:]
        psi0, lam0, _, _ = WS.trajectory_start(pb, x0, u_star, RHO, 60)
        warm = O.solve(pb, x0, RHO, EPS, 500, psi0=psi0, lam0=lam0)
        print(f"  {case} seed {seed}: cold {cold.iters}, optimal-trajectory start {warm.iters}")
        assert exact.converged and warm.converged
        if case == "chain":
            assert warm.iters <= 2
            assert np.abs(warm.u0 - exact.u0).max() <= 1e-6 * np.abs(exact.u0).max()
        else:
            assert warm.iters < cold.iters
            assert np.abs(warm.u0 - exact.u0).max() <= 1e-3 * np.abs(exact.u0).max()
        rng = np.random.default_rng(seed)
        psi0, lam0, _, _ = WS.trajectory_start(pb, x0, u_star * (1 + 0.01 * rng.standard_normal(u_star.shape)),
                                              RHO, 20)
        noisy = O.solve(pb, x0, RHO, EPS, 500, psi0=psi0, lam0=lam0)
        print(f"    1% perturbed trajectory start: {noisy.iters}")
        assert noisy.converged and noisy.iters < cold.iters
