"""Pins of the oracle with neighbour-coupled constraints (nested ADMM in Phi-comp; no GPU).

* The inner ADMM reaches the solution of the Phi-step problem min sum c (y - m)^2 over boxes
  and pair constraints computed directly by a dual active-set method with a KKT certificate
  (random instances: chains and a star of couplings, active boxes and pairs).
* With no couplings the coupled solve is the uncoupled oracle, iterate for iterate.
* The coupled outer ADMM converges to the localised program with the pair constraints written
  out as one dense QP and KKT-certified (the paper's chain plant, limits on the first-state
  difference of chain neighbours that bind).
* A planted mistake in the pair projection (both copies moved the same way) breaks the first pin.
"""
import numpy as np
import pytest

from oracle import certify as C
from oracle import coupled as CP
from oracle import dlmpc_oracle as O
from paper_2103_14990_amd import workloads as W

RHO = 5.0


def _random_phi_step(seed):
    rng = np.random.default_rng(seed)
    n = 8
    c = rng.uniform(0.3, 3.0, n)
    m = rng.normal(0.0, 1.5, n)
    lb, ub = np.full(n, -np.inf), np.full(n, np.inf)
    lb[:4], ub[:4] = -1.0, 1.0
    if seed % 2:  # a chain of couplings
        ra, rb = np.arange(0, 6), np.arange(1, 7)
    else:  # a star around row 3, and one more pair
        ra, rb = np.array([3, 3, 3, 3, 6]), np.array([0, 1, 5, 7, 7])
    lo, hi = -rng.uniform(0.1, 0.5, len(ra)), rng.uniform(0.1, 0.5, len(ra))
    return c, m, lb, ub, ra, rb, lo, hi


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_inner_admm_solves_phi_step_qp(seed):
    c, m, lb, ub, ra, rb, lo, hi = _random_phi_step(seed)
    y_ref, kkt = C.separable_qp(c, m, lb, ub, ra, rb, lo, hi)
    assert max(kkt.values()) < 1e-9
    d = y_ref[ra] - y_ref[rb]
    assert np.any(np.isclose(d, lo, atol=1e-9) | np.isclose(d, hi, atol=1e-9))  # a pair binds
    cp = CP.Coupling(ra, rb, lo, hi, sigma=1.0, inner_max=20000, inner_eps=1e-13)
    st = CP.new_state(cp)
    y = CP.nested_admm(c, m, lb, ub, np.ones(len(c), bool), cp, st)
    assert st.iters[0] < 20000
    assert np.abs(y - y_ref).max() < 1e-9


def test_no_couplings_is_the_uncoupled_oracle():
    wl = W.workload("chain10")
    pb = O.setup_from_network(wl.net, wl.d, wl.T, wl.cost)
    x0 = wl.x0(2)
    e = np.zeros(0, dtype=np.int64)
    cp = CP.Coupling(e, e, np.zeros(0), np.zeros(0))
    res, st = CP.solve(pb, x0, cp, RHO, 1e-4, 500)
    ref = O.solve(pb, x0, RHO, 1e-4, 500)
    assert res.iters == ref.iters and res.converged == ref.converged
    assert np.array_equal(res.u0, ref.u0) and np.array_equal(res.Phi, ref.Phi)
    assert st.iters == [1] * res.iters


@pytest.mark.parametrize("limit,n_active", [(0.5, 3), (0.2, 5)])
def test_coupled_solve_matches_kkt_certified_qp(limit, n_active):
    n, d, T = 10, 1, 5
    net = W.paper_chain(n)
    cost = W.unit_cost(net)
    pb = O.setup_from_network(net, d, T, cost)
    x0 = W.x0(net, 1000, 1.0)
    pairs = W.line_limits(net, T, limit, t0=1)
    qp = C.localized_qp(net.dense_A(), net.dense_B(), n, 2, 2, d, T, pb.w, x0, pb.lb, pb.ub, pairs=pairs)
    assert max(qp.kkt.values()) < 1e-9 and len(qp.active_pairs) == n_active
    cp = CP.Coupling(*pairs, sigma=1.0, inner_max=20, inner_eps=1e-10)
    res, st = CP.solve(pb, x0, cp, RHO, 1e-8, 5000)
    assert res.converged
    assert np.abs(res.y - qp.y).max() < 1e-6
    assert abs(res.J - qp.J) < 1e-7 * qp.J
    ra, rb, lo, hi = pairs
    dd = res.y[ra] - res.y[rb]
    assert np.all(dd >= lo - 1e-6) and np.all(dd <= hi + 1e-6)
    # the uncoupled optimum violates the limits: the couplings change the answer
    plain = O.solve(pb, x0, RHO, 1e-8, 5000)
    assert np.abs(plain.y[ra] - plain.y[rb]).max() > limit + 0.1


def test_planted_wrong_projection_fails_pin(monkeypatch):
    c, m, lb, ub, ra, rb, lo, hi = _random_phi_step(1)
    y_ref, _ = C.separable_qp(c, m, lb, ub, ra, rb, lo, hi)

    def wrong(pa, pb, lo_, hi_):
        d = pa - pb
        shift = 0.5 * (np.clip(d, lo_, hi_) - d)
        return pa + shift, pb + shift  # both copies moved the same way

    monkeypatch.setattr(CP, "project_pairs", wrong)
    cp = CP.Coupling(ra, rb, lo, hi, sigma=1.0, inner_max=20000, inner_eps=1e-13)
    y = CP.nested_admm(c, m, lb, ub, np.ones(len(c), bool), cp, CP.new_state(cp))
    assert np.abs(y - y_ref).max() > 1e-3
