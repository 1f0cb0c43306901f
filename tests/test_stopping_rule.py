"""Pins of the oracle's stopping rule (Algorithm 2, Conv) and of its iterates (no GPU).

The convergence check of Algorithm 2 is per column: the reading used everywhere here is
max over columns c of ||Phi[:,c] - Psi[:,c]||_2 <= eps and of ||Psi^{k+1}[:,c] - Psi^k[:,c]||_2
<= eps (absolute). The pin is a second implementation of the iteration that shares nothing with
the oracle (``certify.admm_entry_space``: entry-vector unknowns, achievability by simulating the
plant, row solves and the projection as linear systems, residuals summed per column by
bincount). Its residual history must equal the oracle's iteration by iteration, and the first
iteration at which the per-column rule holds in that history must be the oracle's iteration
count. The other plausible norms (Frobenius over all columns, largest entry, only one of the two
residuals, relative to ||Psi||) stop at other iterations on these instances, and an oracle with
such a rule planted in it fails the pin.
"""
import numpy as np
import pytest

from oracle import certify as C
from oracle import dlmpc_oracle as O
from paper_2103_14990_amd import workloads as W

RHO, EPS = 5.0, 1e-4


def _chain_case(kind):
    net = W.chain(10)
    if kind == "free":
        return net, W.unit_cost(net), 1.0
    return net, W.box_cost(net, theta_max=0.8, u_max=0.3), 0.4


def _independent(net, cost, x0, n_iter):
    pb = O.setup_from_network(net, 1, 5, cost, blocks=False)  # only for w, lb, ub in row order
    rp, rd, _ = C.admm_entry_space(net.dense_A(), net.dense_B(), net.n_sub, net.nx, net.nu, 1, 5,
                                   pb.w, x0, RHO, n_iter, pb.lb, pb.ub)
    return rp, rd


def _first(mask):
    hit = np.flatnonzero(mask)
    return int(hit[0]) + 1 if hit.size else None


CASES = [("free", 1), ("free", 2), ("free", 3), ("box", 4), ("box", 9)]


@pytest.fixture(scope="module")
def histories():
    out = {}
    for kind, seed in CASES:
        net, cost, sigma = _chain_case(kind)
        x0 = W.x0(net, seed, sigma)
        pb = O.setup_from_network(net, 1, 5, cost)
        hist = []
        res = O.solve(pb, x0, RHO, EPS, 500, progress=lambda k, rp, rd: hist.append((rp, rd)))
        n = res.iters + 40
        rp, rd = _independent(net, cost, x0, n)
        out[(kind, seed)] = (pb, x0, res, np.array(hist), rp, rd)
    return out


@pytest.mark.parametrize("case", CASES)
def test_residual_history_matches_independent_iteration(histories, case):
    _, _, res, hist, rp, rd = histories[case]
    n = res.iters
    assert np.allclose(hist[:, 0], rp[:n].max(axis=1), rtol=1e-8, atol=1e-12)
    assert np.allclose(hist[:, 1], rd[:n].max(axis=1), rtol=1e-8, atol=1e-12)


@pytest.mark.parametrize("case", CASES)
def test_iteration_count_is_first_per_column_pass(histories, case):
    _, _, res, _, rp, rd = histories[case]
    assert res.converged
    assert res.iters == _count(rp, rd)


def test_chain10_iteration_counts(histories):
    """Exact counts, stated so that a change of the rule or of the iteration shows up as a
    changed number: 216 on the unconstrained chain at seed 1 (inside the 202..216 range an
    independent scratch implementation found on this workload), 74 and 93 at seeds 2 and 3."""
    counts = [histories[("free", s)][2].iters for s in (1, 2, 3)]
    assert counts == [216, 74, 93]


def _count(rp, rd):
    return _first((rp.max(axis=1) <= EPS) & (rd.max(axis=1) <= EPS))


def test_other_norms_stop_elsewhere(histories):
    """The pin separates the per-column 2-norm from the plausible alternatives: each of them
    stops at another iteration on at least one of the instances."""
    alts = {
        "frobenius": lambda rp, rd: _first((np.sqrt((rp ** 2).sum(axis=1)) <= EPS)
                                           & (np.sqrt((rd ** 2).sum(axis=1)) <= EPS)),
        "primal only": lambda rp, rd: _first(rp.max(axis=1) <= EPS),
        "dual only": lambda rp, rd: _first(rd.max(axis=1) <= EPS),
    }
    for name, rule in alts.items():
        differs = [rule(h[4], h[5]) != h[2].iters for h in histories.values()]
        assert any(differs), name


def _max_entry(Phi, Psi, Psi_prev):
    return np.abs(Phi - Psi).max(axis=0), np.abs(Psi - Psi_prev).max(axis=0)


def _frobenius(Phi, Psi, Psi_prev):
    return np.array([np.linalg.norm(Phi - Psi)]), np.array([np.linalg.norm(Psi - Psi_prev)])


def _relative(Phi, Psi, Psi_prev):
    nrm = np.maximum(np.linalg.norm(Psi, axis=0), 1e-300)
    return np.linalg.norm(Phi - Psi, axis=0) / nrm, np.linalg.norm(Psi - Psi_prev, axis=0) / nrm


@pytest.mark.parametrize("planted", [_max_entry, _frobenius, _relative])
def test_planted_stopping_rule_fails_pin(histories, monkeypatch, planted):
    monkeypatch.setattr(O, "conv_residuals", planted)
    mismatches = 0
    for pb, x0, res, _, rp, rd in histories.values():
        bad = O.solve(pb, x0, RHO, EPS, 500)
        mismatches += bad.iters != _count(rp, rd)
    assert mismatches > 0
