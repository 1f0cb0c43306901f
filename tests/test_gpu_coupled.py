"""Neighbour-coupled constraints (nested ADMM inside Phi-comp) through the C ABI against the
coupled oracle (needs a GPU).

* FP64, the paper's chain plant with limits on the first-state difference of chain neighbours
  (binding): the oracle's outer iteration count and total nested-ADMM iterations, u(0),
  objective and Phi within 1e-9 relative, under the graph schedule and the per-iteration ones.
* Tight outer eps: the returned trajectory meets the limits and matches the dense localised QP
  with the pair constraints, KKT-certified (oracle/certify.py).
* FP32: u(0) within 1e-4 and the objective within 1e-5 relative of the FP64 oracle.
* Removing the couplings gives the uncoupled solve back; batched entries refuse a coupled
  problem; bad arguments are rejected.
"""
import numpy as np
import pytest

from oracle import certify as C
from oracle import coupled as CP
from oracle import dlmpc_oracle as O
from paper_2103_14990_amd import dlmpc
from paper_2103_14990_amd import workloads as W

pytestmark = pytest.mark.gpu

RHO, EPS = 5.0, 1e-4
SIGMA, INNER_MAX, INNER_EPS = 1.0, 20, 1e-10


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _case(n, d, T, limit):
    net = W.paper_chain(n)
    cost = W.unit_cost(net)
    pairs = W.line_limits(net, T, limit, t0=1)
    return net, cost, pairs, O.setup_from_network(net, d, T, cost)


def _problem(net, cost, d, T, pairs, precision="fp64", **kw):
    pr = dlmpc.Problem.from_network(net, d, T, cost, rho=RHO, eps=kw.pop("eps", EPS), max_iter=kw.pop("max_iter", 3000),
                                    precision=precision, **kw)
    pr.set_coupling(*pairs, sigma=SIGMA, inner_max=INNER_MAX, inner_eps=INNER_EPS)
    return pr


@pytest.mark.parametrize("n,d,T,limit", [(10, 1, 5, 0.5), (10, 1, 5, 0.2), (25, 2, 8, 0.3)])
def test_coupled_fp64_matches_oracle(n, d, T, limit):
    net, cost, pairs, pb = _case(n, d, T, limit)
    cp = CP.Coupling(*pairs, sigma=SIGMA, inner_max=INNER_MAX, inner_eps=INNER_EPS)
    rows = None
    res_graph = {}
    for sched in ("graph", "stepwise", "naive"):
        pr = _problem(net, cost, d, T, pairs, schedule=sched)
        if rows is None:
            rp, ci = pr.phi_pattern()
            rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
        for seed in (1000, 1003):
            x0 = W.x0(net, seed, 1.0)
            ref, st = CP.solve(pb, x0, cp, RHO, EPS, 3000)
            r = pr.solve(x0, want_phi=True)
            s = r.stats
            print(f"  {sched} n {n} limit {limit} seed {seed}: outer gpu {s['iters']} oracle {ref.iters}, inner gpu "
                  f"{s['inner_iters']} oracle {sum(st.iters)}, viol {s['coupling_viol']:.1e}", flush=True)
            assert ref.converged and r.status == dlmpc.OK
            assert s["iters"] == ref.iters and s["inner_iters"] == sum(st.iters)
            assert rel(r.u0, ref.u0) < 1e-9
            assert abs(s["objective"] - ref.J) <= 1e-9 * ref.J
            assert rel(r.phi, ref.Phi[rows, ci]) < 1e-9
            if sched == "graph":
                res_graph[seed] = r
            else:
                assert np.array_equal(r.u0, res_graph[seed].u0)
        pr.close()


def test_coupled_tight_solve_meets_limits_and_certified_qp():
    n, d, T, limit = 10, 1, 5, 0.2
    net, cost, pairs, pb = _case(n, d, T, limit)
    x0 = W.x0(net, 1000, 1.0)
    qp = C.localized_qp(net.dense_A(), net.dense_B(), n, 2, 2, d, T, pb.w, x0, pb.lb, pb.ub, pairs=pairs)
    assert max(qp.kkt.values()) < 1e-9 and len(qp.active_pairs) >= 3
    pr = _problem(net, cost, d, T, pairs, eps=1e-8, max_iter=20000)
    r = pr.solve(x0)
    print(f"  tight: iters {r.stats['iters']} inner {r.stats['inner_iters']} viol {r.stats['coupling_viol']:.2e} "
          f"u0 rel {rel(r.u0, qp.y[pb.lay.u0_rows()]):.2e}", flush=True)
    assert r.status == dlmpc.OK
    assert r.stats["coupling_viol"] < 1e-6
    assert rel(r.u0, qp.y[pb.lay.u0_rows()]) < 1e-6
    assert abs(r.stats["objective"] - qp.J) < 1e-7 * qp.J


def test_coupled_fp32_within_reduced_precision_bar():
    n, d, T, limit = 25, 2, 8, 0.3
    net, cost, pairs, pb = _case(n, d, T, limit)
    cp = CP.Coupling(*pairs, sigma=SIGMA, inner_max=INNER_MAX, inner_eps=INNER_EPS)
    pr = _problem(net, cost, d, T, pairs, precision="fp32")
    for seed in (1000, 1003):
        x0 = W.x0(net, seed, 1.0)
        ref, _ = CP.solve(pb, x0, cp, RHO, EPS, 3000)
        r = pr.solve(x0)
        print(f"  fp32 seed {seed}: iters gpu {r.stats['iters']} oracle {ref.iters}, u0 rel {rel(r.u0, ref.u0):.2e}",
              flush=True)
        assert r.status == dlmpc.OK
        assert rel(r.u0, ref.u0) < 1e-4
        assert abs(r.stats["objective"] - ref.J) <= 1e-5 * ref.J
        assert abs(r.stats["iters"] - ref.iters) <= max(5, 0.05 * ref.iters)


def test_removing_couplings_and_errors():
    n, d, T, limit = 10, 1, 5, 0.2
    net, cost, pairs, pb = _case(n, d, T, limit)
    x0 = W.x0(net, 1003, 1.0)
    pr = _problem(net, cost, d, T, pairs, precision="fp32", max_batch=4, schedule="graph")
    with pytest.raises(dlmpc.DlmpcError) as e:
        pr.solve_batch(np.stack([x0, x0]))
    assert e.value.status == dlmpc.EINVAL
    e0 = np.zeros(0)
    pr.set_coupling(e0, e0, e0, e0)
    r = pr.solve(x0)
    plain = dlmpc.Problem.from_network(net, d, T, cost, rho=RHO, eps=EPS, max_iter=3000, precision="fp32",
                                       schedule="graph")
    q = plain.solve(x0)
    assert r.stats["iters"] == q.stats["iters"] and np.array_equal(r.u0, q.u0) and r.stats["inner_iters"] == 0
    st, u0, _ = pr.solve_batch(np.stack([x0, x0]))  # batched entries work again
    ra, rb, lo, hi = pairs
    Nx = net.n_sub * net.nx
    for bad in [(ra[:1] * 0 + 3, rb[:1], lo[:1], hi[:1]),          # a row of x_0
                (ra[:1], ra[:1], lo[:1], hi[:1]),                  # the same row twice
                (ra[:1], rb[:1], hi[:1], lo[:1]),                  # lo > hi
                (ra[:1] * 0 + 10 * Nx, rb[:1], lo[:1], hi[:1])]:   # out of range
        with pytest.raises(dlmpc.DlmpcError) as e:
            pr.set_coupling(*bad)
        assert e.value.status == dlmpc.EINVAL
    with pytest.raises(dlmpc.DlmpcError):
        pr.set_coupling(*pairs, sigma=0.0)
