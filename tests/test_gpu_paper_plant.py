"""The paper's evaluation plant (Section IV-A: chain of 2-state nodes, B_ii = I, bound -0.2 <=
x_{i,1} <= 1.2) through the C ABI against the FP64 oracle, under every single-instance schedule
(needs a GPU).

* FP64, each schedule (graph, persistent, and the per-iteration designs of Section III that the
  library keeps for comparison: stepwise, host exchange, naive): the oracle's iteration count,
  u(0), objective and Phi within 1e-9 relative. The graph and per-iteration schedules launch the
  same kernels on the same data, so their results are bit-identical; the host round trips of
  the exchange schedules move the iterate unchanged.
* FP32 batched closed loop (Algorithm 1, two inputs per node through the plant step) against
  the oracle's closed loop: u(t) and x(t) within 1e-4 relative.
* dlmpc_set_rho: FP64 single-instance solves of the oracle loop's states x(t) with the loop's
  penalty rho ||x(t)||^2 / ||x(0)||^2 take the oracle's iteration count and u(t) within 1e-9.
"""
import numpy as np
import pytest

from oracle import closed_loop as CL
from oracle import dlmpc_oracle as O
from paper_2103_14990_amd import dlmpc
from paper_2103_14990_amd import workloads as W

pytestmark = pytest.mark.gpu

RHO, EPS, MAXIT = 5.0, 1e-4, 2000
SCHEDULES = ["graph", "persistent", "stepwise", "host_exchange", "naive"]


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


@pytest.fixture(scope="module")
def chain25():
    wl = W.workload("paper_chain25_d2_T10")
    pb = O.setup_from_network(wl.net, wl.d, wl.T, wl.cost)
    seeds = [1000, 1002, 1003]
    return wl, pb, seeds, {s: O.solve(pb, wl.x0(s), RHO, EPS, MAXIT) for s in seeds}


def test_schedules_match_oracle_fp64(chain25):
    wl, pb, seeds, refs = chain25
    rp = ci = None
    results = {}
    for sched in SCHEDULES:
        pr = dlmpc.Problem.from_network(wl.net, wl.d, wl.T, wl.cost, rho=RHO, eps=EPS, max_iter=MAXIT,
                                        precision="fp64", schedule=sched)
        assert dlmpc.SCHEDULE_NAMES[pr.info["schedule"]] == sched
        if rp is None:
            rp, ci = pr.phi_pattern()
            rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
        for s in seeds:
            r = pr.solve(wl.x0(s), want_phi=True)
            o = refs[s]
            print(f"  {sched} seed {s}: iters gpu {r.stats['iters']} oracle {o.iters} "
                  f"t_iter {r.stats['t_iter_ms']:.3f} ms", flush=True)
            assert r.stats["iters"] == o.iters and r.status == dlmpc.OK and o.converged
            assert rel(r.u0, o.u0) < 1e-9
            assert abs(r.stats["objective"] - o.J) <= 1e-9 * o.J
            assert rel(r.phi, o.Phi[rows, ci]) < 1e-9
            results[sched, s] = r
        pr.close()
    # the active bound: some first-state rows of y sit on -0.2 or 1.2
    assert any(np.isclose(refs[s].y, -0.2, atol=1e-6).any() for s in seeds)
    for sched in ("stepwise", "host_exchange", "naive"):
        for s in seeds:
            assert np.array_equal(results[sched, s].u0, results["graph", s].u0)
            assert np.array_equal(results[sched, s].phi, results["graph", s].phi)
            assert results[sched, s].stats["graph_launches"] == results[sched, s].stats["iters"]


def test_two_schedule_flags_rejected():
    wl = W.workload("paper_chain10")
    with pytest.raises(dlmpc.DlmpcError) as e:
        dlmpc.Problem(wl.net.n_sub, wl.net.nx, wl.net.nu, wl.net.a_rowptr, wl.net.a_colidx, wl.net.a_blocks,
                      wl.net.b_blocks, wl.d, wl.T, wl.cost.q_diag, wl.cost.r_diag, wl.cost.x_lo, wl.cost.x_hi,
                      wl.cost.u_lo, wl.cost.u_hi, schedule="naive", flags=dlmpc.FLAG_SCHED_GRAPH)
    assert e.value.status == dlmpc.EINVAL


def test_closed_loop_fp32_matches_oracle(torch):
    wl = W.workload("paper_chain25_d2_T10")
    pb = O.setup_from_network(wl.net, wl.d, wl.T, wl.cost)
    seeds, T_sim = [1000, 1003], 8
    B, G = len(seeds), wl.net.n_sub
    pr = dlmpc.Problem.from_network(wl.net, wl.d, wl.T, wl.cost, rho=RHO, eps=EPS, max_iter=MAXIT,
                                    precision="fp32", max_batch=4)
    x0 = np.stack([wl.x0(s) for s in seeds])
    xd = torch.tensor(x0, dtype=torch.float64, device="cuda")
    xs = torch.zeros((B, T_sim + 1, G * 2), dtype=torch.float64, device="cuda")
    us = torch.zeros((B, T_sim, G * 2), dtype=torch.float64, device="cuda")
    st, stats = pr.closed_loop(B, T_sim, xd.data_ptr(), xs.data_ptr(), us.data_ptr(), scale_rho=True)
    assert st == dlmpc.OK
    xs, us = xs.cpu().numpy(), us.cpu().numpy()
    for b, s in enumerate(seeds):
        ref = CL.closed_loop(pb, x0[b], T_sim, RHO, EPS, MAXIT, scale_rho=True)
        it_g = [stats[t][b]["iters"] for t in range(T_sim)]
        eu = max(rel(us[b, t], ref.u[t]) for t in range(T_sim))
        ex = rel(xs[b], ref.x)
        print(f"  seed {s}: iters gpu {it_g} oracle {ref.iters}; u rel {eu:.2e} x rel {ex:.2e}", flush=True)
        assert all(ref.converged)
        assert all(abs(a - o) <= 5 for a, o in zip(it_g, ref.iters))
        assert eu < 1e-4 and ex < 1e-4


def test_set_rho_reproduces_scaled_loop_steps_fp64():
    wl = W.workload("paper_chain25_d2_T10")
    pb = O.setup_from_network(wl.net, wl.d, wl.T, wl.cost)
    ref = CL.closed_loop(pb, wl.x0(1003), 6, RHO, EPS, MAXIT, scale_rho=True)
    pr = dlmpc.Problem.from_network(wl.net, wl.d, wl.T, wl.cost, rho=RHO, eps=EPS, max_iter=MAXIT,
                                    precision="fp64", schedule="graph")
    for t in range(6):
        rho_t = CL.step_rho(RHO, ref.x[t], ref.x[0])
        pr.set_rho(rho_t)
        r = pr.solve(ref.x[t])
        print(f"  t {t}: rho {rho_t:.3e} iters gpu {r.stats['iters']} oracle {ref.iters[t]}", flush=True)
        assert r.stats["iters"] == ref.iters[t]
        assert rel(r.u0, ref.u[t]) < 1e-9
    with pytest.raises(dlmpc.DlmpcError):
        pr.set_rho(0.0)
    pr.set_rho(RHO)  # back to rho: the first step's solve again
    r = pr.solve(ref.x[0])
    assert r.stats["iters"] == ref.iters[0]
