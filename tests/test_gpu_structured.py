"""Structured Psi-comp (DLMPC_FLAG_STRUCTURED_PSI) against the FP64 oracle (needs a GPU).

A null-space trajectory of column subsystem j is fixed by its input rows (x_0 = 0, the patch
dynamics give the states), so the library's Psi-comp can read only the input rows N_u of each
null basis and rebuild the state rows by simulating the patch (adjoint recursion for N_j' v,
forward simulation for N_j t). Same iteration as the dense Psi-comp up to rounding, hence the
same bars: FP64 the oracle's iteration count, u(0), J and Phi within 1e-9 relative; FP32 u(0)
within 1e-4 and J within 1e-5. Shapes: the swing chain and the 16x16 box grid, generic nx/nu/d/T
(T = 2 included), the paper's plant (two inputs per node), and the 1024 mesh against the stored
oracle values.
"""
import json
import os

import numpy as np
import pytest

from oracle import dlmpc_oracle as O
from paper_2103_14990_amd import dlmpc
from paper_2103_14990_amd import workloads as W

pytestmark = pytest.mark.gpu

RHO, EPS, MAXIT = 5.0, 1e-4, 2000
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "irregular1024_box.json")


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _pair(wl, precision="fp64", **kw):
    mk = lambda s: dlmpc.Problem.from_network(wl.net, wl.d, wl.T, wl.cost, rho=RHO, eps=EPS, max_iter=MAXIT,
                                              precision=precision, schedule="graph", structured_psi=s, **kw)
    return mk(False), mk(True)


def _cases():
    out = [("chain10", W.workload("chain10"), [1, 2, 3]), ("grid16_box", W.workload("grid16_box"), [1000]),
           ("paper_chain25_d2_T10", W.workload("paper_chain25_d2_T10"), [1000, 1003])]
    edges = np.array([(0, 1), (1, 2), (2, 3), (3, 4), (1, 4), (4, 5), (5, 6)])
    for nx, nu, d, T, seed in [(1, 1, 1, 4, 0), (3, 2, 2, 3, 1), (4, 1, 2, 3, 3), (2, 1, 2, 2, 1)]:
        net = W.generic_network(7, edges, nx, nu, seed)
        out.append((f"generic_nx{nx}_nu{nu}_d{d}_T{T}", W.Workload("g", net, d, T, W.unit_cost(net), sigma=1.0), [1, 7]))
    return out


@pytest.mark.parametrize("name,wl,seeds", _cases(), ids=[c[0] for c in _cases()])
def test_structured_fp64_matches_oracle(name, wl, seeds):
    pb = O.setup_from_network(wl.net, wl.d, wl.T, wl.cost)
    if not pb.feasible:
        pytest.skip(f"random plant not localisable at d = {wl.d}")
    dense, structured = _pair(wl)
    rp, ci = structured.phi_pattern()
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    for s in seeds:
        x0 = wl.x0(s)
        ref = O.solve(pb, x0, RHO, EPS, MAXIT)
        r = structured.solve(x0, want_phi=True)
        q = dense.solve(x0)
        print(f"  {name} seed {s}: iters structured {r.stats['iters']} dense {q.stats['iters']} oracle {ref.iters}; "
              f"u0 rel {rel(r.u0, ref.u0):.1e} vs dense {rel(r.u0, q.u0):.1e}", flush=True)
        assert r.stats["iters"] == ref.iters and (r.status == dlmpc.OK) == ref.converged
        assert rel(r.u0, ref.u0) < 1e-9
        assert abs(r.stats["objective"] - ref.J) <= 1e-9 * ref.J
        assert rel(r.phi, ref.Phi[rows, ci]) < 1e-9
        assert rel(r.u0, q.u0) < 1e-11
        assert r.stats["eq_resid"] < 1e-9  # the certificate of the structured iterate


def test_structured_fp32_within_bar():
    wl = W.workload("grid16_box")
    pb = O.setup_from_network(wl.net, wl.d, wl.T, wl.cost)
    _, structured = _pair(wl, "fp32")
    for s in (1000, 1001):
        x0 = wl.x0(s)
        ref = O.solve(pb, x0, RHO, EPS, MAXIT)
        r = structured.solve(x0)
        print(f"  fp32 seed {s}: iters {r.stats['iters']} oracle {ref.iters} u0 rel {rel(r.u0, ref.u0):.2e}", flush=True)
        assert r.status == dlmpc.OK
        assert rel(r.u0, ref.u0) < 1e-4
        assert abs(r.stats["objective"] - ref.J) <= 1e-5 * ref.J
        assert abs(r.stats["iters"] - ref.iters) <= 5


def test_structured_full_size_against_stored_oracle():
    gold = json.load(open(GOLDEN))
    wl = W.workload("irregular1024_box")
    kw = dict(rho=wl.rho, eps=wl.eps, max_iter=wl.max_iter, schedule="graph")
    pr = dlmpc.Problem.from_network(wl.net, wl.d, wl.T, wl.cost, precision="fp64", structured_psi=True, **kw)
    for rec in gold["records"]:
        r = pr.solve(wl.x0(rec["seed"]))
        u0 = np.array(rec["u0"])
        print(f"  mesh seed {rec['seed']}: iters {r.stats['iters']} oracle {rec['iters']} u0 rel {rel(r.u0, u0):.2e} "
              f"t_iter {r.stats['t_iter_ms']:.2f} ms", flush=True)
        assert r.stats["iters"] == rec["iters"]
        assert rel(r.u0, u0) < 1e-9
        assert abs(r.stats["objective"] - rec["J"]) < 1e-9 * rec["J"]
    # per-launch kernel times, dense against structured (FP32, the same x0)
    x = __import__("torch").tensor(wl.x0(1000), dtype=__import__("torch").float64, device="cuda")
    times = {}
    for s in (False, True):
        p_ = dlmpc.Problem.from_network(wl.net, wl.d, wl.T, wl.cost, precision="fp32", structured_psi=s, **kw)
        times[s] = p_.time_kernels(x.data_ptr(), 20)
        p_.close()
    print(f"  FP32 us per launch: dense {times[False]}\n      structured {times[True]}", flush=True)


def test_structured_rejects_persistent():
    wl = W.workload("chain10")
    with pytest.raises(dlmpc.DlmpcError) as e:
        dlmpc.Problem.from_network(wl.net, wl.d, wl.T, wl.cost, precision="fp64", schedule="persistent",
                                   structured_psi=True)
    assert e.value.status == dlmpc.EINVAL


def test_setup_times_structured_against_dense(tmp_path, monkeypatch):
    """Without a schedule flag, setup times the graph schedule with the dense and with the
    structured Psi-comp (and the persistent schedule) and keeps the fastest; the cache replays
    the choice without timing."""
    monkeypatch.setenv("DLMPC_TUNE_CACHE", str(tmp_path / "tune.txt"))
    wl = W.workload("grid16_box")
    mk = lambda: dlmpc.Problem.from_network(wl.net, wl.d, wl.T, wl.cost, rho=RHO, eps=EPS, max_iter=MAXIT,
                                            precision="fp32")
    a = mk()
    ia = a.info
    print(f"  graph {ia['tune_graph_us']:.1f} us, persistent {ia['tune_persistent_us']:.1f} us, structured "
          f"{ia['tune_structured_us']:.1f} us -> schedule {ia['schedule']} structured {ia['psi_structured']}", flush=True)
    assert ia["tune_structured_us"] > 0 and ia["tune_cached"] == 0
    cands = {(0, 0): ia["tune_graph_us"], (0, 1): ia["tune_structured_us"]}
    if ia["tune_persistent_us"] > 0:
        cands[(1, 0)] = ia["tune_persistent_us"]
    assert (ia["schedule"], ia["psi_structured"]) == min(cands, key=cands.get)
    b = mk()
    ib = b.info
    assert ib["tune_cached"] == 1 and (ib["schedule"], ib["psi_structured"]) == (ia["schedule"], ia["psi_structured"])
    x0 = wl.x0(1000)
    ra, rb = a.solve(x0), b.solve(x0)
    assert np.array_equal(ra.u0, rb.u0) and ra.stats["iters"] == rb.stats["iters"]


@pytest.mark.parametrize("name", ["grid8", "paper_chain25_d2_T10"])
def test_batched_structured_psi_matches_oracle(tmp_path, monkeypatch, name):
    """The batched engine's structured Psi-comp (batch_psi_capx 0, forced through the tuning
    cache): FP32-tier bar against the FP64 oracle, instance by instance."""
    wl = W.workload(name)
    pb = O.setup_from_network(wl.net, wl.d, wl.T, wl.cost)
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("DLMPC_TUNE_CACHE", str(cache))
    mk = lambda: dlmpc.Problem.from_network(wl.net, wl.d, wl.T, wl.cost, rho=RHO, eps=EPS, max_iter=MAXIT,
                                            precision="fp32", max_batch=8)
    probe = mk()
    sig = cache.read_text().split("|")[0]
    probe.close()
    cache.write_text(f"{sig}|phi_ntw=1 psi_capx=0 sched=0\n")
    pr = mk()
    assert pr.info["batch_psi_capx"] == 0 and pr.info["tune_cached"] == 1
    seeds = [1000 + i for i in range(8)]
    x0 = np.stack([wl.x0(s) for s in seeds])
    st, u0, stats = pr.solve_batch(x0)
    for i, s in enumerate(seeds):
        ref = O.solve(pb, x0[i], RHO, EPS, MAXIT)
        print(f"  {name} seed {s}: iters {stats[i]['iters']} oracle {ref.iters} u0 rel {rel(u0[i], ref.u0):.2e}",
              flush=True)
        assert stats[i]["converged"] and ref.converged
        assert rel(u0[i], ref.u0) < 1e-4
        assert abs(stats[i]["objective"] - ref.J) <= 1e-5 * ref.J
        assert abs(stats[i]["iters"] - ref.iters) <= 5
