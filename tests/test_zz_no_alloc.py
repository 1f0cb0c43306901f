"""Allocation-free streamed solve (dlmpc_solve_stream_noalloc) against dlmpc_solve_stream, through
the C ABI (needs a GPU).

Per instance a streamed solve is deterministic (same start, same iterates, same stopping rule
whatever slot and moment it joins), so the two entry points must return identical u(0), iteration
counts, convergence flags and FP64 checks: compared on two calls in a row, the second with fewer
instances than the first (the static staging keeps the first call's contents)."""
import numpy as np
import pytest

from paper_2103_14990_amd import dlmpc
from paper_2103_14990_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def _trained(torch, wl, slots):
    pr = dlmpc.Problem.from_network(wl.net, wl.d, wl.T, wl.cost, rho=wl.rho, eps=wl.eps, max_iter=wl.max_iter,
                                    precision="fp32", max_batch=slots)
    G, nx, nu = wl.net.n_sub, wl.net.nx, wl.net.nu
    rs = nx * wl.T + nu * (wl.T - 1)
    n_train = 4 * slots
    xt = torch.tensor(np.stack([wl.x0(10**6 + i) for i in range(n_train)]), dtype=torch.float64, device="cuda")
    yt = torch.zeros((n_train, G * rs), dtype=torch.float64, device="cuda")
    ut = torch.zeros((n_train, G * nu), dtype=torch.float64, device="cuda")
    for s0 in range(0, n_train, slots):
        pr.solve_batch_ex(slots, xt[s0:].data_ptr(), ut[s0:].data_ptr(), "cold", 0, yt[s0:].data_ptr())
    ys = float(yt.view(n_train, G, rs)[:, :, nx * wl.T:].std().item())
    pr.ws_init(16, slots, seed=3, x_scale=wl.sigma, y_scale=ys)
    for k in range(200):
        pr.ws_train_step(slots, xt[(k % 4) * slots:].data_ptr(), yt[(k % 4) * slots:].data_ptr(), 2e-3)
    return pr


def test_noalloc_stream_matches_stream(torch):
    wl = W.workload("grid16_box")
    slots = 16
    pr = _trained(torch, wl, slots)
    G, nu = wl.net.n_sub, wl.net.nu
    for call, n in enumerate((45, 19)):  # the second call is smaller
        x = torch.tensor(np.stack([wl.x0(8000 + 100 * call + i) for i in range(n)]), dtype=torch.float64,
                         device="cuda")
        ua = torch.zeros((n, G * nu), dtype=torch.float64, device="cuda")
        ub = torch.full((n, G * nu), float("nan"), dtype=torch.float64, device="cuda")
        sta, sa, ia = pr.solve_stream(n, x.data_ptr(), ua.data_ptr())
        stb, sb, ib = pr.solve_stream_noalloc(n, x.data_ptr(), ub.data_ptr())
        print(f"  call {call}: n {n}, joins {ib['joins']}, iterations mean {np.mean([q['iters'] for q in sb]):.1f}, "
              f"status {stb}", flush=True)
        assert sta == stb
        assert torch.equal(ua, ub)
        for qa, qb in zip(sa, sb):
            for key in ("iters", "converged", "fell_back", "eq_resid", "u0_check", "objective"):
                assert qa[key] == qb[key], key
        assert ia["joins"] == ib["joins"] and ia["instance_iterations"] == ib["instance_iterations"]
        assert ib["joins"] > 1
    pr.close()


def test_noalloc_stream_rejects_oversize(torch):
    """max_batch * N * (nx*T + nu*(T-1)) above the static staging: a clear error, no device work."""
    net = W.chain(1200)
    cost = W.unit_cost(net)
    pr = dlmpc.Problem.from_network(net, 1, 20, cost, precision="fp32", max_batch=64)
    assert 64 * 1200 * (2 * 20 + 19) > 4 * 2 ** 20
    pr.ws_init(8, 4, seed=1)
    x = torch.zeros((2, 2400), dtype=torch.float64, device="cuda")
    u = torch.zeros((2, 1200), dtype=torch.float64, device="cuda")
    with pytest.raises(dlmpc.DlmpcError) as e:
        pr.solve_stream_noalloc(2, x.data_ptr(), u.data_ptr())
    assert e.value.status == dlmpc.EINVAL and "static staging" in str(e.value)
    pr.close()
