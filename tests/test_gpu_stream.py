"""Streamed solves (instances joining free slots of a running batched solve) through the C ABI
(needs a GPU).

With the learned start every per-instance step of the batched iteration is independent of the
other instances and of the global iteration count, so an instance streamed into any slot at
any moment follows exactly the iterates of the same instance in dlmpc_solve_batch_ex: u(0),
iteration counts, convergence, fallbacks and the FP64 check's values (run on a stash of the
stopped instances' states, emptied whenever it fills: more instances than slots) are compared
for equality."""
import numpy as np
import pytest

from paper_2103_14990_amd import dlmpc
from paper_2103_14990_amd import workloads as W

pytestmark = pytest.mark.gpu

RHO, EPS, CG = 5.0, 1e-4, 16


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def _trained(torch, name, max_batch, n_train=256, steps=300, precision="fp32", eps=EPS):
    """Problem with a warm-start network trained briefly on cold solves (the comparison holds
    for any weights; training only makes the starts realistic)."""
    wl = W.workload(name)
    pr = dlmpc.Problem.from_network(wl.net, wl.d, wl.T, wl.cost, rho=RHO, eps=eps, max_iter=500,
                                    precision=precision, max_batch=max_batch, warm_cg_iters=CG)
    G, rs = wl.net.n_sub, wl.net.nx * wl.T + wl.net.nu * (wl.T - 1)
    xd = torch.tensor(np.stack([wl.x0(10**6 + i) for i in range(n_train)]), dtype=torch.float64, device="cuda")
    yd = torch.zeros((n_train, G * rs), dtype=torch.float64, device="cuda")
    ud = torch.zeros((n_train, G * wl.net.nu), dtype=torch.float64, device="cuda")
    for s0 in range(0, n_train, max_batch):
        n = min(max_batch, n_train - s0)
        pr.solve_batch_ex(n, xd[s0:].data_ptr(), ud[s0:].data_ptr(), "cold", 0, yd[s0:].data_ptr())
    roff = wl.net.nx * wl.T
    ys = float(yd.view(n_train, G, rs)[:, :, roff:].std().item())
    pr.ws_init(32, max_batch, seed=1, x_scale=wl.sigma, y_scale=ys)
    rng = np.random.default_rng(0)
    for step in range(steps):
        idx = int(rng.integers(0, n_train // max_batch)) * max_batch
        pr.ws_train_step(max_batch, xd[idx:].data_ptr(), yd[idx:].data_ptr(), 2e-3 if step < 200 else 5e-4)
    return wl, pr


def _batched_reference(torch, pr, xd, B):
    n = xd.shape[0]
    u = torch.zeros((n, pr.n_sub * pr.nu), dtype=torch.float64, device="cuda")
    stats = []
    for s0 in range(0, n, B):
        c = min(B, n - s0)
        st, s = pr.solve_batch_ex(c, xd[s0:].data_ptr(), u[s0:].data_ptr(), "learned")
        assert st in (dlmpc.OK, dlmpc.ENOCONV)
        stats += s
    return u, stats


@pytest.mark.parametrize("name,n,B,refill_min,check_iters,precision", [
    ("grid8", 57, 16, 4, 3, "fp32"),       # many joins, a few slots at a time
    ("grid8", 40, 16, 0, 0, "fp32"),       # defaults: a tenth of the slots, checks every 12 iterations
    ("grid16_box", 37, 8, 2, 5, "fp32"),   # active bounds
    ("grid8", 5, 16, 0, 0, "fp32"),        # fewer instances than slots: one fill, no join
    ("grid8", 6, 1, 0, 0, "fp32"),         # one slot: the stash holds one instance, checked at every stop
    ("grid8", 30, 4, 1, 1, "fp32"),        # a check after every iteration, joins of single slots
    ("grid16_box", 37, 8, 2, 5, "fp32_bf16"),  # reduced-operator tier (eps 1e-3, above its floor)
])
def test_stream_equals_batched_learned_solves(torch, name, n, B, refill_min, check_iters, precision):
    wl, pr = _trained(torch, name, B, precision=precision, eps=EPS if precision == "fp32" else 1e-3)
    x0s = np.stack([wl.x0(3000 + i) for i in range(n)])
    xd = torch.tensor(x0s, dtype=torch.float64, device="cuda")
    us = torch.zeros((n, pr.n_sub * pr.nu), dtype=torch.float64, device="cuda")
    st, ss, info = pr.solve_stream(n, xd.data_ptr(), us.data_ptr(), refill_min, check_iters)
    ub, sb = _batched_reference(torch, pr, xd, B)
    it_s = [s["iters"] for s in ss]
    print(f"  {name} n {n} slots {B}: iterations mean {np.mean(it_s):.1f} max {max(it_s)}, joins {info['joins']}, "
          f"checks {info['checks']}, slot use {info['instance_iterations'] / max(info['slot_iterations'], 1):.2f}, "
          f"fell back {info['fell_back']}", flush=True)
    assert st in (dlmpc.OK, dlmpc.ENOCONV)
    assert torch.equal(us, ub)
    assert it_s == [s["iters"] for s in sb]
    assert [s["converged"] for s in ss] == [s["converged"] for s in sb]
    assert [s["fell_back"] for s in ss] == [s["fell_back"] for s in sb]
    # the FP64 check of a streamed instance runs on its stashed stopping state (many instances per
    # pass, whichever stash slot holds it): the same values as the batched solve's check
    for f in ("objective", "kkt", "eq_resid", "u0_check"):
        assert [s[f] for s in ss] == [s[f] for s in sb], f
    assert info["fell_back"] == sum(s["fell_back"] for s in ss)
    assert info["instance_iterations"] == sum(it_s)
    if n > B:
        assert info["joins"] > 1
    else:
        assert info["joins"] == 1
    pr.close()


def test_stream_argument_errors(torch):
    wl = W.workload("chain10")
    pr = dlmpc.Problem.from_network(wl.net, wl.d, wl.T, wl.cost, precision="fp32", max_batch=4)
    x = torch.zeros((3, pr.n_sub * pr.nx), dtype=torch.float64, device="cuda")
    u = torch.zeros((3, pr.n_sub * pr.nu), dtype=torch.float64, device="cuda")
    with pytest.raises(dlmpc.DlmpcError):
        pr.solve_stream(3, x.data_ptr(), u.data_ptr())  # no warm-start network
    pr.ws_init(16, 4)
    with pytest.raises(dlmpc.DlmpcError):
        pr.solve_stream(0, x.data_ptr(), u.data_ptr())
    with pytest.raises(dlmpc.DlmpcError):
        pr.solve_stream(3, x.data_ptr(), u.data_ptr(), refill_min=-1)
    st, ss, info = pr.solve_stream(3, x.data_ptr(), u.data_ptr())  # x0 = 0: solved at once
    assert st == dlmpc.OK and all(s["converged"] for s in ss)
    assert float(u.abs().max()) == 0.0
    pr.close()
