"""Instances of several networks advanced together (one captured graph per iteration chunk with
every member's batched iteration as a branch), through the C ABI (needs a GPU).

Every instance's result equals the member's own batched solve (same kernels, same arithmetic
per instance), and sampled instances meet the reduced-precision bar against the FP64 oracle
(u(0) within 1e-4, J within 1e-5, a few iterations of slack)."""
import numpy as np
import pytest

from oracle import dlmpc_oracle as O
from paper_2103_14990_amd import dlmpc
from paper_2103_14990_amd import workloads as W

pytestmark = pytest.mark.gpu

RHO, EPS, MAXIT = 5.0, 1e-4, 500


def _problem(wl, max_batch):
    return dlmpc.Problem.from_network(wl.net, wl.d, wl.T, wl.cost, rho=RHO, eps=EPS, max_iter=MAXIT,
                                      precision="fp32", max_batch=max_batch)


def test_group_equals_members_and_oracle():
    import torch
    names, Bs = ("grid8", "chain10", "grid16_box"), (13, 5, 16)
    wls = [W.workload(n) for n in names]
    probs = [_problem(wl, 16) for wl in wls]
    x0s = [np.stack([wl.x0(7000 + 100 * k + i) for i in range(B)]) for k, (wl, B) in enumerate(zip(wls, Bs))]
    xd = [torch.tensor(x, dtype=torch.float64, device="cuda") for x in x0s]
    ud = [torch.zeros((B, wl.net.n_sub * wl.net.nu), dtype=torch.float64, device="cuda") for wl, B in zip(wls, Bs)]
    group = dlmpc.Group(probs)
    st, gstats = group.solve_batch_device(list(Bs), [x.data_ptr() for x in xd], [u.data_ptr() for u in ud])
    assert st in (dlmpc.OK, dlmpc.ENOCONV)
    for k, (pr, wl, B) in enumerate(zip(probs, wls, Bs)):
        us = torch.zeros_like(ud[k])
        _, sstats = pr.solve_batch_device(B, xd[k].data_ptr(), us.data_ptr())
        print(f"  {names[k]}: B {B}, iters {[s['iters'] for s in gstats[k]][:6]} ...", flush=True)
        assert torch.equal(us, ud[k])
        assert [s["iters"] for s in sstats] == [s["iters"] for s in gstats[k]]
        assert [s["converged"] for s in sstats] == [s["converged"] for s in gstats[k]]
    for k, i in ((0, 4), (1, 2)):
        wl = wls[k]
        pb = O.setup_from_network(wl.net, wl.d, wl.T, wl.cost)
        ref = O.solve(pb, x0s[k][i], RHO, EPS, MAXIT)
        u0 = ud[k][i].cpu().numpy()
        e = np.abs(u0 - ref.u0).max() / np.abs(ref.u0).max()
        je = abs(gstats[k][i]["objective"] - ref.J) / ref.J
        print(f"  {names[k]} instance {i}: iters {gstats[k][i]['iters']} (oracle {ref.iters}) u0 rel {e:.2e} "
              f"J rel {je:.2e}", flush=True)
        assert abs(gstats[k][i]["iters"] - ref.iters) <= 3 and e < 1e-4 and je < 1e-5
    group.close()


def test_group_argument_errors():
    wl = W.workload("chain10")
    plain = dlmpc.Problem.from_network(wl.net, wl.d, wl.T, wl.cost, precision="fp32")
    with pytest.raises(dlmpc.DlmpcError):
        dlmpc.Group([plain])  # no batched engine
    pr = _problem(wl, 4)
    with pytest.raises(dlmpc.DlmpcError):
        dlmpc.Group([pr, pr])  # the same member twice
    import torch
    g = dlmpc.Group([pr])
    x = torch.zeros((5, 20), dtype=torch.float64, device="cuda")
    u = torch.zeros((5, 10), dtype=torch.float64, device="cuda")
    with pytest.raises(dlmpc.DlmpcError):
        g.solve_batch_device([5], [x.data_ptr()], [u.data_ptr()])  # above max_batch
    g.close()
