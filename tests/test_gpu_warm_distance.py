"""Warm and cold starts side by side against the exact optimum (needs a GPU).

u(0) of the convex program (eq. (MPC) under the SLS parametrisation) is unique even though Phi
is not, and ADMM only approaches it: an eps-converged iterate sits at a distance of the order of
eps from it, by an amount that depends on where the iteration started. The stored values of
tests/golden/*_tight.json are the FP64 oracle run to eps = 1e-8 (u(0) within ~1e-8 of the
optimum). Here the batched cold start (eps), the batched learned start and the streamed learned
start (eps * warm_eps_scale, the library default) are all held to one bar against them, and the
learned start must land within the cold start's distance (mean and worst over the stored x0).
"""
import json
import os

import numpy as np
import pytest

from paper_2103_14990_amd import dlmpc
from paper_2103_14990_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
# One bar for the three starts: u(0) relative to the exact optimum. The eps = 1e-4 rule bounds
# residuals, not this distance; the cold start reaches up to 1.3e-3 on the 16x16 box grid.
BAR = 20 * 1e-4


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def _train(torch, pr, wl, n_solves, steps, hidden=64, B=64):
    G, nx, nu = wl.net.n_sub, wl.net.nx, wl.net.nu
    rs = nx * wl.T + nu * (wl.T - 1)
    xt = torch.tensor(np.stack([wl.x0(10**6 + i) for i in range(n_solves)]), dtype=torch.float64, device="cuda")
    yt = torch.zeros((n_solves, G * rs), dtype=torch.float64, device="cuda")
    ut = torch.zeros((n_solves, G * nu), dtype=torch.float64, device="cuda")
    conv = []
    for s0 in range(0, n_solves, B):
        _, s = pr.solve_batch_ex(B, xt[s0:].data_ptr(), ut[s0:].data_ptr(), "cold", 0, yt[s0:].data_ptr())
        conv += [s0 + i for i, q in enumerate(s) if q["converged"]]
    keep = torch.tensor(conv[:(len(conv) // B) * B], device="cuda")
    xt, yt = xt[keep].contiguous(), yt[keep].contiguous()
    ys = float(yt.view(-1, G, rs)[:, :, nx * wl.T:].std().item())
    pr.ws_init(hidden, B, seed=1, x_scale=wl.sigma, y_scale=ys)
    rng = np.random.default_rng(0)
    nb = xt.shape[0] // B
    for k in range(steps):
        i = int(rng.integers(0, nb)) * B
        f = k / steps
        lr = 2e-3 if f < 0.6 else (5e-4 if f < 0.85 else 1e-4)
        pr.ws_train_step(B, xt[i:].data_ptr(), yt[i:].data_ptr(), lr)


def _rel(u, ref):
    return float(np.abs(u - ref).max() / np.abs(ref).max())


@pytest.mark.parametrize("name,n_train,steps", [("grid16_box", 1024, 2000), ("irregular1024_box", 4096, 4000)])
def test_learned_within_cold_distance_of_optimum(torch, tmp_path, name, n_train, steps):
    path = os.path.join(GOLD, f"{name}_tight.json")
    if not os.path.exists(path):
        pytest.skip(f"no stored tight oracle values for {name}")
    gold = json.load(open(path))
    wl = W.workload(name)
    recs = gold["records"]
    assert all(r["eps"] <= 1e-8 and r["converged"] for r in recs)
    G, nu = wl.net.n_sub, wl.net.nu
    pr = dlmpc.Problem.from_network(wl.net, wl.d, wl.T, wl.cost, rho=wl.rho, eps=wl.eps, max_iter=wl.max_iter,
                                    precision="fp32", max_batch=64)
    _train(torch, pr, wl, n_train, steps)
    seeds = [r["seed"] for r in recs] + [2000 + i for i in range(64 - len(recs))]
    xd = torch.tensor(np.stack([wl.x0(s) for s in seeds]), dtype=torch.float64, device="cuda")
    uc, ul = (torch.zeros((64, G * nu), dtype=torch.float64, device="cuda") for _ in range(2))
    _, sc = pr.solve_batch_ex(64, xd.data_ptr(), uc.data_ptr(), "cold")
    _, sl = pr.solve_batch_ex(64, xd.data_ptr(), ul.data_ptr(), "learned")
    n = 96  # joins into freed slots
    xs = torch.cat([xd, torch.tensor(np.stack([wl.x0(7000 + i) for i in range(n - 64)]), dtype=torch.float64,
                                     device="cuda")])
    us = torch.zeros((n, G * nu), dtype=torch.float64, device="cuda")
    _, ss, info = pr.solve_stream(n, xs.data_ptr(), us.data_ptr())
    # other eps scales of the learned start (same network), for the record
    pr.ws_save(str(tmp_path / "ws.bin"))
    other = {}
    for scale in (1.0, 1.0 / 3.0):
        p1 = dlmpc.Problem.from_network(wl.net, wl.d, wl.T, wl.cost, rho=wl.rho, eps=wl.eps, max_iter=wl.max_iter,
                                        precision="fp32", max_batch=64, warm_eps_scale=scale)
        p1.warmstart_load(str(tmp_path / "ws.bin"))
        u1 = torch.zeros_like(ul)
        _, s1 = p1.solve_batch_ex(64, xd.data_ptr(), u1.data_ptr(), "learned")
        p1.close()
        other[scale] = (u1.cpu().numpy(), np.mean([q["iters"] for q in s1]))
    dist = {"cold": [], "learned": [], "streamed": [], "learned_scale1": [], "learned_scale1/3": []}
    u_c, u_l, u_s = uc.cpu().numpy(), ul.cpu().numpy(), us.cpu().numpy()
    for i, r in enumerate(recs):
        ref = np.array(r["u0"])
        dist["cold"].append(_rel(u_c[i], ref))
        dist["learned"].append(_rel(u_l[i], ref))
        dist["streamed"].append(_rel(u_s[i], ref))
        dist["learned_scale1"].append(_rel(other[1.0][0][i], ref))
        dist["learned_scale1/3"].append(_rel(other[1.0 / 3.0][0][i], ref))
    ic = np.mean([q["iters"] for q in sc])
    il = np.mean([q["iters"] for q in sl])
    print(f"  {name}: iterations cold {ic:.1f} learned {il:.1f} (streamed {np.mean([q['iters'] for q in ss]):.1f}, "
          f"joins {info['joins']}); fell back {sum(q['fell_back'] for q in sl)}", flush=True)
    print(f"  {name}: learned start at eps scale 1: iterations {other[1.0][1]:.1f}; "
          f"at 1/3: {other[1.0 / 3.0][1]:.1f}", flush=True)
    for k in ("cold", "learned", "streamed", "learned_scale1", "learned_scale1/3"):
        d = np.array(dist[k])
        print(f"  {name} {k}: u0 distance to the optimum mean {d.mean():.2e} max {d.max():.2e}", flush=True)
    ng = len(recs)  # the x0 with stored optimum values; the oracle converged on them
    assert all(q["converged"] for q in sc[:ng] + sl[:ng] + ss[:ng])
    assert not any(q["fell_back"] for q in sl[:ng] + ss[:ng])
    for k in ("cold", "learned", "streamed"):
        assert max(dist[k]) < BAR, k
    for k in ("learned", "streamed"):
        assert np.mean(dist[k]) <= np.mean(dist["cold"]), k
        assert max(dist[k]) <= max(dist["cold"]), k
    assert il < ic
