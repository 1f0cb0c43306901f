"""Learned warm start through the C ABI (needs a GPU).

* The warm-start network's loss, gradient, prediction and Adam steps against the FP64 reference
  network (oracle/mlp_ref.py, pinned by finite differences), with inputs gathered on the oracle
  side from its own hop distances. Bar: the products run as split-bf16 matrix-core GEMMs with
  FP32 accumulation, so loss and predictions within 1e-5 and each gradient block within 1e-4
  relative (norm-wise) of FP64.
* A batched solve warm-started from given row multipliers alpha0 against the oracle's ADMM run
  from the equivalent standard-form initial iterate Psi^0[:,c] = o_c, Lambda^0[:,c] =
  x0_c (I - P_j) alpha0 on the support of c (reduced-precision bar: u(0) 1e-4, J 1e-5, a few
  iterations of slack).
* The learned start end to end: trained on cold solves, every held-out warm solve meets the
  same eps, needs fewer iterations than the cold start, and agrees with the cold u(0); a warm
  start that cannot converge within max_iter falls back to the cold start (counted in stats).
"""
import numpy as np
import pytest

from oracle import dlmpc_oracle as O
from oracle import mlp_ref as M
from paper_2103_14990_amd import dlmpc
from paper_2103_14990_amd import workloads as W

pytestmark = pytest.mark.gpu

RHO, EPS = 5.0, 1e-4


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def lib_rows_to_canonical(lay: O.Layout) -> np.ndarray:
    """Canonical Phi row of library row g*rs + l (rows of subsystem g: x_0..x_{T-1}, then
    u_0..u_{T-2}, each block nx resp. nu entries)."""
    nx, nu, T, N = lay.nx, lay.nu, lay.T, lay.n_sub
    rs = nx * T + nu * (T - 1)
    out = np.zeros(N * rs, dtype=np.int64)
    for g in range(N):
        for l in range(rs):
            if l < nx * T:
                out[g * rs + l] = (l // nx) * lay.Nx + g * nx + l % nx
            else:
                lu = l - nx * T
                out[g * rs + l] = lay.Nx * T + (lu // nu) * lay.Nu + g * nu + lu % nu
    return out


def network_inputs(pb: O.Problem, x0s: np.ndarray, IN: int, xs: float) -> np.ndarray:
    """X [G, S, IN]: x0 of the subsystems within d hops of g, ascending, / xs, zero-padded."""
    G, nx = pb.lay.n_sub, pb.lay.nx
    X = np.zeros((G, x0s.shape[0], IN))
    for g in range(G):
        members = np.flatnonzero((pb.dist[g] >= 0) & (pb.dist[g] <= pb.d))
        cols = (members[:, None] * nx + np.arange(nx)[None, :]).ravel()
        X[g, :, :cols.size] = x0s[:, cols] / xs
    return X


def standard_form_start(pb: O.Problem, x0: np.ndarray, alpha_canon: np.ndarray):
    """Psi^0 = o_c and Lambda^0 = x0_c (I - P_j) alpha on the support of every column c."""
    R, Nx, nx = pb.lay.R, pb.lay.Nx, pb.lay.nx
    psi0, lam0 = np.zeros((R, Nx)), np.zeros((R, Nx))
    for blk in pb.blocks:
        a = alpha_canon[blk.rows]
        q = a - blk.P @ a
        for ci in range(nx):
            c = blk.j * nx + ci
            psi0[blk.rows, c] = blk.O[:, ci]
            lam0[blk.rows, c] = x0[c] * q
    return psi0, lam0


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


@pytest.fixture(scope="module")
def grid8():
    wl = W.workload("grid8")
    pb = O.setup_from_network(wl.net, wl.d, wl.T, wl.cost)
    return wl, pb


def make_problem(wl, max_batch=64, max_iter=500):
    return dlmpc.Problem.from_network(wl.net, wl.d, wl.T, wl.cost, rho=RHO, eps=EPS, max_iter=max_iter,
                                      precision="fp32", max_batch=max_batch)


# ------------------------------------------------------------------ network kernels vs FP64


def _net_case(torch, wl, pb, S=37, H=40, xs=0.7, ys=0.05, seed=3):
    pr = make_problem(wl)
    pr.ws_init(H, 64, seed=seed, x_scale=xs, y_scale=ys)
    sh = pr.ws_shape()
    G, rs = wl.net.n_sub, sh["OUT"]
    rng = np.random.default_rng(seed)
    x0s = rng.standard_normal((S, G * wl.net.nx))
    alpha = ys * rng.standard_normal((S, G * rs))
    xd = torch.tensor(x0s, dtype=torch.float64, device="cuda")
    ad = torch.tensor(alpha, dtype=torch.float64, device="cuda")
    X = network_inputs(pb, x0s, sh["IN"], xs)
    Yt = (alpha / ys).reshape(S, G, rs).transpose(1, 0, 2)
    return pr, sh, x0s, alpha, xd, ad, X, Yt


def test_network_loss_and_gradient_match_fp64(torch, grid8):
    wl, pb = grid8
    pr, sh, x0s, alpha, xd, ad, X, Yt = _net_case(torch, wl, pb)
    G, IN, H, OUT = wl.net.n_sub, sh["IN"], sh["H"], sh["OUT"]
    theta = pr.ws_params().astype(np.float64)
    assert theta.size == sh["n_params"] == G * (IN * H + H + H * H + H + (H + IN) * OUT + OUT)
    loss, g = pr.ws_loss_grad(x0s.shape[0], xd.data_ptr(), ad.data_ptr())
    L, grads = M.loss_and_grads(M.unflatten(theta, G, IN, H, OUT), X, Yt)
    print(f"  loss {loss:.8e} (FP64 {L:.8e})", flush=True)
    assert abs(loss - L) / L < 1e-5
    gl = M.unflatten(g.astype(np.float64), G, IN, H, OUT)
    for name, a, b in zip(("W1", "b1", "W2", "b2", "W3", "b3"), gl, grads):
        e = np.linalg.norm(a - b) / np.linalg.norm(b)
        print(f"  d{name}: rel {e:.2e}", flush=True)
        assert e < 1e-4


def test_network_prediction_matches_fp64(torch, grid8):
    wl, pb = grid8
    pr, sh, x0s, alpha, xd, ad, X, Yt = _net_case(torch, wl, pb, S=64, H=64, seed=5)
    G, IN, H, OUT = wl.net.n_sub, sh["IN"], sh["H"], sh["OUT"]
    theta = pr.ws_params().astype(np.float64)
    out = torch.zeros((64, G * OUT), dtype=torch.float64, device="cuda")
    pr.ws_predict(64, xd.data_ptr(), out.data_ptr())
    Y, _ = M.forward(M.unflatten(theta, G, IN, H, OUT), X)
    ref = 0.05 * Y.transpose(1, 0, 2).reshape(64, G * OUT)
    e = rel(out.cpu().numpy(), ref)
    print(f"  prediction rel {e:.2e}", flush=True)
    assert e < 1e-5


def test_adam_steps_match_fp64(torch, grid8):
    wl, pb = grid8
    pr, sh, x0s, alpha, xd, ad, X, Yt = _net_case(torch, wl, pb, S=21, H=24, seed=7)
    G, IN, H, OUT = wl.net.n_sub, sh["IN"], sh["H"], sh["OUT"]
    th = pr.ws_params().astype(np.float64)
    m, v = np.zeros_like(th), np.zeros_like(th)
    lr = 1e-3
    gmax = 0.0
    for t in (1, 2):
        pr.ws_train_step(x0s.shape[0], xd.data_ptr(), ad.data_ptr(), lr)
        _, grads = M.loss_and_grads(M.unflatten(th, G, IN, H, OUT), X, Yt)
        gf = M.flatten(grads)
        gmax = max(gmax, np.abs(gf).max())
        th, m, v = M.adam_step(th, gf, m, v, t, lr)
    got = pr.ws_params().astype(np.float64)
    # entries whose gradient is far from zero: the update direction is decided, compare tightly
    big = np.abs(gf) > 1e-2 * gmax
    err = np.abs(got - th)
    print(f"  max |dtheta| err {err[big].max():.2e} on {big.sum()} entries; overall {err.max():.2e}", flush=True)
    assert err[big].max() < 1e-2 * lr
    assert err.max() < 2 * lr + 1e-6  # Adam moves each entry by at most about lr per step


def test_weights_save_load_roundtrip(torch, grid8, tmp_path):
    wl, pb = grid8
    pr, sh, x0s, alpha, xd, ad, X, Yt = _net_case(torch, wl, pb, S=8, H=16, seed=9)
    path = str(tmp_path / "ws.bin")
    pr.ws_save(path)
    other = make_problem(wl, max_batch=8)
    other.warmstart_load(path)
    assert np.array_equal(other.ws_params(), pr.ws_params())
    a1 = torch.zeros((8, alpha.shape[1]), dtype=torch.float64, device="cuda")
    a2 = torch.zeros_like(a1)
    pr.ws_predict(8, xd.data_ptr(), a1.data_ptr())
    other.ws_predict(8, xd.data_ptr(), a2.data_ptr())
    assert torch.equal(a1, a2)
    bad = make_problem(W.workload("chain10"), max_batch=4)
    with pytest.raises(dlmpc.DlmpcError):
        bad.warmstart_load(path)  # other network shape


# ------------------------------------------------------------------ warm-started ADMM vs oracle


def test_alpha_start_matches_oracle(torch, grid8):
    """Seeded alpha0 (any point is a valid start) on both sides; same iteration as the oracle."""
    wl, pb = grid8
    pr = make_problem(wl, max_batch=8)
    rs = wl.net.nx * wl.T + wl.net.nu * (wl.T - 1)
    perm = lib_rows_to_canonical(pb.lay)
    B = 3
    x0s = np.stack([wl.x0(6000 + i) for i in range(B)])
    rng = np.random.default_rng(11)
    alpha0 = 0.3 * rng.standard_normal((B, wl.net.n_sub * rs))
    xd = torch.tensor(x0s, dtype=torch.float64, device="cuda")
    a0 = torch.tensor(alpha0, dtype=torch.float64, device="cuda")
    ud = torch.zeros((B, wl.net.n_sub * wl.net.nu), dtype=torch.float64, device="cuda")
    aout = torch.zeros_like(a0)
    st, stats = pr.solve_batch_ex(B, xd.data_ptr(), ud.data_ptr(), "alpha", a0.data_ptr(), aout.data_ptr())
    assert st == dlmpc.OK
    u0 = ud.cpu().numpy()
    aout = aout.cpu().numpy()
    for i in range(B):
        ac = np.zeros(pb.lay.R)
        ac[perm] = alpha0[i]
        psi0, lam0 = standard_form_start(pb, x0s[i], ac)
        ref = O.solve(pb, x0s[i], RHO, EPS, 500, psi0=psi0, lam0=lam0)
        cold = O.solve(pb, x0s[i], RHO, EPS, 500)
        e, je = rel(u0[i], ref.u0), abs(stats[i]["objective"] - ref.J) / ref.J
        print(f"  instance {i}: iters {stats[i]['iters']} (oracle {ref.iters}, cold {cold.iters}) "
              f"u0 rel {e:.2e} J rel {je:.2e} start {stats[i]['start']} fell_back {stats[i]['fell_back']}",
              flush=True)
        assert stats[i]["start"] == dlmpc.STARTS["alpha"] and stats[i]["fell_back"] == 0
        assert abs(stats[i]["iters"] - ref.iters) <= 3
        assert e < 1e-4 and je < 1e-5
        # stopping multipliers against the fixed-point relation alpha* = -2 w y / rho (no bounds)
        astar = (-2.0 * pb.w * ref.y / RHO)[perm]
        ea = rel(aout[i], astar)
        print(f"    alpha_out vs -2wy/rho: rel {ea:.2e}", flush=True)
        assert ea < 2e-2


# ------------------------------------------------------------------ learned start end to end


def _cold_data(torch, pr, wl, seeds, B=64):
    G, rs = wl.net.n_sub, wl.net.nx * wl.T + wl.net.nu * (wl.T - 1)
    x0s = np.stack([wl.x0(s) for s in seeds])
    xd = torch.tensor(x0s, dtype=torch.float64, device="cuda")
    ad = torch.zeros((len(seeds), G * rs), dtype=torch.float64, device="cuda")
    ud = torch.zeros((len(seeds), G * wl.net.nu), dtype=torch.float64, device="cuda")
    stats = []
    for s0 in range(0, len(seeds), B):
        n = min(B, len(seeds) - s0)
        st, s = pr.solve_batch_ex(n, xd[s0:].data_ptr(), ud[s0:].data_ptr(), "cold", 0, ad[s0:].data_ptr())
        assert st == dlmpc.OK
        stats += s
    return x0s, xd, ad, ud, stats


def test_learned_start_reduces_iterations(torch, grid8):
    wl, pb = grid8
    pr = make_problem(wl)
    x0s, xd, ad, _, cold_train = _cold_data(torch, pr, wl, [10**6 + i for i in range(1024)])
    ys = float(ad.std().item())
    pr.ws_init(64, 64, seed=1, x_scale=1.0, y_scale=ys)
    rng = np.random.default_rng(0)
    losses = []
    for step in range(1500):
        idx = int(rng.integers(0, 1024 // 64)) * 64
        lr = 2e-3 if step < 1000 else 5e-4
        losses.append(pr.ws_train_step(64, xd[idx:].data_ptr(), ad[idx:].data_ptr(), lr))
    print(f"  training loss {losses[0]:.3e} -> {np.mean(losses[-50:]):.3e}", flush=True)
    assert np.mean(losses[-50:]) < 0.05 * losses[0]
    # held-out instances: cold vs learned start
    hx, hxd, _, hu_cold, hs_cold = _cold_data(torch, pr, wl, [2000 + i for i in range(64)])
    hu = torch.zeros_like(hu_cold)
    st, hs = pr.solve_batch_ex(64, hxd.data_ptr(), hu.data_ptr(), "learned")
    assert st == dlmpc.OK
    ic = np.array([s["iters"] for s in hs_cold])
    iw = np.array([s["iters"] for s in hs])
    print(f"  held-out iterations: cold {ic.mean():.1f}, learned {iw.mean():.1f}; "
          f"fell back {sum(s['fell_back'] for s in hs)}; inference {hs[0]['t_warm_ms']:.3f} ms", flush=True)
    assert all(s["converged"] and s["start"] == dlmpc.STARTS["learned"] for s in hs)
    assert iw.mean() < 0.8 * ic.mean()
    e = rel(hu.cpu().numpy(), hu_cold.cpu().numpy())
    print(f"  learned vs cold u0 rel {e:.2e}", flush=True)
    assert e < 1e-3
    for i in (0, 31):
        ref = O.solve(pb, hx[i], RHO, EPS, 500)
        assert rel(hu[i].cpu().numpy(), ref.u0) < 1e-4


def test_unconvergent_warm_start_falls_back_to_cold(torch, grid8):
    wl, pb = grid8
    B = 4
    probe = make_problem(wl, max_batch=B)
    x0s, xd, _, u_cold, s_cold = _cold_data(torch, probe, wl, [7000 + i for i in range(B)], B=B)
    cap = max(s["iters"] for s in s_cold) + 10
    pr = make_problem(wl, max_batch=B, max_iter=cap)
    rs = wl.net.nx * wl.T + wl.net.nu * (wl.T - 1)
    rng = np.random.default_rng(5)
    a0 = torch.tensor(1e4 * rng.standard_normal((B, wl.net.n_sub * rs)), dtype=torch.float64, device="cuda")
    a0[1].zero_()  # instance 1 starts from alpha0 = 0: a valid start that converges
    ud = torch.zeros_like(u_cold)
    st, stats = pr.solve_batch_ex(B, xd.data_ptr(), ud.data_ptr(), "alpha", a0.data_ptr())
    assert st == dlmpc.OK
    fb = [s["fell_back"] for s in stats]
    print(f"  fell_back {fb}, iters {[s['iters'] for s in stats]} (cold {[s['iters'] for s in s_cold]})",
          flush=True)
    assert fb[0] == fb[2] == fb[3] == 1 and fb[1] == 0
    for i in (0, 2, 3):
        assert stats[i]["converged"] and abs(stats[i]["iters"] - (cap + s_cold[i]["iters"])) <= 1
        assert rel(ud[i].cpu().numpy(), u_cold[i].cpu().numpy()) < 1e-6


def test_warm_start_argument_errors(torch, grid8):
    wl, _ = grid8
    pr = make_problem(wl, max_batch=4)
    xd = torch.zeros((2, wl.net.n_sub * wl.net.nx), dtype=torch.float64, device="cuda")
    ud = torch.zeros((2, wl.net.n_sub * wl.net.nu), dtype=torch.float64, device="cuda")
    with pytest.raises(dlmpc.DlmpcError):
        pr.solve_batch_ex(2, xd.data_ptr(), ud.data_ptr(), "learned")  # no network yet
    with pytest.raises(dlmpc.DlmpcError):
        pr.solve_batch_ex(2, xd.data_ptr(), ud.data_ptr(), "alpha")  # alpha0 missing
    with pytest.raises(dlmpc.DlmpcError):
        pr.ws_init(0, 4)
    pr.ws_init(8, 4)
    ad = torch.zeros((8, 10), dtype=torch.float64, device="cuda")
    with pytest.raises(dlmpc.DlmpcError):
        pr.ws_predict(5, xd.data_ptr(), ad.data_ptr())  # above max_samples
