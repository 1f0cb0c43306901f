"""HIP path against the FP64 oracle, element by element, through the C ABI (needs a GPU).

Bars: FP64 — same iteration count, u(0), objective and Phi within 1e-9 relative;
FP32 — u(0) within 1e-4 and the objective within 1e-5 relative of the FP64 oracle run with
the same eps and stopping rule.
"""
import numpy as np
import pytest

from oracle import dlmpc_oracle as O
from paper_2103_14990_amd import dlmpc
from paper_2103_14990_amd import workloads as W

pytestmark = pytest.mark.gpu

RHO, EPS, MAXIT = 5.0, 1e-4, 500


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def csr_values(pr, dense):
    rp, ci = pr.phi_pattern()
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    return dense[rows, ci]


def csr_to_dense(pr, vals, shape):
    rp, ci = pr.phi_pattern()
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    out = np.zeros(shape)
    out[rows, ci] = vals
    return out


SCHEDULES = ["graph", "persistent"]


class Case:
    def __init__(self, wl, precision="fp64", **kw):
        self.wl = wl
        self.pb = O.setup_from_network(wl.net, wl.d, wl.T, wl.cost)
        self.pr = dlmpc.Problem.from_network(wl.net, wl.d, wl.T, wl.cost, rho=RHO, eps=EPS,
                                             max_iter=kw.pop("max_iter", MAXIT),
                                             precision=precision, **kw)


@pytest.fixture(scope="module", params=SCHEDULES)
def chain10(request):
    return Case(W.workload("chain10"), schedule=request.param)


@pytest.fixture(scope="module", params=SCHEDULES)
def grid16_box(request):
    return Case(W.workload("grid16_box"), schedule=request.param)


def check_fp64(case, x0, res, ores):
    print(f"  iters gpu={res.stats['iters']} oracle={ores.iters}", flush=True)
    assert res.stats["iters"] == ores.iters
    assert (res.status == dlmpc.OK) == ores.converged
    assert rel(res.u0, ores.u0) < 1e-9
    assert abs(res.stats["objective"] - ores.J) <= 1e-9 * ores.J + 1e-300
    if res.phi is not None:
        assert rel(res.phi, csr_values(case.pr, ores.Phi)) < 1e-9


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_chain10_fp64(chain10, seed):
    x0 = chain10.wl.x0(seed)
    ores = O.solve(chain10.pb, x0, RHO, EPS, MAXIT)
    res = chain10.pr.solve(x0, want_phi=True)
    check_fp64(chain10, x0, res, ores)


def test_grid16_box_fp64(grid16_box):
    x0 = grid16_box.wl.x0(1000)
    ores = O.solve(grid16_box.pb, x0, RHO, EPS, MAXIT)
    res = grid16_box.pr.solve(x0, want_phi=True)
    check_fp64(grid16_box, x0, res, ores)


@pytest.mark.parametrize("schedule", SCHEDULES)
def test_grid16_box_active_bounds_fp64(schedule):
    """Tighter input bound so that the clip of the row solve is active on the GPU path."""
    net = W.grid(16)
    cost = W.box_cost(net, theta_max=0.8, u_max=0.05)
    wl = W.Workload("grid16_tight", net, 2, 10, cost, sigma=0.2)
    case = Case(wl, schedule=schedule)
    x0 = wl.x0(1001)
    ores = O.solve(case.pb, x0, RHO, EPS, MAXIT)
    n_active = int(np.sum(np.isclose(np.abs(ores.y[case.pb.lay.Nx * 10:]), 0.05, atol=1e-12)))
    print(f"  active input bounds {n_active}", flush=True)
    assert n_active > 0
    check_fp64(case, x0, case.pr.solve(x0, want_phi=True), ores)


@pytest.mark.parametrize("schedule", SCHEDULES)
def test_not_converged_returns_last_iterate(chain10, schedule):
    c = Case(chain10.wl, max_iter=7, schedule=schedule)
    x0 = chain10.wl.x0(1)
    ores = O.solve(c.pb, x0, RHO, EPS, 7)
    res = c.pr.solve(x0, want_phi=True)
    assert res.status == dlmpc.ENOCONV and res.stats["iters"] == 7 and not ores.converged
    check_fp64(c, x0, res, ores)


def test_warm_start_fp64(chain10):
    rng = np.random.default_rng(42)
    mask = chain10.pb.mask
    psi0 = rng.standard_normal(mask.shape) * mask
    lam0 = rng.standard_normal(mask.shape) * mask
    x0 = chain10.wl.x0(5)
    ores = O.solve(chain10.pb, x0, RHO, EPS, MAXIT, psi0=psi0, lam0=lam0)
    res = chain10.pr.solve(x0, psi0=csr_values(chain10.pr, psi0), lambda0=csr_values(chain10.pr, lam0),
                           want_phi=True)
    check_fp64(chain10, x0, res, ores)


def test_zero_x0_and_zero_patch(chain10):
    """x0 = 0 everywhere (every row keeps phi = v) and x0 zero on whole patches."""
    x0 = np.zeros(20)
    ores = O.solve(chain10.pb, x0, RHO, EPS, MAXIT)
    res = chain10.pr.solve(x0, want_phi=True)
    check_fp64(chain10, x0, res, ores)
    assert np.all(res.u0 == 0.0)
    x0 = chain10.wl.x0(3)
    x0[:6] = 0.0
    ores = O.solve(chain10.pb, x0, RHO, EPS, MAXIT)
    check_fp64(chain10, x0, chain10.pr.solve(x0, want_phi=True), ores)


def test_deterministic(grid16_box):
    x0 = grid16_box.wl.x0(1002)
    a = grid16_box.pr.solve(x0, want_phi=True)
    b = grid16_box.pr.solve(x0, want_phi=True)
    assert np.array_equal(a.u0, b.u0) and np.array_equal(a.phi, b.phi)
    assert a.stats["iters"] == b.stats["iters"]


@pytest.mark.parametrize("schedule", SCHEDULES)
# (nx > nu plants of this graph are not localisable at d = 1 for T = 3: the oracle finds no
# solution of the ring equations, so those shapes run at d = 2)
@pytest.mark.parametrize("nx,nu,d,T,seed", [(1, 1, 1, 4, 0), (3, 2, 2, 3, 1), (4, 1, 2, 3, 3)])
def test_generic_shapes_fp64(nx, nu, d, T, seed, schedule):
    edges = np.array([(0, 1), (1, 2), (2, 3), (3, 4), (1, 4), (4, 5), (5, 6)])
    net = W.generic_network(7, edges, nx, nu, seed)
    wl = W.Workload("generic", net, d, T, W.unit_cost(net), sigma=1.0)
    pb = O.setup_from_network(net, d, T, wl.cost)
    if not pb.feasible:
        pytest.skip(f"random plant not localisable at d = {d}")
    case = Case(wl, schedule=schedule)
    x0 = wl.x0(7)
    ores = O.solve(case.pb, x0, RHO, EPS, MAXIT)
    check_fp64(case, x0, case.pr.solve(x0, want_phi=True), ores)


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("name,seed", [("chain10", 1), ("grid16_box", 1000)])
def test_fp32_tier(name, seed, schedule):
    wl = W.workload(name)
    case = Case(wl, precision="fp32", schedule=schedule)
    x0 = wl.x0(seed)
    ores = O.solve(case.pb, x0, RHO, EPS, MAXIT)
    res = case.pr.solve(x0)
    print(f"  fp32 iters {res.stats['iters']} oracle {ores.iters} u0 rel {rel(res.u0, ores.u0):.2e} "
          f"J rel {abs(res.stats['objective'] - ores.J) / ores.J:.2e}", flush=True)
    assert res.status == dlmpc.OK
    assert rel(res.u0, ores.u0) < 1e-4
    assert abs(res.stats["objective"] - ores.J) < 1e-5 * ores.J


def test_fixed_check_interval(chain10):
    """check_every > 0: fixed chunks of iterations between host checks, same result."""
    c = Case(chain10.wl, check_every=7, schedule="graph")
    x0 = chain10.wl.x0(2)
    ores = O.solve(c.pb, x0, RHO, EPS, MAXIT)
    check_fp64(c, x0, c.pr.solve(x0, want_phi=True), ores)


def test_schedules_agree():
    """The two schedules sum the projection in different orders (split over waves vs one
    thread per row) but follow the same trajectory: same iterations, FP64 results to 1e-12."""
    wl = W.workload("grid16_box")
    a = Case(wl, schedule="graph").pr.solve(wl.x0(1003), want_phi=True)
    b = Case(wl, schedule="persistent").pr.solve(wl.x0(1003), want_phi=True)
    assert a.stats["iters"] == b.stats["iters"]
    assert rel(a.u0, b.u0) < 1e-12 and rel(a.phi, b.phi) < 1e-12


def test_auto_schedule_reports_tuning():
    wl = W.workload("chain10")
    pr = dlmpc.Problem.from_network(wl.net, wl.d, wl.T, wl.cost)
    print(f"  chain10 tuning: {pr.info}", flush=True)
    assert pr.info["tune_graph_us"] > 0
    assert pr.info["schedule"] in (0, 1)


def test_kernel_timing_entry(chain10):
    import torch
    xd = torch.tensor(chain10.wl.x0(1), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    us = chain10.pr.time_kernels(xd.data_ptr(), 10)
    assert set(us) == set(dlmpc.KERNEL_NAMES) and all(v > 0 for v in us.values())
    # the problem still solves correctly afterwards
    x0 = chain10.wl.x0(1)
    ores = O.solve(chain10.pb, x0, RHO, EPS, MAXIT)
    check_fp64(chain10, x0, chain10.pr.solve(x0, want_phi=True), ores)


def test_solve_device_matches_host_entry(chain10):
    import torch
    x0 = chain10.wl.x0(2)
    ref = chain10.pr.solve(x0, want_phi=True)
    xd = torch.tensor(x0, dtype=torch.float64, device="cuda")
    ud = torch.zeros(10, dtype=torch.float64, device="cuda")
    pd = torch.zeros(chain10.pr.nnz, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    st, stats = chain10.pr.solve_device(xd.data_ptr(), ud.data_ptr(), pd.data_ptr())
    assert st == dlmpc.OK and stats["iters"] == ref.stats["iters"]
    assert np.array_equal(ud.cpu().numpy(), ref.u0)
    assert np.array_equal(pd.cpu().numpy(), ref.phi)
