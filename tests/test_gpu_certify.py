"""FP64 certificate of a single-instance solve (dlmpc_certify) against the oracle's KKT
residuals of the same solve (same trajectory in the FP64 tier), through the C ABI (needs a
GPU). The certificate recomputes Z_AB Psi - I on every column's support and ring, |Phi - Psi|,
the column norms of Phi - Psi, the bound violation of Phi x0 and the Psi-step stationarity
N_j N_j' rho Lambda_c in FP64 on the device."""
import numpy as np
import pytest

from oracle import dlmpc_oracle as O
from paper_2103_14990_amd import dlmpc
from paper_2103_14990_amd import workloads as W

pytestmark = pytest.mark.gpu

RHO, EPS = 5.0, 1e-4


def _cases():
    net = W.chain(10)
    tight = W.box_cost(net, theta_max=0.8, u_max=0.3)
    return [("chain10", W.workload("chain10"), 1), ("grid8", W.workload("grid8"), 4),
            ("chain10_tight", W.Workload("chain10_tight", net, 1, 5, tight, sigma=0.4), 9)]


@pytest.mark.parametrize("name,wl,seed", _cases())
def test_certificate_matches_oracle_kkt(name, wl, seed):
    pb = O.setup_from_network(wl.net, wl.d, wl.T, wl.cost)
    x0 = wl.x0(seed)
    ref = O.solve(pb, x0, RHO, EPS, 500)
    kkt = O.kkt_residuals(pb, ref, x0, RHO)
    pr = dlmpc.Problem.from_network(wl.net, wl.d, wl.T, wl.cost, rho=RHO, eps=EPS, max_iter=500,
                                    precision="fp64")
    r = pr.solve(x0)
    assert r.stats["iters"] == ref.iters
    c = pr.certify()
    rp_ref = max(np.linalg.norm(ref.Phi[:, k] - ref.Psi[:, k]) for k in range(pb.lay.Nx))
    print(f"  {name}: certificate {c}; oracle {kkt}, rp {rp_ref:.3e}", flush=True)
    assert c["eq"] < 1e-11 and kkt["eq"] < 1e-11
    for key, gpu, cpu in (("pf", c["pf"], kkt["pf"]), ("stat", c["stat"], kkt["stat"]), ("rp", c["rp"], rp_ref)):
        assert abs(gpu - cpu) <= 1e-6 * cpu + 1e-12, key
    assert abs(c["box"] - kkt["box"]) <= 1e-9
    assert abs(c["rp"] - r.stats["r_primal"]) <= 1e-9 * max(c["rp"], 1e-300) + 1e-15


def test_certificate_fp32_full_mesh():
    """FP32 tier at the 1024 mesh: the certificate (FP64 arithmetic on the FP32 state) agrees
    with the stopping rule and shows the FP32 feasibility level."""
    import torch
    wl = W.workload("irregular1024_box")
    pr = dlmpc.Problem.from_network(wl.net, wl.d, wl.T, wl.cost, rho=wl.rho, eps=wl.eps,
                                    max_iter=wl.max_iter, precision="fp32")
    xd = torch.tensor(wl.x0(1000), dtype=torch.float64, device="cuda")
    ud = torch.zeros(wl.net.n_sub * wl.net.nu, dtype=torch.float64, device="cuda")
    st, stats = pr.solve_device(xd.data_ptr(), ud.data_ptr())
    c = pr.certify(xd.data_ptr())
    print(f"  certificate {c}; stats rp {stats['r_primal']:.3e}", flush=True)
    assert st == dlmpc.OK
    assert c["eq"] < 1e-4 and c["rp"] <= 1.01 * wl.eps and c["box"] < 1e-5  # FP32 state, FP64 check
