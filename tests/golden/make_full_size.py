"""Writes oracle reference values for the full-size workloads (FP64 CPU oracle only).

    python tests/golden/make_full_size.py irregular1024_box 1000 1001 > tests/golden/irregular1024_box.json

Each record: workload, seed, sigma, eps, rho, max_iter, iters, converged, u0, J, r_primal,
r_dual. The oracle's setup factors every column block by SVD (minutes on 8 cores) and each
iteration works on dense R x N_x arrays, so this is run offline, never inside the tests.
"""
import json
import os
import sys
import time

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

from oracle import dlmpc_oracle as O  # noqa: E402
from paper_2103_14990_amd import workloads as W  # noqa: E402


def main():
    name = sys.argv[1]
    seeds = [int(s) for s in sys.argv[2:]]
    wl = W.workload(name)
    t0 = time.time()
    pb = O.setup_from_network(wl.net, wl.d, wl.T, wl.cost)
    t_setup = time.time() - t0
    assert pb.feasible
    out = {"workload": name, "setup_s": t_setup, "records": []}
    for seed in seeds:
        x0 = wl.x0(seed)
        t0 = time.time()
        res = O.solve(pb, x0, wl.rho, wl.eps, wl.max_iter)
        out["records"].append({"seed": seed, "sigma": wl.sigma, "eps": wl.eps, "rho": wl.rho,
                               "max_iter": wl.max_iter, "iters": res.iters,
                               "converged": res.converged, "u0": res.u0.tolist(), "J": res.J,
                               "r_primal": res.r_primal, "r_dual": res.r_dual,
                               "solve_s": time.time() - t0})
        print(f"seed {seed}: iters {res.iters} converged {res.converged} J {res.J:.6f} "
              f"({time.time() - t0:.0f} s)", file=sys.stderr, flush=True)
    json.dump(out, sys.stdout)


if __name__ == "__main__":
    main()
