"""Writes oracle reference values for the full-size workloads (FP64 CPU oracle only).

    python tests/golden/make_full_size.py irregular1024_box 1000 1001 > tests/golden/irregular1024_box.json
    python tests/golden/make_full_size.py --eps 1e-8 --max-iter 20000 --jobs 6 \
        irregular1024_box 1000 > tests/golden/irregular1024_box_tight.json

Each record: workload, seed, sigma, eps, rho, max_iter, iters, converged, u0, J, r_primal,
r_dual. The oracle's setup factors every column block by SVD (minutes on 8 cores) and each
iteration works on dense R x N_x arrays, so this is run offline, never inside the tests.
``--eps``/``--max-iter`` override the workload's stopping rule (a tight eps gives values
close to the exact optimum: u(0) and J of the convex program are unique even though Phi is
not). ``--jobs`` factors the column blocks in that many forked processes; every block is
still the oracle's own ``column_block``.
"""
import argparse
import json
import multiprocessing as mp
import os
import sys
import time

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

from oracle import dlmpc_oracle as O  # noqa: E402
from paper_2103_14990_amd import workloads as W  # noqa: E402

_SHARED = {}


def _block(j):
    Z, mask, lay = _SHARED["args"]
    return O.column_block(Z, mask, lay, j)


def setup(wl, jobs):
    if jobs <= 1:
        return O.setup_from_network(wl.net, wl.d, wl.T, wl.cost)
    pb = O.setup_from_network(wl.net, wl.d, wl.T, wl.cost, blocks=False)
    _SHARED["args"] = (O.build_zab(pb.A, pb.B, wl.T).tocsc(), pb.mask, pb.lay)
    with mp.get_context("fork").Pool(jobs) as pool:
        pb.blocks = pool.map(_block, range(pb.lay.n_sub), chunksize=4)
    return pb


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("name")
    ap.add_argument("seeds", type=int, nargs="+")
    ap.add_argument("--eps", type=float, default=None)
    ap.add_argument("--max-iter", type=int, default=None)
    ap.add_argument("--jobs", type=int, default=1)
    ap.add_argument("--every", type=int, default=50, help="progress line interval (iterations)")
    a = ap.parse_args()
    wl = W.workload(a.name)
    eps = wl.eps if a.eps is None else a.eps
    max_iter = wl.max_iter if a.max_iter is None else a.max_iter
    t0 = time.time()
    pb = setup(wl, a.jobs)
    t_setup = time.time() - t0
    print(f"setup {t_setup:.0f} s", file=sys.stderr, flush=True)
    assert pb.feasible
    out = {"workload": a.name, "setup_s": t_setup, "records": []}
    for seed in a.seeds:
        x0 = wl.x0(seed)
        t0 = time.time()

        def progress(k, rp, rd, seed=seed, t0=t0):
            if k % a.every == 0:
                print(f"seed {seed} iter {k}: r_primal {rp:.3e} r_dual {rd:.3e} "
                      f"({time.time() - t0:.0f} s)", file=sys.stderr, flush=True)

        res = O.solve(pb, x0, wl.rho, eps, max_iter, progress=progress)
        out["records"].append({"seed": seed, "sigma": wl.sigma, "eps": eps, "rho": wl.rho,
                               "max_iter": max_iter, "iters": res.iters,
                               "converged": res.converged, "u0": res.u0.tolist(), "J": res.J,
                               "r_primal": res.r_primal, "r_dual": res.r_dual,
                               "solve_s": time.time() - t0})
        print(f"seed {seed}: iters {res.iters} converged {res.converged} J {res.J:.6f} "
              f"({time.time() - t0:.0f} s)", file=sys.stderr, flush=True)
    json.dump(out, sys.stdout)


if __name__ == "__main__":
    main()
