"""Reference pressures of the benchmark workloads from the oracle (test
infrastructure only: run by hand, never by the library).

    python -m oracle.make_pref --config 5 --rhs 0 [--rtol 1e-11]

Builds the workload with the seeded generator, its coarse grids with the
oracle's own grid code, runs the oracle's F-AMS setup (Decoupled-AMS: the
converged pressure does not depend on the coupling strategy) and its GMRES(30)
to `rtol`, and stores the pressure rounded to float32 under
oracle/_pref/<key>.npy with a JSON sidecar (achieved residual, iterations,
timings).  The key is the SHA-256 of the system (A, its right-hand side),
so a stored pressure is only ever compared with the input it was computed
for.  Rounding to float32 perturbs the reference by at most 6e-8 relative,
well under the 1e-6 pressure-error target it is used for.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "_pref")
# coarse grid of each benchmark workload: (cx, cy, cz), d_min, r_z
GRIDS = {2: ((10, 10, 10), 8, 8), 3: ((10, 10, 10), 10, 10), 5: ((10, 10, 10), 10, 10)}


def cache_path(key: str) -> str:
    return os.path.join(CACHE, key + ".npy")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--config", type=int, default=5)
    ap.add_argument("--rhs", type=int, default=0,
                    help="index into the config's right-hand sides; -1: the boundary term alone")
    ap.add_argument("--flux", action="store_true",
                    help="also reconstruct the conservative flux and store its balance")
    ap.add_argument("--contrast", type=float, default=None)
    ap.add_argument("--rtol", type=float, default=1e-11)
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(HERE))
    from workloads import make_config
    from workloads.configs import config_rhs
    from workloads.edfm import system_key
    from oracle import fams, grids

    t0 = time.perf_counter()
    s = make_config(args.config, contrast=args.contrast)
    q = s.q if args.rhs < 0 else config_rhs(s, args.config, args.rhs + 1)[args.rhs]
    key = system_key(s.row_ptr, s.col, s.val, q)
    coarse, d_min, r_z = GRIDS[args.config]
    wb, primal, vertex, _ = grids.full_grid(s, coarse, d_min, r_z)
    t1 = time.perf_counter()
    F = fams.FAMS(s.csr(), wb, vertex, s.n_matrix, fams.DECOUPLED, alpha=0.0)
    t2 = time.perf_counter()
    p, info = F.gmres(q, rtol=args.rtol, max_iter=2000)
    t3 = time.perf_counter()
    balance = None
    if args.flux:
        from oracle import flux
        balance = float(flux.reconstruct_flux(F.A, F.P, primal, vertex, q, p)[3])
    os.makedirs(CACHE, exist_ok=True)
    np.save(cache_path(key), p.astype(np.float32))
    meta = dict(config=args.config, rhs=args.rhs, contrast=args.contrast, key=key, n=int(s.n),
                rtol=args.rtol, status=int(info["status"]), iterations=int(info["iterations"]),
                rel_residual=float(info["rel_residual"]), variant="decoupled", alpha=0.0,
                balance=balance,
                input_s=t1 - t0, setup_s=t2 - t1, solve_s=t3 - t2)
    with open(os.path.join(CACHE, key + ".json"), "w") as f:
        json.dump(meta, f, indent=1)
    print(json.dumps(meta))


if __name__ == "__main__":
    main()
