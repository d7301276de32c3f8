"""Write the oracle's sigma_min at seeded sample points of the sparse
convection-diffusion grid (N = 500, n = 250,000, 100 x 100 grid near the
spectral boundary; workloads.convection_diffusion defaults).  The sample is
drawn from the grid points on every STRIDE-th line in each direction, so that
a GPU run on that 20 x 20 sub-grid (same region) meets every sampled point.

Every value comes from the scale oracle O2 for square sparse C
(oracle.sigma_min_sparse_lu: banded LU of C - z I, block inverse subspace
iteration on (A^* A)^{-1}), itself checked against the dense Jacobi oracle on
reduced instances by tests/test_oracle.py.  ||C||_2 comes from the oracle's
power iteration.  Nothing here calls the GPU library.  The sample: 64 of the
400 sub-grid points drawn without replacement by workloads.sample_indices
(seed 3003), stored as indices j * nx + i of the full grid.

Each point needs a ~6 GB banded factorisation, so the sample is split into
parts that can run side by side, then merged:

    OMP_NUM_THREADS=2 python tests/golden/make_convdiff_ref.py --part 0 --parts 4
    ...
    python tests/golden/make_convdiff_ref.py --merge --parts 4
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle      # noqa: E402
import workloads   # noqa: E402

OUT = os.path.join(HERE, "convdiff_n250000_grid100_sigma.json")
NPTS = 64
SEED = 3003
STRIDE = 5


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--part", type=int, default=0)
    ap.add_argument("--parts", type=int, default=1)
    ap.add_argument("--merge", action="store_true")
    args = ap.parse_args()
    wl = workloads.convection_diffusion()
    if args.merge:
        idx, sig, steps = [], [], []
        meta = None
        for p in range(args.parts):
            d = json.load(open(OUT + ".part%d" % p))
            meta = d
            idx += d["indices"]
            sig += d["sigma"]
            steps += d["steps"]
        order = np.argsort(idx)
        out = {k: meta[k] for k in ("workload", "N", "n", "nx", "ny", "region", "oracle")}
        wl = workloads.convection_diffusion()
        out["normC"] = oracle.norm2_sparse(wl.m, wl.n, wl.rowptr, wl.colind, wl.vals)
        out["indices"] = [int(idx[i]) for i in order]
        out["sigma"] = [float(sig[i]) for i in order]
        out["steps"] = [int(steps[i]) for i in order]
        with open(OUT, "w") as f:
            json.dump(out, f)
        for p in range(args.parts):
            os.remove(OUT + ".part%d" % p)
        return
    zs = oracle.grid_points(*wl.region, wl.nx, wl.ny)
    sub = np.array([j * wl.nx + i for j in range(0, wl.ny, STRIDE) for i in range(0, wl.nx, STRIDE)])
    idx = sub[workloads.sample_indices(sub.size, NPTS, SEED)]
    mine = [int(i) for k, i in enumerate(idx) if k % args.parts == args.part]
    normC = oracle.norm2_sparse(wl.m, wl.n, wl.rowptr, wl.colind, wl.vals)
    t0 = time.time()
    sig, steps = [], []
    for c, i in enumerate(mine):
        s, it = oracle.sigma_min_sparse_lu(wl.m, wl.n, wl.rowptr, wl.colind, wl.vals, zs[i:i + 1], normC=normC)
        sig.append(float(s[0]))
        steps.append(int(it[0]))
        print("part %d: %d/%d points, %.0f s" % (args.part, c + 1, len(mine), time.time() - t0), file=sys.stderr,
              flush=True)
    with open(OUT + ".part%d" % args.part, "w") as f:
        json.dump({"workload": "convection_diffusion", "N": wl.info["N"], "n": wl.n, "nx": wl.nx, "ny": wl.ny,
                   "region": list(wl.region), "normC": normC, "oracle": "O2 sparse (banded LU + inverse subspace "
                   "iteration)", "indices": mine, "sigma": sig, "steps": steps}, f)


if __name__ == "__main__":
    main()
