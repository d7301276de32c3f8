"""Write the oracle's sigma_min on the whole dense-Toeplitz grid.

Workload: the seeded dense nonnormal banded Toeplitz matrix, n = 4000, on
the 200 x 200 grid over its padded numerical-range box (workloads.
toeplitz_band defaults).  Every value comes from the banded oracle O2
(Givens QR of the band, bulge chasing to bidiagonal form, Sturm bisection);
nothing here calls the GPU library.  Output: a float64 .npy of nx*ny values
in grid order (index j*nx + i) and a small JSON file with the workload
fingerprint.  Runs for hours on a few cores; progress goes to stderr and
finished chunks are kept in <out>.part so an interrupted run resumes.
The JSON file also holds ||C||_2, the largest singular value of C from the
same oracle at z = 0 (all n singular values by Sturm bisection); it scales
the parity tolerance.  ``--norm`` (re)computes only that value.

    OMP_NUM_THREADS=8 python tests/golden/make_toeplitz_ref.py
    python tests/golden/make_toeplitz_ref.py --norm
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle      # noqa: E402
import workloads   # noqa: E402

OUT = os.path.join(HERE, "toeplitz_n4000_grid200_sigma.npy")
CHUNK = 400


def fingerprint(wl):
    return {"workload": "toeplitz_band", "n": wl.n, "nx": wl.nx, "ny": wl.ny,
            "region": list(wl.region), "c00": [float(wl.dense[0, 0].real), float(wl.dense[0, 0].imag)],
            "c01": [float(wl.dense[0, 1].real), float(wl.dense[0, 1].imag)]}


def norm2(wl):
    band, kl, ku = oracle.band_from_dense(wl.dense)
    return float(oracle.banded_smallest(band, wl.m, wl.n, kl, ku, 0.0, k=wl.n)[-1])


def main():
    wl = workloads.toeplitz_band()
    meta_path = OUT.replace(".npy", ".json")
    if "--norm" in sys.argv[1:]:
        meta = json.load(open(meta_path))
        meta["normC"] = norm2(wl)
        with open(meta_path, "w") as f:
            json.dump(meta, f)
        return
    zs = oracle.grid_points(*wl.region, wl.nx, wl.ny)
    band, kl, ku = oracle.band_from_dense(wl.dense)
    part = OUT + ".part.npy"
    sig = np.load(part) if os.path.exists(part) else np.full(zs.size, np.nan)
    t0 = time.time()
    for c0 in range(0, zs.size, CHUNK):
        c1 = min(zs.size, c0 + CHUNK)
        if not np.isnan(sig[c0:c1]).any():
            continue
        sig[c0:c1] = oracle.sigma_min_banded(band, wl.m, wl.n, kl, ku, zs[c0:c1])
        np.save(part, sig)
        print("%d/%d points, %.0f s" % (c1, zs.size, time.time() - t0), file=sys.stderr, flush=True)
    np.save(OUT, sig)
    with open(meta_path, "w") as f:
        json.dump(dict(fingerprint(wl), threads=oracle.num_threads(), oracle="O2 banded", normC=norm2(wl)), f)
    os.remove(part)


if __name__ == "__main__":
    main()
