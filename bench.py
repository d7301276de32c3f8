#!/usr/bin/env python3
"""Throughput of the recycled sigma_min path on one MI355X.

Workload (default): dense nonnormal banded Toeplitz C, n = 4000, one sub- and
three superdiagonals drawn from CN(0,1) by seed, stored dense; 200 x 200 grid
over the bounding box of the numerical range padded by 10%; recycled
subspace k <= 32, block r = 8.  One step is one ps_eval over the whole grid
(every point certified), with C already resident on the device.

Printed (one JSON line): grid points per second of the recycled path, the
plain per-point solver on the same GPU (LOBPCG-SVD from a seeded random
start, no recycling) measured on a sub-grid of the same region, the roofline
of the dominant kernel class from HIP events recorded around its launches,
and the oracle timed on the host cores on a bounded sample of points.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6      # MI355X dense FP64 (matrix and vector)
PEAK_HBM_GBS = 8000.0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--n", type=int, default=4000)
    ap.add_argument("--grid", type=int, default=200)
    ap.add_argument("--plain-grid", type=int, default=5, help="side of the sub-grid timed with the plain solver")
    ap.add_argument("--cpu-points", type=int, default=16, help="grid points in the oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--verbose", action="store_true", help="progress lines on stderr (the default)")
    ap.add_argument("--quiet", action="store_true", help="no progress lines")
    ap.add_argument("--tiles-x", type=int, default=0)
    ap.add_argument("--tiles-y", type=int, default=0)
    ap.add_argument("--batch", type=int, default=20)
    ap.add_argument("--save-sigma", default="", help="write the grid's sigma and flags to this .npy")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: measures one GPU only (the path would shard by grid tile, one band of tiles per GPU)",
              file=sys.stderr)
        sys.exit(2)

    def log(msg):
        print("[bench] " + msg, file=sys.stderr, flush=True)

    log("loading torch and the library")
    import numpy as np
    import torch
    import paper_2606_26785_amd as P
    import workloads

    wl = workloads.toeplitz_band(n=args.n, grid=args.grid)
    npts = wl.npts
    # progress lines go to stderr every few seconds: a sweep of the full grid
    # takes minutes, and the one JSON line stays alone on stdout
    params = P.default_params(profile=1, verbose=0 if args.quiet else 1, tiles_x=args.tiles_x,
                              tiles_y=args.tiles_y, batch=args.batch)
    t0 = time.perf_counter()
    mat = P.create_from_workload(wl, params=params)
    t_create = time.perf_counter() - t0
    grid = P.ps_grid(*wl.region, wl.nx, wl.ny)
    log("created n=%d in %.2f s; grid %dx%d" % (wl.n, t_create, wl.nx, wl.ny))
    for w in range(args.warmup):
        res = P.ps_eval(mat, grid, wl.eps)
        log("warmup %d: %.1f ms" % (w, res.stats["t_total_ms"]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        res = P.ps_eval(mat, grid, wl.eps)
        log("step %d: %.1f ms accepted %d refined %d rebuilds %d" % (
            k, res.stats["t_total_ms"], res.stats["accepted"], res.stats["refined"], res.stats["rebuilds"]))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    value = npts / (ms_per_step / 1000.0)
    st = res.stats

    # dominant kernel class by event-timed device time
    names = ["operator_apply_zgemm_mfma", "precond_apply_zgemm_mfma", "ritz_jacobi", "factorization_zgemm_mfma"]
    c = int(np.argmax([st["k_ms"][i] if i != 2 else 0.0 for i in range(4)]))
    launches = st["k_launches"][c]
    roofline = None
    if launches > 0 and st["k_ms"][c] > 0:
        avg_ms = st["k_ms"][c] / launches
        fl = st["k_flops"][c] / launches
        achieved = fl / (avg_ms * 1e-3) / 1e12
        roofline = {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                    "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None, "kernel": names[c],
                    "launches": int(launches), "avg_launch_ms": avg_ms,
                    "flops_per_launch": fl, "bytes_per_launch": st["k_bytes"][c] / launches,
                    "device_ms_by_class": dict(zip(names, st["k_ms"][:4]))}

    plain = None
    if not args.no_plain:
        g = args.plain_grid
        pp = P.default_params(recycle=0, tiles_x=1, tiles_y=1)
        matp = P.create_from_workload(wl, params=pp)
        gp = P.ps_grid(*wl.region, g, g)
        torch.cuda.synchronize()
        tp0 = time.perf_counter()
        resp = P.ps_eval(matp, gp, wl.eps)
        torch.cuda.synchronize()
        tp = time.perf_counter() - tp0
        plain = {"value": g * g / tp, "unit": "pts/s", "points": g * g,
                 "lobpcg_iters": resp.stats["lobpcg_iters"], "uncertified": resp.stats["uncertified"]}
        matp.close()
        log("plain solver: %d points in %.2f s" % (g * g, tp))

    if args.save_sigma:
        np.save(args.save_sigma, np.stack([res.sigma, res.flags.astype(np.float64)]))

    # full-grid parity against the stored oracle values (tests/golden), when present
    parity = None
    gold = os.path.join(ROOT, "tests", "golden", "toeplitz_n4000_grid200_sigma.npy")
    if args.n == 4000 and args.grid == 200 and os.path.exists(gold):
        ref = np.load(gold)
        normC = mat.norm_estimate / 1.01
        err = np.abs(res.sigma - ref) / normC
        parity = {"points": int(ref.size), "max_abs_err_over_normC": float(err.max()),
                  "points_over_1e-8": int((err > 1e-8).sum()),
                  "min_signed_err_over_normC": float(((res.sigma - ref) / normC).min()),
                  "oracle": "O2 banded, every grid point (tests/golden)"}
        log("full-grid parity: max |err|/||C|| = %.2e, %d points over 1e-8" % (
            parity["max_abs_err_over_normC"], parity["points_over_1e-8"]))

    cpu = None
    if not args.no_cpu:
        import oracle
        zs = oracle.grid_points(*wl.region, wl.nx, wl.ny)
        idx = workloads.sample_indices(zs.size, args.cpu_points, 4242)
        band, kl, ku = oracle.band_from_dense(wl.dense)
        tc0 = time.perf_counter()
        ref = oracle.sigma_min_banded(band, wl.m, wl.n, kl, ku, zs[idx])
        tc = time.perf_counter() - tc0
        normC = mat.norm_estimate / 1.01
        err = float(np.max(np.abs(res.sigma[idx] - ref)) / normC)
        cpu = {"value": len(idx) / tc, "unit": "pts/s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": "%d seeded grid points of the same grid, banded O2 oracle (Givens QR + bulge "
                         "chasing + Sturm bisection), %.1f s wall" % (len(idx), tc),
               "sample_max_abs_err_over_normC": err}
        log("oracle sample: %d points in %.2f s, max |err|/||C|| = %.2e" % (len(idx), tc, err))

    out = {
        "metric": "sigma_min grid pts/s (recycled path, certified at 1e-8 ||C||)",
        "value": value,
        "unit": "pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic (seeded dense banded Toeplitz)",
        "config": {"workload": "dense-toeplitz-n%d-grid%dx%d" % (wl.n, wl.nx, wl.ny), "n": wl.n,
                   "grid": [wl.nx, wl.ny], "r": params.r, "k_max": params.k_max, "points": npts},
        "stats": {k: st[k] for k in ("accepted", "refined", "uncertified", "certified", "lipschitz_redo",
                                     "lobpcg_iters", "rebuilds", "rounds", "mv_M", "sv_F", "t_ritz_ms",
                                     "t_lobpcg_ms", "t_update_ms", "t_precond_ms")},
        "parity": parity,
        "create_s": t_create,
        "plain_per_point": plain,
        "recycled_vs_plain": (value / plain["value"]) if plain else None,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    mat.close()


if __name__ == "__main__":
    main()
