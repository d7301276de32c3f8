#!/usr/bin/env python3
"""Throughput of the recycled sigma_min path on one MI355X.

Workload (default): dense nonnormal banded Toeplitz C, n = 4000, one sub- and
three superdiagonals drawn from CN(0,1) by seed, stored dense; 200 x 200 grid
over the bounding box of the numerical range padded by 10%; recycled
subspace k <= 32, block r = 8.  One step is one ps_eval over the whole grid
(every point evaluated to 1e-8 ||C||_2), with C already resident on the
device; each ps_eval starts from empty recycled stores.

Wall-clock budget: a step takes tens of seconds, so the run is bounded by
--budget-s (whole process).  Kernels are loaded by a warm-up ps_eval on a
16 x 16 window of the grid; then full-grid steps are timed while the next one
still fits the budget (at least one, at most --steps).  The line reports the
steps requested and run.

Printed (one JSON line on stdout; progress on stderr):
  value            grid points per second of the recycled path;
  roofline         the event-timed kernel class with the most device time:
                   algorithmic flops per launch / average launch duration
                   (HIP events on the library's stream);
  roofline_path    the whole path: the time the algorithmic work counted by
                   the library (Ritz tests, LOBPCG iterations, store updates,
                   factorizations) needs at the FP64 peak, over the step time;
  plain_per_point  the plain solver (LOBPCG-SVD from a random start, no
                   recycling, same kernels and batching) on a strided
                   sub-grid of the same region;
  cpu_baseline     the oracle on a bounded seeded sample, on the host cores;
  parity           the full grid against the stored oracle values.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6      # MI355X dense FP64 (matrix cores and vector units alike)
PEAK_HBM_GBS = 8000.0
CLASS_NAMES = ["operator_apply", "precond_apply", "ritz_extraction", "factorization_gemm",
               "factorization_diag", "small_per_tile", "tall_skinny", "other", "factorization_gemm_narrow"]
CLASS_BOUND = ["mfma", "mfma", "alu", "mfma", "alu", "alu", "hbm", "hbm", "mfma"]
CLASS_KERNELS = ["k_dense_gemm + k_dense_reduce (dense) or k_csr_apply (CSR)", "k_zgemm (+ k_zgemm_reduce)",
                 "k_ritz", "k_zgemm_fact_wide", "k_chol_step, k_form_normal",
                 "k_rr_hl, k_chol_dd, k_svqb, k_rotations", "k_gram_part, k_gemm_ts, k_colnorm_part",
                 "copies, fills", "k_zgemm_fact (+ k_zgemm_reduce)"]


# The paper's own timings (Sec. 4, Tables 1 and 2), for context only: other
# matrices (its dense examples are basor, a Toeplitz matrix of n = 2,000, and
# landau_40pi, n = 5,000), no stated accuracy bar, and other hardware (Julia,
# one thread of a 2.90 GHz Intel Core i5); 200 x 200 grids throughout.
PAPER_CONTEXT = {
    "hardware": "Julia v1.12, single thread, 2.90 GHz Intel Core i5, 16 GB",
    "grid_points": 40000,
    "dense": [
        {"matrix": "basor", "n": 2000, "psTriRecy_s": 1352, "psTriRecy_pts_per_s": 40000 / 1352,
         "psInvLanc_s": 7251, "psInvLanc_pts_per_s": 40000 / 7251},
        {"matrix": "landau_40pi", "n": 5000, "psTriRecy_s": 2006, "psTriRecy_pts_per_s": 40000 / 2006,
         "psInvLanc_s": 9069, "psInvLanc_pts_per_s": 40000 / 9069},
    ],
    "note": "different matrices, accuracy and hardware: context, not a baseline for this workload",
}


def measured_traffic(kernel):
    """The HBM traffic per launch of `kernel` stored in profiles/<kernel>_traffic.md
    (rocprofv3 FETCH_SIZE and WRITE_SIZE passes scaled by a copy of known
    size), or None when there is none or the kernel's source has changed
    since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "%s_traffic.md" % kernel)
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        line = line.strip()
        if ":" in line and line.split(":", 1)[0] in ("kernel_source", "kernel_source_sha256",
                                                      "traffic_bytes_per_launch", "algorithmic_bytes_per_launch",
                                                      "workload"):
            k, v = line.split(":", 1)
            fields[k] = v.strip()
    try:
        src = open(os.path.join(ROOT, fields["kernel_source"]), "rb").read()
    except (KeyError, OSError):
        return None
    if hashlib.sha256(src).hexdigest() != fields.get("kernel_source_sha256"):
        return None
    t = float(fields["traffic_bytes_per_launch"])
    a = float(fields["algorithmic_bytes_per_launch"])
    return {"counted_bytes_per_launch": t, "counted_algorithmic_bytes_per_launch": a, "over_algorithmic": t / a,
            "counted_workload": fields.get("workload"), "source": "profiles/%s_traffic.md" % kernel}


def path_work(st, n, r, k):
    """Algorithmic flops and HBM bytes of one ps_eval from the library's
    counters.  Complex multiply-add = 8 real flops.
      Ritz test (per tested point): QR of the 2k x k B(z) plus about eight
        one-sided Jacobi sweeps with right vectors: ~250 k^3;
      LOBPCG iteration (per point): C(z) W and C(z)^* (C X) on r columns,
        2 * 8 n^2 r, plus 2 * 4 n^2 r for K^{-1} = F^{-1} F^{-*} (triangular
        explicit inverse) where a preconditioner is applied;
      store update (per point): 3 r operator columns, 3 * 8 n^2 r;
      inertia test: Cholesky of N(z) - mu I, 8 n^3 / 3;
      preconditioner site: Cholesky plus explicit inverse, 16 n^3 / 3.
    Bytes: the tall-skinny traffic of a LOBPCG iteration, about 30 sweeps
    over n x r complex blocks, and the operator read once per apply launch."""
    n = float(n)
    fl = (st["ritz_jobs"] * 250.0 * k ** 3
          + st["lobpcg_iters"] * 16.0 * n * n * r
          + st["precond_iters"] * 8.0 * n * n * r
          + st["store_updates"] * 24.0 * n * n * r
          + st["cert_tests"] * 8.0 * n ** 3 / 3.0
          + st["rebuilds"] * 16.0 * n ** 3 / 3.0)
    by = st["lobpcg_iters"] * 30.0 * n * r * 16.0 + st["k_launches"][0] * 16.0 * n * n
    return fl, by


def path_work_sparse(st, wl, r, k):
    """Algorithmic HBM bytes (and flops) of one ps_eval on the sparse path
    from the library's counters: per operator column-apply the CSR arrays
    (20 B per nonzero) plus one read of x and one write of y (32 n B); per
    preconditioner column-solve the factor values and indices (20 B per
    nonzero) plus x, y; per LOBPCG iteration about 30 sweeps over n x r
    blocks; the Ritz tests as in the dense path."""
    nnz = float(len(wl.vals) + wl.n)
    n = float(wl.n)
    by = (st["mv_M"] * (20.0 * nnz / max(r, 1) + 32.0 * n) + st["sv_F"] * (20.0 * nnz / max(r, 1) + 32.0 * n)
          + st["lobpcg_iters"] * 30.0 * n * r * 16.0)
    fl = st["ritz_jobs"] * 250.0 * k ** 3 + 8.0 * nnz * (st["mv_M"] + st["sv_F"])
    return fl, by


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--budget-s", type=float, default=500.0,
                    help="wall-clock budget of the whole run (timed steps stop when the next would not fit)")
    ap.add_argument("--workload", default="toeplitz", choices=["toeplitz", "convdiff", "serving", "batched"],
                    help="toeplitz: dense Toeplitz n=4000, 200x200 (default); convdiff: sparse CSR n=250,000, "
                         "100x100; serving: a Poisson stream of mixed requests (reduced sizes, see --serve-*)")
    ap.add_argument("--serve-requests", type=int, default=24)
    ap.add_argument("--serve-max-active", type=int, default=8)
    ap.add_argument("--serve-seed", type=int, default=1005)
    ap.add_argument("--serve-dense", default="256,1024", help="dense n range (full stream: 256,4096)")
    ap.add_argument("--serve-sparse", default="40,100", help="stencil side N range (full stream: 100,447)")
    ap.add_argument("--serve-grid", default="16,32", help="grid side range (full stream: 32,128)")
    ap.add_argument("--batch-dense", type=int, default=24, help="batched: dense matrices (full batch: 192)")
    ap.add_argument("--batch-fold", type=int, default=8, help="batched: rectangular foldings (full batch: 64)")
    ap.add_argument("--batch-dense-n", default="64,512", help="batched: dense n range (full batch: 64,1024)")
    ap.add_argument("--batch-fold-n", default="1000,4000", help="batched: folding n range (full: 1000,20000)")
    ap.add_argument("--batch-grid", type=int, default=16, help="batched: grid side (full batch: 64)")
    ap.add_argument("--n", type=int, default=4000)
    ap.add_argument("--grid", type=int, default=200)
    ap.add_argument("--plain-stride", type=int, default=10,
                    help="plain solver on every k-th grid line in each direction (0: skip)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target length of the oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--quiet", action="store_true", help="no progress lines")
    ap.add_argument("--profile", type=int, default=1, help="event-timed kernel classes (1: 0-4, 2: all)")
    ap.add_argument("--tiles-x", type=int, default=0)
    ap.add_argument("--tiles-y", type=int, default=0)
    ap.add_argument("--batch", type=int, default=20)
    ap.add_argument("--precond", type=int, default=-1, help="ps_params.precond (-1: the library default)")
    ap.add_argument("--save-sigma", default="", help="write the grid's sigma and flags to this .npy")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-mebibyte device buffer 4 times and exit (the known-size copy that "
                         "scales the HBM byte counters of a profile)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: measures one GPU only (the path would shard by grid tile, one band of tiles per GPU)",
              file=sys.stderr)
        sys.exit(2)
    t_start = time.perf_counter()

    def log(msg):
        if not args.quiet:
            print("[bench %6.1fs] %s" % (time.perf_counter() - t_start, msg), file=sys.stderr, flush=True)

    log("loading torch and the library")
    import numpy as np
    import torch
    import paper_2606_26785_amd as P
    import workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calib > 0:
        nb = args.copy_calib << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib_bytes": nb, "copies": 4}), flush=True)
        return
    if args.workload == "serving":
        return serve_main(args, log)
    if args.workload == "batched":
        return batched_main(args, log)
    if args.workload == "convdiff":
        wl = workloads.convection_diffusion()
        params = P.default_params(profile=args.profile, verbose=0 if args.quiet else 1, tiles_x=args.tiles_x,
                                  tiles_y=args.tiles_y, batch=args.batch, k_max=64, tile_mem_gb=96,
                                  precond=args.precond)
    else:
        wl = workloads.toeplitz_band(n=args.n, grid=args.grid)
        params = P.default_params(profile=args.profile, verbose=0 if args.quiet else 1, tiles_x=args.tiles_x,
                                  tiles_y=args.tiles_y, batch=args.batch, precond=args.precond)
    npts = wl.npts
    t0 = time.perf_counter()
    mat = P.create_from_workload(wl, params=params)
    t_create = time.perf_counter() - t0
    grid = P.ps_grid(*wl.region, wl.nx, wl.ny)
    log("created n=%d in %.2f s; grid %dx%d" % (wl.n, t_create, wl.nx, wl.ny))

    # kernel warm-up on a 16 x 16 window of the same grid
    re_lo, re_hi, im_lo, im_hi = wl.region
    hx = (re_hi - re_lo) / max(wl.nx - 1, 1)
    hy = (im_hi - im_lo) / max(wl.ny - 1, 1)
    w = min(16, wl.nx, wl.ny)
    gwin = P.ps_grid(re_lo, re_lo + (w - 1) * hx, im_lo, im_lo + (w - 1) * hy, w, w)
    warm_run = 0
    for _ in range(max(args.warmup, 0)):
        rw = P.ps_eval(mat, gwin, wl.eps)
        warm_run += 1
        log("warm-up window %dx%d: %.1f ms" % (w, w, rw.stats["t_total_ms"]))
    torch.cuda.synchronize()

    reserve = 45.0 + (0 if args.no_cpu else args.cpu_seconds)
    times = []
    res = None
    while len(times) < max(args.steps, 1):
        elapsed = time.perf_counter() - t_start
        if times and elapsed + max(times) * 1.1 + reserve > args.budget_s:
            break
        torch.cuda.synchronize()
        ts = time.perf_counter()
        res = P.ps_eval(mat, grid, wl.eps)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts)
        st = res.stats
        log("step %d: %.1f s accepted %d refined %d certified %d rebuilds %d cert_tests %d iters %d" % (
            len(times) - 1, times[-1], st["accepted"], st["refined"], st["certified"], st["rebuilds"],
            st["cert_tests"], st["lobpcg_iters"]))
    ms_per_step = 1000.0 * sum(times) / len(times)
    value = npts / (ms_per_step / 1000.0)
    st = res.stats

    # dominant event-timed kernel class (device time of the last step)
    kms = st["k_ms"]
    c = int(np.argmax(kms))
    roofline = None
    if st["k_launches"][c] > 0 and kms[c] > 0:
        launches = st["k_launches"][c]
        avg_ms = kms[c] / launches
        fl = st["k_flops"][c] / launches
        by = st["k_bytes"][c] / launches
        if CLASS_BOUND[c] == "hbm":
            achieved, peak, unit = by / (avg_ms * 1e-3) / 1e9, PEAK_HBM_GBS, "GB/s"
        else:
            achieved, peak, unit = fl / (avg_ms * 1e-3) / 1e12, PEAK_FP64_TFLOPS, "TFLOP/s"
        tr = measured_traffic(CLASS_KERNELS[c]) if " " not in CLASS_KERNELS[c] else None
        roofline = {"bound": CLASS_BOUND[c], "achieved": achieved, "peak": peak, "unit": unit,
                    "frac": achieved / peak,
                    # measured traffic / algorithmic bytes of the counted run, applied to
                    # this run's algorithmic bytes per launch
                    "traffic": tr["over_algorithmic"] * by if tr else None,
                    "traffic_detail": tr, "kernel_class": CLASS_NAMES[c], "kernels": CLASS_KERNELS[c],
                    "launches": int(launches), "avg_launch_ms": avg_ms, "flops_per_launch": fl,
                    "bytes_per_launch": by,
                    "device_ms_by_class": {CLASS_NAMES[i]: kms[i] for i in range(len(kms)) if kms[i] > 0},
                    "launches_by_class": {CLASS_NAMES[i]: int(st["k_launches"][i]) for i in range(len(kms))
                                          if kms[i] > 0},
                    "frac_by_class": {CLASS_NAMES[i]: (st["k_flops"][i] / (kms[i] * 1e-3) / 1e12 / PEAK_FP64_TFLOPS
                                                       if CLASS_BOUND[i] != "hbm" else
                                                       st["k_bytes"][i] / (kms[i] * 1e-3) / 1e9 / PEAK_HBM_GBS)
                                      for i in range(len(kms)) if kms[i] > 0}}
    fl_path, by_path = path_work(st, wl.n, params.r, params.k_max) if wl.kind == "dense" else \
        path_work_sparse(st, wl, params.r, params.k_max)
    t_roof = fl_path / (PEAK_FP64_TFLOPS * 1e12) + by_path / (PEAK_HBM_GBS * 1e9)
    roofline_path = {"bound": "mfma", "algorithmic_tflop": fl_path / 1e12, "algorithmic_gb": by_path / 1e9,
                     "t_roof_s": t_roof, "t_step_s": ms_per_step / 1000.0,
                     "frac": t_roof / (ms_per_step / 1000.0),
                     "achieved_tflops": fl_path / (ms_per_step / 1000.0) / 1e12}

    if args.save_sigma:
        np.save(args.save_sigma, np.stack([res.sigma, res.flags.astype(np.float64)]))

    # full-grid parity against the stored oracle values (tests/golden), when present
    parity = None
    gold = os.path.join(ROOT, "tests", "golden", "toeplitz_n4000_grid200_sigma.npy")
    meta = gold.replace(".npy", ".json")
    gold_cd = os.path.join(ROOT, "tests", "golden", "convdiff_n250000_grid100_sigma.json")
    if args.workload == "convdiff" and os.path.exists(gold_cd):
        d = json.load(open(gold_cd))
        idx = np.asarray(d["indices"])
        ref = np.asarray(d["sigma"])
        normC = float(d["normC"])
        err = (res.sigma[idx] - ref) / normC
        parity = {"points": int(ref.size), "max_abs_err_over_normC": float(np.abs(err).max()),
                  "points_over_1e-8": int((np.abs(err) > 1e-8).sum()),
                  "min_signed_err_over_normC": float(err.min()),
                  "oracle": "O2 sparse (banded LU + inverse subspace iteration), 64 seeded points (tests/golden)"}
        log("sample parity: max |err|/||C|| = %.2e over %d points" % (parity["max_abs_err_over_normC"], ref.size))
    elif args.workload == "toeplitz" and args.n == 4000 and args.grid == 200 and os.path.exists(gold) and \
            os.path.exists(meta):
        ref = np.load(gold)
        normC = float(json.load(open(meta))["normC"])      # oracle-side ||C||_2
        err = (res.sigma - ref) / normC
        parity = {"points": int(ref.size), "max_abs_err_over_normC": float(np.abs(err).max()),
                  "points_over_1e-8": int((np.abs(err) > 1e-8).sum()),
                  "min_signed_err_over_normC": float(err.min()),
                  "oracle": "O2 banded, every grid point (tests/golden)"}
        log("full-grid parity: max |err|/||C|| = %.2e, %d points over 1e-8, min signed %.2e" % (
            parity["max_abs_err_over_normC"], parity["points_over_1e-8"], parity["min_signed_err_over_normC"]))

    plain = None
    if args.plain_stride > 0:
        k = args.plain_stride
        nxp = (wl.nx - 1) // k + 1
        nyp = (wl.ny - 1) // k + 1
        gp = P.ps_grid(re_lo, re_lo + (nxp - 1) * k * hx, im_lo, im_lo + (nyp - 1) * k * hy, nxp, nyp)
        # no recycling: every point is its own tile, all in flight together
        pp = P.default_params(recycle=0, verbose=0, tile_points=1, batch=args.batch,
                              **({"k_max": 64, "tile_mem_gb": 96} if args.workload == "convdiff" else {}))
        matp = P.create_from_workload(wl, params=pp)
        torch.cuda.synchronize()
        tp0 = time.perf_counter()
        resp = P.ps_eval(matp, gp, wl.eps)
        torch.cuda.synchronize()
        tp = time.perf_counter() - tp0
        plain = {"value": nxp * nyp / tp, "unit": "pts/s", "points": nxp * nyp,
                 "sample": "every %d-th grid line in each direction of the same grid (%dx%d points, %.1f%% of "
                           "the grid), no recycling, one point per tile, all points batched" % (k, nxp, nyp,
                                                                                 100.0 * nxp * nyp / npts),
                 "lobpcg_iters": resp.stats["lobpcg_iters"], "cert_tests": resp.stats["cert_tests"],
                 "rebuilds": resp.stats["rebuilds"], "uncertified": resp.stats["uncertified"]}
        matp.close()
        log("plain solver: %d points in %.2f s" % (nxp * nyp, tp))

    cpu = None
    if not args.no_cpu and args.workload == "convdiff":
        import oracle
        zs = oracle.grid_points(*wl.region, wl.nx, wl.ny)
        idx = workloads.sample_indices(zs.size, 1, 4242)
        tc0 = time.perf_counter()
        ref, _ = oracle.sigma_min_sparse_lu(wl.m, wl.n, wl.rowptr, wl.colind, wl.vals, zs[idx], normC=8.0)
        tc = time.perf_counter() - tc0
        cpu = {"value": len(idx) / tc, "unit": "pts/s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": "%d seeded point of the same grid, sparse oracle O2 (banded LU with bandwidth 500 + block "
                         "inverse subspace iteration), %.1f s wall" % (len(idx), tc)}
        log("oracle sample: %d points in %.2f s" % (len(idx), tc))
    elif not args.no_cpu:
        import oracle
        zs = oracle.grid_points(*wl.region, wl.nx, wl.ny)
        band, kl, ku = oracle.band_from_dense(wl.dense)
        probe = workloads.sample_indices(zs.size, 8, 4242)
        tc0 = time.perf_counter()
        oracle.sigma_min_banded(band, wl.m, wl.n, kl, ku, zs[probe])
        per = (time.perf_counter() - tc0) / len(probe)
        cnt = int(min(zs.size, max(8, args.cpu_seconds / max(per, 1e-6))))
        idx = workloads.sample_indices(zs.size, cnt, 4243)
        tc0 = time.perf_counter()
        ref = oracle.sigma_min_banded(band, wl.m, wl.n, kl, ku, zs[idx])
        tc = time.perf_counter() - tc0
        cpu = {"value": len(idx) / tc, "unit": "pts/s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": "%d seeded points of the same grid, banded oracle O2 (Givens QR of the band, bulge "
                         "chasing, Sturm bisection), %.1f s wall" % (len(idx), tc),
               "sample_max_abs_err_over_normC": float(np.max(np.abs(res.sigma[idx] - ref)) /
                                                      wl_norm(wl, meta if parity else None))}
        log("oracle sample: %d points in %.2f s" % (len(idx), tc))

    out = {
        "metric": "sigma_min grid pts/s (recycled path, every point within 1e-8 ||C||_2)",
        "value": value,
        "unit": "pts/s",
        "n_gpus": 1,
        "steps": len(times),
        "warmup": warm_run,
        "steps_requested": args.steps,
        "warmup_requested": args.warmup,
        "warmup_kind": "ps_eval on a %dx%d window of the grid (kernel loading)" % (w, w),
        "budget_s": args.budget_s,
        "ms_per_step": ms_per_step,
        "step_s": times,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic (seeded dense banded Toeplitz, stored dense)" if args.workload == "toeplitz" else
                "synthetic (seeded convection-diffusion CSR with random row phases)",
        "config": {"workload": ("dense-toeplitz-n%d-grid%dx%d" if args.workload == "toeplitz" else
                                "csr-convdiff-n%d-grid%dx%d") % (wl.n, wl.nx, wl.ny), "n": wl.n,
                   "grid": [wl.nx, wl.ny], "r": params.r, "k_max": params.k_max, "points": npts,
                   "precond": {0: "none (K = I)", 1: "base (exact Cholesky sites)" if wl.kind == "dense" else
                               "base (incomplete Cholesky sites)",
                               2: "two-level (%s base + recycled projection subspace)" % (
                                   "regularised Cholesky" if wl.kind == "dense" else
                                   "incomplete Cholesky of N(z_dag)")}[params.precond if params.precond >= 0 else
                                                                        (1 if wl.kind == "dense" else 2)]},
        "stats": {k: st[k] for k in ("accepted", "refined", "uncertified", "certified", "lipschitz_redo",
                                     "lobpcg_iters", "precond_iters", "ritz_jobs", "store_updates", "rebuilds",
                                     "cert_tests", "repairs", "rounds", "mv_M", "sv_F", "proj_accepted",
                                     "proj_refined", "proj_iters", "ic_retries", "builds_shared",
                                     "builds_private", "t_ritz_ms",
                                     "t_lobpcg_ms", "t_update_ms", "t_precond_ms")},
        "parity": parity,
        "create_s": t_create,
        "plain_per_point": plain,
        "recycled_vs_plain": (value / plain["value"]) if plain else None,
        "roofline": roofline,
        "roofline_path": roofline_path,
        "cpu_baseline": cpu,
        "paper_context": PAPER_CONTEXT if wl.kind == "dense" else None,
    }
    print(json.dumps(out), flush=True)
    mat.close()


def serve_main(args, log):
    """Serving run: a closed-loop pre-run (the first requests, all arriving
    at once) gives the saturated capacity in requests/s; then the whole
    stream arrives as a Poisson process at 0.7 x that rate.  Reports the
    served grid points/s over the stream's makespan and the p50/p99
    latency (completion minus arrival)."""
    import numpy as np
    import torch
    import workloads
    from paper_2606_26785_amd import serving

    rng2 = lambda s: tuple(int(x) for x in s.split(","))
    wls = workloads.serving_requests(seed=args.serve_seed, n_req=args.serve_requests,
                                     dense_range=rng2(args.serve_dense), sparse_N_range=rng2(args.serve_sparse),
                                     grid_range=rng2(args.serve_grid))
    free, total = torch.cuda.mem_get_info()
    budget = int(0.8 * free)
    be = serving.LibraryBackend()
    # kernel loading
    warm = workloads.triangular_disk(seed=1, n=64, grid=4)
    be.run(serving.Request(-1, warm, 0.0))
    m = min(args.serve_max_active, len(wls))
    log("closed-loop pre-run: %d requests at once" % m)
    srv = serving.Server(be, hbm_budget=budget, max_active=args.serve_max_active)
    t0 = time.perf_counter()
    pre = srv.run([serving.Request(i, wls[i], 0.0) for i in range(m)], time_limit=args.budget_s)
    t_pre = time.perf_counter() - t0
    cap = m / max(max(r.done for r in pre), 1e-9)
    rate = 0.7 * cap
    arr = serving.poisson_arrivals(len(wls), rate, args.serve_seed + 1)
    log("capacity %.3f req/s; stream of %d requests at %.3f req/s" % (cap, len(wls), rate))
    srv = serving.Server(be, hbm_budget=budget, max_active=args.serve_max_active)
    reqs = [serving.Request(i, wl, float(a)) for i, (wl, a) in enumerate(zip(wls, arr))]
    res = srv.run(reqs, time_limit=max(args.budget_s - t_pre, 60.0))
    span = max(r.done for r in res)
    pts = sum(wl.npts for wl in wls)
    p50, p99 = serving.latency_percentiles(res)
    unc = sum(int(r.stats["uncertified"]) for r in res)
    out = {
        "metric": "served sigma_min grid pts/s (Poisson request stream at 0.7x closed-loop capacity)",
        "value": pts / span,
        "unit": "pts/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": span * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic (seeded request stream: dense triangular and convection-diffusion CSR)",
        "config": {"workload": "serving-%d-requests" % len(wls), "dense_n": args.serve_dense,
                   "stencil_N": args.serve_sparse, "grid_side": args.serve_grid,
                   "reduced": "from 512 requests, dense n 256..4096, stencil N 100..447, grid side 32..128",
                   "max_active": args.serve_max_active, "hbm_budget_gb": budget / 1e9},
        "p50_s": p50,
        "p99_s": p99,
        "capacity_req_s": cap,
        "rate_req_s": rate,
        "points": pts,
        "uncertified": unc,
        "peak_active": srv.peak_active,
        "peak_footprint_gb": srv.peak_bytes / 1e9,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def batched_main(args, log):
    """Batched uneven matrices: every matrix of the batch arrives at once and
    the serving loop runs them with continuous batching (one handle and HIP
    stream each, up to --serve-max-active at a time, admission by device
    memory).  Reports grid points/s over the whole batch."""
    import torch
    import workloads
    from paper_2606_26785_amd import serving

    rng2 = lambda s: tuple(int(x) for x in s.split(","))
    wls = workloads.batched_uneven(seed=1004, n_dense=args.batch_dense, n_fold=args.batch_fold,
                                   grid=args.batch_grid, dense_range=rng2(args.batch_dense_n),
                                   fold_range=rng2(args.batch_fold_n))
    free, total = torch.cuda.mem_get_info()
    budget = int(0.8 * free)
    be = serving.LibraryBackend()
    be.run(serving.Request(-1, workloads.triangular_disk(seed=1, n=64, grid=4), 0.0))
    log("batch of %d matrices (%d dense, %d foldings), grid %dx%d" % (
        len(wls), args.batch_dense, args.batch_fold, args.batch_grid, args.batch_grid))
    srv = serving.Server(be, hbm_budget=budget, max_active=args.serve_max_active)
    reqs = [serving.Request(i, wl, 0.0) for i, wl in enumerate(wls)]
    t0 = time.perf_counter()
    res = srv.run(reqs, time_limit=args.budget_s)
    span = time.perf_counter() - t0
    pts = sum(wl.npts for wl in wls)
    unc = sum(int(r.stats["uncertified"]) for r in res)
    out = {
        "metric": "batched sigma_min grid pts/s (uneven dense and rectangular CSR matrices, continuous batching)",
        "value": pts / span,
        "unit": "pts/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": span * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic (seeded uneven batch: dense triangular and rectangular banded foldings)",
        "config": {"workload": "batched-uneven-%d" % len(wls), "dense": args.batch_dense,
                   "dense_n": args.batch_dense_n, "foldings": args.batch_fold, "folding_n": args.batch_fold_n,
                   "grid": args.batch_grid, "max_active": args.serve_max_active,
                   "reduced": "from 192 dense (n 64..1024) + 64 foldings (n 1000..20000) on 64 x 64 grids"},
        "points": pts,
        "uncertified": unc,
        "peak_active": srv.peak_active,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def wl_norm(wl, meta):
    import numpy as np
    if meta and os.path.exists(meta):
        return float(json.load(open(meta))["normC"])
    return float(np.linalg.norm(wl.dense, 2))


if __name__ == "__main__":
    main()
