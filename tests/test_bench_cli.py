"""bench.py's command line: more than one GPU is refused with a message (this
path measures one GPU), without touching a GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _bench_module():
    sys.path.insert(0, ROOT)
    import bench
    return bench


def test_traffic_reader_checks_the_kernel_source(tmp_path, monkeypatch):
    """roofline.traffic comes from profiles/<kernel>_traffic.md only while the
    kernel source still has the hash recorded there; the reported ratio is
    measured over algorithmic bytes of the counted run."""
    import hashlib
    bench = _bench_module()
    src = tmp_path / "k.hip"
    src.write_text("kernel text\n")
    (tmp_path / "profiles").mkdir()
    doc = tmp_path / "profiles" / "k_demo_traffic.md"

    def write(sha):
        doc.write_text("# demo\n\n    kernel_source: k.hip\n    kernel_source_sha256: %s\n"
                       "    traffic_bytes_per_launch: 150\n    algorithmic_bytes_per_launch: 100\n"
                       "    workload: demo\n" % sha)

    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    write(hashlib.sha256(src.read_bytes()).hexdigest())
    tr = bench.measured_traffic("k_demo")
    assert tr is not None and abs(tr["over_algorithmic"] - 1.5) < 1e-12
    assert tr["counted_bytes_per_launch"] == 150.0
    write("0" * 64)
    assert bench.measured_traffic("k_demo") is None
    assert bench.measured_traffic("k_missing") is None


def test_committed_traffic_profile_is_readable():
    """The committed counter summary of the dominant dense kernel parses, and
    names a kernel source that exists."""
    bench = _bench_module()
    path = os.path.join(ROOT, "profiles", "k_zgemm_fact_wide_traffic.md")
    assert os.path.exists(path)
    fields = {}
    for line in open(path):
        line = line.strip()
        if ":" in line:
            k, v = line.split(":", 1)
            fields[k] = v.strip()
    assert os.path.exists(os.path.join(ROOT, fields["kernel_source"]))
    assert float(fields["traffic_bytes_per_launch"]) > float(fields["algorithmic_bytes_per_launch"]) > 0
    assert "k_zgemm_fact_wide" in bench.CLASS_KERNELS


def test_paper_context_is_the_published_table():
    """The context block of the bench line restates the paper's Table 2 times
    for its dense examples (40,000 grid points each) and serialises to JSON."""
    import json
    bench = _bench_module()
    ctx = json.loads(json.dumps(bench.PAPER_CONTEXT))
    rows = {r["matrix"]: r for r in ctx["dense"]}
    assert rows["basor"]["psTriRecy_s"] == 1352 and rows["basor"]["psInvLanc_s"] == 7251
    assert rows["landau_40pi"]["psTriRecy_s"] == 2006 and rows["landau_40pi"]["psInvLanc_s"] == 9069
    for r in ctx["dense"]:
        assert abs(r["psTriRecy_pts_per_s"] - ctx["grid_points"] / r["psTriRecy_s"]) < 1e-9


def test_path_work_per_unit_figures():
    """The per-unit algorithmic work bench.py charges, at the dense workload's
    n = 4000, r = 8, k = 32: a Ritz test 8.2 MFLOP, a LOBPCG iteration two
    operator products of 8 n^2 r flops each (2.05 GFLOP), a preconditioned
    iteration 1.02 GFLOP more, a store update 3.07 GFLOP, an inertia test
    8 n^3 / 3 and a site twice that."""
    bench = _bench_module()
    n, r, k = 4000, 8, 32
    keys = ("ritz_jobs", "lobpcg_iters", "precond_iters", "store_updates", "cert_tests", "rebuilds")

    def one(key):
        st = {x: 0 for x in keys}
        st[key] = 1
        st["k_launches"] = [0] * 9
        return bench.path_work(st, n, r, k)[0]

    assert abs(one("ritz_jobs") - 8.192e6) < 1e3
    assert abs(one("lobpcg_iters") - 2.048e9) < 1e3
    assert abs(one("precond_iters") - 1.024e9) < 1e3
    assert abs(one("store_updates") - 3.072e9) < 1e3
    assert abs(one("cert_tests") - 8 * n ** 3 / 3) < 1e3
    assert abs(one("rebuilds") - 16 * n ** 3 / 3) < 1e3
