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
