"""The profile summariser that writes profiles/: per-kernel averages from a
kernel-stats table and per-dispatch counter means, on small hand-made CSVs."""
import contextlib
import io

from paper_2606_26785_amd import profsum


def _run(fn, *a):
    out = io.StringIO()
    with contextlib.redirect_stdout(out):
        fn(*a)
    return out.getvalue().splitlines()


def test_stats_averages_and_shares(tmp_path):
    p = tmp_path / "stats.csv"
    p.write_text("Name,Calls,TotalDurationNs\n"
                 "k_a(int),4,4000000\n"
                 "k_b,1,1000000\n")
    lines = _run(profsum.stats, str(p))
    assert lines[0] == "total kernel time 5.0 ms over 2 kernels"
    a = lines[2].split()
    assert a[0] == "k_a" and a[1] == "4" and float(a[2]) == 4.0 and float(a[3]) == 1000.0 and a[4] == "80.0%"
    b = lines[3].split()
    assert b[0] == "k_b" and float(b[3]) == 1000.0 and b[4] == "20.0%"


def test_pmc_means_per_dispatch_and_copy_calibration(tmp_path):
    p = tmp_path / "pmc.csv"
    p.write_text("Kernel_Name,Counter_Name,Counter_Value,Grid_Size\n"
                 "k_x(double*),FETCH_SIZE,100,256\n"
                 "k_x(double*),FETCH_SIZE,300,256\n"
                 "k_x(double*),WRITE_SIZE,7,256\n"
                 "__amd_rocclr_copyBuffer,FETCH_SIZE,50,64\n"
                 "__amd_rocclr_copyBuffer,FETCH_SIZE,500,1024\n"
                 "__amd_rocclr_copyBuffer,FETCH_SIZE,520,1024\n")
    lines = _run(profsum.pmc, str(p), "FETCH_SIZE")
    rows = {l.split()[0]: l.split() for l in lines[2:] if not l.startswith("calibration")}
    assert rows["k_x"][1] == "2" and float(rows["k_x"][2]) == 200.0
    cal = [l for l in lines if l.startswith("calibration")][0]
    assert "grid 1024" in cal and "2 dispatches" in cal and "mean 510.0 KiB" in cal
