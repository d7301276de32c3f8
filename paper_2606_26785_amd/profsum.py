"""Summaries of rocprofv3 CSV output, as short text for profiles/.

    python profsum.py stats <kernel_stats.csv> [top]
        per-kernel calls, total and average duration, share of device time
    python profsum.py pmc <counter_collection.csv> <COUNTER>
        per-kernel dispatches and mean counter value per dispatch, plus the
        calibration line for the runtime's copy kernel (its largest
        dispatches), whose bytes are known to the caller
"""
import csv
import sys
from collections import defaultdict


def _col(row, *names):
    low = {k.lower(): k for k in row}
    for n in names:
        if n.lower() in low:
            return row[low[n.lower()]]
    raise KeyError(names)


def stats(path, top=25):
    rows = list(csv.DictReader(open(path)))
    tot = sum(float(_col(r, "TotalDurationNs")) for r in rows)
    print("total kernel time %.1f ms over %d kernels" % (tot / 1e6, len(rows)))
    print("%-44s %10s %12s %12s %7s" % ("kernel", "calls", "total ms", "avg us", "share"))
    for r in rows[:top]:
        name = _col(r, "Name", "Kernel_Name")
        calls = int(_col(r, "Calls"))
        t = float(_col(r, "TotalDurationNs"))
        print("%-44s %10d %12.1f %12.2f %6.1f%%" % (name.split("(")[0][:44], calls, t / 1e6, t / calls / 1e3,
                                                    100.0 * t / tot))


def pmc(path, counter):
    acc = defaultdict(lambda: [0, 0.0])
    copy_sizes = []
    for r in csv.DictReader(open(path)):
        if _col(r, "Counter_Name") != counter:
            continue
        name = _col(r, "Kernel_Name").split("(")[0]
        v = float(_col(r, "Counter_Value"))
        a = acc[name]
        a[0] += 1
        a[1] += v
        if "copyBuffer" in name:
            copy_sizes.append((int(float(_col(r, "Grid_Size"))), v))
    print("%s per dispatch (KiB)" % counter)
    print("%-44s %10s %14s" % ("kernel", "dispatches", "mean KiB"))
    for name, (c, s) in sorted(acc.items(), key=lambda kv: -kv[1][1]):
        print("%-44s %10d %14.1f" % (name[:44], c, s / c))
    if copy_sizes:
        gmax = max(g for g, _ in copy_sizes)
        big = [v for g, v in copy_sizes if g == gmax]
        print("calibration: runtime copy kernel, largest dispatches (grid %d): %d dispatches, mean %.1f KiB"
              % (gmax, len(big), sum(big) / len(big)))


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2], int(sys.argv[3]) if len(sys.argv) > 3 else 25)
    elif sys.argv[1] == "pmc":
        pmc(sys.argv[2], sys.argv[3])
    else:
        raise SystemExit(__doc__)
