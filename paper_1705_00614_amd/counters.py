"""Summarise rocprofv3 runs of the step kernel: HBM counter passes and
kernel traces.

python -m paper_1705_00614_amd.counters traffic --fetch F.csv --write W.csv \\
    --kernel k_step --last 20 --copy-mib 256 --run-key "floodplain n=4096 tile=0x0" \\
    --window "steps 5..25" --alg-bytes B [--command-fetch ...] [--command-write ...]
python -m paper_1705_00614_amd.counters trace --csv kernel_trace.csv \\
    --kernel "k_step<float, 32, 32" --first 5 --count 20

Reads the counter-collection CSVs of two rocprofv3 --pmc passes (FETCH_SIZE,
then WRITE_SIZE, both in KiB per dispatch), averages the last N dispatches of
the kernel whose name contains --kernel, scales each counter by what it read
for the plain device copy of --copy-mib MiB in the same run (the largest copy
dispatch), and prints one block in the format of profiles/k_step_traffic.txt
(bench.py reports hbm_bytes_per_launch as roofline.traffic while the kernel
source digest still matches).
"""
import argparse
import csv
import hashlib
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def kernel_source_digest():
    with open(os.path.join(HERE, "csrc", "swe_step.hpp"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def read_counter(path, counter):
    """(dispatch id, kernel name, value) of every row of `counter`, in dispatch order."""
    rows = []
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            if r.get("Counter_Name", "").strip() != counter:
                continue
            rows.append((int(r.get("Dispatch_Id") or r.get("Correlation_Id") or len(rows)),
                         r.get("Kernel_Name", ""), float(r["Counter_Value"])))
    rows.sort(key=lambda x: x[0])
    return rows


def summarise(rows, kernel, last, copy_bytes):
    ks = [v for _, name, v in rows if kernel in name]
    if len(ks) < last:
        raise SystemExit("only %d dispatches of %s" % (len(ks), kernel))
    copies = [v for _, name, v in rows if "copy" in name.lower()]
    if not copies:
        raise SystemExit("no copy dispatch in the run")
    copy_kib = max(copies)
    factor = copy_bytes / (copy_kib * 1024.0)
    mean_kib = sum(ks[-last:]) / last
    return mean_kib * 1024.0 * factor, copy_kib, factor


def trace(a):
    """Mean, min and max duration of dispatches first..first+count-1 (in
    dispatch order) of the kernels whose name contains --kernel, from a
    rocprofv3 --kernel-trace CSV, and the mean over all of them."""
    rows = []
    with open(a.csv, newline="") as f:
        for r in csv.DictReader(f):
            name = r.get("Kernel_Name", "")
            if a.kernel in name:
                d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3
                rows.append((int(r.get("Dispatch_Id") or r.get("Correlation_Id") or len(rows)), d, name))
    rows.sort(key=lambda x: x[0])
    if len(rows) < a.first + a.count:
        raise SystemExit("only %d dispatches of %s" % (len(rows), a.kernel))
    w = [d for _, d, _ in rows[a.first:a.first + a.count]]
    allv = [d for _, d, _ in rows]
    print("kernel: %s" % rows[0][2])
    print("window: dispatches %d..%d of %d" % (a.first + 1, a.first + a.count, len(rows)))
    print("window_mean_us: %.3f" % (sum(w) / len(w)))
    print("window_min_max_us: %.3f %.3f" % (min(w), max(w)))
    print("all_dispatches_mean_us: %.3f" % (sum(allv) / len(allv)))


def main():
    import sys
    if len(sys.argv) > 1 and sys.argv[1] == "trace":
        ap = argparse.ArgumentParser()
        ap.add_argument("--csv", required=True)
        ap.add_argument("--kernel", required=True)
        ap.add_argument("--first", type=int, default=0)
        ap.add_argument("--count", type=int, required=True)
        return trace(ap.parse_args(sys.argv[2:]))
    if len(sys.argv) > 1 and sys.argv[1] == "traffic":
        del sys.argv[1]
    ap = argparse.ArgumentParser()
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--kernel", default="k_step")
    ap.add_argument("--last", type=int, required=True)
    ap.add_argument("--copy-mib", type=int, default=256)
    ap.add_argument("--run-key", required=True)
    ap.add_argument("--window", required=True)
    ap.add_argument("--alg-bytes", type=float, required=True, help="algorithmic bytes per launch")
    ap.add_argument("--alg-read-fraction", type=float, default=20.0 / 32.0)
    ap.add_argument("--command-fetch", default="")
    ap.add_argument("--command-write", default="")
    a = ap.parse_args()
    cb = a.copy_mib * float(1 << 20)
    fetch, fk, ff = summarise(read_counter(a.fetch, "FETCH_SIZE"), a.kernel, a.last, cb)
    write, wk, wf = summarise(read_counter(a.write, "WRITE_SIZE"), a.kernel, a.last, cb)
    alg = a.alg_bytes
    lines = [
        "run_key: %s" % a.run_key,
        "window: %s" % a.window,
        "kernel_source_sha256_16: %s" % kernel_source_digest(),
        "hbm_bytes_per_launch: %.6e" % (fetch + write),
        "fetch_bytes_per_launch: %.6e" % fetch,
        "write_bytes_per_launch: %.6e" % write,
        "algorithmic_bytes_per_launch: %.6e" % alg,
        "traffic_over_algorithmic: %.3f" % ((fetch + write) / alg),
        "fetch_over_algorithmic_reads: %.3f" % (fetch / (alg * a.alg_read_fraction)),
        "write_over_algorithmic_writes: %.3f" % (write / (alg * (1.0 - a.alg_read_fraction))),
        "copy_calibration: %d MiB device copy read FETCH_SIZE %.1f KiB -> factor %.4f, WRITE_SIZE %.1f KiB "
        "-> factor %.4f" % (a.copy_mib, fk, ff, wk, wf),
        "dispatches_averaged: %d (the timed steps)" % a.last,
    ]
    if a.command_fetch:
        lines.append("command_fetch: %s" % a.command_fetch)
    if a.command_write:
        lines.append("command_write: %s" % a.command_write)
    print("\n".join(lines))


if __name__ == "__main__":
    main()
