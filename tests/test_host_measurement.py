"""Host logic of the measurement plumbing, no GPU: the HBM-traffic summary
of two rocprofv3 counter passes (paper_1705_00614_amd/counters.py), its
kernel-trace window, and bench.py's lookup of a committed summary (the run
key and the kernel source digest must both match)."""
import csv
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1705_00614_amd import counters as C  # noqa: E402


def _counter_csv(path, counter, rows):
    """rows: (dispatch id, kernel name, value in KiB)."""
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for d, name, v in rows:
            w.writerow([d, name, counter, v])


def test_traffic_scales_by_the_copy_and_averages_the_last_dispatches(tmp_path):
    # a 256 MiB copy that FETCH_SIZE reads as half its size (factor 2) and
    # WRITE_SIZE as its size (factor 1); three step dispatches, the last two
    # averaged
    mib = 256
    fetch = [(1, "__amd_rocclr_copyBuffer", mib * 1024 / 2), (2, "void swe::k_step<float>", 999.0),
             (3, "void swe::k_step<float>", 100.0), (4, "void swe::k_step<float>", 300.0)]
    write = [(1, "__amd_rocclr_copyBuffer", mib * 1024.0), (2, "void swe::k_step<float>", 5.0),
             (3, "void swe::k_step<float>", 10.0), (4, "void swe::k_step<float>", 30.0)]
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    _counter_csv(f, "FETCH_SIZE", fetch)
    _counter_csv(w, "WRITE_SIZE", write)
    fb, fk, ff = C.summarise(C.read_counter(str(f), "FETCH_SIZE"), "k_step", 2, mib * float(1 << 20))
    wb, wk, wf = C.summarise(C.read_counter(str(w), "WRITE_SIZE"), "k_step", 2, mib * float(1 << 20))
    assert ff == pytest.approx(2.0) and wf == pytest.approx(1.0)
    assert fb == pytest.approx(200.0 * 1024 * 2.0) and wb == pytest.approx(20.0 * 1024)
    # too few dispatches, or no copy in the run, is an error
    with pytest.raises(SystemExit):
        C.summarise(C.read_counter(str(f), "FETCH_SIZE"), "k_step", 4, mib * float(1 << 20))
    _counter_csv(f, "FETCH_SIZE", fetch[1:])
    with pytest.raises(SystemExit):
        C.summarise(C.read_counter(str(f), "FETCH_SIZE"), "k_step", 2, mib * float(1 << 20))


def test_trace_window_mean(tmp_path, capsys):
    p = tmp_path / "t.csv"
    with open(p, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        for d, dur in enumerate([50, 10, 20, 30, 99], start=1):
            w.writerow([d, "void swe::k_step<float, 32, 32>", 1000 * d, 1000 * d + 1000 * dur])
        w.writerow([9, "other", 0, 5])

    class A:
        csv = str(p)
        kernel = "k_step<float, 32, 32"
        first = 1
        count = 3
    C.trace(A)
    out = capsys.readouterr().out
    assert "window_mean_us: 20.000" in out and "window_min_max_us: 10.000 30.000" in out


def test_bench_reports_traffic_only_for_the_current_kernel_source(tmp_path, monkeypatch):
    import bench
    prof = tmp_path / "profiles"
    prof.mkdir()
    digest = bench.kernel_source_digest()
    (prof / "k_step_traffic.txt").write_text(
        "# header\n\nrun_key: floodplain n=4096 tile=0x0\nkernel_source_sha256_16: %s\n"
        "hbm_bytes_per_launch: 4.0e7\n\nrun_key: wet n=4096 tile=0x0\nkernel_source_sha256_16: 0000000000000000\n"
        "hbm_bytes_per_launch: 9.0e8\n" % digest)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "paper_1705_00614_amd" / "csrc")
    with open(os.path.join(ROOT, "paper_1705_00614_amd", "csrc", "swe_step.hpp"), "rb") as src:
        (tmp_path / "paper_1705_00614_amd" / "csrc" / "swe_step.hpp").write_bytes(src.read())
    assert bench.profiled_traffic("floodplain n=4096 tile=0x0") == 4.0e7
    assert bench.profiled_traffic("wet n=4096 tile=0x0") is None        # another source digest
    assert bench.profiled_traffic("nest n=2048 tile=0x0") is None       # no block for the key


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
