"""CPU tests of bench.py's host logic: the one-GPU guard and the accounting behind the roofline
figures it reports (the bisection's flop count, the Golub-Kahan path's algorithmic bytes, and the
HBM traffic summed from two rocprofv3 counter runs).  Nothing here touches a GPU."""
import csv
import os
import re
import shutil
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--no-cpu-baseline"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""          # no JSON line


def test_tests_per_lane_matches_the_kernels_choice(tmp_path):
    """The bench prices a pass by the tests the kernel makes in it; that count is a compile-time
    function in the bisection header.  Compile that function alone on the host and compare it
    with the bench's copy for every half-bandwidth and test mode."""
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    src = open(os.path.join(ROOT, "paper_2605_04550_amd", "csrc", "ps_bisect.hpp")).read()
    m = re.search(r"constexpr int tests_per_lane\(int hb, int ktm\) \{.*?\n\}", src, re.S)
    assert m, "tests_per_lane not found in the bisection header"
    body = m.group(0)
    # the library's ps_opts.tests -> the kernel's test-count mode (ps_api.cpp: ktm_of)
    api = open(os.path.join(ROOT, "paper_2605_04550_amd", "csrc", "ps_api.cpp")).read()
    k = re.search(r"int ktm_of\(const ps_opts &o\) \{ return (.*?); \}", api)
    assert k, "ktm_of not found"
    ktm = k.group(1).replace("o.tests", "t")
    prog = ("#include <cstdio>\n%s\nint ktm_of(int t) { return %s; }\n"
            "int main() { for (int t = 0; t <= 3; ++t) for (int hb = 1; hb <= 8; ++hb)"
            " std::printf(\"%%d %%d %%d\\n\", t, hb, tests_per_lane(hb, ktm_of(t))); }\n" % (body, ktm))
    cpp, exe = str(tmp_path / "tpl.cpp"), str(tmp_path / "tpl")
    open(cpp, "w").write(prog)
    subprocess.run([gxx, "-std=c++17", "-O0", cpp, "-o", exe], check=True, timeout=120)
    out = subprocess.run([exe], capture_output=True, text=True, check=True, timeout=60).stdout.split("\n")
    rows = [tuple(map(int, line.split())) for line in out if line.strip()]
    assert len(rows) == 32
    for t, hb, want in rows:
        assert bench.tests_per_lane(hb, t) == want, (t, hb)


def test_row_flops_hand_counts():
    # hb = 1: forming the row of H is 8 + 5 = 13; a test on a 1-wide window has no off-diagonal
    # update (4 hb (hb - 1) = 0), 6 pivot-column/diagonal operations and 10 for the shift and
    # the refined reciprocal: 16 per test
    assert bench.row_flops(1, 1) == 13 + 16
    assert bench.row_flops(1, 3) == 13 + 3 * 16
    # hb = 8 (kl + ku = 8, the widest band the bisection takes): 69 + t (224 + 48 + 10)
    assert bench.row_flops(8, 1) == 69 + 282
    assert bench.row_flops(8, 2) == 69 + 2 * 282


def test_bisection_flops_counts_only_bisected_shifts():
    n, hb = 1000, 2
    # bits 8..31 hold the passes of a bisected shift (PS_PT_BISECT = 8); a Golub-Kahan shift's
    # high bits may hold an underflow exponent (PS_PT_UNDERFLOW = 4) and must not count
    info = np.array([8 | (30 << 8), 8 | 2 | (128 << 8), 4 | (1000 << 8), 0, 8 | (1 << 8)], dtype=np.int32)
    per_row = bench.row_flops(hb, 1 * bench.tests_per_lane(hb, 0))
    assert bench.bisection_flops(n, hb, info) == (30 + 128 + 1) * n * per_row
    # two lanes per shift, three tests each (hb = 2, default mode): a pass forms the row once
    per_row2 = bench.row_flops(hb, 2 * 3)
    assert bench.bisection_flops(n, hb, info, lanes=2) == (30 + 128 + 1) * n * per_row2
    assert bench.bisection_flops(n, hb, np.zeros(4, dtype=np.int32)) == 0.0


def test_algorithmic_bytes():
    n, kl, ku = 100, 1, 2
    wl, wu = kl, kl + ku + 1
    lu = (wl + wu) * 16 * n + n
    step = (2 * (wl + wu) + 10) * 16 * n + 2 * n
    band = (kl + ku + 1) * 16 * n
    iters = np.array([3, 0, 7])
    info = np.array([0, 8 | (20 << 8), 2])
    # the band once; each Golub-Kahan shift its LU and steps; every shift 16 bytes of result
    want = band + (lu + 3 * step) + (lu + 7 * step) + 3 * 16
    assert bench.algorithmic_bytes(n, kl, ku, iters, info) == want
    # without info every shift is taken as Golub-Kahan
    assert bench.algorithmic_bytes(n, kl, ku, iters) == band + 3 * lu + 10 * step + 3 * 16


def _write_pmc(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for d, k, v in rows:
            w.writerow([d, k, counter, v])
            w.writerow([d, k, "OTHER_COUNTER", 1e9])     # other counters are ignored


def test_counter_summary_scales_by_the_calibration_copy(tmp_path, monkeypatch):
    """FETCH_SIZE / WRITE_SIZE (KiB) of the library kernels after the calibration copy, each scaled
    so that the copy reads exactly its known size."""
    calib_kib = bench.CALIB_BYTES / 1024.0
    fetch = [(1, "ps::k_sort_lists(...)", 50.0),                        # before the copy: ignored
             (2, "__amd_rocclr_copyBuffer", 10.0),                      # a small copy: not the calibration
             (3, "__amd_rocclr_copyBuffer", calib_kib * 1.25),
             (4, "void ps::bis::k_bis<2, 2, 1, 1>(ps::BisArgs)", 400.0),
             (5, "void ps::bis::k_bis<2, 2, 1, 1>(ps::BisArgs)", 100.0),
             (6, "void ps::k_sort_lists(long*, long)", 20.0),
             (7, "void ps::k_eval<1, 1, false, false>(ps::EvalArgs)", 980.0),
             (8, "elementwise_kernel<float>", 7777.0)]                   # not the library's
    write = [(3, "__amd_rocclr_copyBuffer", calib_kib * 0.8),
             (4, "void ps::bis::k_bis<2, 2, 1, 1>(ps::BisArgs)", 8.0),
             (7, "void ps::k_eval<1, 1, false, false>(ps::EvalArgs)", 32.0)]
    fp, wp = str(tmp_path / "fetch.csv"), str(tmp_path / "write.csv")
    _write_pmc(fp, "FETCH_SIZE", fetch)
    _write_pmc(wp, "WRITE_SIZE", write)
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    bench.summarize_counters(fp, wp)
    import json
    doc = json.load(open(out))
    want_fetch = (400 + 100 + 20 + 980) * 1024.0 / 1.25
    want_write = (8 + 32) * 1024.0 / 0.8
    assert doc["fetch"]["bytes"] == pytest.approx(want_fetch, rel=1e-12)
    assert doc["write"]["bytes"] == pytest.approx(want_write, rel=1e-12)
    assert doc["traffic_bytes_per_launch"] == pytest.approx(want_fetch + want_write, rel=1e-12)
    assert doc["fetch"]["per_kernel_kib"]["ps::bis::k_bis<2, 2, 1, 1>"] == 500.0
    assert doc["source_hash"] == bench.source_hash()

    # the batch summary keeps only the bisection kernel's launches
    bout = tmp_path / "batch.json"
    monkeypatch.setattr(bench, "BATCH_TRAFFIC_FILE", str(bout))
    bench.summarize_batch_counters(fp, wp, lanes=2, tests=3)
    bdoc = json.load(open(bout))
    assert bdoc["fetch"]["launches"] == 2 and bdoc["write"]["launches"] == 1
    assert bdoc["traffic_bytes_per_launch"] == pytest.approx(500 * 1024.0 / 1.25 + 8 * 1024.0 / 0.8, rel=1e-12)
    assert bdoc["plan"] == {"lanes": 2, "tests_mode": 3}
    # a stored summary is used only for the plan and the sources it was taken with
    assert bench.batch_stored_traffic(2, 3) == bdoc["traffic_bytes_per_launch"]
    assert bench.batch_stored_traffic(1, 2) is None
