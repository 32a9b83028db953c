"""Host tests of the measurement tools.  The rocprofv3 summaries
(paper_2604_00546_amd.profsum) on small synthetic CSV files: the timed
region starts after the calibration copy (the first device copy at least
half as long as the longest one, so the result downloads of later
service-time steps, also copy kernels, do not move it), the queries in the
region are counted, and the byte counters are scaled by what they read for
the calibration copy.  And bench.py's refusal of more than one GPU."""
import contextlib
import csv
import io

import pytest

from paper_2604_00546_amd import profsum

TRACE_COLS = ["Kernel_Name", "Start_Timestamp", "End_Timestamp", "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z"]


def _write(path, cols, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=cols)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def _trace_rows(steps_before, steps_after, with_downloads):
    """A warmup query, the calibration copy (100 us), the timed queries and,
    optionally, a longer copy after them (a 130 us result download)."""
    rows, t = [], 0

    def k(name, us, gy=1, gz=1):
        nonlocal t
        rows.append({"Kernel_Name": name, "Start_Timestamp": t, "End_Timestamp": t + us * 1000,
                     "Grid_Size_X": 65536, "Grid_Size_Y": gy, "Grid_Size_Z": gz})
        t += us * 1000 + 500

    def query():
        k("void (anonymous namespace)::k_automorph_sum(unsigned long*)", 9, 20, 1)
        k("void (anonymous namespace)::k_fwd_cols2<4>(NttLaunch)", 40, 14, 32)
        k("void (anonymous namespace)::k_fwd_rows2<4, true>(NttLaunch)", 60, 32, 14)
        k("void (anonymous namespace)::k_inv_cols4(NttLaunch)", 10, 1, 2)

    k("__amd_rocclr_copyBuffer", 5)
    for _ in range(steps_before):
        query()
    k("__amd_rocclr_copyBuffer", 100)  # calibration
    for i in range(steps_after):
        query()
        if with_downloads and i == 0:
            k("__amd_rocclr_copyBuffer", 130)  # a result download, longer than the calibration copy
    return rows


def _run(fn, *args):
    out = io.StringIO()
    with contextlib.redirect_stdout(out):
        fn(*args)
    return out.getvalue()


@pytest.mark.parametrize("with_downloads", [False, True])
def test_trace_region_starts_after_the_calibration_copy(tmp_path, with_downloads):
    p = tmp_path / "trace.csv"
    _write(p, TRACE_COLS, _trace_rows(steps_before=2, steps_after=5, with_downloads=with_downloads))
    text = _run(profsum.trace, str(p), 0, 256)
    head = text.splitlines()[0]
    assert "over 5 step(s)" in head  # the queries counted after the calibration copy
    line = next(l for l in text.splitlines() if l.startswith("k_fwd_rows2<4, true>"))
    calls, ms, avg = (float(x) for x in line.split()[-4:-1])
    assert (calls, ms, avg) == (1.0, 0.06, 60.0)
    copies = [l for l in text.splitlines() if l.startswith("__amd_rocclr_copyBuffer")]
    assert bool(copies) == with_downloads  # the download is inside the region, the calibration copy is not


def test_ntt_sizes_group_by_launch_size(tmp_path):
    p = tmp_path / "trace.csv"
    _write(p, TRACE_COLS, _trace_rows(steps_before=1, steps_after=3, with_downloads=False))
    text = _run(profsum.ntt_sizes, str(p), 256)
    rows = {tuple(l.split()[:-5]): l.split()[-5:] for l in text.splitlines()[1:]}
    lp, n, mean = rows[("k_fwd_cols2<4>",)][:3]
    assert (int(lp), int(n), float(mean)) == (448, 3, 40.0)
    lp, n, mean = rows[("k_inv_cols4",)][:3]
    assert (int(lp), int(n), float(mean)) == (2, 3, 10.0)


def test_counters_scaled_by_the_calibration_copy(tmp_path):
    cols = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    # the counter reads half the calibration copy's 256 MiB (FETCH) and all of it (WRITE)
    fetch = [
        {"Dispatch_Id": 1, "Kernel_Name": "k_mac", "Counter_Name": "FETCH_SIZE", "Counter_Value": 999},
        {"Dispatch_Id": 2, "Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": "FETCH_SIZE",
         "Counter_Value": 128 * 1024},
        {"Dispatch_Id": 3, "Kernel_Name": "k_mac", "Counter_Name": "FETCH_SIZE", "Counter_Value": 1024},
        {"Dispatch_Id": 4, "Kernel_Name": "k_mac", "Counter_Name": "FETCH_SIZE", "Counter_Value": 3072},
        {"Dispatch_Id": 5, "Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": "FETCH_SIZE",
         "Counter_Value": 10},
    ]
    write = [dict(r, Counter_Name="WRITE_SIZE", Counter_Value=(256 * 1024 if r["Dispatch_Id"] == 2 else 512))
             for r in fetch]
    pf, pw = tmp_path / "f.csv", tmp_path / "w.csv"
    _write(pf, cols, fetch)
    _write(pw, cols, write)
    text = _run(profsum.counters, str(pf), str(pw), 256)
    assert "factor 2.0000" in text and "factor 1.0000" in text
    line = next(l for l in text.splitlines() if l.startswith("k_mac"))
    n, rd, wr = line.split()[1:]
    # dispatches after the calibration copy only: (1024 + 3072) / 2 KiB x 2 = 4 MiB read, 512 KiB written
    assert (int(n), float(rd), float(wr)) == (2, 4.0, 0.5)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: asked for more, it exits with status 2 and
    says so, before touching a device."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=root)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""
