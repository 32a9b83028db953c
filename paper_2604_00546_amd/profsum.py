"""Summaries of rocprofv3 CSV output for one benchmark run.

bench.py --calib-copy-mib M issues one device-to-device copy of M MiB just
before the timed steps; every dispatch after that copy belongs to the timed
region.  This script restricts the trace (or the counter collection) to
those dispatches and prints per-kernel figures per step.

usage:
  python -m paper_2604_00546_amd.profsum trace <run_kernel_trace.csv> [--steps S] --calib-mib M
  python -m paper_2604_00546_amd.profsum counters <fetch.csv> <write.csv> --calib-mib M
  python -m paper_2604_00546_amd.profsum sq <sq_counter_collection.csv>
  python -m paper_2604_00546_amd.profsum ntt <run_kernel_trace.csv> --calib-mib M
"""
import argparse
import collections
import csv


def _short(name: str) -> str:
    n = name.replace("(anonymous namespace)::", "").replace("void ", "")
    return n.split("(")[0]


def _calib_index(rows):
    """Index of the calibration copy in a time-ordered kernel trace: the
    first device copy that takes at least half as long as the longest one.
    (Copies to pinned host memory later in the run, such as the result
    downloads of the service-time steps, are copy kernels of similar
    duration; the calibration copy comes before all of them.)"""
    dur = lambda r: int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    cand = [i for i, r in enumerate(rows) if _short(r["Kernel_Name"]) == "__amd_rocclr_copyBuffer"]
    if not cand:
        raise SystemExit("calibration copy not found in the trace")
    longest = max(dur(rows[i]) for i in cand)
    return next(i for i in cand if 2 * dur(rows[i]) >= longest)


def trace(path, steps, calib_mib):
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    dur = lambda r: int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    timed = rows[_calib_index(rows) + 1:]
    if steps <= 0:
        # one k_automorph_sum per hoisted product: the number of queries in the region
        steps = sum(1 for r in timed if _short(r["Kernel_Name"]) == "k_automorph_sum")
    agg = collections.defaultdict(lambda: [0, 0])
    for r in timed:
        a = agg[_short(r["Kernel_Name"])]
        a[0] += 1
        a[1] += dur(r)
    total = sum(v[1] for v in agg.values())
    span = int(timed[-1]["End_Timestamp"]) - int(timed[0]["Start_Timestamp"])
    print(f"timed region: {len(timed)} dispatches over {steps} step(s); kernel time {total / 1e6 / steps:.3f} ms/step; "
          f"wall span {span / 1e6 / steps:.3f} ms/step")
    print(f"{'kernel':40s} {'calls/step':>10s} {'ms/step':>9s} {'avg us':>8s} {'share':>6s}")
    for k, (n, t) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        print(f"{k[:40]:40s} {n / steps:10.1f} {t / 1e6 / steps:9.3f} {t / n / 1e3:8.2f} {100 * t / total:5.1f}%")


def ntt_sizes(path, calib_mib, n_coeff=65536):
    """NTT passes of the timed region by launch size: limb polynomials per
    launch (grid y x z for every pass at N = 2^16), mean duration and the
    pass's algorithmic HBM rate (16 B per coefficient: one read, one write)."""
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    dur = lambda r: int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    agg = collections.defaultdict(lambda: [0, 0])
    for r in rows[_calib_index(rows) + 1:]:
        k = _short(r["Kernel_Name"])
        if not k.startswith(("k_fwd_", "k_inv_")):
            continue
        lp = int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
        a = agg[(k, lp)]
        a[0] += 1
        a[1] += dur(r)
    print(f"{'pass':28s} {'limb polys':>10s} {'launches':>8s} {'mean us':>8s} {'GB/s':>7s} {'total ms':>9s}")
    for (k, lp), (n, t) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        us = t / n / 1e3
        print(f"{k[:28]:28s} {lp:10d} {n:8d} {us:8.2f} {lp * n_coeff * 16 / (us * 1e3):7.0f} {t / 1e6:9.3f}")


def counters(fpath, wpath, calib_mib):
    def load(path, ctr):
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == ctr]
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        return rows
    f, w = load(fpath, "FETCH_SIZE"), load(wpath, "WRITE_SIZE")
    ref_kib = calib_mib * 1024.0
    # calibration: the largest copy's counters against its known size
    def is_copy(r):
        return _short(r["Kernel_Name"]) == "__amd_rocclr_copyBuffer"
    fc = max((r for r in f if is_copy(r)), key=lambda r: float(r["Counter_Value"]))
    wc = max((r for r in w if is_copy(r)), key=lambda r: float(r["Counter_Value"]))
    kf, kw = ref_kib / float(fc["Counter_Value"]), ref_kib / float(wc["Counter_Value"])
    print(f"calibration copy of {calib_mib} MiB: FETCH_SIZE {float(fc['Counter_Value']):.1f} KiB -> factor {kf:.4f}; "
          f"WRITE_SIZE {float(wc['Counter_Value']):.1f} KiB -> factor {kw:.4f}")
    fi = [r for r in f if int(r["Dispatch_Id"]) > int(fc["Dispatch_Id"])]
    wi = {r["Dispatch_Id"]: float(r["Counter_Value"]) for r in w}
    agg = collections.defaultdict(lambda: [0, 0.0, 0.0])
    for r in fi:
        a = agg[_short(r["Kernel_Name"])]
        a[0] += 1
        a[1] += float(r["Counter_Value"]) * kf
        a[2] += wi.get(r["Dispatch_Id"], 0.0) * kw
    print(f"{'kernel':40s} {'dispatches':>10s} {'read MiB/disp':>14s} {'write MiB/disp':>15s}")
    for k, (n, rd, wr) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        print(f"{k[:40]:40s} {n:10d} {rd / n / 1024:14.3f} {wr / n / 1024:15.3f}")
    # one NTT transform = one column kernel plus one row kernel
    ntt = [k for k in agg if k.startswith(("k_fwd_", "k_inv_"))]
    transforms = sum(agg[k][0] for k in ntt if "cols" in k)
    if transforms:
        rd = sum(agg[k][1] for k in ntt) * 1024.0
        wr = sum(agg[k][2] for k in ntt) * 1024.0
        print(f"NTT per transform (both passes): {transforms} transforms, read {rd / transforms / 2**20:.3f} MiB, "
              f"write {wr / transforms / 2**20:.3f} MiB, total {(rd + wr) / transforms:.0f} B")


def sq(path):
    """Per-wave SQ counters of every dispatch in the run, by kernel."""
    per = collections.defaultdict(dict)
    names = {}
    for r in csv.DictReader(open(path)):
        per[r["Dispatch_Id"]][r["Counter_Name"]] = float(r["Counter_Value"])
        names[r["Dispatch_Id"]] = _short(r["Kernel_Name"])
    agg = collections.defaultdict(lambda: collections.Counter())
    disp = collections.Counter()
    for d, cs in per.items():
        agg[names[d]].update(cs)
        disp[names[d]] += 1
    cols = [("VALU/wave", "SQ_INSTS_VALU"), ("SALU/wave", "SQ_INSTS_SALU"), ("LDS/wave", "SQ_INSTS_LDS"),
            ("wave_cyc/wave", "SQ_WAVE_CYCLES"), ("wait_any/wave", "SQ_WAIT_INST_ANY")]
    print(f"{'kernel':28s} {'disp':>5s} " + " ".join(f"{h:>{max(9, len(h))}s}" for h, _ in cols))
    for k, a in sorted(agg.items(), key=lambda kv: -kv[1]["SQ_WAVE_CYCLES"]):
        w = max(a["SQ_WAVES"], 1.0)
        print(f"{k[:28]:28s} {disp[k]:5d} " + " ".join(f"{a[c] / w:{max(9, len(h))}.0f}" for h, c in cols))
    same = all(abs(a["SQ_ACTIVE_INST_VALU"] - a["SQ_INSTS_VALU"]) <= 0.01 * a["SQ_INSTS_VALU"] for a in agg.values())
    print(f"SQ_ACTIVE_INST_VALU within 1% of SQ_INSTS_VALU for every kernel: {same}")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("path")
    t.add_argument("--steps", type=int, default=0,
                   help="queries in the timed region (default: counted, one k_automorph_sum per hoisted product)")
    t.add_argument("--calib-mib", type=int, required=True)
    c = sub.add_parser("counters")
    c.add_argument("fetch")
    c.add_argument("write")
    c.add_argument("--calib-mib", type=int, required=True)
    q = sub.add_parser("sq")
    q.add_argument("path")
    n = sub.add_parser("ntt")
    n.add_argument("path")
    n.add_argument("--calib-mib", type=int, required=True)
    a = ap.parse_args()
    if a.cmd == "trace":
        trace(a.path, a.steps, a.calib_mib)
    elif a.cmd == "ntt":
        ntt_sizes(a.path, a.calib_mib)
    elif a.cmd == "counters":
        counters(a.fetch, a.write, a.calib_mib)
    else:
        sq(a.path)


if __name__ == "__main__":
    main()
