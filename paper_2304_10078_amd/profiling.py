"""Summaries of rocprofv3 output for the measurement of the semisort kernels.

Three sub-commands turn the profiler's CSV files into the small text files
kept with the project:

  kstats  <kernel_stats.csv> <out.md> --command "<command that produced it>"
      per-kernel call count and durations (``rocprofv3 --kernel-trace
      --stats --output-format csv``);
  pmc     <counter_collection.csv> <out.json>
      per-dispatch values of one counter (``rocprofv3 --pmc FETCH_SIZE`` or
      ``WRITE_SIZE``) for the engine's kernels and for the copy dispatches;
      the copies after the engine's last kernel are the calibration copy of
      known size that bench.py --calib-copy makes;
  traffic <fetch.json> <write.json> <out.json> --calib-bytes B --workload W --n N
      HBM bytes per distribution launch: each counter (KiB per dispatch) is
      scaled by known_bytes / counter_bytes of the calibration copy;
  passes  <fetch.json> <write.json> <out.json> --calib-bytes B --workload W --op O --n N --calls C
      HBM bytes per call of every pass (sampling, counting, prefix,
      distribution, planning, base cases, compaction, key fills), scaled the
      same way.

Nothing here runs on the GPU.
"""
import argparse
import csv
import hashlib
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCES = ("paper_2304_10078_amd/csrc/ss_device.h", "paper_2304_10078_amd/csrc/engine.hip")


def source_digest():
    """Digest of the kernel sources, stored with counter results so that stale
    numbers are recognised once the kernels change."""
    h = hashlib.sha256()
    for rel in SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def short_name(name):
    s = re.sub(r"\(.*$", "", name.strip())
    s = s.replace("void ", "").replace("ssd::", "")
    s = s.replace("unsigned long", "u64").replace("unsigned int", "u32")
    return s[:90]


def _col(header, *want):
    for w in want:
        for i, h in enumerate(header):
            if h.strip().lower() == w.lower():
                return i
    raise KeyError(f"none of {want} in {header}")


def kstats(path, out, cmd, top=10):
    with open(path, newline="") as f:
        r = csv.reader(f)
        hdr = next(r)
        rows = list(r)
    ni, ci, ti, ai = (_col(hdr, "Name"), _col(hdr, "Calls"), _col(hdr, "TotalDurationNs"), _col(hdr, "AverageNs"))
    mi, xi, pi = _col(hdr, "MinNs"), _col(hdr, "MaxNs"), _col(hdr, "Percentage")
    rows.sort(key=lambda x: -float(x[ti]))
    # every kernel of the engine, then the largest others (the input's
    # generation and statistics, outside the timed region)
    ours = [x for x in rows if short_name(x[ni]).startswith("k_")]
    others = [x for x in rows if not short_name(x[ni]).startswith("k_")]
    lines = ["# rocprofv3 kernel statistics", "", "Command:", "", "```", cmd, "```", ""]
    head = ["| kernel | calls | total ms | avg ms | min ms | max ms | % |", "|---|---|---|---|---|---|---|"]

    def row(x):
        return (f"| `{short_name(x[ni])}` | {int(x[ci])} | {float(x[ti]) / 1e6:.3f} | {float(x[ai]) / 1e6:.4f} "
                f"| {float(x[mi]) / 1e6:.4f} | {float(x[xi]) / 1e6:.4f} | {float(x[pi]):.2f} |")
    lines += ["Engine kernels:", ""] + head + [row(x) for x in ours]
    lines += ["", f"Largest other kernels (of {len(others)}):", ""] + head + [row(x) for x in others[:top]]
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def pmc(path, out):
    with open(path, newline="") as f:
        r = csv.reader(f)
        hdr = next(r)
        rows = list(r)
    ki = _col(hdr, "Kernel_Name", "Kernel-Name", "Name")
    cn = _col(hdr, "Counter_Name", "Counter-Name")
    cv = _col(hdr, "Counter_Value", "Counter-Value")
    di = _col(hdr, "Dispatch_Id", "Dispatch-Id", "Dispatch_ID")
    agg = {}
    counter = None
    for x in rows:
        counter = x[cn]
        key = (int(x[di]), x[ki])
        agg[key] = agg.get(key, 0.0) + float(x[cv])  # summed over dimensions (e.g. XCC)
    res = {"counter": counter, "unit": "KiB per dispatch", "kernels": {}, "copies": []}
    for (d, name), v in sorted(agg.items()):
        s = short_name(name)
        if s.startswith("k_"):
            res["kernels"].setdefault(s, []).append([d, v])
        elif "copybuffer" in name.lower():
            res["copies"].append([d, v])
    with open(out, "w") as f:
        json.dump(res, f, indent=1)


def traffic(fetch, write, out, calib_bytes, workload, n, kernel_prefix="k_distribute", commands=None):
    F = json.load(open(fetch))
    W = json.load(open(write))

    def per_launch(d):
        vals = []
        for name, lst in d["kernels"].items():
            if name.startswith(kernel_prefix):
                vals += [v for _, v in lst]
        return vals

    def calib(d):
        # the calibration copy is the last GPU work of the run: every copy
        # dispatch after the engine's last kernel belongs to it
        last = max(x for lst in d["kernels"].values() for x, _ in lst)
        return sum(v for x, v in d["copies"] if x > last) * 1024.0

    fv, wv = per_launch(F), per_launch(W)
    f_scale = calib_bytes / calib(F)
    w_scale = calib_bytes / calib(W)
    fb = sum(fv) / len(fv) * 1024.0 * f_scale
    wb = sum(wv) / len(wv) * 1024.0 * w_scale
    res = {"workload": workload, "n": n, "kernel": kernel_prefix, "source_digest": source_digest(),
           "launches": len(fv), "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
           "bytes_per_launch": fb + wb, "calib_copy_bytes": calib_bytes,
           "fetch_scale": f_scale, "write_scale": w_scale, "commands": commands or []}
    with open(out, "w") as f:
        json.dump(res, f, indent=1)
    return res


# pass of each engine kernel (the passes of ss_profile_read)
PASS_OF = (("k_sample", "sample"), ("k_count", "count"), ("k_scan", "scan"), ("k_distribute", "distribute"),
           ("k_plan", "plan"), ("k_seg_prefix", "plan"), ("k_heavy_results", "plan"), ("k_base", "finish"),
           ("k_copy", "finish"), ("k_sum_job", "finish"), ("k_flag", "compact"), ("k_fill", "fill"),
           ("k_sfold", "fold"), ("k_iota", "fold"), ("k_gather_at", "fold"), ("k_pack", "pack"),
           ("k_inst", "pack"))


def pass_of(kernel):
    for prefix, name in PASS_OF:
        if kernel.startswith(prefix):
            return name
    return "other"


def passes(fetch, write, out, calib_bytes, workload, op, n, calls, commands=None):
    """HBM bytes per call of every pass: each counter (KiB per dispatch) is
    scaled by the calibration copy, summed over the pass's kernels and divided
    by the number of calls in the profiled run."""
    F = json.load(open(fetch))
    W = json.load(open(write))

    def calib(d):
        last = max(x for lst in d["kernels"].values() for x, _ in lst)
        return sum(v for x, v in d["copies"] if x > last) * 1024.0

    res = {"workload": workload, "op": op, "n": n, "source_digest": source_digest(), "calls": calls,
           "calib_copy_bytes": calib_bytes, "passes": {}, "commands": commands or []}
    for key, d in (("fetch_bytes", F), ("write_bytes", W)):
        scale = calib_bytes / calib(d)
        res[key + "_scale"] = scale
        for name, lst in d["kernels"].items():
            p = res["passes"].setdefault(pass_of(name), {"fetch_bytes": 0.0, "write_bytes": 0.0})
            p[key] += sum(v for _, v in lst) * 1024.0 * scale / calls
    with open(out, "w") as f:
        json.dump(res, f, indent=1)
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="action", required=True)
    a = sub.add_parser("kstats")
    a.add_argument("csv")
    a.add_argument("out")
    a.add_argument("--command", required=True)
    b = sub.add_parser("pmc")
    b.add_argument("csv")
    b.add_argument("out")
    c = sub.add_parser("traffic")
    c.add_argument("fetch")
    c.add_argument("write")
    c.add_argument("out")
    c.add_argument("--calib-bytes", type=float, required=True)
    c.add_argument("--workload", required=True)
    c.add_argument("--n", type=int, required=True)
    c.add_argument("--command", action="append", default=[], help="profiler command of a counter run (repeat)")
    e = sub.add_parser("passes")
    e.add_argument("fetch")
    e.add_argument("write")
    e.add_argument("out")
    e.add_argument("--calib-bytes", type=float, required=True)
    e.add_argument("--workload", required=True)
    e.add_argument("--op", required=True)
    e.add_argument("--n", type=int, required=True)
    e.add_argument("--calls", type=int, required=True)
    e.add_argument("--command", action="append", default=[], help="profiler command of a counter run (repeat)")
    args = ap.parse_args(argv)
    if args.action == "passes":
        print(json.dumps(passes(args.fetch, args.write, args.out, args.calib_bytes, args.workload, args.op, args.n,
                                args.calls, commands=args.command)))
        return
    if args.action == "kstats":
        kstats(args.csv, args.out, args.command)
    elif args.action == "pmc":
        pmc(args.csv, args.out)
    else:
        print(json.dumps(traffic(args.fetch, args.write, args.out, args.calib_bytes, args.workload, args.n,
                                 commands=args.command)))


if __name__ == "__main__":
    main()
