"""Summaries of rocprofv3 output for the solver's kernels.

    python -m paper_2407_16144_amd.rocprof_summary stats DIR
        Markdown table of the kernel-trace statistics (*_kernel_stats.csv
        under DIR): calls, average / min / max duration, share of GPU time.

    python -m paper_2407_16144_amd.rocprof_summary traffic \\
            --fetch CSV --write CSV --copy-kernel NAME --copy-bytes B [--json OUT]
        Per-dispatch HBM traffic from two --pmc runs (FETCH_SIZE, WRITE_SIZE;
        both in KiB per dispatch).  Each counter is scaled by the factor that
        makes it read B bytes for a plain streaming kernel (NAME, a substring
        of its name) that reads B bytes and writes B bytes.  With --json the
        per-kernel figures are stored together with a hash of the kernel
        sources, so that a reader can tell whether the kernels have changed
        since the counters were taken.

Reads only CSV text; needs neither the GPU nor the solver library.
"""
import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import re
import sys

_CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
KERNEL_SOURCES = ("kernels.hip", "kernels.h", "halp_types.h")


def kernel_source_hash():
    """sha256 over the sources the per-step kernels are compiled from."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(_CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read() + b"\0")
    return h.hexdigest()


def short_name(name):
    """'void halp::primal_step<double>(halp::IterArgs<double>, int)' ->
    'primal_step<double>'; other kernels keep their name up to '('."""
    n = name.strip('"')
    n = re.sub(r"^void\s+", "", n)
    n = n.split("(", 1)[0]
    return n.replace("halp::", "")


def read_stats(directory):
    files = sorted(glob.glob(os.path.join(directory, "**", "*kernel_stats.csv"), recursive=True))
    if not files:
        raise SystemExit(f"no *kernel_stats.csv under {directory}")
    rows = []
    for f in files:
        with open(f, newline="") as fh:
            rows += list(csv.DictReader(fh))
    return rows


def stats_table(directory, top=20):
    rows = read_stats(directory)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = ["| kernel | calls | avg us | min us | max us | % GPU time |",
           "|---|---:|---:|---:|---:|---:|"]
    for r in rows[:top]:
        out.append(f"| {short_name(r['Name'])} | {int(r['Calls'])} | {float(r['AverageNs']) / 1e3:.2f} | "
                   f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                   f"{float(r['Percentage']):.2f} |")
    return "\n".join(out)


def counter_means(path, counter):
    """{short kernel name: (dispatches, mean counter value)} for one counter."""
    acc = collections.defaultdict(lambda: [0, 0.0])
    with open(path, newline="") as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] != counter:
                continue
            a = acc[short_name(r["Kernel_Name"])]
            a[0] += 1
            a[1] += float(r["Counter_Value"])
    return {k: (n, v / n) for k, (n, v) in acc.items() if n}


def traffic(fetch_csv, write_csv, copy_kernel, copy_bytes):
    f = counter_means(fetch_csv, "FETCH_SIZE")
    w = counter_means(write_csv, "WRITE_SIZE")
    ck = [k for k in f if copy_kernel in k]
    cw = [k for k in w if copy_kernel in k]
    if len(ck) != 1 or len(cw) != 1:
        raise SystemExit(f"copy kernel '{copy_kernel}' matched {ck} / {cw}")
    sf = copy_bytes / (f[ck[0]][1] * 1024.0)
    sw = copy_bytes / (w[cw[0]][1] * 1024.0)
    kernels = {}
    for k in sorted(set(f) & set(w)):
        fb = f[k][1] * 1024.0 * sf
        wb = w[k][1] * 1024.0 * sw
        kernels[k] = {"dispatches": f[k][0], "fetch_kib": round(f[k][1], 3), "write_kib": round(w[k][1], 3),
                      "fetch_bytes": fb, "write_bytes": wb, "traffic_bytes": fb + wb}
    return {"copy_kernel": ck[0], "copy_bytes": copy_bytes, "scale_fetch": sf, "scale_write": sw,
            "kernels": kernels}


def traffic_table(t, names=None):
    out = [f"copy calibration: {t['copy_kernel']} reads and writes {t['copy_bytes']} B per dispatch; "
           f"FETCH_SIZE scale {t['scale_fetch']:.4f}, WRITE_SIZE scale {t['scale_write']:.4f}", "",
           "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | fetch MB | write MB | traffic MB |",
           "|---|---:|---:|---:|---:|---:|---:|"]
    for k, v in sorted(t["kernels"].items(), key=lambda kv: -kv[1]["traffic_bytes"]):
        if names and not any(n in k for n in names):
            continue
        out.append(f"| {k} | {v['dispatches']} | {v['fetch_kib']:.1f} | {v['write_kib']:.1f} | "
                   f"{v['fetch_bytes'] / 1e6:.2f} | {v['write_bytes'] / 1e6:.2f} | "
                   f"{v['traffic_bytes'] / 1e6:.2f} |")
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("dir")
    a.add_argument("--top", type=int, default=20)
    b = sub.add_parser("traffic")
    b.add_argument("--fetch", required=True)
    b.add_argument("--write", required=True)
    b.add_argument("--copy-kernel", required=True)
    b.add_argument("--copy-bytes", type=float, required=True)
    b.add_argument("--only", nargs="*", default=None, help="kernel name substrings to list")
    b.add_argument("--json", default=None)
    b.add_argument("--workload", default="")
    args = ap.parse_args(argv)
    if args.cmd == "stats":
        print(stats_table(args.dir, args.top))
        return 0
    t = traffic(args.fetch, args.write, args.copy_kernel, args.copy_bytes)
    print(traffic_table(t, args.only))
    if args.json:
        if args.only:
            t["kernels"] = {k: v for k, v in t["kernels"].items() if any(n in k for n in args.only)}
        t["source_sha256"] = kernel_source_hash()
        t["workload"] = args.workload
        with open(args.json, "w") as fh:
            json.dump(t, fh, indent=1, sort_keys=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
