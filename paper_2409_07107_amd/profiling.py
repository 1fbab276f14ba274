"""Reads rocprofv3 CSV output into the figures the benchmark reports.

    python -m paper_2409_07107_amd.profiling stats DIR --kernel SUBSTR --cmd "..." --out FILE.md
        kernel-trace statistics (--kernel-trace --stats) of the kernels whose
        name contains SUBSTR, written as a short text summary with the command.

    python -m paper_2409_07107_amd.profiling traffic --fetch DIR --write DIR \
        --copy-fetch DIR --copy-write DIR --copy-bytes N --kernel SUBSTR \
        --copy-kernel SUBSTR --cmd "..." --out FILE.json
        HBM bytes per dispatch of the kernel from two counter runs (FETCH_SIZE,
        then WRITE_SIZE, KiB per dispatch), each scaled by the reading of the
        same counter for a plain copy of N bytes (which reads and writes N).

The JSON records a digest of the HIP sources, so that a traffic figure stops
being reported once the kernel it was measured on has changed.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def source_digest() -> str:
    """SHA-1 over the HIP sources and the C header."""
    h = hashlib.sha1()
    csrc = os.path.join(ROOT, "paper_2409_07107_amd", "csrc")
    files = sorted(os.path.join(csrc, f) for f in os.listdir(csrc) if f.endswith((".h", ".hip")))
    for f in files + [os.path.join(ROOT, "include", "dsim.h")]:
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()


def _find(d: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits[-1]


def kernel_stats(d: str, substr: str) -> list[dict]:
    rows = []
    with open(_find(d, "kernel_stats.csv")) as fh:
        for r in csv.DictReader(fh):
            if substr in r["Name"]:
                rows.append(r)
    return rows


def counter_per_dispatch(d: str, counter: str, substr: str, first: int = 0) -> tuple[float, int]:
    """Mean over matching dispatches (the first `first` of them when > 0) of
    the counter summed over its instances (one row per dispatch and counter
    in rocprofv3's CSV)."""
    per = {}
    with open(_find(d, "counter_collection.csv")) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] != counter or substr not in r["Kernel_Name"]:
                continue
            key = r["Dispatch_Id"]
            per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    if not per:
        raise ValueError(f"no {counter} rows for kernels matching {substr!r} in {d}")
    if first > 0:
        keep = sorted(per, key=int)[:first]
        per = {k: per[k] for k in keep}
    return sum(per.values()) / len(per), len(per)


def cmd_stats(a):
    rows = kernel_stats(a.dir, a.kernel)
    lines = [f"# rocprofv3 kernel statistics: {a.title}", "", "Command:", "", "```", a.cmd, "```", "",
             "| kernel | calls | average ms | min ms | max ms | share % |", "|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.3f} | "
                     f"{float(r['MinNs']) / 1e6:.3f} | {float(r['MaxNs']) / 1e6:.3f} | {float(r['Percentage']):.1f} |")
    if a.note:
        lines += ["", a.note]
    with open(a.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def cmd_traffic(a):
    kib = 1024.0
    f_k, n_f = counter_per_dispatch(a.fetch, "FETCH_SIZE", a.kernel, a.first)
    w_k, n_w = counter_per_dispatch(a.write, "WRITE_SIZE", a.kernel, a.first)
    cf_k, _ = counter_per_dispatch(a.copy_fetch, "FETCH_SIZE", a.copy_kernel)
    cw_k, _ = counter_per_dispatch(a.copy_write, "WRITE_SIZE", a.copy_kernel)
    ff = a.copy_bytes / (cf_k * kib)
    wf = a.copy_bytes / (cw_k * kib)
    fetch = f_k * kib * ff
    write = w_k * kib * wf
    out = dict(kernel=a.kernel, source_sha1=source_digest(), command=a.cmd, dispatches_used=a.first or "all",
               fetch_kib_per_dispatch=f_k, write_kib_per_dispatch=w_k, dispatches=[n_f, n_w],
               copy_bytes=a.copy_bytes, copy_fetch_kib=cf_k, copy_write_kib=cw_k,
               fetch_scale=ff, write_scale=wf, fetch_bytes=fetch, write_bytes=write,
               bytes_per_launch=fetch + write)
    with open(a.out, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(json.dumps(out, indent=1))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--kernel", default="")
    s.add_argument("--title", default="")
    s.add_argument("--cmd", required=True)
    s.add_argument("--note", default="")
    s.add_argument("--out", required=True)
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write"):
        t.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--copy-kernel", required=True)
    t.add_argument("--first", type=int, default=0, help="use only the first N matching dispatches")
    t.add_argument("--cmd", required=True)
    t.add_argument("--out", required=True)
    a = ap.parse_args()
    {"stats": cmd_stats, "traffic": cmd_traffic}[a.what](a)


if __name__ == "__main__":
    main()
