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

    python -m paper_2409_07107_amd.profiling dispatches DIR --kernel SUBSTR \
        [--alternate LABEL,LABEL] --cmd "..." --out FILE.md
        per-dispatch durations (--kernel-trace) of the matching kernels; with
        --alternate, a kernel's successive dispatches are dealt to the labels
        in turn (the step kernel's first and fallback passes alternate).

    python -m paper_2409_07107_amd.profiling counters DIR [DIR ...] --kernel SUBSTR \
        [--alternate LABEL,LABEL] --cmd "..." --out FILE.md
        SQ/GRBM counters per dispatch (--pmc runs), averaged per kernel (and
        label), with the derived ratios named in the output.

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


def counter_per_dispatch(d: str, counter: str, substr: str, first: int = 0, stride: int = 1,
                         offset: int = 0) -> tuple[float, int]:
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
    order = sorted(per, key=int)[offset::stride]
    if first > 0:
        order = order[:first]
    per = {k: per[k] for k in order}
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
    f_k, n_f = counter_per_dispatch(a.fetch, "FETCH_SIZE", a.kernel, a.first, a.stride, a.offset)
    w_k, n_w = counter_per_dispatch(a.write, "WRITE_SIZE", a.kernel, a.first, a.stride, a.offset)
    cf_k, _ = counter_per_dispatch(a.copy_fetch, "FETCH_SIZE", a.copy_kernel)
    cw_k, _ = counter_per_dispatch(a.copy_write, "WRITE_SIZE", a.copy_kernel)
    ff = a.copy_bytes / (cf_k * kib)
    wf = a.copy_bytes / (cw_k * kib)
    fetch = f_k * kib * ff
    write = w_k * kib * wf
    out = dict(kernel=a.kernel, source_sha1=source_digest(), command=a.cmd, dispatches_used=a.first or "all",
               dispatch_stride=a.stride, dispatch_offset=a.offset,
               fetch_kib_per_dispatch=f_k, write_kib_per_dispatch=w_k, dispatches=[n_f, n_w],
               copy_bytes=a.copy_bytes, copy_fetch_kib=cf_k, copy_write_kib=cw_k,
               fetch_scale=ff, write_scale=wf, fetch_bytes=fetch, write_bytes=write,
               bytes_per_launch=fetch + write)
    with open(a.out, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(json.dumps(out, indent=1))


def _label(name: str, alternate, seen: dict) -> str:
    """The label of this kernel's next dispatch: `alternate` is a list of
    labels dealt in turn, or (labels, n, rest): the first n dispatches dealt
    the labels in turn, every later one `rest`."""
    i = seen.get(name, 0)
    seen[name] = i + 1
    if not alternate:
        return ""
    if isinstance(alternate, tuple):
        labels, n, rest = alternate
        return labels[i % len(labels)] if i < n else rest
    return alternate[i % len(alternate)]


def _labels_for(name: str, a):
    """The labels dealt to this kernel's dispatches: from --alternate-spec
    ("SUBSTR=LABEL,LABEL;..." or "SUBSTR=LABEL,LABEL@N,REST": the first N
    dispatches in turn, then REST), else --alternate with --alternate-kernel."""
    for part in filter(None, (getattr(a, "alternate_spec", "") or "").split(";")):
        key, labels = part.split("=", 1)
        if key in name:
            if "@" in labels:
                cyc, tail = labels.split("@", 1)
                n, rest = tail.split(",", 1)
                return (cyc.split(","), int(n), rest)
            return labels.split(",")
    if a.alternate and a.alternate_kernel and a.alternate_kernel in name:
        return a.alternate.split(",")
    return None


def cmd_dispatches(a):
    alt = a.alternate.split(",") if a.alternate else None
    groups, seen = {}, {}
    with open(_find(a.dir, "kernel_trace.csv")) as fh:
        rows = sorted(csv.DictReader(fh), key=lambda r: int(r["Dispatch_Id"]))
    for r in rows:
        if a.kernel not in r["Kernel_Name"]:
            continue
        name = r["Kernel_Name"]
        lab = _label(name, _labels_for(name, a), seen)
        ms = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
        groups.setdefault((name, lab), []).append(ms)
    lines = [f"# rocprofv3 dispatch durations: {a.title}", "", "Command:", "", "```", a.cmd, "```", "",
             "| kernel | pass | dispatches | average ms | min ms | max ms |", "|---|---|---|---|---|---|"]
    for (name, lab), d in groups.items():
        lines.append(f"| `{name[:80]}` | {lab or '-'} | {len(d)} | {sum(d) / len(d):.3f} | {min(d):.3f} | "
                     f"{max(d):.3f} |")
    if a.note:
        lines += ["", a.note]
    with open(a.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


SIMDS = 256 * 4  # gfx950: 256 compute units x 4 SIMDs


def cmd_counters(a):
    alt = a.alternate.split(",") if a.alternate else None
    per = {}  # (kernel, label) -> {dispatch: {counter: value}}
    for d in a.dirs:
        seen, lab_of = {}, {}
        with open(_find(d, "counter_collection.csv")) as fh:
            rows = sorted(csv.DictReader(fh), key=lambda r: int(r["Dispatch_Id"]))
        for r in rows:
            name = r["Kernel_Name"]
            if a.kernel not in name:
                continue
            key = (d, r["Dispatch_Id"])
            if key not in lab_of:
                lab_of[key] = _label(name, _labels_for(name, a), seen)
            slot = per.setdefault((name, lab_of[key]), {}).setdefault(key, {})
            c, x = r["Counter_Name"], float(r["Counter_Value"])
            # SQ counters add over their instances; the GRBM clock is one per
            # XCD, each the length of the dispatch, so its largest is taken
            slot[c] = max(slot.get(c, 0.0), x) if c.startswith("GRBM_") else slot.get(c, 0.0) + x
    lines = [f"# rocprofv3 counters per dispatch: {a.title}", "", "Commands:", "", "```", a.cmd, "```", ""]
    for (name, lab), disp in per.items():
        names = sorted({c for v in disp.values() for c in v})
        mean = {c: sum(v.get(c, 0.0) for v in disp.values()) / max(1, sum(c in v for v in disp.values()))
                for c in names}
        lines += [f"## `{name[:80]}` {('(' + lab + ')') if lab else ''}", "",
                  f"{len(disp)} dispatches (counters averaged over the dispatches that carry them)", "",
                  "| counter | per dispatch |", "|---|---|"]
        lines += [f"| {c} | {mean[c]:.4g} |" for c in names]
        der = []
        if "SQ_INSTS_VALU" in mean and mean.get("SQ_WAVES"):
            der.append(("VALU instructions per wave (SQ_INSTS_VALU / SQ_WAVES)", mean["SQ_INSTS_VALU"] / mean["SQ_WAVES"]))
        if "SQ_INSTS_LDS" in mean and mean.get("SQ_WAVES"):
            der.append(("LDS instructions per wave (SQ_INSTS_LDS / SQ_WAVES)", mean["SQ_INSTS_LDS"] / mean["SQ_WAVES"]))
        if mean.get("SQ_ACTIVE_INST_VALU") and "SQ_THREAD_CYCLES_VALU" in mean:
            der.append(("VALU utilization, active lanes of 64 (SQ_THREAD_CYCLES_VALU / (64 SQ_ACTIVE_INST_VALU))",
                        mean["SQ_THREAD_CYCLES_VALU"] / (64.0 * mean["SQ_ACTIVE_INST_VALU"])))
        if a.ms and "SQ_INSTS_VALU" in mean:
            ms = next((v for k, v in (x.split("=") for x in a.ms.split(";"))
                       if (lab and k == lab) or (not lab and k in name)), None)
            if ms:
                der.append((f"VALU issue share: 4 cycles per wave64 VALU instruction over {SIMDS} SIMDs for the "
                            f"launch's {float(ms):.3f} ms at 2.4 GHz (4 SQ_INSTS_VALU / (SIMDs cycles))",
                            4.0 * mean["SQ_INSTS_VALU"] / (SIMDS * float(ms) * 1e-3 * 2.4e9)))
        if mean.get("SQ_ACTIVE_INST_LDS") and "SQ_LDS_BANK_CONFLICT" in mean:
            der.append(("LDS bank-conflict cycles per LDS instruction cycle (SQ_LDS_BANK_CONFLICT / "
                        "SQ_ACTIVE_INST_LDS)", mean["SQ_LDS_BANK_CONFLICT"] / mean["SQ_ACTIVE_INST_LDS"]))
        if der:
            lines += ["", "| derived | value |", "|---|---|"] + [f"| {k} | {v:.4g} |" for k, v in der]
        lines.append("")
    if a.note:
        lines += [a.note]
    with open(a.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


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
    t.add_argument("--stride", type=int, default=1, help="use every STRIDE-th matching dispatch ...")
    t.add_argument("--offset", type=int, default=0, help="... starting at this one")
    t.add_argument("--cmd", required=True)
    t.add_argument("--out", required=True)
    for name in ("dispatches", "counters"):
        c = sub.add_parser(name)
        if name == "dispatches":
            c.add_argument("dir")
        else:
            c.add_argument("dirs", nargs="+")
        c.add_argument("--kernel", default="")
        c.add_argument("--alternate", default="", help="labels dealt in turn to a kernel's dispatches")
        c.add_argument("--alternate-kernel", default="", help="the kernel (substring) whose dispatches alternate")
        c.add_argument("--alternate-spec", default="", help="SUBSTR=LABEL,LABEL;... per kernel")
        c.add_argument("--title", default="")
        c.add_argument("--cmd", required=True)
        c.add_argument("--note", default="")
        c.add_argument("--out", required=True)
        if name == "counters":
            c.add_argument("--ms", default="", help="KEY=ms;... launch durations (from the kernel trace); KEY is a label or a kernel-name substring")
    a = ap.parse_args()
    {"stats": cmd_stats, "traffic": cmd_traffic, "dispatches": cmd_dispatches, "counters": cmd_counters}[a.what](a)


if __name__ == "__main__":
    main()
