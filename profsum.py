"""Summaries for profiles/ from rocprofv3 output (measurement tooling, not the product path).

    python profsum.py stats  <kernel_stats.csv> <out.md> "<title>" "<command>"
    python profsum.py traffic <fetch_dir> <write_dir> <copy_fetch_dir> <copy_write_dir> <out.md> "<commands>" ["<workload>" "<json path or empty>"]
    python profsum.py counters <out.md> "<title>" "<commands>" <pmc_dir> [<pmc_dir> ...]

`traffic` scales FETCH_SIZE and WRITE_SIZE (KiB per dispatch, from two --pmc runs of the same
command) by what the same counters read for a plain 1 GiB device copy, writes a markdown table
per kernel and profiles/traffic.json keyed by kernel name with the hash of the kernel sources
they were taken on (bench.py reports the dominant kernel's bytes only while that hash holds).
"""
import csv
import glob
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))


def short(name: str) -> str:
    return re.sub(r"\(.*", "", name).replace("void ", "").replace("sps::", "")


def stats(src, out, title, cmd):
    rows = list(csv.DictReader(open(src)))
    lines = [f"# {title}", "", "Command (repository root, one MI355X, ROCm 7.2):", "", "```", cmd, "```",
             "", "| kernel | calls | avg µs | min µs | max µs | share of GPU time |",
             "|---|---|---|---|---|---|"]
    for r in rows[:12]:
        lines.append(f"| `{short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                     f"{float(r['Percentage']):.1f} % |")
    open(out, "w").write("\n".join(lines) + "\n")


def _counter(d):
    f = glob.glob(os.path.join(d, "*counter_collection.csv"))[0]
    vals = {}
    for r in csv.DictReader(open(f)):
        vals.setdefault(short(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
    return vals


def traffic(fd, wd, cfd, cwd, out, cmds, workload="config-2 workload",
            json_out="profiles/traffic.json"):
    sys.path.insert(0, ROOT)
    from bench import kernel_source_hash
    fe, wr, cf, cw = _counter(fd), _counter(wd), _counter(cfd), _counter(cwd)
    kib = (1 << 30) / 1024
    kf = kib / cf["__amd_rocclr_copyBuffer"][0]
    kw = kib / cw["__amd_rocclr_copyBuffer"][0]
    h = kernel_source_hash()
    table, js = [], {}
    for k in sorted(fe):
        if not k.startswith("k_"):
            continue
        f = sum(fe[k]) / len(fe[k]) * kf * 1024
        w = sum(wr.get(k, [0.0])) / max(1, len(wr.get(k, []))) * kw * 1024
        js[k] = {"bytes_per_launch": int(f + w), "fetch_bytes": int(f), "write_bytes": int(w),
                    "dispatches": len(fe[k]), "source_hash": h}
        table.append(f"| `{k}` | {len(fe[k])} | {f / 1e6:.2f} | {w / 1e6:.2f} | {(f + w) / 1e6:.2f} |")
    lines = [f"# HBM traffic per launch, {workload} (rocprofv3 PMC)", "",
             "Commands (repository root, one MI355X, ROCm 7.2):", "", "```", cmds, "```", "",
             f"Calibration: a 1 GiB device copy reads {cf['__amd_rocclr_copyBuffer'][0]:.0f} KiB in "
             f"FETCH_SIZE and {cw['__amd_rocclr_copyBuffer'][0]:.0f} KiB in WRITE_SIZE, so FETCH_SIZE "
             f"is scaled by {kf:.3f} and WRITE_SIZE by {kw:.3f}.", "",
             f"Kernel sources hash: `{h}`.", "",
             "| kernel | dispatches | fetch MB | write MB | total MB |", "|---|---|---|---|---|"] + table
    open(out, "w").write("\n".join(lines) + "\n")
    if json_out:  # the per-kernel bytes bench.py reports (config-2 kernels only)
        json.dump(js, open(os.path.join(ROOT, json_out), "w"), indent=1)


def _counters_all(d):
    """{kernel: {counter: [value per dispatch]}} from one --pmc run."""
    f = glob.glob(os.path.join(d, "*counter_collection.csv"))[0]
    out = {}
    for r in csv.DictReader(open(f)):
        k = short(r["Kernel_Name"])
        out.setdefault(k, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    return out


def counters(out, title, cmds, *dirs):
    """Per-kernel mean of every counter of several --pmc runs (one dispatch = one value per
    counter), as a markdown table and as profiles/counters.json keyed by kernel with the
    kernel-source hash they were taken on."""
    sys.path.insert(0, ROOT)
    from bench import kernel_source_hash
    merged = {}
    for d in dirs:
        for k, cs in _counters_all(d).items():
            for c, v in cs.items():
                merged.setdefault(k, {})[c] = (sum(v) / len(v), len(v))
    names = sorted({c for cs in merged.values() for c in cs})
    h = kernel_source_hash()
    lines = [f"# {title}", "", "Commands (repository root, one MI355X, ROCm 7.2):", "", "```",
             cmds, "```", "", f"Kernel sources hash: `{h}`.  Values: mean per dispatch.", ""]
    js = {}
    for k in sorted(merged):
        if not k.startswith("k_"):
            continue
        lines += [f"## `{k}`", "", "| counter | mean per dispatch | dispatches |", "|---|---|---|"]
        for c in names:
            if c in merged[k]:
                m, n = merged[k][c]
                lines.append(f"| {c} | {m:.4g} | {n} |")
        lines.append("")
        js[k] = {"counters": {c: merged[k][c][0] for c in merged[k]}, "source_hash": h}
    open(out, "w").write("\n".join(lines) + "\n")
    json.dump(js, open(os.path.join(ROOT, "profiles", "counters.json"), "w"), indent=1)


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(*sys.argv[2:6])
    elif sys.argv[1] == "counters":
        counters(sys.argv[2], sys.argv[3], sys.argv[4], *sys.argv[5:])
    else:
        traffic(*sys.argv[2:10])
