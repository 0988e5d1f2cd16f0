"""Short text summaries of rocprofv3 output for the profiles folder.

pmc: HBM traffic per launch of the dominant entry point from two rocprofv3
counter runs (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) of
`bench.py --pmc-probe`, calibrated by the plain copy kernel of known size the
probe runs in the same process:

    python -m paper_2307_14837_amd.profile_summary pmc --fetch F.csv --write W.csv \\
        --probe probe.log --out profiles/pmc_<workload>.json

F.csv / W.csv are rocprofv3 `*_counter_collection.csv` files; probe.log is
what `bench.py --pmc-probe` printed (its last JSON line is used).

sq: a Markdown table of SQ counters (one or more `--pmc` passes, each its own
csv) for the one kernel whose name contains --kernel, averaged over its
dispatches, with per-wave values:

    python -m paper_2307_14837_amd.profile_summary sq --kernel "k_residual<4, false>" \
        --csv P1.csv --csv P2.csv --out profiles/sq_<kernel>_<workload>.md --command "..." --command "..."

stats: a Markdown table of a `--kernel-trace --stats` run's kernel_stats.csv,
or of its kernel_trace.csv restricted to the dispatches after the last one
matching --after:

    python -m paper_2307_14837_amd.profile_summary stats --csv K.csv --out profiles/<name>.md \\
        --command "<the rocprofv3 command>"
    python -m paper_2307_14837_amd.profile_summary stats --trace T.csv --after k_adamw ...
"""
from __future__ import annotations

import argparse
import csv
import json
from collections import defaultdict

ENTRY_KERNELS = {"dnnmg_residual_b": ("k_residual<4, false>", "k_lps_corners"),
                 "dnnmg_residual_rhs_b": ("k_residual_rhs_b", "k_lps_corners"),
                 "dnnmg_prolong_residual_b": ("k_residual<3, false>",),
                 "dnnmg_patch_gather_forward": ("k_mlp_fwd<2, 512",),
                 "dnnmg_q2_residual_b": ("k_q2_element<0>", "k_q2_sum_nodes<0>")}
COPY_KERNEL = "neg"


def per_kernel(path, counter):
    """Average counter value per dispatch for each kernel name."""
    vals = defaultdict(dict)
    for row in csv.DictReader(open(path)):
        if row.get("Counter_Name") != counter:
            continue
        # one value per dispatch (summed over dimensions if the tool splits it)
        d = vals[row["Kernel_Name"]]
        d[row["Dispatch_Id"]] = d.get(row["Dispatch_Id"], 0.0) + float(row["Counter_Value"])
    return {k: sum(v.values()) / len(v) for k, v in vals.items() if v}


def find(avgs, needle):
    hits = [v for k, v in avgs.items() if needle in k]
    if len(hits) != 1:
        raise SystemExit(f"expected one kernel matching {needle!r}, found {len(hits)}")
    return hits[0]


def trace_stats(path, after, tail=0):
    """kernel_stats-like rows from a kernel_trace.csv, over the dispatches
    after the last one whose name contains `after` (the setup before the
    measured section, e.g. network training, is left out), or over the last
    `tail` dispatches when tail > 0."""
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    if tail > 0:
        rows = rows[-tail:]
    else:
        last = max((i for i, r in enumerate(rows) if after in r["Kernel_Name"]), default=-1)
        rows = rows[last + 1:]
    per = defaultdict(list)
    for r in rows:
        per[r["Kernel_Name"]].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    total = sum(sum(v) for v in per.values()) or 1
    out = []
    for name, d in per.items():
        out.append({"Name": name, "Calls": len(d), "TotalDurationNs": sum(d), "AverageNs": sum(d) / len(d),
                    "MinNs": min(d), "MaxNs": max(d), "Percentage": 100.0 * sum(d) / total})
    return out


def stats(a):
    rows = trace_stats(a.trace, a.after, a.last) if a.trace else list(csv.DictReader(open(a.csv)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"# {a.title}", "", "Command:", "", "```", a.command, "```", "",
             "| kernel | calls | avg us | min us | max us | share % |", "|---|---:|---:|---:|---:|---:|"]
    for r in rows[: a.top]:
        name = r["Name"]
        short = name.split("(")[0] if "(" in name else name
        lines.append(f"| `{short[:90]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.1f} |")
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def sq(a):
    vals = {}
    for path in a.csv:
        names = {r["Counter_Name"] for r in csv.DictReader(open(path))}
        for c in names:
            vals[c] = find(per_kernel(path, c), a.kernel)
    waves = vals.get("SQ_WAVES", 0.0) or 1.0
    lines = [f"# {a.title}", "", "Commands (one counter pass each; values averaged over the dispatches of the kernel):",
             "", "```", *a.command, "```", "", "| counter | total | per wave |", "|---|---:|---:|"]
    for c in sorted(vals):
        lines.append(f"| {c} | {vals[c]:.4g} | {vals[c] / waves:.1f} |")
    if a.note:
        lines += ["", *a.note]
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    sp = sub.add_parser("stats")
    sp.add_argument("--csv", default=None, help="kernel_stats.csv of a --stats run")
    sp.add_argument("--trace", default=None, help="kernel_trace.csv (with --after)")
    sp.add_argument("--after", default="", help="count only dispatches after the last kernel matching this")
    sp.add_argument("--last", type=int, default=0, help="count only the last N dispatches (with --trace)")
    sp.add_argument("--out", required=True)
    sp.add_argument("--command", default="")
    sp.add_argument("--title", default="rocprofv3 kernel statistics")
    sp.add_argument("--top", type=int, default=20)
    sq_p = sub.add_parser("sq")
    sq_p.add_argument("--csv", action="append", required=True, help="counter_collection.csv of one --pmc pass")
    sq_p.add_argument("--kernel", required=True, help="substring naming exactly one kernel")
    sq_p.add_argument("--out", required=True)
    sq_p.add_argument("--command", action="append", default=[])
    sq_p.add_argument("--note", action="append", default=[], help="a line of text appended after the table")
    sq_p.add_argument("--title", default="SQ counters")
    ap_p = sub.add_parser("pmc")
    ap_p.add_argument("--fetch", required=True)
    ap_p.add_argument("--write", required=True)
    ap_p.add_argument("--probe", required=True)
    ap_p.add_argument("--out", required=True)
    ap_p.add_argument("--command", default="")
    a = ap.parse_args()
    if a.mode == "stats":
        return stats(a)
    if a.mode == "sq":
        return sq(a)
    probe = [json.loads(l) for l in open(a.probe) if l.startswith('{"pmc_probe"')][-1]
    fetch = per_kernel(a.fetch, "FETCH_SIZE")
    write = per_kernel(a.write, "WRITE_SIZE")
    # calibration: counter KiB of the copy vs its known bytes
    f_scale = probe["copy_bytes_read"] / (1024.0 * find(fetch, COPY_KERNEL))
    w_scale = probe["copy_bytes_written"] / (1024.0 * find(write, COPY_KERNEL))
    entries = {}
    for entry, kernels in ENTRY_KERNELS.items():
        ks = {}
        fb = wb = 0.0
        for kname in kernels:
            fk, wk = find(fetch, kname), find(write, kname)
            ks[kname] = {"fetch_kib": fk, "write_kib": wk}
            fb += fk * 1024.0 * f_scale
            wb += wk * 1024.0 * w_scale
        h = probe["src_hash"]
        entries[entry] = {"src_hash": h[entry] if isinstance(h, dict) else h, "kernels": ks, "fetch_bytes": fb, "write_bytes": wb,
                          "bytes_per_launch": fb + wb}
    out = {"workload": probe["pmc_probe"], "command": a.command,
           "copy": {"bytes_read": probe["copy_bytes_read"], "bytes_written": probe["copy_bytes_written"],
                    "fetch_kib": find(fetch, COPY_KERNEL), "write_kib": find(write, COPY_KERNEL),
                    "fetch_scale": f_scale, "write_scale": w_scale},
           "entries": entries}
    with open(a.out, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
