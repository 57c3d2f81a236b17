"""Summaries of rocprofv3 output for the profiles/ folder.

    python -m paper_1305_7313_amd.profsum stats <kernel_stats.csv> <out.md> "<command>"
    python -m paper_1305_7313_amd.profsum traffic <fetch.csv> <write.csv> <workload> <out.json> "<command>"

``stats`` turns a --kernel-trace --stats CSV into a short table.  ``traffic``
averages FETCH_SIZE / WRITE_SIZE (KiB per dispatch) per kernel class of the
band-pair path, calibrated against the plain device copy the benchmark runs
with --copy-probe (a copy reads as many bytes as it writes: fetch_scale =
copy WRITE / copy FETCH; write_scale = bytes copied / copy WRITE).
"""
from __future__ import annotations

import collections
import csv
import json
import re
import sys

COPY_BYTES = 3 * (1 << 30)  # bench.py --copy-probe: three 1 GiB copies


def short(name: str) -> str:
    name = re.sub(r"\(fockx::[A-Za-z]+Args\)|\(.*\)$", "", name)
    return name.replace("void ", "").replace("fockx::", "")


def kernel_class(name: str):
    m = re.search(r"plane_kernel<\w+, \d+, \d+, \d+, \w+, (\d), \d>", name)
    if m:
        return {"0": "p1_pair_plane_fwd", "1": "p3_plane_inv_mac", "2": "a7_plane_fwd", "3": "plane_inv",
                "4": "p3_second", "5": "band_plane_density", "6": "band_plane_vmul", "7": "p1_pair_plane_fwd",
                "8": "p3_plane_inv_mac", "9": "p3_second"}.get(m.group(1))
    m = re.search(r"pencil_kernel<\w+, \d+, \d+, \d+, \w+, (\d), \d>", name)
    if m:
        return {"0": "p2_pencil_kernel", "1": "p2_pencil_energy", "2": "a7_pencil_fwd", "3": "a1_pencil_inv"}[m.group(1)]
    if "mac_conj_kernel" in name or "mac_pair_kernel" in name or "mac_gamma_kernel" in name:
        return "p3_second"
    if "force_gather_kernel" in name:
        return "band_force_gather"
    return None


def stats(csv_path, out_md, command):
    rows = list(csv.DictReader(open(csv_path)))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = [f"# rocprofv3 kernel statistics", "", "Command:", "", "```", command, "```", "",
             "| kernel | calls | average (us) | total (ms) | share |", "|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| `{short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.2f} | {100 * float(r['TotalDurationNs']) / total:.1f}% |")
    open(out_md, "w").write("\n".join(lines) + "\n")


def dispatch_classes(rows):
    """Kernel class of every dispatch.  The in-place inverse plane pass runs in
    two roles: after P2 it is the pair pass P3 of the streaming schedule
    (class p3_plane_inv_mac, like the fused P3), after the inverse pencil pass
    it takes orbitals to real space (class plane_inv).  Its role is read from
    the dispatch before it on the same queue (a stream's kernels run in order
    on one queue)."""
    out = {}
    last = {}
    for r in sorted(rows, key=lambda r: int(r["Dispatch_Id"])):
        k = kernel_class(r["Kernel_Name"])
        if k == "plane_inv" and last.get(r["Queue_Id"]) == "p2_pencil_kernel":
            k = "p3_plane_inv_mac"
        out[r["Dispatch_Id"]] = k
        last[r["Queue_Id"]] = k
    return out


def traffic(fetch_csv, write_csv, workload, out_json, command, sha):
    def load(p):
        rows = list(csv.DictReader(open(p)))
        cls = dispatch_classes(rows)
        agg = collections.defaultdict(list)
        copy = 0.0
        for r in rows:
            if r["Kernel_Name"] == "__amd_rocclr_copyBuffer":
                copy += float(r["Counter_Value"])
            elif cls[r["Dispatch_Id"]]:
                agg[cls[r["Dispatch_Id"]]].append(float(r["Counter_Value"]))
        return agg, copy
    (f, cf), (w, cw) = load(fetch_csv), load(write_csv)
    rec = {"workload": workload, "command": command, "source_sha256": sha,
           "fetch_scale": cw / cf if cf else None, "write_scale": COPY_BYTES / 1024.0 / cw if cw else None,
           "copy_probe": {"bytes": COPY_BYTES, "fetch_kib": cf, "write_kib": cw}, "kernels": {}}
    by_class = collections.defaultdict(lambda: [[], []])
    for k, vals in f.items():
        by_class[k][0].extend(vals)
    for k, vals in w.items():
        by_class[k][1].extend(vals)
    for k, (fv, wv) in by_class.items():
        rec["kernels"][k] = {"dispatches": len(fv), "fetch_kib": sum(fv) / len(fv), "write_kib": sum(wv) / len(wv)}
    open(out_json, "w").write(json.dumps(rec, indent=1) + "\n")


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "traffic":
        import os
        sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
        import bench
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], sys.argv[6], bench.sources_sha())
    else:
        raise SystemExit(__doc__)
