"""Summaries of rocprofv3 output for the step kernels (kernel-trace statistics and HBM
counters), written as short text/JSON files.

    python -m paper_1311_7239_amd.profiling stats <kernel_stats.csv> <out.txt> <command...>
    python -m paper_1311_7239_amd.profiling counters <fetch.csv> <write.csv> <out.json> <command...>
    python -m paper_1311_7239_amd.profiling sq <counters.csv> <out.txt> <command...>

FETCH_SIZE and WRITE_SIZE are read per dispatch (KiB) and scaled by what the same
counters read for a plain device copy of known size recorded in the same run
(hipMemcpy of 1 GiB: 1 GiB read, 1 GiB written).
"""
from __future__ import annotations

import csv
import hashlib
import json
import pathlib
import sys

PKG = pathlib.Path(__file__).resolve().parent


def kernel_sources():
    """Every source of the library (kernels, device header, launch interface, C ABI):
    a change to any of them, launch choices included, marks older summaries stale."""
    return sorted(p for p in (PKG / "csrc").iterdir() if p.suffix in (".hip", ".h", ".cpp"))


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for path in kernel_sources():
        h.update(path.name.encode() + b"\0")
        h.update(path.read_bytes())
    return h.hexdigest()[:16]


def _rows(path):
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def _short(name, width=150):
    return name if len(name) <= width else name[:width] + " ..."


def stats_summary(stats_csv, out_txt, command):
    rows = _rows(stats_csv)
    lines = [f"# rocprofv3 --kernel-trace --stats summary", f"# command: {command}",
             f"# kernel sources sha256[:16]: {kernel_source_hash()}",
             "calls  avg_us  min_us  max_us  pct  kernel"]
    for r in rows:
        lines.append(f"{int(r['Calls']):5d} {float(r['AverageNs']) / 1e3:8.1f} {float(r['MinNs']) / 1e3:8.1f} "
                     f"{float(r['MaxNs']) / 1e3:8.1f} {float(r['Percentage']):5.1f}  {_short(r['Name'])}")
    pathlib.Path(out_txt).write_text("\n".join(lines) + "\n")


def _per_kernel(rows, counter):
    out = {}
    for r in rows:
        if r["Counter_Name"] != counter:
            continue
        out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return out


def counters_summary(fetch_csv, write_csv, out_json, command, kernel_prefix="void mrt::k_step"):
    fetch = _per_kernel(_rows(fetch_csv), "FETCH_SIZE")
    write = _per_kernel(_rows(write_csv), "WRITE_SIZE")
    copy_f = max(fetch.get("__amd_rocclr_copyBuffer", [0.0]))
    copy_w = max(write.get("__amd_rocclr_copyBuffer", [0.0]))
    gib_kib = float(1 << 20)
    fscale = gib_kib / copy_f if copy_f > 0 else None
    wscale = gib_kib / copy_w if copy_w > 0 else None
    kernels = {}
    for name, vals in fetch.items():
        if not name.startswith(kernel_prefix) or "k_step_batch" in name:
            continue
        w = write.get(name, [])
        kernels[name] = {"dispatches": len(vals), "fetch_kib": sum(vals) / len(vals),
                         "write_kib": (sum(w) / len(w)) if w else None}
    out = {"command": command, "kernel_source_hash": kernel_source_hash(),
           "copy_reference": {"bytes_read": 1 << 30, "bytes_written": 1 << 30,
                              "fetch_kib": copy_f, "write_kib": copy_w},
           "fetch_scale": fscale, "write_scale": wscale, "kernels": kernels}
    pathlib.Path(out_json).write_text(json.dumps(out, indent=1) + "\n")


def sq_summary(counters_csv, out_txt, command, kernel_prefix="void mrt::k_step"):
    """Per-kernel sums of SQ counters (instruction mix, waves) over the dispatches."""
    rows = _rows(counters_csv)
    agg, disp = {}, {}
    for r in rows:
        name = r["Kernel_Name"]
        if not name.startswith(kernel_prefix):
            continue
        agg.setdefault(name, {})
        agg[name][r["Counter_Name"]] = agg[name].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        disp.setdefault(name, set()).add(r.get("Dispatch_Id", r.get("Correlation_Id", "")))
    lines = ["# rocprofv3 --pmc SQ counter summary (sums over the dispatches)", f"# command: {command}",
             f"# kernel sources sha256[:16]: {kernel_source_hash()}"]
    for name, c in agg.items():
        waves = c.get("SQ_WAVES", 0.0)
        lines.append(f"{_short(name)}")
        lines.append(f"    dispatches {len(disp[name])}  " + "  ".join(f"{k} {v:.4g}" for k, v in sorted(c.items())))
        if waves:
            lines.append(f"    SQ_INSTS_VALU per wave {c.get('SQ_INSTS_VALU', 0.0) / waves:.1f}")
    pathlib.Path(out_txt).write_text("\n".join(lines) + "\n")


def traffic_bytes(summary_json, kernel_name=None):
    """HBM bytes per dispatch of the step kernel from a counters summary, or None if the
    kernel sources changed since the counters were taken. kernel_name: the full name or a
    prefix of it (the first match); None takes the most dispatched kernel."""
    p = pathlib.Path(summary_json)
    if not p.exists():
        return None
    s = json.loads(p.read_text())
    if s.get("kernel_source_hash") != kernel_source_hash() or not s.get("kernels"):
        return None
    if kernel_name:
        k = s["kernels"].get(kernel_name)
        if k is None:
            k = next((v for n, v in s["kernels"].items() if n.startswith(kernel_name)), None)
    else:
        k = max(s["kernels"].values(), key=lambda v: v["dispatches"])
    if not k or k["write_kib"] is None or not s["fetch_scale"] or not s["write_scale"]:
        return None
    return 1024.0 * (k["fetch_kib"] * s["fetch_scale"] + k["write_kib"] * s["write_scale"])


if __name__ == "__main__":
    mode = sys.argv[1]
    if mode == "stats":
        stats_summary(sys.argv[2], sys.argv[3], " ".join(sys.argv[4:]))
    elif mode == "counters":
        counters_summary(sys.argv[2], sys.argv[3], sys.argv[4], " ".join(sys.argv[5:]))
    elif mode == "sq":
        sq_summary(sys.argv[2], sys.argv[3], " ".join(sys.argv[4:]))
    elif mode == "sq-all":   # every library kernel (the adjoint's as well as the step's)
        sq_summary(sys.argv[2], sys.argv[3], " ".join(sys.argv[4:]), kernel_prefix="void mrt::k_")
    else:
        raise SystemExit("usage: profiling.py stats|counters|sq|sq-all ...")
