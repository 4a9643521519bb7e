"""Summaries of rocprofv3 output for the profiles/ folder (command-line tool; no device needed).

  python -m paper_2205_11935_amd.profdigest stats --trace T.csv --stats S.csv --cmd "..." --title "..." \
      --out profiles/x.md
      per-kernel time table (rocprofv3 --stats) and per-instance table (kernel name and grid size,
      from the --kernel-trace dispatches)
  python -m paper_2205_11935_amd.profdigest counters --fetch F.csv --write W.csv [--valu V.csv] \
      --trace T.csv --copy-mib 1024 --cmd-fetch "..." --cmd-write "..." [--cmd-valu "..."] \
      --json profiles/hbm_traffic.json --md profiles/y.md
      HBM bytes per launch of each instance from FETCH_SIZE / WRITE_SIZE (KiB per dispatch), scaled
      by what the same counters read for the device copy of --copy-mib MiB that the profiled
      command makes (bench.py --copy-calibration-mib), and VALU issue figures from SQ_INSTS_VALU,
      SQ_ACTIVE_INST_VALU and GRBM_GUI_ACTIVE with durations from the trace

An instance is a kernel (its full template name) launched with one grid size: for the library's
kernels that identifies the call site (layer and phase) within a forward pass.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import statistics
from collections import defaultdict
from typing import Dict, List, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
VALU_LANES = 64
CUS, SIMDS_PER_CU = 256, 4


def source_digest() -> str:
    """Digest of the kernel sources, the same as bench.py's (counter figures only hold for it)."""
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.h", "ctl_internal.h"):
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _rows(path: str) -> List[Dict[str, str]]:
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _col(row: Dict[str, str], *names: str) -> str:
    for n in names:
        if n in row:
            return row[n]
    raise KeyError("none of %s in %s" % (names, sorted(row)))


def _grid(row: Dict[str, str]) -> int:
    if "Grid_Size" in row:
        return int(row["Grid_Size"])
    return int(row["Grid_Size_X"]) * int(row.get("Grid_Size_Y", 1) or 1) * int(row.get("Grid_Size_Z", 1) or 1)


def _short(name: str) -> str:
    n = name.split("(")[0].replace("void ", "").strip()
    return n.replace("ctl::", "")


def trace_instances(trace: str) -> Dict[Tuple[str, int], List[float]]:
    """{(kernel, grid threads): [durations in ms]} of every dispatch of a kernel trace."""
    out: Dict[Tuple[str, int], List[float]] = defaultdict(list)
    for r in _rows(trace):
        ms = (int(_col(r, "End_Timestamp")) - int(_col(r, "Start_Timestamp"))) * 1e-6
        out[(_short(_col(r, "Kernel_Name")), _grid(r))].append(ms)
    return out


def counter_values(path: str) -> Dict[Tuple[str, int], Dict[str, List[float]]]:
    """{(kernel, grid threads): {counter: [value per dispatch]}}."""
    per: Dict[Tuple[int, str], Dict] = {}
    for r in _rows(path):
        did = int(_col(r, "Dispatch_Id"))
        key = (did, _col(r, "Counter_Name"))
        e = per.setdefault(key, {"kernel": _short(_col(r, "Kernel_Name")), "grid": _grid(r), "value": 0.0})
        e["value"] += float(_col(r, "Counter_Value"))          # summed over dimensions (XCDs, SEs)
    out: Dict[Tuple[str, int], Dict[str, List[float]]] = defaultdict(lambda: defaultdict(list))
    for (_, counter), e in per.items():
        out[(e["kernel"], e["grid"])][counter].append(e["value"])
    return out


def copy_dispatch(values, counter: str):
    """The calibration copy among the dispatches of a counter run: the largest reading of a copy
    kernel (the runtime's blit kernel for a device-to-device copy, or an elementwise copy); the
    library's own kernels (k_*) are never taken, whatever they read."""
    cands = [(k, v[counter]) for k, v in values.items()
             if counter in v and not k[0].startswith("k_") and "copy" in k[0].lower()]
    if not cands:
        raise SystemExit("no copy kernel among the %s dispatches: run the profiled command with "
                         "--copy-calibration-mib" % counter)
    return max(cands, key=lambda x: max(x[1]))


def cmd_stats(a):
    stats = sorted(_rows(a.stats), key=lambda r: -float(_col(r, "TotalDurationNs")))
    inst = trace_instances(a.trace)
    total = sum(sum(v) for v in inst.values())
    lines = ["# %s" % a.title, "", "Command (from the repository root, one MI355X):", "", "```", a.cmd, "```", ""]
    if a.note:
        lines += [a.note, ""]
    lines += ["Per kernel (rocprofv3 --stats):", "", "| kernel | calls | avg ms | total ms | % |", "|---|---:|---:|---:|---:|"]
    for r in stats[: a.top]:
        lines.append("| `%s` | %s | %.4f | %.3f | %.2f |" % (_short(_col(r, "Name")), _col(r, "Calls"),
                                                            float(_col(r, "AverageNs")) * 1e-6,
                                                            float(_col(r, "TotalDurationNs")) * 1e-6,
                                                            float(_col(r, "Percentage"))))
    lines += ["", "Per instance (kernel and grid size, from the dispatch trace):", "",
              "| kernel | grid threads | calls | avg ms | min ms | max ms | total ms | % |",
              "|---|---:|---:|---:|---:|---:|---:|---:|"]
    for (k, g), d in sorted(inst.items(), key=lambda x: -sum(x[1]))[: a.top]:
        lines.append("| `%s` | %d | %d | %.4f | %.4f | %.4f | %.3f | %.2f |" % (
            k, g, len(d), statistics.mean(d), min(d), max(d), sum(d), 100.0 * sum(d) / total))
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")


def cmd_counters(a):
    fetch, write = counter_values(a.fetch), counter_values(a.write)
    copy_bytes = a.copy_mib * (1 << 20)
    cf = copy_dispatch(fetch, "FETCH_SIZE")
    cw = copy_dispatch(write, "WRITE_SIZE")
    fs = copy_bytes / (max(cf[1]) * 1024.0)
    ws = copy_bytes / (max(cw[1]) * 1024.0)
    inst = trace_instances(a.trace) if a.trace else {}
    rec = {"source_digest": source_digest(),
           "copy_calibration": {"bytes": copy_bytes, "fetch_kernel": cf[0][0], "write_kernel": cw[0][0],
                                "fetch_scale": fs, "write_scale": ws},
           "command_fetch": a.cmd_fetch, "command_write": a.cmd_write, "note": a.note or "", "instances": {}}
    for key in sorted(set(fetch) & set(write)):
        k, g = key
        if not k.startswith("k_") or "FETCH_SIZE" not in fetch[key] or "WRITE_SIZE" not in write[key]:
            continue
        fb = statistics.mean(fetch[key]["FETCH_SIZE"]) * 1024.0 * fs
        wb = statistics.mean(write[key]["WRITE_SIZE"]) * 1024.0 * ws
        e = {"kernel": k, "grid_threads": g, "launches_counted": len(fetch[key]["FETCH_SIZE"]),
             "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb, "bytes_per_launch": fb + wb}
        if key in inst:
            e["trace_avg_ms"] = statistics.mean(inst[key])
            e["gbs"] = (fb + wb) / (e["trace_avg_ms"] * 1e-3) / 1e9
        rec["instances"]["%s grid %d" % (k, g)] = e
    for name, key in (a.site or []):
        # bench.py's name for an instance ("<family> @ <site>") -> the rocprof instance given
        if name not in rec["instances"]:
            raise SystemExit("no instance %r in the counter runs" % name)
        rec["instances"][key] = rec["instances"][name]
    lines = ["# HBM traffic and VALU issue per kernel instance", "",
             "Counter passes (each its own run; from the repository root, one MI355X):", "",
             "```", a.cmd_fetch, a.cmd_write] + ([a.cmd_valu] if a.cmd_valu else []) + ["```", ""]
    if a.trace_cmd:
        lines += ["Durations from the dispatch trace of:", "", "```", a.trace_cmd, "```", ""]
    lines += ["FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are scaled by what they read for a %d MiB device "
              "copy in the same run (`%s`): fetch x%.3f, write x%.3f." % (a.copy_mib, cf[0][0], fs, ws), "",
              "| instance | launches | fetched GB | written GB | total GB | avg ms | GB/s |",
              "|---|---:|---:|---:|---:|---:|---:|"]
    for name, e in sorted(rec["instances"].items(), key=lambda x: -x[1]["bytes_per_launch"]):
        if " @ " in name:
            continue
        lines.append("| `%s` | %d | %.4f | %.4f | %.4f | %s | %s |" % (
            name, e["launches_counted"], e["fetch_bytes_per_launch"] / 1e9, e["write_bytes_per_launch"] / 1e9,
            e["bytes_per_launch"] / 1e9, "%.4f" % e["trace_avg_ms"] if "trace_avg_ms" in e else "-",
            "%.0f" % e["gbs"] if "gbs" in e else "-"))
    if a.valu:
        val = counter_values(a.valu)
        rec["valu"] = {}
        lines += ["", "VALU issue (SQ_INSTS_VALU: wave-level VALU instructions, SQ_ACTIVE_INST_VALU: cycles "
                  "of VALU activity summed over waves, GRBM_GUI_ACTIVE: GPU-busy cycles; lane-instructions/s = "
                  "SQ_INSTS_VALU x 64 / trace duration, against the unit-count peak of %d CUs x 64 lanes x 2.4 GHz "
                  "= 39.3 T):" % CUS, "",
                  "| instance | launches | VALU instr / launch | T lane-instr/s | of 39.3 T | VALU-active cycles / launch | GUI-active cycles / launch |",
                  "|---|---:|---:|---:|---:|---:|---:|"]
        for key, cs in sorted(val.items(), key=lambda x: -statistics.mean(x[1].get("SQ_INSTS_VALU", [0]))):
            k, g = key
            if not k.startswith("k_") or "SQ_INSTS_VALU" not in cs:
                continue
            ins = statistics.mean(cs["SQ_INSTS_VALU"])
            act = statistics.mean(cs.get("SQ_ACTIVE_INST_VALU", [0]))
            gui = statistics.mean(cs.get("GRBM_GUI_ACTIVE", [0]))
            e = {"launches": len(cs["SQ_INSTS_VALU"]), "valu_instr": ins, "valu_active_cycles": act, "gui_active": gui}
            rate = None
            if key in inst:
                rate = ins * VALU_LANES / (statistics.mean(inst[key]) * 1e-3)
                e["lane_instr_per_s"] = rate
            rec["valu"]["%s grid %d" % (k, g)] = e
            lines.append("| `%s grid %d` | %d | %.4g | %s | %s | %.4g | %.4g |" % (
                k, g, e["launches"], ins, "%.2f" % (rate / 1e12) if rate else "-",
                "%.3f" % (rate / 39.3216e12) if rate else "-", act, gui))
    with open(a.json, "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
    with open(a.md, "w") as f:
        f.write("\n".join(lines) + "\n")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("--trace", required=True)
    s.add_argument("--stats", required=True)
    s.add_argument("--cmd", required=True)
    s.add_argument("--title", required=True)
    s.add_argument("--note", default="")
    s.add_argument("--top", type=int, default=24)
    s.add_argument("--out", required=True)
    c = sub.add_parser("counters")
    c.add_argument("--fetch", required=True)
    c.add_argument("--write", required=True)
    c.add_argument("--valu")
    c.add_argument("--trace")
    c.add_argument("--trace-cmd", default="")
    c.add_argument("--copy-mib", type=int, required=True)
    c.add_argument("--cmd-fetch", required=True)
    c.add_argument("--cmd-write", required=True)
    c.add_argument("--cmd-valu", default="")
    c.add_argument("--note", default="")
    c.add_argument("--site", nargs=2, action="append", metavar=("INSTANCE", "KEY"),
                   help="also key an instance ('k_x<..> grid G') by bench.py's name for it "
                        "('family @ site')")
    c.add_argument("--json", required=True)
    c.add_argument("--md", required=True)
    a = ap.parse_args(argv)
    (cmd_stats if a.what == "stats" else cmd_counters)(a)


if __name__ == "__main__":
    main()
