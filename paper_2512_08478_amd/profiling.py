"""Summaries of rocprofv3 output for the committed profiles.

Subcommands (each prints a short text summary; `traffic` also records the
per-launch HBM bytes that bench.py reports as roofline.traffic):

  stats   DIR [--title T --command C]
      per-kernel launches, total and average duration from the
      `--kernel-trace --stats` CSVs under DIR.
  traffic --fetch DIR --write DIR --calib-mib M --key KEY --kernel REGEX
          [--sources f1,f2,...] [--json PATH] [--title T --command C]
      FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of every kernel, scaled
      by what the same counters read for the M MiB device copy the run
      starts with; the average bytes per launch of the kernels matching
      REGEX go into PATH under KEY, with a hash of their sources.
  counters DIR [DIR ...] --kernel REGEX [--key KEY --json PATH --sources f1,...]
           [--title T --command C]
      the SQ counters of the matching kernels (one or more --pmc passes),
      averaged per dispatch, with VALU-busy % and LDS bank conflicts per
      LDS instruction; with --json, the VALU-busy and issue fractions,
      resident waves and instructions per wave go into PATH under KEY, with
      a hash of the kernel's sources.

rocprofv3 writes its CSVs under DIR/<host>/<pid>_*.csv (or directly under
DIR); every `*_kernel_stats.csv`, `*_kernel_trace.csv` and
`*_counter_collection.csv` below DIR is read.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")


def _files(d, suffix):
    out = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not out:
        raise SystemExit(f"no *{suffix} under {d}")
    return out


def _rows(d, suffix):
    for f in _files(d, suffix):
        with open(f, newline="") as fh:
            yield from csv.DictReader(fh)


def short_name(name):
    """Kernel name without its namespace, return type and parameter list."""
    n = re.sub(r"^void\s+", "", name.strip())
    n = n.replace("(anonymous namespace)::", "")
    n = re.sub(r"^gs::", "", n)
    depth, cut = 0, len(n)
    for i, ch in enumerate(n):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            cut = i
            break
    return n[:cut]


def _header(title, command):
    lines = []
    if title:
        lines.append(f"# {title}")
    if command:
        lines.append(f"# command: {command}")
    return lines


def cmd_stats(a):
    lines = _header(a.title, a.command)
    rows = list(_rows(a.dir, "kernel_stats.csv"))
    tot = sum(float(r["TotalDurationNs"]) for r in rows) or 1.0
    lines.append(f"{'kernel':60s} {'calls':>7s} {'total us':>11s} {'avg us':>9s} {'%':>6s}")
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        t = float(r["TotalDurationNs"])
        lines.append(f"{short_name(r['Name'])[:60]:60s} {int(r['Calls']):7d} {t / 1e3:11.1f} "
                     f"{float(r['AverageNs']) / 1e3:9.2f} {100 * t / tot:6.2f}")
    print("\n".join(lines))


def _per_dispatch(d, counter):
    """{dispatch id: (kernel name, grid, value)} of one counter."""
    out = {}
    for r in _rows(d, "counter_collection.csv"):
        if r["Counter_Name"] != counter:
            continue
        k = r["Dispatch_Id"]
        v = float(r["Counter_Value"])
        if k in out:
            out[k] = (out[k][0], out[k][1], out[k][2] + v)
        else:
            out[k] = (r["Kernel_Name"], int(r["Grid_Size"]), v)
    if not out:
        raise SystemExit(f"no {counter} rows under {d}")
    return out


def _calibration(disp, mib):
    """Counter KiB of the largest copy kernel vs the copy's own KiB."""
    cands = [v for v in disp.values() if "copy" in v[0].lower() or "elementwise" in v[0].lower()]
    if not cands:
        raise SystemExit("no copy kernel found for the calibration")
    best = max(cands, key=lambda v: v[2])
    return (mib * 1024.0) / best[2], best


def source_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def cmd_traffic(a):
    fetch = _per_dispatch(a.fetch, "FETCH_SIZE")
    write = _per_dispatch(a.write, "WRITE_SIZE")
    ff, fc = _calibration(fetch, a.calib_mib)
    wf, wc = _calibration(write, a.calib_mib)
    lines = _header(a.title, a.command)
    lines.append(f"# calibration: a {a.calib_mib} MiB device copy reads FETCH_SIZE {fc[2]:.1f} KiB "
                 f"(factor {ff:.4f}) and WRITE_SIZE {wc[2]:.1f} KiB (factor {wf:.4f})")
    lines.append("# values: counter KiB x factor, averaged over dispatches, in MB (1e6 B)")
    agg = defaultdict(lambda: [0, 0.0, 0.0])
    for k, (name, grid, v) in fetch.items():
        g = agg[(short_name(name), grid)]
        g[0] += 1
        g[1] += v * ff * 1024
    for k, (name, grid, v) in write.items():
        agg[(short_name(name), grid)][2] += v * wf * 1024
    lines.append(f"{'kernel':52s} {'grid':>10s} {'n':>5s} {'fetch MB':>10s} {'write MB':>10s}")
    pat = re.compile(a.kernel)
    sel = []
    for (name, grid), (n, fb, wb) in sorted(agg.items()):
        lines.append(f"{name[:52]:52s} {grid:10d} {n:5d} {fb / n / 1e6:10.2f} {wb / n / 1e6:10.2f}")
        if pat.search(name):
            sel.append((n, fb, wb))
    if not sel:
        raise SystemExit(f"no kernel matches {a.kernel}")
    n = sum(s[0] for s in sel)
    per = (sum(s[1] for s in sel) + sum(s[2] for s in sel)) / n
    lines.append(f"# {a.key}: {n} launches matching {a.kernel!r}, {per / 1e6:.2f} MB per launch")
    print("\n".join(lines))
    if a.json:
        try:
            db = json.load(open(a.json))
        except (OSError, ValueError):
            db = {}
        srcs = a.sources.split(",")
        db[a.key] = {"bytes_per_launch": int(round(per)), "launches": n,
                     "fetch_bytes_per_launch": int(round(sum(s[1] for s in sel) / n)),
                     "write_bytes_per_launch": int(round(sum(s[2] for s in sel) / n)),
                     "sources": srcs, "source_sha256_16": source_hash(srcs)}
        with open(a.json, "w") as fh:
            json.dump(db, fh, indent=1, sort_keys=True)
            fh.write("\n")


def cmd_counters(a):
    pat = re.compile(a.kernel)
    vals = defaultdict(lambda: defaultdict(list))
    meta = {}
    for d in a.dirs:
        per = defaultdict(dict)
        for r in _rows(d, "counter_collection.csv"):
            name = short_name(r["Kernel_Name"])
            if not pat.search(name):
                continue
            per[(r["Dispatch_Id"], name)][r["Counter_Name"]] = \
                per[(r["Dispatch_Id"], name)].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
            meta[name] = (int(r["Grid_Size"]), int(r["Workgroup_Size"]), int(r.get("VGPR_Count", 0) or 0),
                          int(r.get("LDS_Block_Size", 0) or 0))
        for (disp, name), cs in per.items():
            for c, v in cs.items():
                vals[name][c].append(v)
    lines = _header(a.title, a.command)
    for name, cs in sorted(vals.items()):
        g, wg, vg, lds = meta[name]
        lines.append(f"{name}: grid {g}, workgroup {wg}, VGPRs {vg}, LDS bytes {lds}")
        avg = {c: sum(v) / len(v) for c, v in cs.items()}
        for c in sorted(avg):
            lines.append(f"  {c:28s} {avg[c]:18.1f}   ({len(cs[c])} dispatches)")
        if "GRBM_GUI_ACTIVE" in avg and avg["GRBM_GUI_ACTIVE"] > 0:
            # GRBM_GUI_ACTIVE is summed over the XCDs: the kernel's GPU-busy
            # cycles are the per-XCD value; SQ_ACTIVE_INST_VALU counts
            # quad-cycles summed over the SIMDs, so VALU busy (rocprof's
            # definition) = 100 x ACTIVE_INST_VALU x 4 / SIMDs / cycles
            cyc = avg["GRBM_GUI_ACTIVE"] / a.xcds
            lines.append(f"  kernel cycles (GRBM_GUI_ACTIVE / {a.xcds} XCDs): {cyc:.0f}")
            if "SQ_ACTIVE_INST_VALU" in avg:
                lines.append(f"  VALU busy: {100 * avg['SQ_ACTIVE_INST_VALU'] * 4 / a.simds / cyc:.1f} % "
                             f"(100 x SQ_ACTIVE_INST_VALU x 4 / {a.simds} SIMDs / cycles)")
            if "SQ_INSTS_VALU" in avg:
                lines.append(f"  VALU issue: {100 * avg['SQ_INSTS_VALU'] * 4 / a.simds / cyc:.1f} % "
                             f"(wave64 FP32 instructions x 4 cycles / {a.simds} SIMDs / cycles)")
            if "SQ_WAVE_CYCLES" in avg:
                lines.append(f"  waves resident per SIMD: {avg['SQ_WAVE_CYCLES'] * 4 / a.simds / cyc:.2f} "
                             f"(SQ_WAVE_CYCLES x 4 / SIMDs / cycles)")
        if "SQ_INSTS_LDS" in avg and "SQ_LDS_BANK_CONFLICT" in avg and avg["SQ_INSTS_LDS"] > 0:
            lines.append(f"  LDS bank-conflict cycles per LDS instruction: "
                         f"{avg['SQ_LDS_BANK_CONFLICT'] / avg['SQ_INSTS_LDS']:.3f}")
        if "SQ_INSTS_VALU" in avg and "SQ_WAVES" in avg and avg["SQ_WAVES"] > 0:
            lines.append(f"  VALU instructions per wave: {avg['SQ_INSTS_VALU'] / avg['SQ_WAVES']:.1f}")
        if a.json and a.key and "GRBM_GUI_ACTIVE" in avg and avg["GRBM_GUI_ACTIVE"] > 0:
            cyc = avg["GRBM_GUI_ACTIVE"] / a.xcds
            rec = {"kernel": name, "dispatches": len(next(iter(cs.values()))),
                   "sources": a.sources.split(","), "source_sha256_16": source_hash(a.sources.split(","))}
            if "SQ_ACTIVE_INST_VALU" in avg:
                rec["valu_busy"] = round(avg["SQ_ACTIVE_INST_VALU"] * 4 / a.simds / cyc, 4)
            if "SQ_INSTS_VALU" in avg:
                rec["valu_issue"] = round(avg["SQ_INSTS_VALU"] * 4 / a.simds / cyc, 4)
            if "SQ_WAVE_CYCLES" in avg:
                rec["waves_per_simd"] = round(avg["SQ_WAVE_CYCLES"] * 4 / a.simds / cyc, 3)
            if "SQ_INSTS_VALU" in avg and avg.get("SQ_WAVES", 0) > 0:
                rec["valu_insts_per_wave"] = round(avg["SQ_INSTS_VALU"] / avg["SQ_WAVES"], 1)
            try:
                db = json.load(open(a.json))
            except (OSError, ValueError):
                db = {}
            db[a.key] = rec
            with open(a.json, "w") as fh:
                json.dump(db, fh, indent=1, sort_keys=True)
                fh.write("\n")
    print("\n".join(lines))


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_2512_08478_amd.profiling")
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--calib-mib", type=float, required=True)
    t.add_argument("--key", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--sources", default="raster.hip,gs_device.h,gs_internal.h")
    t.add_argument("--json")
    c = sub.add_parser("counters")
    c.add_argument("dirs", nargs="+")
    c.add_argument("--kernel", required=True)
    c.add_argument("--simds", type=int, default=1024)
    c.add_argument("--xcds", type=int, default=8)
    c.add_argument("--key")
    c.add_argument("--json")
    c.add_argument("--sources", default="raster.hip,gs_device.h,gs_internal.h")
    for p in (s, t, c):
        p.add_argument("--title", default="")
        p.add_argument("--command", default="")
    a = ap.parse_args(argv)
    {"stats": cmd_stats, "traffic": cmd_traffic, "counters": cmd_counters}[a.cmd](a)


if __name__ == "__main__":
    sys.exit(main())
