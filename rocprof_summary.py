"""Summaries of rocprofv3 output for the profiles/ directory.

    python rocprof_summary.py stats <kernel_stats.csv> [--title T] [--command C]
        -> a Markdown table of per-kernel calls and durations.

    python rocprof_summary.py traffic --fetch <dir> --write <dir>
           --copy-fetch <dir> --copy-write <dir> --kernels a,b,c [--durations <kernel_stats.csv>]
        -> a Markdown table of calibrated DRAM bytes per dispatch for several kernels.

    python rocprof_summary.py counters --fetch <dir> --write <dir>
           --copy-fetch <dir> --copy-write <dir> --kernels a,b --names id_a,id_b --prec <p> --source-hash <h>
           [--out profiles/vx_counters.json] [--command C]
        -> HBM traffic per launch of each kernel from FETCH_SIZE and WRITE_SIZE
           (KiB per dispatch), each scaled by the factor that makes a plain
           1 GiB device copy read and write exactly 1 GiB.

    python rocprof_summary.py table <dir> [<dir> ...] --kernels a,b,c
        -> a Markdown table of the mean of every counter per dispatch for each kernel.

    python rocprof_summary.py mfma <dir> [--kernel k_tn_mfma]
        -> executed MFMA TFLOP/s, fraction of the dense peak and matrix-core busy
           fraction of each matrix-core kernel instantiation.

Input directories are rocprofv3 -d output folders written with
--output-format csv (the counter runs produce *counter_collection.csv).
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import sys


def _find(d, pattern):
    hits = sorted(glob.glob(os.path.join(d, "**", pattern), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no {pattern} under {d}")
    return hits[0]


def stats(path, title=None, command=None):
    rows = list(csv.DictReader(open(path)))
    out = []
    if title:
        out.append(f"# {title}\n")
    if command:
        out.append(f"Command:\n\n```\n{command}\n```\n")
    out.append("| kernel | calls | total ms | average ms | min ms | max ms | % |")
    out.append("|---|---|---|---|---|---|---|")
    for r in rows:
        name = r.get("Name", r.get("KernelName", ""))
        calls = int(float(r.get("Calls", 0)))
        tot = float(r.get("TotalDurationNs", 0)) / 1e6
        avg = float(r.get("AverageNs", 0)) / 1e6
        mn = float(r.get("MinNs", 0)) / 1e6
        mx = float(r.get("MaxNs", 0)) / 1e6
        pct = float(r.get("Percentage", 0))
        out.append(f"| `{name[:90]}` | {calls} | {tot:.2f} | {avg:.4f} | {mn:.4f} | {mx:.4f} | {pct:.1f} |")
    return "\n".join(out) + "\n"


def _counter_rows(d, counter):
    path = _find(d, "*counter_collection.csv")
    rows = []
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name", r.get("Counter-Name", "")) != counter:
            continue
        name = r.get("Kernel_Name", r.get("Kernel-Name", ""))
        val = float(r.get("Counter_Value", r.get("Counter-Value", 0)))
        disp = r.get("Dispatch_Id", r.get("Dispatch-Id", ""))
        rows.append((disp, name, val))
    return rows


def _per_dispatch(rows):
    acc = {}
    for disp, name, val in rows:
        key = (disp, name)
        acc[key] = acc.get(key, 0.0) + val
    return acc


def counters(fetch, write, copy_fetch, copy_write, kernels, names, prec, source_hash, command=None):
    """Copy-calibrated DRAM bytes per launch for each kernel (name substring -> library id)."""
    one_gib_kib = float(1 << 20)
    # calibration: the largest dispatch of the copy run is the 1 GiB copy
    cf = max(_per_dispatch(_counter_rows(copy_fetch, "FETCH_SIZE")).values())
    cw = max(_per_dispatch(_counter_rows(copy_write, "WRITE_SIZE")).values())
    sf, sw = one_gib_kib / cf, one_gib_kib / cw
    fr = _per_dispatch(_counter_rows(fetch, "FETCH_SIZE"))
    wr = _per_dispatch(_counter_rows(write, "WRITE_SIZE"))
    out = {}
    for kernel, name in zip(kernels, names):
        f = [v for (d, n), v in fr.items() if kernel in n]
        w = [v for (d, n), v in wr.items() if kernel in n]
        if not f or not w:
            raise ValueError(f"kernel {kernel!r} not found in the counter runs")
        fetch_b = sum(f) / len(f) * 1024 * sf
        write_b = sum(w) / len(w) * 1024 * sw
        out[name] = {"kernel": kernel, "fetch_bytes_per_launch": fetch_b, "write_bytes_per_launch": write_b,
                     "bytes_per_launch": fetch_b + write_b, "launches": [len(f), len(w)]}
    return {"prec": prec, "source_hash": source_hash, "copy_scale_fetch": sf, "copy_scale_write": sw,
            "kernels": out, "command": command}


def traffic_table(fetch, write, copy_fetch, copy_write, kernels, title=None, command=None, durations=None):
    """Markdown table: calibrated DRAM read/write bytes per dispatch for each kernel
    whose name contains one of `kernels`; with `durations` (kernel_stats.csv of a
    kernel-trace run of the same command) also the measured rate."""
    one_gib_kib = float(1 << 20)
    cf = max(_per_dispatch(_counter_rows(copy_fetch, "FETCH_SIZE")).values())
    cw = max(_per_dispatch(_counter_rows(copy_write, "WRITE_SIZE")).values())
    sf, sw = one_gib_kib / cf, one_gib_kib / cw
    fr = _per_dispatch(_counter_rows(fetch, "FETCH_SIZE"))
    wr = _per_dispatch(_counter_rows(write, "WRITE_SIZE"))
    avg_ms = {}
    if durations:
        for r in csv.DictReader(open(durations)):
            avg_ms[r.get("Name", r.get("KernelName", ""))] = float(r.get("AverageNs", 0)) / 1e6
    out = []
    if title:
        out.append(f"# {title}\n")
    if command:
        out.append(f"Commands:\n\n```\n{command}\n```\n")
    out.append(f"Calibration: a 1 GiB device copy reads {cf / one_gib_kib:.4f} GiB by FETCH_SIZE and writes "
               f"{cw / one_gib_kib:.4f} GiB by WRITE_SIZE; counts below are scaled by {sf:.4f} and {sw:.4f}.\n")
    out.append("| kernel | dispatches | read GB / dispatch | write GB / dispatch | total GB | avg ms | DRAM GB/s |")
    out.append("|---|---|---|---|---|---|---|")
    for k in kernels:
        f = [v for (d, n), v in fr.items() if k in n]
        w = [v for (d, n), v in wr.items() if k in n]
        if not f or not w:
            continue
        fb = sum(f) / len(f) * 1024 * sf / 1e9
        wb = sum(w) / len(w) * 1024 * sw / 1e9
        ms = [v for n, v in avg_ms.items() if k in n]
        msv = sum(ms) / len(ms) if ms else None
        rate = f"{(fb + wb) / (msv * 1e-3):.0f}" if msv else "-"
        mss = f"{msv:.3f}" if msv else "-"
        out.append(f"| `{k}` | {len(f)} | {fb:.3f} | {wb:.3f} | {fb + wb:.3f} | {mss} | {rate} |")
    return "\n".join(out) + "\n"


def counter_table(dirs, kernels, title=None, command=None):
    """Markdown table: mean of every counter per dispatch, for each kernel (name substring),
    over one or more rocprofv3 --pmc output folders."""
    vals = {}
    for d in dirs:
        path = _find(d, "*counter_collection.csv")
        per = {}
        for r in csv.DictReader(open(path)):
            name = r.get("Kernel_Name", r.get("Kernel-Name", ""))
            k = next((k for k in kernels if k in name), None)
            if k is None:
                continue
            c = r.get("Counter_Name", r.get("Counter-Name", ""))
            disp = r.get("Dispatch_Id", r.get("Dispatch-Id", ""))
            per.setdefault((k, c), {}).setdefault(disp, 0.0)
            per[(k, c)][disp] += float(r.get("Counter_Value", r.get("Counter-Value", 0)))
        for (k, c), byd in per.items():
            vals.setdefault(c, {})[k] = sum(byd.values()) / len(byd)
    out = []
    if title:
        out.append(f"# {title}\n")
    if command:
        out.append(f"Commands:\n\n```\n{command}\n```\n")
    out.append("| counter (mean per dispatch) | " + " | ".join(f"`{k}`" for k in kernels) + " |")
    out.append("|---|" + "---|" * len(kernels))
    for c in sorted(vals):
        out.append(f"| {c} | " + " | ".join(f"{vals[c].get(k, float('nan')):.4g}" for k in kernels) + " |")
    return "\n".join(out) + "\n"


MFMA_PEAK_TFLOPS = {"F32": 157.3, "BF16": 2500.0, "F16": 2500.0, "F64": 78.6}


def mfma_table(d, kernel_substr, title=None, command=None, xcds=8, simds=1024):
    """Markdown table for the matrix-core kernels of one rocprofv3 --pmc folder with
    SQ_INSTS_VALU_MFMA_MOPS_* (MFMA flops = MOPS x 512), SQ_VALU_MFMA_BUSY_CYCLES and
    GRBM_GUI_ACTIVE: per kernel instantiation, the mean dispatch duration, the executed MFMA
    TFLOP/s and its fraction of the published dense peak of the operand type, and the matrix
    cores' busy fraction BUSY / (GUI_ACTIVE / xcds x simds).  GRBM_GUI_ACTIVE is reported
    summed over the XCDs; the clock column (GUI_ACTIVE / xcds / duration) checks that."""
    path = _find(d, "*counter_collection.csv")
    per = {}
    for r in csv.DictReader(open(path)):
        name = r.get("Kernel_Name", "")
        if kernel_substr not in name:
            continue
        disp = r.get("Dispatch_Id", "")
        e = per.setdefault(name, {}).setdefault(disp, {})
        e[r.get("Counter_Name", "")] = float(r.get("Counter_Value", 0))
        e["_ns"] = float(r["End_Timestamp"]) - float(r["Start_Timestamp"])
    out = []
    if title:
        out.append(f"# {title}\n")
    if command:
        out.append(f"Command:\n\n```\n{command}\n```\n")
    out.append("| kernel | dispatches | mean ms | MFMA TFLOP/s | operand type | of dense peak | MFMA busy | clock GHz |")
    out.append("|---|---|---|---|---|---|---|---|")
    for name, byd in per.items():
        n = len(byd)
        ms = sum(e["_ns"] for e in byd.values()) / n / 1e6
        mops = {t: sum(e.get(f"SQ_INSTS_VALU_MFMA_MOPS_{t}", 0.0) for e in byd.values()) / n for t in MFMA_PEAK_TFLOPS}
        t_main = max(mops, key=mops.get)
        flops = 512.0 * sum(mops.values())
        tf = flops / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
        gui = sum(e.get("GRBM_GUI_ACTIVE", 0.0) for e in byd.values()) / n
        busy = sum(e.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) for e in byd.values()) / n
        util = busy / (gui / xcds * simds) if gui > 0 else float("nan")
        ghz = gui / xcds / (ms * 1e-3) / 1e9 if ms > 0 else float("nan")
        short = name.split("(")[0].replace("void ", "")
        out.append(f"| `{short}` | {n} | {ms:.2f} | {tf:.1f} | {t_main} | {tf / MFMA_PEAK_TFLOPS[t_main]:.1%} | "
                   f"{util:.1%} | {ghz:.2f} |")
    return "\n".join(out) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--title")
    s.add_argument("--command")
    c = sub.add_parser("counters")
    for k in ("--fetch", "--write", "--copy-fetch", "--copy-write", "--prec", "--source-hash"):
        c.add_argument(k, required=True)
    c.add_argument("--kernels", required=True, help="comma-separated kernel name substrings")
    c.add_argument("--names", required=True,
                   help="comma-separated library ids of the same kernels (fock_prof.h), e.g. vx_plane_fwd")
    c.add_argument("--out")
    c.add_argument("--command")
    t = sub.add_parser("traffic")
    for k in ("--fetch", "--write", "--copy-fetch", "--copy-write"):
        t.add_argument(k, required=True)
    t.add_argument("--kernels", required=True, help="comma-separated name substrings")
    t.add_argument("--durations")
    t.add_argument("--title")
    t.add_argument("--command")
    m = sub.add_parser("mfma")
    m.add_argument("dir")
    m.add_argument("--kernel", default="k_tn_mfma", help="name substring of the matrix-core kernels")
    m.add_argument("--title")
    m.add_argument("--command")
    q = sub.add_parser("table")
    q.add_argument("dirs", nargs="+")
    q.add_argument("--kernels", required=True, help="comma-separated name substrings")
    q.add_argument("--title")
    q.add_argument("--command")
    a = ap.parse_args(argv)
    if a.cmd == "table":
        sys.stdout.write(counter_table(a.dirs, a.kernels.split(","), a.title, a.command))
        return
    if a.cmd == "mfma":
        sys.stdout.write(mfma_table(a.dir, a.kernel, a.title, a.command))
        return
    if a.cmd == "stats":
        sys.stdout.write(stats(a.csv, a.title, a.command))
    elif a.cmd == "traffic":
        sys.stdout.write(traffic_table(a.fetch, a.write, a.copy_fetch, a.copy_write, a.kernels.split(","), a.title,
                                       a.command, a.durations))
    else:
        res = counters(a.fetch, a.write, a.copy_fetch, a.copy_write, a.kernels.split(","), a.names.split(","),
                       a.prec, a.source_hash, a.command)
        txt = json.dumps(res, indent=1)
        if a.out:
            open(a.out, "w").write(txt + "\n")
        print(txt)


if __name__ == "__main__":
    main()
