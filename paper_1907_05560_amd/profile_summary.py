"""Summaries of rocprofv3 output for the kernels (text for profiles/).

Two inputs, both written by ``rocprofv3`` runs of ``bench.py``:

* a kernel-trace run (``--kernel-trace --stats``): its ``*_kernel_trace.csv``
  gives the duration of every dispatch;
* two counter runs (``--pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE``) of a bench
  invocation that also copies a buffer of known size
  (``bench.py --copy-calibration-mib M``).  The HBM counters are scaled by
  the ratio between the bytes that copy moves (M MiB read and M MiB written)
  and what the same counter reports for it, so the kernel figures are in
  bytes that a plain copy would count as moved.  The JSON file keys them by
  ``kernel_key`` (e.g. ``k_final<float,float,3,DP54,2>``), as bench.py looks
  them up.

Dispatches made after a run has reached its end radius (the attempts a host
loop enqueues past the end) return at once; a dispatch is counted as such, and
left out of the means, when its duration (or counter value) is below a quarter
of the largest one of the same kernel.

Usage::

    python -m paper_1907_05560_amd.profile_summary trace <kernel_trace.csv> --command "..." > profiles/x.md
    python -m paper_1907_05560_amd.profile_summary traffic --fetch <csv> --write <csv> \
        --copy-mib M --command-fetch "..." --command-write "..." \
        --json profiles/traffic.json > profiles/y.md
    python -m paper_1907_05560_amd.profile_summary valu <counter_collection.csv> --command "..." \
        --json profiles/exp_valu.json > profiles/z.md
"""

from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import re
import sys

_HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SRC = os.path.join(_HERE, "csrc", "nuosc_kernels.hip")
EXP_SRC = os.path.join(_HERE, "csrc", "nuosc_exp.hip")
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def kernel_source_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def exp_source_hash() -> str:
    """Hash of the exponential-stepper kernel source (nuosc_exp.hip)."""
    with open(EXP_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def exp_launch(name: str):
    """Beam launch (1..3) of a three-flavor exponential-stepper kernel, or None."""
    m = re.search(r"k_exp_beam<3,(\d)>", short_name(name))
    return int(m.group(1)) if m and m.group(1) != "0" else None


def valu_summary(csv_path: str, command: str):
    """VALU wavefront-instruction counts (rocprofv3 SQ_INSTS_VALU) of the
    exponential-stepper beam kernels, per launch (full dispatches only)."""
    per = _counter_means(csv_path, "SQ_INSTS_VALU")
    waves = _counter_means(csv_path, "SQ_WAVES")
    lines = ["# VALU instructions of the exponential-stepper beam kernels (rocprofv3 SQ_INSTS_VALU)", "",
             "Command:", "", "```", command, "```", "",
             f"Kernel source (nuosc_exp.hip) sha256[:16]: `{exp_source_hash()}`", "",
             "| kernel | dispatches | VALU wave-instructions / dispatch | waves / dispatch | per wave |",
             "|---|---|---|---|---|"]
    doc = {"source_sha256_16": exp_source_hash(), "valu_wave_instr_per_launch": {}}
    for name in sorted(per, key=lambda n: (exp_launch(n) or 9, n)):
        L = exp_launch(name)
        if L is None:
            continue
        v = _full(per[name])
        wv = _full(waves.get(name, [])) or [0.0]
        vm, wm = sum(v) / len(v), sum(wv) / len(wv)
        lines.append(f"| `{short_name(name)}` | {len(v)} | {vm:.4g} | {wm:.0f} | {vm / wm if wm else 0:.0f} |")
        doc["valu_wave_instr_per_launch"][f"launch{L}"] = round(vm)
    return "\n".join(lines) + "\n", doc


def short_name(name: str) -> str:
    """'void nuosc::(anonymous namespace)::k_final_one<float, float, 3, ...TabDP54, 2>(nuosc::RunConst)'
    -> 'k_final_one<float,float,3,DP54,2>'."""
    n = name.replace("nuosc::(anonymous namespace)::", "").replace("void ", "")
    n = re.sub(r"\(nuosc::(RunConst|LaunchSet).*\)$", "", n)
    n = n.replace("TabDP54", "DP54").replace("TabRK4", "RK4").replace(" ", "")
    return n


def kernel_key(name: str) -> str:
    """Short name of a kernel with the single-run suffix dropped, so that the
    one-run and launch-set instantiations of a kernel share a key:
    'k_final_one<float,float,3,DP54,2>' -> 'k_final<float,float,3,DP54,2>'."""
    return re.sub(r"_one<", "<", short_name(name), count=1)


def _full(values):
    """Values of full dispatches (at least a quarter of the largest)."""
    if not values:
        return []
    top = max(values)
    return [v for v in values if v >= 0.25 * top]


def trace_summary(trace_csv: str, command: str) -> str:
    per = collections.defaultdict(list)
    regs = {}
    for r in csv.DictReader(open(trace_csv)):
        name = r["Kernel_Name"]
        per[name].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
        regs[name] = (r["VGPR_Count"], r["Accum_VGPR_Count"], r["SGPR_Count"], r["LDS_Block_Size"],
                      r["Workgroup_Size_X"], r["Grid_Size_X"])
    total = sum(sum(v) for v in per.values())
    out = ["# Kernel trace summary", "", "Command:", "", "```", command, "```", "",
           "Means are over full dispatches; `early` counts dispatches that returned at once because the "
           "run had already reached its end radius.", "",
           "| kernel | full | early | mean us | min us | max us | share % | VGPR | AGPR | SGPR | LDS B | WG | grid |",
           "|---|---|---|---|---|---|---|---|---|---|---|---|---|"]
    for name in sorted(per, key=lambda n: -sum(per[n])):
        v = per[name]
        f = _full(v)
        vg, ag, sg, lds, wg, grid = regs[name]
        out.append(f"| `{short_name(name)}` | {len(f)} | {len(v) - len(f)} | {sum(f) / len(f):.2f} | "
                   f"{min(f):.2f} | {max(f):.2f} | {100 * sum(v) / total:.2f} | {vg} | {ag} | {sg} | {lds} | "
                   f"{wg} | {grid} |")
    return "\n".join(out) + "\n"


def _counter_means(path: str, counter: str):
    """Mean counter value (KiB as reported) per kernel name; copy kernel: per-dispatch values."""
    per = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        per[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return per


def traffic_summary(fetch_csv: str, write_csv: str, copy_mib: float, cmd_f: str, cmd_w: str):
    fetch = _counter_means(fetch_csv, "FETCH_SIZE")
    write = _counter_means(write_csv, "WRITE_SIZE")
    copy_bytes = copy_mib * 2 ** 20
    # the calibration copy is the largest copy dispatch of the run
    cf = max(fetch.get(COPY_KERNEL, [0.0]))
    cw = max(write.get(COPY_KERNEL, [0.0]))
    if cf <= 0 or cw <= 0:
        raise SystemExit("calibration copy kernel not found in the counter runs")
    scale_f = copy_bytes / (cf * 1024.0)
    scale_w = copy_bytes / (cw * 1024.0)
    per_launch = {}
    lines = ["# HBM traffic of the kernels (rocprofv3 FETCH_SIZE / WRITE_SIZE)", "",
             "Commands:", "", "```", cmd_f, cmd_w, "```", "",
             f"Calibration: a device-to-device copy of {copy_mib:g} MiB ({COPY_KERNEL}) reads "
             f"{cf:.0f} KiB by FETCH_SIZE and writes {cw:.0f} KiB by WRITE_SIZE, so FETCH_SIZE is scaled by "
             f"{scale_f:.3f} and WRITE_SIZE by {scale_w:.3f}.", "",
             f"Kernel source sha256[:16]: `{kernel_source_hash()}`", "",
             "| kernel | dispatches | FETCH KiB (raw) | WRITE KiB (raw) | read MB (scaled) | write MB (scaled) | total MB |",
             "|---|---|---|---|---|---|---|"]
    for name in sorted(set(fetch) | set(write), key=kernel_key):
        if name == COPY_KERNEL:
            continue
        f = fetch.get(name, [])
        w = write.get(name, [])
        if not f or not w:
            continue
        f, w = _full(f), _full(w)
        fm, wm = sum(f) / len(f), sum(w) / len(w)
        rb, wb = fm * 1024 * scale_f, wm * 1024 * scale_w
        lines.append(f"| `{short_name(name)}` | {len(f)} | {fm:.0f} | {wm:.0f} | {rb / 1e6:.2f} | "
                     f"{wb / 1e6:.2f} | {(rb + wb) / 1e6:.2f} |")
        per_launch[kernel_key(name)] = round(rb + wb)
    doc = {
        "kernel_source_sha256_16": kernel_source_hash(),
        "copy_calibration_mib": copy_mib,
        "fetch_scale": scale_f,
        "write_scale": scale_w,
        "bytes_per_launch": per_launch,
    }
    return "\n".join(lines) + "\n", doc


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("trace_csv")
    t.add_argument("--command", required=True)
    f = sub.add_parser("traffic")
    f.add_argument("--fetch", required=True)
    f.add_argument("--write", required=True)
    f.add_argument("--copy-mib", type=float, required=True)
    f.add_argument("--command-fetch", required=True)
    f.add_argument("--command-write", required=True)
    f.add_argument("--json", required=True)
    v = sub.add_parser("valu")
    v.add_argument("counter_csv")
    v.add_argument("--command", required=True)
    v.add_argument("--json", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "valu":
        text, doc = valu_summary(a.counter_csv, a.command)
        with open(a.json, "w") as fh:
            json.dump(doc, fh, indent=1)
            fh.write("\n")
        sys.stdout.write(text)
        return 0
    if a.cmd == "trace":
        sys.stdout.write(trace_summary(a.trace_csv, a.command))
    else:
        text, doc = traffic_summary(a.fetch, a.write, a.copy_mib, a.command_fetch, a.command_write)
        with open(a.json, "w") as fh:
            json.dump(doc, fh, indent=1)
            fh.write("\n")
        sys.stdout.write(text)
    return 0


if __name__ == "__main__":
    sys.exit(main())
