"""Summaries of rocprofv3 output for the committed profiles.

Reads only rocprofv3's CSV files (kernel statistics, counter collection) and writes
text: a markdown table of per-kernel times, and the HBM traffic per launch of the
Kronecker matvec from FETCH_SIZE / WRITE_SIZE counter runs, scaled by what the same
counters read for a plain device copy of known size taken in the same runs.

    python -m paper_2609_02394_amd.profiling stats <kernel_stats.csv> <out.md> <title> <command>
    python -m paper_2609_02394_amd.profiling traffic <fetch_dir> <write_dir> <out.json> <out.md> \
        <fetch command> <write command>
    python -m paper_2609_02394_amd.profiling mfma <counter_dir> <out.md> <title> <command>

The mfma summary reads one counter run with SQ_VALU_MFMA_BUSY_CYCLES, GRBM_GUI_ACTIVE and
the SQ_INSTS_VALU_MFMA_MOPS_* counters: per kernel, the share of the MI355X SIMDs'
cycles their MFMA units were busy (the busy cycles summed over the SIMDs over
GRBM_GUI_ACTIVE / 8 XCDs times 1024 SIMDs), and the MFMA flops (MOPS x 512) per second
of dispatch time, dispatches being serialised while counters are collected.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 256 << 20  # the calibration copy bench.py --calibrate-copy makes
PREC_NAMES = {"0": "fp64", "1": "fp32", "2": "bf16"}


def kron_source_hash() -> str:
    p = os.path.join(ROOT, "paper_2609_02394_amd", "csrc", "kron.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def _short(name: str) -> str:
    name = name.strip().replace("(anonymous namespace)::", "")
    name = re.sub(r"\(.*\)$", "", name)
    return name.replace("void ", "")


def stats_md(csv_path: str, title: str, command: str, top: int = 25) -> str:
    rows = list(csv.DictReader(open(csv_path)))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    out = [f"# {title}", "", "Command (from the repository root on the GPU host):", "", "```",
           command, "```", "",
           "| kernel | calls | total ms | avg us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    for r in rows[:top]:
        out.append("| `{}` | {} | {:.3f} | {:.2f} | {:.2f} | {:.2f} | {:.1f} |".format(
            _short(r["Name"]), r["Calls"], float(r["TotalDurationNs"]) / 1e6,
            float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3,
            100.0 * float(r["TotalDurationNs"]) / total))
    out += ["", f"Total kernel time: {total / 1e6:.2f} ms over {len(rows)} kernels.", ""]
    return "\n".join(out)


def _counter_rows(d: str):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    rows = []
    for f in files:
        rows += list(csv.DictReader(open(f)))
    return rows


def _per_dispatch(rows, counter: str):
    """{dispatch id: (kernel name, summed counter value in KiB)}"""
    acc = {}
    for r in rows:
        if r["Counter_Name"] != counter:
            continue
        key = r.get("Dispatch_Id") or r.get("Correlation_Id")
        name, v = r["Kernel_Name"], float(r["Counter_Value"])
        if key in acc:
            acc[key] = (name, acc[key][1] + v)
        else:
            acc[key] = (name, v)
    return acc


def _kron_key(name: str):
    """'kron_step:fp64' or 'kron_filter_kernel:fp32' style key of a Kronecker launch: the
    one-step matvec (streaming or tiled kernel) or the whole fused filter (64- or
    96-wide form), by precision, as the benchmark's event timing groups them."""
    m = re.search(r"kron_(stream|batched|filter|filter_wide)_kernel<(\d)", name)
    if not m:
        return None
    kind = "kron_filter_kernel" if m.group(1).startswith("filter") else "kron_step"
    return f"{kind}:{PREC_NAMES.get(m.group(2))}"


def traffic(fetch_dir: str, write_dir: str):
    res = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        disp = _per_dispatch(_counter_rows(d), counter)
        copies = [v for n, v in disp.values() if "copy" in n.lower()]
        big = max(copies) if copies else 0.0
        scale = (COPY_BYTES / 1024.0) / big if big > 0 else None
        per = defaultdict(list)
        for n, v in disp.values():
            p = _kron_key(n)
            if p:
                per[p].append(v)
        res[counter] = {"scale": scale, "copy_kib": big,
                        "kron_kib_avg": {p: sum(v) / len(v) for p, v in per.items()},
                        "kron_dispatches": {p: len(v) for p, v in per.items()}}
    out = {"kron_source_sha": kron_source_hash(), "bytes_per_launch": {},
           "fetch_scale": res["FETCH_SIZE"]["scale"], "write_scale": res["WRITE_SIZE"]["scale"],
           "fetch_kib_avg": res["FETCH_SIZE"]["kron_kib_avg"],
           "write_kib_avg": res["WRITE_SIZE"]["kron_kib_avg"],
           "dispatches": res["FETCH_SIZE"]["kron_dispatches"]}
    fs, ws = out["fetch_scale"], out["write_scale"]
    if fs and ws:
        for p in out["fetch_kib_avg"]:
            if p in out["write_kib_avg"]:
                out["bytes_per_launch"][p] = 1024.0 * (out["fetch_kib_avg"][p] * fs +
                                                       out["write_kib_avg"][p] * ws)
    return out


def traffic_md(t: dict, fetch_cmd: str, write_cmd: str) -> str:
    lines = ["# HBM traffic of the Kronecker kernels (rocprofv3 counters)", "",
             "FETCH_SIZE and WRITE_SIZE per dispatch (KiB), averaged over the Kronecker "
             "launches of each precision, each scaled by the reading of the same counter for "
             f"a plain {COPY_BYTES >> 20} MiB device copy in the same run.", "",
             f"kron.hip sha256[:16] = `{t['kron_source_sha']}`", "",
             f"Scale factors: FETCH x{t['fetch_scale']:.3f}, WRITE x{t['write_scale']:.3f}", "",
             "| kernel:precision | launches | FETCH KiB avg | WRITE KiB avg | HBM bytes / launch |",
             "|---|---|---|---|---|"]
    for p, b in sorted(t["bytes_per_launch"].items()):
        lines.append(f"| {p} | {t['dispatches'].get(p, 0)} | {t['fetch_kib_avg'][p]:.1f} | "
                     f"{t['write_kib_avg'][p]:.1f} | {b / 1e6:.2f} MB |")
    lines += ["", "Commands:", "", "```", fetch_cmd, write_cmd, "```", ""]
    return "\n".join(lines)


SIMDS = 1024  # 256 CUs x 4 SIMDs
XCDS = 8      # GRBM_GUI_ACTIVE reads summed over the XCDs


def mfma(d: str):
    per_disp = defaultdict(lambda: defaultdict(float))
    info = {}
    for r in _counter_rows(d):
        key = r.get("Dispatch_Id") or r.get("Correlation_Id")
        per_disp[key][r["Counter_Name"]] += float(r["Counter_Value"])
        info[key] = (_short(r["Kernel_Name"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    per = defaultdict(lambda: defaultdict(float))
    for key, c in per_disp.items():
        name, ns = info[key]
        a = per[name]
        a["n"] += 1
        a["ns"] += ns
        for cn, v in c.items():
            a[cn] += v
    rows = []
    for name, a in per.items():
        cyc = a.get("GRBM_GUI_ACTIVE", 0.0) / XCDS
        busy = a.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) / (cyc * SIMDS) if cyc > 0 else 0.0
        sec = a["ns"] * 1e-9
        tf = {p: a.get(f"SQ_INSTS_VALU_MFMA_MOPS_{p}", 0.0) * 512 / sec / 1e12 if sec > 0 else 0.0
              for p in ("F64", "F32", "BF16")}
        rows.append((name, int(a["n"]), a["ns"] / 1e6, busy, tf))
    rows.sort(key=lambda x: -x[2])
    return rows


def mfma_md(rows, title: str, command: str) -> str:
    out = [f"# {title}", "", "Command (from the repository root on the GPU host):", "", "```",
           command, "```", "",
           "Dispatches are serialised while counters are collected, so the times and rates "
           "are per kernel alone on the chip.", "",
           "| kernel | dispatches | ms | MFMA busy | FP64 TF/s | FP32 TF/s | BF16 TF/s |",
           "|---|---|---|---|---|---|---|"]
    for name, n, ms, busy, tf in rows:
        out.append(f"| `{name}` | {n} | {ms:.1f} | {100 * busy:.1f}% | {tf['F64']:.1f} | "
                   f"{tf['F32']:.1f} | {tf['BF16']:.1f} |")
    out.append("")
    return "\n".join(out)


def main(argv):
    if argv[0] == "stats":
        _, csv_path, out, title, cmd = argv
        open(out, "w").write(stats_md(csv_path, title, cmd))
    elif argv[0] == "traffic":
        _, fd, wd, out_json, out_md, fcmd, wcmd = argv
        t = traffic(fd, wd)
        t["commands"] = [fcmd, wcmd]
        json.dump(t, open(out_json, "w"), indent=1)
        open(out_md, "w").write(traffic_md(t, fcmd, wcmd))
    elif argv[0] == "mfma":
        _, d, out, title, cmd = argv
        open(out, "w").write(mfma_md(mfma(d), title, cmd))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
