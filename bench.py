#!/usr/bin/env python3
"""Benchmark: coupled eigensolves/s of the recursive module-coupling eigensolver.

Default line (the metric's workload): 512 random-field Heisenberg chains N=32, J=1,
h_i ~ U[-2, 2] seeded per chain, 8-site leaves (dense 256-dim leaf ED), retained k
drawn per chain from {32, 48, 64, 96}, three bond operators per cut, lowest 8 states.
One step solves every chain once (leaf EDs, projections, every coupling step with its
Kronecker-sum eigensolve, edge-operator transforms), all modules of a tree level across
all chains in batched launches, with FP32 (or BF16) Kronecker matvecs and FP64
correction. A chain counts as a solve only if its 8 energies match the FP64 reference
to |dE|/max(|E|,1) <= 1e-8; the FP64 references are the GPU's FP64 path, itself
checked against the oracle's stored energies (tests/golden) on a 32-chain subset.

Beside it, in the same run: the plain per-job FP64 recursion of the same chains, the
roofline of the dominant kernel (HIP events on the library's stream inside the timed
region), the oracle timed on the host cores (all cores and one thread), and extra
keys for the other workloads: the XXZ chain N=64 k=64 (32 jobs per step, and one job
at a time), the TFIM ladder 2x48 k=128, and a bounded serving run.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# Kronecker kernel variants measured on MI355X for the benchmark shapes (the
# autotuner's cache format); used through a private copy so that runs do not edit it.
TUNE_FILE = os.path.join(ROOT, "paper_2609_02394_amd", "kron_tune_gfx950.txt")
GOLDEN_RFHEIS = os.path.join(ROOT, "tests", "golden", "recursion_rfheis_subset.txt")
GOLDEN_LADDER = os.path.join(ROOT, "tests", "golden", "recursion_ladder96_k128.txt")

METRIC = "coupled eigensolves/s (lowest 8, rel err≤1e-8 vs FP64) + p50/p99 latency"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}
HBM_GBS = 8000.0
PREC = {"fp64": 0, "fp32": 1, "bf16": 2}
KINDS = {0: "kron_step", 1: "kron_filter_kernel"}
# the one-step launches run the streaming kernel or, where its tiles do not fit, the
# tiled one; the profiler counts them as one kind
KIND_NAMES = {0: "kron_stream_kernel|kron_batched_kernel", 1: "kron_filter_kernel"}


def use_tune_file():
    if "RMC_TUNE_CACHE" in os.environ or not os.path.exists(TUNE_FILE):
        return
    import shutil
    import tempfile

    fd, path = tempfile.mkstemp(prefix="rmc_tune_", suffix=".txt")
    os.close(fd)
    shutil.copyfile(TUNE_FILE, path)
    os.environ["RMC_TUNE_CACHE"] = path


def kron_source_hash() -> str:
    p = os.path.join(ROOT, "paper_2609_02394_amd", "csrc", "kron.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def measured_traffic(workload: str, kernel: str, prec: str):
    """HBM bytes per launch of a Kronecker kernel kind from committed rocprofv3 counter
    runs of this workload (scaled by a copy kernel of known size), or None when the
    counters were taken on another kernel source."""
    try:
        d = json.load(open(os.path.join(ROOT, "profiles", f"kron_traffic_{workload}.json")))
    except Exception:
        return None
    if d.get("kron_source_sha") != kron_source_hash():
        return None
    return d.get("bytes_per_launch", {}).get(f"{kernel}:{prec}")


def rel_err(a, b):
    import numpy as np

    a, b = np.asarray(a, dtype=float), np.asarray(b, dtype=float)
    e = np.abs(a - b) / np.maximum(np.abs(b), 1.0)
    return float(np.max(e)) if np.all(np.isfinite(e)) else float("inf")


def read_golden(path):
    """{name: (k, q, energies)} from a golden file written by the oracle."""
    out, cur = {}, None
    if not os.path.exists(path):
        return out
    for line in open(path):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue
        if f[0] == "job":
            kv = dict(x.split("=") for x in f[2:])
            cur = f[1]
            out[cur] = (int(kv["k"]), int(kv["q"]), [])
        elif f[0] == "E":
            out[cur][2].extend(float(x) for x in f[1:])
    return out


# ---- measurement helpers -------------------------------------------------------------

def kron_profile(ctx, steps):
    """Per (kind, precision) totals of the Kronecker launches since profile(True)."""
    table = {}
    for kk in KINDS:
        for name in PREC:
            pr = ctx.profile_read(PREC[name], kernel=kk)
            if pr["launches"]:
                table[(kk, name)] = pr
    out = {}
    for (kk, name), pr in table.items():
        sec = pr["ms"] * 1e-3
        out[f"{KINDS[kk]}:{name}"] = {
            "kernel": KIND_NAMES[kk], "launches": pr["launches"],
            "ms_per_step": pr["ms"] / steps, "avg_launch_us": pr["ms"] * 1e3 / pr["launches"],
            "tflops": pr["flops"] / sec / 1e12 if sec > 0 else 0.0,
            "frac_of_mfma_peak": (pr["flops"] / sec / 1e12 / PEAK_TFLOPS[name]) if sec > 0 else 0.0,
            "gbs": pr["bytes"] / sec / 1e9 if sec > 0 else 0.0,
            "flops_per_launch": pr["flops"] / pr["launches"],
            "bytes_per_launch": pr["bytes"] / pr["launches"]}
    return table, out


def roofline(table, workload):
    """Roofline of the dominant Kronecker kernel kind and precision (most event time)."""
    if not table:
        return None
    (kk, name) = max(table, key=lambda k: table[k]["ms"])
    pr = table[(kk, name)]
    sec = pr["ms"] * 1e-3
    # the bound is the roof the kernel's algorithmic intensity meets first: HBM below the
    # ridge (peak flops / 8 TB/s), the MFMA peak of its precision above it
    intensity = pr["flops"] / pr["bytes"] if pr["bytes"] > 0 else float("inf")
    if intensity < PEAK_TFLOPS[name] * 1e12 / (HBM_GBS * 1e9):
        achieved = pr["bytes"] / sec / 1e9 if sec > 0 else 0.0
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_GBS, "unit": "GB/s",
                "frac": achieved / HBM_GBS}
    else:
        achieved = pr["flops"] / sec / 1e12 if sec > 0 else 0.0
        roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS[name],
                "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS[name]}
    roof.update({"traffic": measured_traffic(workload, KINDS[kk], name),
                 "kernel": KIND_NAMES[kk], "precision": name, "intensity_flop_per_byte": intensity,
                 "launches": pr["launches"],
                 "avg_launch_us": pr["ms"] * 1e3 / max(1, pr["launches"]),
                 "flops_per_launch": pr["flops"] / max(1, pr["launches"]),
                 "bytes_per_launch": pr["bytes"] / max(1, pr["launches"])})
    return roof


def timed_batches(ctx, jobs, refs, opts, steps, warmup, qs):
    """Time `steps` solves of the whole batch after `warmup` untimed ones; a job counts
    when its energies match refs to 1e-8. Returns the measurement and the kernel table."""
    import numpy as np
    import torch

    from paper_2609_02394_amd import rmc

    # the jobs' descriptors are inputs: marshalled from Python once, before the clock
    batch = rmc.JobBatch(jobs)
    for _ in range(warmup):
        ctx.recurse_batch(batch, opts=opts)
    lat, ok, max_err, results = [], 0, 0.0, []
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        s0 = time.perf_counter()
        e, st, top = ctx.recurse_batch(batch, opts=opts)
        lat.append(time.perf_counter() - s0)
        results.append((e, st))
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    # every job of every timed step against its FP64 reference, once the clock has stopped
    for e, st in results:
        for i in range(len(jobs)):
            err = rel_err(e[i, : qs[i]], refs[i]) if st[i] == 0 else float("inf")
            max_err = max(max_err, err)
            ok += err <= 1e-8
    table, ktab = kron_profile(ctx, steps)
    ctx.profile(False)
    lat_ms = np.array(lat) * 1e3
    return {"value": ok / total, "ms_per_step": total / steps * 1e3,
            "p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99)),
            "accurate_solves": ok, "jobs_per_step": len(jobs), "max_rel_err": max_err}, table, ktab


def plain_per_job(ctx, jobs, refs, qs, reps=1):
    """The plain per-job FP64 recursion: one job at a time, every job FP64."""
    from paper_2609_02394_amd import rmc

    fp64 = rmc.default_opts(precision=0)
    ctx.recurse(*jobs[0], opts=fp64)
    ok, t0 = 0, time.perf_counter()
    for _ in range(reps):
        for j, r, q in zip(jobs, refs, qs):
            e, _ = ctx.recurse(*j, opts=fp64)
            ok += rel_err(e[:q], r) <= 1e-8
    dt = time.perf_counter() - t0
    return {"form": "plain per-job FP64 recursion, one job at a time", "jobs": len(jobs) * reps,
            "value": ok / dt, "unit": "solves/s", "seconds": dt}


def host_info():
    info = {"nproc": os.cpu_count(), "cpu_model": platform.processor() or None, "blas": None}
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                info["cpu_model"] = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        r = subprocess.run(["nproc"], capture_output=True, text=True, timeout=10)
        info["nproc"] = int(r.stdout.strip())
    except Exception:
        pass
    try:
        from threadpoolctl import threadpool_info

        b = [d for d in threadpool_info() if d.get("user_api") == "blas"]
        if b:
            info["blas"] = f"{b[0].get('internal_api')} {b[0].get('version')} ({b[0].get('architecture')})"
            info["blas_threads_default"] = b[0].get("num_threads")
    except Exception:
        pass
    return info


def cpu_baseline_rfheis(jobs_all):
    """The oracle (dense LAPACK recursion via NumPy, as it stands) on a bounded sample of
    the 512 chains: the first chain of each k in {32, 48, 64} on all host cores, and the
    k = 32 and k = 48 ones on one thread. A k = 96 chain alone takes minutes on the host
    (three dense 9216 x 9216 eigensolves), so it is left out of the sample; the rate is
    the sample's, not the workload mix's."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import recursion as OR

    first = {}
    for i, j in enumerate(jobs_all):
        first.setdefault(j.k, i)
    info = host_info()
    out = {"kind": "oracle", "unit": "solves/s", **info}
    runs = {}
    for label, ks, threads in (("all_cores", (32, 48, 64), None), ("one_thread", (32, 48), 1)):
        with threadpool_limits(limits=threads):
            used = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
            per = {}
            t0 = time.perf_counter()
            for k in ks:
                s0 = time.perf_counter()
                OR.recurse(jobs_all[first[k]])
                per[str(k)] = time.perf_counter() - s0
            dt = time.perf_counter() - t0
        runs[label] = {"value": len(ks) / dt, "cores": used, "seconds": dt,
                       "chains": [first[k] for k in ks], "seconds_per_chain_by_k": per}
    out.update({"value": runs["all_cores"]["value"], "cores": runs["all_cores"]["cores"],
                "sample": "chains " + ", ".join(str(first[k]) for k in (32, 48, 64)) +
                          " of the 512 (the first with k = 32, 48, 64; one whole recursion each; "
                          "k = 96 left out: one such chain takes minutes on the host)",
                "one_thread": runs["one_thread"], "all_cores": runs["all_cores"]})
    return out


# ---- workloads ---------------------------------------------------------------------------

def bench_rfheis(args, ctx, extras_out):
    """The default line: 512 random-field chains per step."""
    from paper_2609_02394_amd import rmc, workloads as W

    jobs_all = W.rfheis_batch(512)
    jobs = [rmc.job_chain(j) for j in jobs_all]
    qs = [j.q for j in jobs_all]
    # FP64 references: the GPU's FP64 path for all chains, checked against the oracle's
    # stored energies on the golden subset
    e64, st64, _ = ctx.recurse_batch(jobs, opts=rmc.default_opts(precision=0))
    assert all(s == 0 for s in st64), "FP64 reference batch failed"
    refs = [e64[i, : qs[i]] for i in range(len(jobs))]
    gold = read_golden(GOLDEN_RFHEIS)
    gold_err = 0.0
    for name, (k, q, E) in gold.items():
        i = int(name.split(":")[1])
        gold_err = max(gold_err, rel_err(refs[i], E))
    assert not gold or gold_err <= 1e-10, f"FP64 path vs oracle golden {gold_err}"
    opts = rmc.default_opts(precision=PREC[args.precision], max_degree=args.max_degree)
    meas, table, ktab = timed_batches(ctx, jobs, refs, opts, args.steps, args.warmup, qs)
    oracle_err = max((rel_err(refs[int(n.split(":")[1])], E) for n, (_, _, E) in gold.items()),
                     default=None)
    # the other precision forms of the same batch, after the timed region (same gate)
    forms = {}
    if not args.no_extras:
        for name, steps in (("bf16", 3), ("fp32", 3), ("fp64", 2)):
            if name == args.precision:
                continue
            o = rmc.default_opts(precision=PREC[name], max_degree=args.max_degree)
            m, t, kt = timed_batches(ctx, jobs, refs, o, steps, 1, qs)
            m["roofline"] = roofline(t, "rfheis512")
            m["kron_by_kernel"] = kt
            forms[f"rfheis512_{name}"] = m
    plain = None
    if not args.no_plain:
        idx = list(range(0, 512, 16))  # 32 chains, every k
        plain = plain_per_job(ctx, [jobs[i] for i in idx], [refs[i] for i in idx],
                              [qs[i] for i in idx])
        plain["sample"] = "chains 0, 16, ..., 496 (32 of the 512)"
    config = {"workload": "512 random-field Heisenberg chains N=32, J=1, h_i~U[-2,2] seeded per "
                          "chain, 8-site leaves (dense 256 ED), k per chain from {32,48,64,96}, "
                          "3 bond ops per cut, lowest 8; every chain solved once per step, all "
                          "modules of a tree level across all chains in batched launches",
              "precision": args.precision, "form": "batched levels",
              "max_rel_err_vs_fp64": meas["max_rel_err"],
              "fp64_path_vs_oracle_golden": {"chains": len(gold), "max_rel_err": oracle_err},
              "jobs_per_step": meas["jobs_per_step"], "accurate_solves": meas["accurate_solves"]}
    return meas, table, ktab, config, plain, (lambda: cpu_baseline_rfheis(jobs_all)), forms


def bench_chain_batch(args, ctx, job, batch, golden=None):
    """`batch` copies of one chain job per step."""
    from paper_2609_02394_amd import rmc

    chain = rmc.job_chain(job)
    ref, _ = ctx.recurse(*chain, opts=rmc.default_opts(precision=0))
    gerr = rel_err(ref, golden) if golden is not None else None
    assert gerr is None or gerr <= 1e-10, f"FP64 path vs oracle golden {gerr}"
    opts = rmc.default_opts(precision=PREC[args.precision], max_degree=args.max_degree)
    jobs = [chain] * batch
    meas, table, ktab = timed_batches(ctx, jobs, [ref] * batch, opts, args.steps, args.warmup,
                                      [job.q] * batch)
    meas["fp64_path_vs_oracle_golden"] = gerr
    return meas, table, ktab, ref


def serve_run(ctx, precision, rate, n_jobs, warm, check_every=8):
    """Open-loop Poisson stream through rmc_submit / rmc_poll: achieved rate, p50/p99
    latency (submission to completion) of the measured jobs, and accuracy against the
    FP64 per-job path on a sample."""
    import threading

    import numpy as np

    from paper_2609_02394_amd import rmc, workloads as W

    stream = W.serving_stream(warm + n_jobs, rate=rate)
    sample = list(range(warm, warm + n_jobs, check_every))
    refs = {i: ctx.recurse(*rmc.job_chain(stream[i][1]))[0] for i in sample}
    ctx.serve_start(opts=rmc.default_opts(precision=precision), max_inflight=64)
    ids = [None] * len(stream)
    t0 = time.perf_counter()

    def feeder():
        for i, (t, job) in enumerate(stream):
            d = t - (time.perf_counter() - t0)
            if d > 0:
                time.sleep(d)
            ids[i] = ctx.submit(*rmc.job_chain(job))

    th = threading.Thread(target=feeder)
    th.start()
    res, t_done = {}, {}
    try:
        while len(res) < len(stream):
            for i, (t, job) in enumerate(stream):
                if i in res or ids[i] is None:
                    continue
                done, e, st, lat = ctx.poll(ids[i], job.q)
                if done:
                    res[i] = (e, st, lat)
                    t_done[i] = time.perf_counter() - t0
            time.sleep(0.0005)
    finally:
        th.join()
        ctx.serve_stop()
    meas = list(range(warm, len(stream)))
    lat = np.array([res[i][2] for i in meas])
    ok = sum(res[i][1] == 0 for i in meas)
    errs = [rel_err(res[i][0], refs[i]) for i in sample]
    span = max(t_done[i] for i in meas) - stream[warm][0]
    offered = n_jobs / max(stream[-1][0] - stream[warm][0], 1e-9)
    # the rate is sustained when the server keeps up (completions at >= 90% of the
    # offered rate) and the queue does not grow (the last quarter of the jobs waits not
    # much longer than the first)
    q = max(1, len(lat) // 4)
    first, last = float(np.median(lat[:q])), float(np.median(lat[-q:]))
    return {"rate_offered_per_s": rate, "offered_measured_per_s": offered, "value": ok / span,
            "unit": "solves/s", "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "jobs": n_jobs, "warmup_jobs": warm,
            "completed_ok": int(ok), "median_latency_first_quarter_ms": first,
            "median_latency_last_quarter_ms": last,
            "sustained": bool(ok / span >= 0.9 * offered and last <= 2.0 * first + 50.0),
            "max_rel_err_sample": max(errs), "sample_size": len(sample)}


def extras(args, ctx):
    """The other workloads, short runs, as extra keys of the line."""
    import numpy as np

    from paper_2609_02394_amd import rmc, workloads as W

    out = {}
    ns = argparse.Namespace(**vars(args))
    ns.steps, ns.warmup = 5, 1
    t0 = time.perf_counter()
    # XXZ chain N=64, k=64: 32 jobs per step, and one job at a time (FP32 and plain FP64)
    job = W.xxz_chain64()
    m, table, ktab, ref = bench_chain_batch(ns, ctx, job, 32)
    m["roofline"] = roofline(table, "xxz64")
    m["workload"] = "open XXZ chain N=64, J=1, Delta=1, 8-site leaves, k=64, 3 bond ops, lowest 8"
    out["xxz64_batch32"] = m
    chain = rmc.job_chain(job)
    fp32 = rmc.default_opts(precision=PREC[args.precision])
    lat = []
    for _ in range(6):
        s0 = time.perf_counter()
        e, _ = ctx.recurse(*chain, opts=fp32)
        lat.append(time.perf_counter() - s0)
    lat = np.array(lat[1:]) * 1e3
    out["xxz64_single_job"] = {"value": 1e3 / float(np.mean(lat)), "unit": "solves/s",
                               "p50_ms": float(np.percentile(lat, 50)),
                               "p99_ms": float(np.percentile(lat, 99)),
                               "max_rel_err": rel_err(e, ref),
                               "plain_per_job_fp64": plain_per_job(ctx, [chain], [ref], [job.q], 3)}
    # TFIM ladder 2x48, k = 128
    lad = W.tfim_ladder96()
    gold = read_golden(GOLDEN_LADDER).get("ladder96")
    ns.steps = 3
    m, table, ktab, ref = bench_chain_batch(ns, ctx, lad, 8, gold[2] if gold else None)
    m["roofline"] = roofline(table, "ladder96")
    m["workload"] = ("TFIM ladder 2x48, J_leg=1, J_rung=0.5, h=0.9, 2x4 leaves, k=128, 2 bond ops "
                     "per cut, lowest 8; 8 jobs per step")
    m["plain_per_job_fp64"] = plain_per_job(ctx, [rmc.job_chain(lad)], [ref], [lad.q], 1)
    out["ladder96"] = m
    # serving: the seeded Poisson stream at the configured 200 jobs/s, and a lower rate
    srv = {}
    for rate in (200.0, 60.0):
        srv[f"rate_{int(rate)}"] = serve_run(ctx, PREC[args.precision], rate, 200, 40)
    srv["workload"] = ("Poisson arrivals, open XXZ or TFIM chains N in {16,32,64,128}, Delta or "
                       "h ~ U[0.5,1.5], 8-site leaves, k in {32,64,128}, lowest 4-8; 40 warm-up "
                       "and 200 measured jobs per rate")
    out["serve"] = srv
    out["seconds"] = time.perf_counter() - t0
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=list(PREC), default="fp32",
                    help="precision of the Kronecker matvecs of the filter (Rayleigh-Ritz, "
                         "CholeskyQR2, residuals and the defect correction stay FP64)")
    ap.add_argument("--workload", choices=["rfheis512", "xxz64", "ladder96"], default="rfheis512",
                    help="rfheis512: 512 random-field chains per step (the metric's workload); "
                         "xxz64: XXZ N=64 k=64, --batch jobs per step; ladder96: TFIM ladder "
                         "2x48 k=128, --batch jobs per step")
    ap.add_argument("--batch", type=int, default=32, help="jobs per step for xxz64 / ladder96")
    ap.add_argument("--mode", choices=["recurse", "serve", "bound"], default="recurse")
    ap.add_argument("--jobs", type=int, default=200, help="serve mode: measured jobs")
    ap.add_argument("--rate", type=float, default=200.0, help="serve mode: arrivals per second")
    ap.add_argument("--max-degree", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    # the device arena, sized for the MI355X's 288 GB: at 128 GB every merge of a
    # random-field level fits one memory chunk (32 GB split the first level in two)
    ap.add_argument("--arena-gb", type=float, default=128.0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain 256 MiB device copy (scales HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU (the path is measured on one "
                                   "GPU's share); --gpus must be 1", "n_gpus": args.gpus}))
        sys.exit(2)
    use_tune_file()

    import torch

    from paper_2609_02394_amd import rmc, workloads as W

    ctx = rmc.Context(arena_bytes=int(args.arena_gb * (1 << 30)))
    if args.calibrate_copy:  # a copy kernel of known size for HBM counter scaling
        src = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.mode == "serve":
        r = serve_run(ctx, PREC[args.precision], args.rate, args.jobs, max(0, args.warmup))
        print(json.dumps({"metric": METRIC, "n_gpus": 1, "higher_is_better": True,
                          "data": "synthetic", **r}))
        ctx.close()
        return
    if args.mode == "bound":
        bound_bench(args, ctx)
        ctx.close()
        return

    cpu_fn, plain, forms = None, None, {}
    if args.workload == "rfheis512":
        meas, table, ktab, config, plain, cpu_fn, forms = bench_rfheis(args, ctx, None)
    else:
        job = W.xxz_chain64() if args.workload == "xxz64" else W.tfim_ladder96()
        gold = read_golden(GOLDEN_LADDER).get("ladder96") if args.workload == "ladder96" else None
        meas, table, ktab, ref = bench_chain_batch(args, ctx, job, max(1, args.batch),
                                                   gold[2] if gold else None)
        if not args.no_plain:
            plain = plain_per_job(ctx, [rmc.job_chain(job)], [ref], [job.q], 3)
        config = {"workload": ("open XXZ chain N=64, J=1, Delta=1, 8-site leaves, k=64, 3 bond "
                               "ops per cut, lowest 8" if args.workload == "xxz64" else
                               "TFIM ladder 2x48, J_leg=1, J_rung=0.5, h=0.9, 2x4 leaves, k=128, "
                               "2 bond ops per cut, lowest 8"),
                  "precision": args.precision, "form": "batched levels",
                  "jobs_per_step": meas["jobs_per_step"],
                  "max_rel_err_vs_fp64": meas["max_rel_err"],
                  "fp64_path_vs_oracle_golden": meas.get("fp64_path_vs_oracle_golden")}
    roof = roofline(table, args.workload)
    ext = None if args.no_extras else {**forms, **extras(args, ctx)}
    cpu = None
    if not args.no_cpu_baseline and cpu_fn is not None:
        cpu = cpu_fn()
    out = {
        "metric": METRIC, "value": meas["value"], "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": meas["ms_per_step"],
        "p50_ms": meas["p50_ms"], "p99_ms": meas["p99_ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32+f64", "bf16": "bf16+f64"}[args.precision],
        "data": "synthetic", "config": config, "roofline": roof, "kron_by_kernel": ktab,
        "plain_per_job_fp64": plain, "cpu_baseline": cpu, "extras": ext,
    }
    print(json.dumps(out))
    ctx.close()


def bound_bench(args, ctx):
    """Single-merge truncation diagnostics (a, ||PHQ||, lambda_min(QHQ), gamma, r, E0) of
    the open TFIM chain L = 20 as two ten-site leaves, J = 1, g = 0.7, k = 8: a step is
    one rmc_merge_bound call on the two leaf modules (built once). Checked against the
    free-fermion ground energy and the stored oracle values of the same merge."""
    import numpy as np

    from oracle import exact as OX
    from paper_2609_02394_amd import rmc, spin_models as SM, workloads as W

    k, L, nA = 8, 20, 10
    job = W.ChainJob("tfim", L, nA, k, 1, J=1.0, h=0.7)
    tA, tB = SM.block_terms(job, 0, nA), SM.block_terms(job, nA, L)
    A = ctx.module_ed(nA, tA, k)
    B = ctx.module_ed(L - nA, tB, k)
    cut = [(c, ops) for c, ops in SM.chain_terms(job) if len(ops) == 2 and ops[0][0] < nA <= ops[1][0]]
    opA = A.project_ops([o[0][0] for _, o in cut], [o[0][1] for _, o in cut])
    opB = B.project_ops([o[1][0] - nA for _, o in cut], [o[1][1] for _, o in cut])
    coefs = [c for c, _ in cut]

    def step():
        return ctx.merge_bound(A, tA, B, tB, coefs, opA, opB)

    for _ in range(max(1, args.warmup)):
        step()
    e0 = float(OX.tfim_free_fermion(L, 1.0, 0.7, 1)[0])
    gold = None
    gp = os.path.join(ROOT, "tests", "golden", "merge_bounds_tfim20.txt")
    for line in open(gp):
        if line.strip() and not line.startswith("#") and int(line.split()[0]) == k:
            gold = [float(x) for x in line.split()[3:]]
    steps = max(1, min(args.steps, 5))
    lat, ok, d = [], 0, None
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        s0 = time.perf_counter()
        d = step()
        lat.append(time.perf_counter() - s0)
        good = abs(d["E0"] - e0) <= 1e-10 * abs(e0) and gold is not None and \
            abs(d["a"] - gold[0]) <= 1e-10 * abs(gold[0]) and abs(d["b"] - gold[1]) <= 1e-10 and \
            abs(d["c"] - gold[2]) <= 1e-10 * abs(gold[2])
        ok += bool(good)
    total = time.perf_counter() - t0
    pr = ctx.profile_read(rmc.FP64, kernel=rmc.PROF_PAULI)
    ctx.profile(False)
    sec = pr["ms"] * 1e-3
    gbs = pr["bytes"] / sec / 1e9 if sec > 0 else 0.0
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import bounds as OB
        c0 = time.perf_counter()
        OB.merge_bound_sparse(job, nA, k)
        cs = time.perf_counter() - c0
        cpu = {"value": 1.0 / cs, "unit": "diagnostics/s", "cores": os.cpu_count() or 1,
               "kind": "oracle", "sample": "one whole diagnostic of the same merge (retained-space "
                                           "b, ARPACK Lanczos on scipy sparse H for E0 and c)",
               "seconds": cs}
    lat_ms = np.array(lat) * 1e3
    out = {
        "metric": "single-merge truncation diagnostics/s (a, ||PHQ||_2, lambda_min(QHQ), r, E0)",
        "value": ok / total, "unit": "diagnostics/s", "n_gpus": 1, "steps": steps,
        "warmup": max(1, args.warmup), "ms_per_step": total / steps * 1e3,
        "p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99)),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "open TFIM chain L=20 = 10 + 10 leaves, J=1, g=0.7, k=8, one "
                               "rmc_merge_bound per step", "checked_ok": ok, "last": d},
        "roofline": {"bound": "hbm", "kernel": "pauli_batched_kernel", "achieved": gbs,
                     "peak": HBM_GBS, "unit": "GB/s", "frac": gbs / HBM_GBS, "traffic": None,
                     "launches": pr["launches"],
                     "avg_launch_us": pr["ms"] * 1e3 / max(1, pr["launches"]),
                     "bytes_per_launch": pr["bytes"] / max(1, pr["launches"]),
                     "ms_per_step": pr["ms"] / steps},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
