#!/usr/bin/env python3
"""Benchmark: coupled eigensolves/s of the recursive module-coupling eigensolver.

A step is one whole recursion (leaf ED, projections, every coupling step with its
Kronecker-sum eigensolve, edge-operator transforms) of the open XXZ chain N=64,
J=1, Delta=1, 8-site leaves (dense 256-dim ED), k=64 (coupled space 4096), three
bond operators per cut, lowest 8 states, on synthetic parameters. Only steps whose
8 energies match the FP64 reference to |dE|/max(|E|,1) <= 1e-8 count as solves.

Prints one JSON line with the metric, p50/p99 step latency, the roofline of the
dominant kernel (the Kronecker matvec, timed with HIP events on the library's
stream inside the timed region) and the CPU oracle timed on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# Kronecker kernel variants measured on MI355X for the benchmark shapes (the
# autotuner's cache format); used through a private copy so that runs do not edit it.
TUNE_FILE = os.path.join(ROOT, "paper_2609_02394_amd", "kron_tune_gfx950.txt")


def use_tune_file():
    if "RMC_TUNE_CACHE" in os.environ or not os.path.exists(TUNE_FILE):
        return
    import shutil
    import tempfile

    fd, path = tempfile.mkstemp(prefix="rmc_tune_", suffix=".txt")
    os.close(fd)
    shutil.copyfile(TUNE_FILE, path)
    os.environ["RMC_TUNE_CACHE"] = path

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}
HBM_GBS = 8000.0
PREC = {"fp64": 0, "fp32": 1, "bf16": 2}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "kron_traffic.json")


def kron_source_hash() -> str:
    p = os.path.join(ROOT, "paper_2609_02394_amd", "csrc", "kron.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def cpu_baseline(job):
    """The oracle (dense LAPACK recursion) on the host cores, one whole job."""
    import numpy as np
    from oracle import recursion as OR

    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    t0 = time.perf_counter()
    res = OR.recurse(job)
    dt = time.perf_counter() - t0
    return np.asarray(res.energies), dt, threads


KERNELS = {0: "kron_stream_kernel", 1: "kron_filter_kernel"}


def measured_traffic(kernel: str, prec: str):
    """HBM bytes per launch of a Kronecker kernel from committed rocprofv3 counter runs
    (scaled by a copy kernel of known size), if taken on the current kernel source."""
    try:
        d = json.load(open(TRAFFIC_FILE))
    except Exception:
        return None
    if d.get("kron_source_sha") != kron_source_hash():
        return None
    return d.get("bytes_per_launch", {}).get(f"{kernel}:{prec}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=list(PREC), default="fp32",
                    help="precision of the Kronecker matvecs (Rayleigh-Ritz, CholQR2, "
                         "residuals and the defect correction stay FP64)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--arena-gb", type=float, default=8.0)
    ap.add_argument("--mode", choices=["recurse", "serve", "bound"], default="recurse",
                    help="recurse: timed recursions of the XXZ N=64 workload; serve: the "
                         "Poisson serving stream through the continuous-batching scheduler; "
                         "bound: single-merge truncation diagnostics of the L=20 TFIM chain")
    ap.add_argument("--workload", choices=["xxz64", "ladder96", "rfheis512"], default="xxz64",
                    help="xxz64: XXZ N=64 k=64 (the metric's configuration); ladder96: TFIM "
                         "ladder 2x48 k=128; rfheis512: 512 random-field Heisenberg chains N=32 "
                         "with k in {32,48,64,96}, all solved as one batch per step")
    ap.add_argument("--jobs", type=int, default=200, help="serve mode: measured jobs")
    ap.add_argument("--rate", type=float, default=200.0, help="serve mode: arrivals per second")
    ap.add_argument("--max-degree", type=int, default=0,
                    help="cap of the Chebyshev degree per outer iteration (0 = library default)")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the plain per-job FP64 comparison run after the timed region")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain 256 MiB device copy (scales HBM counters)")
    ap.add_argument("--batch", type=int, default=32,
                    help="independent jobs of the workload solved together per step "
                         "(batched levels); 1 = the plain per-job recursion")
    args = ap.parse_args()
    use_tune_file()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2609_02394_amd import rmc, workloads as W

    if args.mode == "serve":
        serve_bench(args)
        return
    if args.mode == "bound":
        bound_bench(args)
        return

    if args.workload == "rfheis512":
        batch_bench(args)
        return
    job = W.xxz_chain64() if args.workload == "xxz64" else W.tfim_ladder96()
    chain = rmc.job_chain(job)

    ref = None
    cpu = None
    if not args.no_cpu_baseline and args.workload == "xxz64":
        ref, cpu_s, threads = cpu_baseline(job)
        cpu = {"value": 1.0 / cpu_s, "unit": "solves/s", "cores": threads, "kind": "oracle",
               "sample": "1 whole job of the benchmark workload (dense 256 leaf ED + 3 dense "
                         "4096x4096 eigh merges, LAPACK via NumPy)",
               "seconds": cpu_s}

    ctx = rmc.Context(arena_bytes=int(args.arena_gb * (1 << 30)))
    opts = rmc.default_opts(precision=PREC[args.precision], max_degree=args.max_degree)
    fp64_opts = rmc.default_opts(precision=0)
    if args.calibrate_copy:  # a copy kernel of known size for HBM counter scaling
        src = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if ref is None:  # FP64 GPU path as the reference when the oracle is skipped
        ref, _ = ctx.recurse(*chain, opts=fp64_opts)

    B = max(1, args.batch)

    def step():
        if B == 1:
            e, rep = ctx.recurse(*chain, opts=opts)
            return [e], rep
        e, st, top = ctx.recurse_batch([chain] * B, opts=opts)
        return [e[i, : job.q] if st[i] == 0 else np.full(job.q, np.nan) for i in range(B)], None

    for _ in range(args.warmup):
        step()

    lat = []
    ok = 0
    max_err = 0.0
    rep = None
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        es, r = step()
        rep = r if r is not None else rep
        lat.append(time.perf_counter() - s0)
        for e in es:
            err = float(np.max(np.abs(e - ref) / np.maximum(np.abs(ref), 1.0)))
            max_err = max(max_err, err if err == err else np.inf)
            ok += err <= 1e-8
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    by_prec = {name: ctx.profile_read(PREC[name]) for name in PREC}
    by_kernel = {(kk, name): ctx.profile_read(PREC[name], kernel=kk) for kk in KERNELS for name in PREC}
    ctx.profile(False)

    # the plain per-job FP64 recursion of the same workload, for comparison
    plain = None
    if not args.no_plain:
        for _ in range(2):
            ctx.recurse(*chain, opts=fp64_opts)
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        for _ in range(5):
            ctx.recurse(*chain, opts=fp64_opts)
        torch.cuda.synchronize()
        plain = {"form": "plain per-job FP64 recursion, one job at a time",
                 "value": 5 / (time.perf_counter() - p0), "unit": "solves/s"}

    lat_ms = np.array(lat) * 1e3
    # dominant kernel: the Kronecker kernel kind (one matvec step, or the whole filter)
    # and precision that took most of the Kronecker time
    dk, dom = max(by_kernel, key=lambda k: by_kernel[k]["ms"])
    prof = by_kernel[(dk, dom)]
    kron_table = {}
    for (kk, name), pr in by_kernel.items():
        if pr["launches"] == 0:
            continue
        sec = pr["ms"] * 1e-3
        kron_table[f"{KERNELS[kk]}:{name}"] = {
            "launches": pr["launches"], "ms_per_step": pr["ms"] / args.steps,
            "avg_launch_us": pr["ms"] * 1e3 / pr["launches"],
            "tflops": pr["flops"] / sec / 1e12, "gbs": pr["bytes"] / sec / 1e9,
            "flops_per_launch": pr["flops"] / pr["launches"],
            "bytes_per_launch": pr["bytes"] / pr["launches"]}
    sec = prof["ms"] * 1e-3
    tr = measured_traffic(KERNELS[dk], dom)
    if dom == "bf16":  # HBM-bound: the BF16 MFMA roof lies far above the HBM roof
        achieved = prof["bytes"] / sec / 1e9 if sec > 0 else 0.0
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_GBS, "unit": "GB/s",
                "frac": achieved / HBM_GBS}
    else:
        achieved = prof["flops"] / sec / 1e12 if sec > 0 else 0.0
        peak = PEAK_TFLOPS[dom]
        roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak}
    roof.update({"traffic": tr, "kernel": KERNELS[dk], "precision": dom,
                 "launches": prof["launches"],
                 "avg_launch_us": prof["ms"] * 1e3 / max(1, prof["launches"]),
                 "flops_per_launch": prof["flops"] / max(1, prof["launches"]),
                 "bytes_per_launch": prof["bytes"] / max(1, prof["launches"])})
    out = {
        "metric": "coupled eigensolves/s (lowest 8, rel err<=1e-8 vs FP64)",
        "value": ok / total,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total / args.steps * 1e3,
        "p50_ms": float(np.percentile(lat_ms, 50)),
        "p99_ms": float(np.percentile(lat_ms, 99)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32+f64", "bf16": "bf16+f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": ("open XXZ chain N=64, J=1, Delta=1, 8-site leaves, k=64, "
                                "3 bond ops per cut, lowest 8, one whole recursion per job")
                   if args.workload == "xxz64" else
                   ("TFIM ladder 2x48, J_leg=1, J_rung=0.5, h=0.9, 2x4 leaves, k=128, 2 bond "
                    "ops per cut, lowest 8, one whole recursion per job"),
                   "precision": args.precision, "max_rel_err": max_err,
                   "jobs_per_step": B, "accurate_solves": ok,
                   "form": "per-job recursion" if B == 1 else "batched levels"},
        "roofline": roof,
        "kron_by_kernel": kron_table,
        "plain_per_job_fp64": plain,
        "cpu_baseline": cpu,
        "report_last_step": rep["records"] if rep else None,
    }
    print(json.dumps(out))
    ctx.close()


def batch_bench(args):
    """512 random-field Heisenberg chains (N=32, h_i ~ U[-2,2] seeded per chain, 8-site
    leaves, k in {32,48,64,96}, lowest 8): one step solves all of them as one batch
    (every level of every chain in batched launches). Accuracy: FP64 per-chain
    references for a sample of chains."""
    import numpy as np

    from paper_2609_02394_amd import rmc, workloads as W

    jobs = W.rfheis_batch(512)
    chains = [rmc.job_chain(j) for j in jobs]
    ctx = rmc.Context(arena_bytes=int(max(args.arena_gb, 32.0) * (1 << 30)))
    opts = rmc.default_opts(precision=PREC[args.precision], max_degree=args.max_degree)
    sample = list(range(0, 512, 37))
    refs = {i: ctx.recurse(*chains[i])[0] for i in sample}
    for _ in range(args.warmup):
        ctx.recurse_batch(chains, opts=opts)
    lat, ok, max_err = [], 0, 0.0
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        e, st, top = ctx.recurse_batch(chains, opts=opts)
        lat.append(time.perf_counter() - s0)
        ok += sum(1 for x in st if x == 0)
        for i in sample:
            err = float(np.max(np.abs(e[i] - refs[i]) / np.maximum(np.abs(refs[i]), 1.0)))
            max_err = max(max_err, err)
    total = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.profile(False)
    achieved = prof["flops"] / (prof["ms"] * 1e-3) / 1e12 if prof["ms"] > 0 else 0.0
    peak = PEAK_TFLOPS[args.precision]
    lat_ms = np.array(lat) * 1e3
    out = {
        "metric": "coupled eigensolves/s (lowest 8, rel err<=1e-8 vs FP64), batched levels",
        "value": ok / total if max_err <= 1e-8 else 0.0, "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": total / args.steps * 1e3,
        "p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99)),
        "higher_is_better": True, "data": "synthetic",
        "config": {"workload": "512 random-field Heisenberg chains N=32, W=2, 8-site leaves, "
                               "k in {32,48,64,96}, lowest 8, all chains per step",
                   "precision": args.precision, "max_rel_err_sample": max_err,
                   "sample_size": len(sample)},
        "roofline": {"bound": "mfma", "kernel": "kron_batched_kernel", "achieved": achieved,
                     "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                     "launches": prof["launches"],
                     "avg_launch_us": prof["ms"] * 1e3 / max(1, prof["launches"])},
    }
    print(json.dumps(out))
    ctx.close()


def bound_bench(args):
    """Single-merge truncation diagnostics (a, ||PHQ||, lambda_min(QHQ), gamma, r, E0) of
    the open TFIM chain L = 20 as two ten-site leaves, J = 1, g = 0.7, k = 8: a step is
    one rmc_merge_bound call on the two leaf modules (built once). Checked against the
    free-fermion ground energy and the stored oracle values of the same merge."""
    import numpy as np

    from oracle import exact as OX
    from paper_2609_02394_amd import rmc, spin_models as SM, workloads as W

    k, L, nA = 8, 20, 10
    job = W.ChainJob("tfim", L, nA, k, 1, J=1.0, h=0.7)
    ctx = rmc.Context(arena_bytes=int(args.arena_gb * (1 << 30)))
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
    ctx.close()


def serve_bench(args):
    """Open-loop Poisson stream of XXZ / TFIM jobs (N in {16,32,64,128}, k in
    {32,64,128}, lowest 4-8) through rmc_submit / rmc_poll: throughput, p50/p99
    latency (submission to completion), accuracy vs the FP64 per-job path on a sample."""
    import threading

    import numpy as np

    from paper_2609_02394_amd import rmc, workloads as W

    warm = max(0, args.warmup)
    stream = W.serving_stream(warm + args.jobs, rate=args.rate)
    ctx = rmc.Context(arena_bytes=int(args.arena_gb * (1 << 30)))
    opts = rmc.default_opts(precision=PREC[args.precision])
    # FP64 per-job references for a sample of the measured jobs (accuracy gate)
    sample = list(range(warm, warm + args.jobs, max(1, args.jobs // 8)))
    refs = {i: ctx.recurse(*rmc.job_chain(stream[i][1]))[0] for i in sample}
    ctx.serve_start(opts=opts, max_inflight=64)
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
    res = {}
    t_done = {}
    while len(res) < len(stream):
        for i, (t, job) in enumerate(stream):
            if i in res or ids[i] is None:
                continue
            done, e, st, lat = ctx.poll(ids[i], job.q)
            if done:
                res[i] = (e, st, lat)
                t_done[i] = time.perf_counter() - t0
        time.sleep(0.0005)
    th.join()
    ctx.serve_stop()
    # the plain per-job FP64 recursion over the first measured jobs, one at a time
    plain = None
    if not args.no_plain:
        nplain = min(24, args.jobs)
        p0 = time.perf_counter()
        for i in range(warm, warm + nplain):
            ctx.recurse(*rmc.job_chain(stream[i][1]))
        plain = {"form": "plain per-job FP64 recursion, one job at a time (first jobs of the "
                         "measured stream)", "jobs": nplain,
                 "value": nplain / (time.perf_counter() - p0), "unit": "solves/s"}
    meas = list(range(warm, len(stream)))
    lat = np.array([res[i][2] for i in meas])
    ok = sum(res[i][1] == 0 for i in meas)
    errs = [float(np.max(np.abs(res[i][0] - refs[i]) / np.maximum(np.abs(refs[i]), 1.0)))
            for i in sample]
    span = max(t_done[i] for i in meas) - stream[warm][0]
    out = {
        "metric": "coupled eigensolves/s (lowest 4-8, rel err<=1e-8 vs FP64), serving",
        "value": ok / span, "unit": "solves/s", "n_gpus": 1,
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "higher_is_better": True, "data": "synthetic",
        "config": {"workload": "Poisson stream, XXZ/TFIM N in {16,32,64,128}, 8-site leaves, "
                               "k in {32,64,128}, lowest 4-8", "rate_per_s": args.rate,
                   "jobs": args.jobs, "warmup_jobs": warm, "precision": args.precision,
                   "completed_ok": ok, "offered_span_s": stream[-1][0] - stream[warm][0],
                   "max_rel_err_sample": max(errs), "sample_size": len(sample)},
        "plain_per_job_fp64": plain,
    }
    print(json.dumps(out))
    ctx.close()


if __name__ == "__main__":
    main()
