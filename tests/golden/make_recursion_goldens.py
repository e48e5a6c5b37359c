"""Writes the oracle's whole-recursion results at the shapes of the large workloads:

* recursion_ladder96_k128.txt: the TFIM ladder 2x48 (J_leg = 1, J_rung = 0.5,
  h = 0.9, 2x4 leaves, k = 128, lowest 8): four dense 16384 x 16384 eigensolves;
* recursion_rfheis_subset.txt: a seeded subset of the 512 random-field Heisenberg
  chains (N = 32, h_i ~ U[-2, 2], 8-site leaves, k from {32, 48, 64, 96}, lowest 8):
  the first 8 chains of each k, in chain order.

Each job block holds the lowest q energies of the root merge and one record per
computed module (level, width, kind, k_req, k_eff, cut gap), in the oracle's order:
Algorithm 1 run literally with dense LAPACK at every merge (oracle.recursion).
Only the oracle and the seeded parameter generator are used.

    python tests/golden/make_recursion_goldens.py ladder     # about half an hour
    python tests/golden/make_recursion_goldens.py rfheis     # about twenty minutes
"""
import os
import sys
import time

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

from oracle import recursion as OR  # noqa: E402
from paper_2609_02394_amd import workloads as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
PER_K = 8


def rfheis_subset():
    """Indices of the subset: the first PER_K chains of each k value, ascending."""
    jobs = W.rfheis_batch(512)
    out = []
    for k in (32, 48, 64, 96):
        out += [i for i, j in enumerate(jobs) if j.k == k][:PER_K]
    return sorted(out), jobs


def job_block(name, job):
    t0 = time.time()
    res = OR.recurse(job)
    lines = [f"job {name} k={job.k} q={job.q} seconds={time.time() - t0:.1f}",
             "E " + " ".join(f"{x:.17g}" for x in res.energies)]
    for r in res.records:
        lines.append(f"R {r.level} {r.width} {r.kind} {r.k_req} {r.k_eff} {r.gap:.17g}")
    print("\n".join(lines), flush=True)
    return lines


def main(which):
    if which == "ladder":
        head = ["# TFIM ladder 2x48, J_leg=1, J_rung=0.5, h=0.9, 2x4 leaves, k=128, lowest 8",
                "# oracle.recursion.recurse (dense Kronecker-sum H_eff and eigh at every merge)",
                "# E: lowest q energies; R: level width kind k_req k_eff gap, one per computed module"]
        lines = head + job_block("ladder96", W.tfim_ladder96())
        path = os.path.join(HERE, "recursion_ladder96_k128.txt")
    elif which == "rfheis":
        idx, jobs = rfheis_subset()
        lines = ["# random-field Heisenberg N=32, W=2, 8-site leaves, seeded chains "
                 "(workloads.rfheis_batch(512)); the first 8 chains of each k in {32,48,64,96}",
                 "# oracle.recursion.recurse (dense Kronecker-sum H_eff and eigh at every merge)",
                 "# E: lowest q energies; R: level width kind k_req k_eff gap, one per computed module"]
        for i in idx:
            lines += job_block(f"rfheis:{i}", jobs[i])
        path = os.path.join(HERE, "recursion_rfheis_subset.txt")
    else:
        raise SystemExit("usage: make_recursion_goldens.py ladder|rfheis")
    open(path, "w").write("\n".join(lines) + "\n")


def read(path):
    """{name: {"k": k, "q": q, "E": [...], "R": [(level, width, kind, k_req, k_eff, gap)]}}."""
    out, cur = {}, None
    for line in open(path):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue
        if f[0] == "job":
            kv = dict(x.split("=") for x in f[2:])
            cur = out[f[1]] = {"k": int(kv["k"]), "q": int(kv["q"]), "E": [], "R": []}
        elif f[0] == "E":
            cur["E"] = [float(x) for x in f[1:]]
        elif f[0] == "R":
            cur["R"].append((int(f[1]), int(f[2]), f[3], int(f[4]), int(f[5]), float(f[6])))
    return out


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "")
