"""Writes merge_bounds_tfim20.txt: single-merge diagnostics of the open TFIM chain,
L = 20 as two ten-site leaves, J = 1, g = 0.7 (the paper's bound validation, App. on
the error bounds), through the oracle's sparse full-space route only.

    python tests/golden/make_merge_bounds.py
"""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

from oracle import bounds as BD  # noqa: E402
from paper_2609_02394_amd.workloads import ChainJob  # noqa: E402

KS = (2, 4, 8, 16)


def main():
    job = ChainJob(model="tfim", n_sites=20, leaf_sites=10, k=4, q=1, J=1.0, h=0.7)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "merge_bounds_tfim20.txt")
    lines = ["# open TFIM, L = 20 = 10 + 10, J = 1, g = 0.7; oracle.bounds.merge_bound_sparse",
             "# k kA kB a b c E0"]
    for k in KS:
        d = BD.merge_bound_sparse(job, 10, k)
        lines.append(f"{k} {d.kA} {d.kB} {d.a:.17g} {d.b:.17g} {d.c:.17g} {d.E0:.17g}")
        print(lines[-1], flush=True)
    open(out, "w").write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
