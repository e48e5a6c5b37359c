"""Spin-model Hamiltonians for the oracle, as term lists and dense FP64 matrices.

Conventions (the paper is silent on them; both implementations follow the same
reading):

* Real operator alphabet {X, T, Z}: X = sigma^x, Z = sigma^z and
  T = -i sigma^y = [[0, -1], [1, 0]], so that sigma^y (x) sigma^y = -T (x) T and
  every Hamiltonian here is a real symmetric matrix.
* Site j of an L-site block is kron factor j counted from the left, i.e. bit
  (L-1-j) of the basis index; bit value 0 is sigma^z = +1.
* Ladder spins are numbered s = 2*x + y (x = column, y = leg).
* Canonical term order (which is also the accumulation order of a dense block
  Hamiltonian): all two-site terms first, ordered by the site pair (s, t), s < t,
  lexicographically, each pair expanding in the order XX, TT, ZZ; then all
  one-site terms by site.

Models (J, h, Delta, fields as in ``ChainJob``):
  tfim        : H = -J sum Z_s Z_{s+1} - h sum X_s        (Sec. III, TFIM)
  xxz         : H = J sum (Sx Sx + Sy Sy + Delta Sz Sz), S = sigma/2
                  = sum (J/4) XX - (J/4) TT + (J Delta/4) ZZ
  rfheis      : H = J sum S_s . S_{s+1} + sum h_s Sz_s
  tfim_ladder : H = -J sum_legs ZZ - J_rung sum_rungs ZZ - h sum X
  tfim_nnn    : H = -J sum Z_s Z_{s+1} - j2 sum Z_s Z_{s+2} - h sum X_s
"""
from __future__ import annotations

from functools import reduce

import numpy as np

PAULI = {
    "I": np.eye(2),
    "X": np.array([[0.0, 1.0], [1.0, 0.0]]),
    "T": np.array([[0.0, -1.0], [1.0, 0.0]]),
    "Z": np.array([[1.0, 0.0], [0.0, -1.0]]),
}


def bonds(job):
    """Bonded site pairs (s, t), s < t, in lexicographic order."""
    n = job.n_sites
    if job.model == "tfim_nnn":
        pairs = [(s, s + 1) for s in range(n - 1)] + [(s, s + 2) for s in range(n - 2)]
        return sorted(pairs)
    if job.model == "tfim_ladder":
        out = []
        for s in range(n):
            x, y = divmod(s, 2)
            if y == 0:
                out.append((s, s + 1))          # rung
            if s + 2 < n:
                out.append((s, s + 2))          # leg
        return sorted(out)
    return [(s, s + 1) for s in range(n - 1)]


def bond_terms(job, s, t):
    """Terms of the bond (s, t) as (coef, op_s, op_t), in the order XX, TT, ZZ."""
    if job.model == "tfim":
        return [(-job.J, "Z", "Z")]
    if job.model == "tfim_ladder":
        if t - s == 2:
            return [(-job.J, "Z", "Z")]
        return [(-job.j_rung, "Z", "Z")]
    if job.model == "tfim_nnn":
        return [(-job.J if t - s == 1 else -job.j2, "Z", "Z")]
    if job.model == "xxz":
        return [(0.25 * job.J, "X", "X"), (-0.25 * job.J, "T", "T"),
                (0.25 * job.J * job.delta, "Z", "Z")]
    if job.model == "rfheis":
        return [(0.25 * job.J, "X", "X"), (-0.25 * job.J, "T", "T"),
                (0.25 * job.J, "Z", "Z")]
    raise ValueError(job.model)


def site_terms(job, s):
    """One-site terms at site s as (coef, op)."""
    if job.model in ("tfim", "tfim_ladder", "tfim_nnn"):
        return [(-job.h, "X")]
    if job.model == "rfheis":
        return [(0.5 * job.fields[s], "Z")]
    return []


def block_terms(job, a, b):
    """Canonical term list of the block of sites [a, b): bonds with both ends in
    the block, then fields. Each term is (coef, ((site, op), ...)) with global
    site numbers."""
    out = []
    for (s, t) in bonds(job):
        if a <= s and t < b:
            for c, os_, ot in bond_terms(job, s, t):
                out.append((c, ((s, os_), (t, ot))))
    for s in range(a, b):
        for c, o in site_terms(job, s):
            out.append((c, ((s, o),)))
    return out


def cut_terms(job, a, m, b):
    """Bond terms crossing the cut between A = [a, m) and B = [m, b), as
    (coef, site_in_A, op_A, site_in_B, op_B) with global sites, canonical order."""
    out = []
    for (s, t) in bonds(job):
        if a <= s < m <= t < b:
            for c, os_, ot in bond_terms(job, s, t):
                out.append((c, s, os_, t, ot))
    return out


def site_operator(n_local, j, op):
    """Dense 2^n x 2^n matrix of a one-site operator at local site j."""
    return reduce(np.kron, [PAULI[op] if i == j else PAULI["I"] for i in range(n_local)])


def term_matrix(n_local, local_ops):
    """Dense matrix of a product of one-site operators {local_site: op}."""
    return reduce(np.kron, [PAULI[local_ops.get(i, "I")] for i in range(n_local)])


def block_hamiltonian(job, a, b):
    """Dense FP64 Hamiltonian of the sites [a, b), accumulated term by term from
    +0.0 in canonical order (the leaf-module Hamiltonian of Algorithm 1)."""
    n = b - a
    H = np.zeros((2 ** n, 2 ** n))
    for c, ops in block_terms(job, a, b):
        H = H + c * term_matrix(n, {s - a: o for s, o in ops})
    return H


def full_hamiltonian(job):
    """Dense Hamiltonian of the whole system (brute-force reference)."""
    return block_hamiltonian(job, 0, job.n_sites)
