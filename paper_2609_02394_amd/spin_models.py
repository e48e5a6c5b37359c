"""Term lists of the spin models, as handed to librmc (rmc_term arrays).

A term is (coef, ((site, op), ...)) with op in {"X", "T", "Z"}: X = sigma^x,
Z = sigma^z, T = -i sigma^y (real), so sigma^y sigma^y = -T T. Spin-1/2 operators
are S = sigma / 2.

Canonical order (also the accumulation order of each leaf Hamiltonian): two-site
terms first, by site pair (s, t), s < t, lexicographically, each pair in the
order XX, TT, ZZ; then one-site terms by site.

Models (parameters from ``workloads.ChainJob``):
  tfim        : -J Z_s Z_{s+1}, -h X_s                   (the paper's Sec. III TFIM)
  xxz         : J/4 XX - J/4 TT + J Delta/4 ZZ per bond  (J (SxSx + SySy + Delta SzSz))
  rfheis      : J/4 XX - J/4 TT + J/4 ZZ per bond, h_s/2 Z_s   (J S.S + h_s Sz_s)
  tfim_ladder : spins s = 2x + y; legs (s, s+2) -J ZZ, rungs (2x, 2x+1) -J_rung ZZ,
                fields -h X_s
  tfim_nnn    : -J Z_s Z_{s+1}, -j2 Z_s Z_{s+2}, -h X_s
"""
from __future__ import annotations

from typing import List, Tuple

Term = Tuple[float, Tuple[Tuple[int, str], ...]]


def _pairs(job) -> List[Tuple[int, int]]:
    n = job.n_sites
    if job.model == "tfim_ladder":
        out = [(s, s + 1) for s in range(0, n, 2)] + [(s, s + 2) for s in range(n - 2)]
        return sorted(out)
    if job.model == "tfim_nnn":
        return sorted([(s, s + 1) for s in range(n - 1)] + [(s, s + 2) for s in range(n - 2)])
    return [(s, s + 1) for s in range(n - 1)]


def _pair_terms(job, s, t):
    m = job.model
    if m == "tfim":
        return [(-job.J, "Z", "Z")]
    if m == "tfim_ladder":
        return [(-job.J if t - s == 2 else -job.j_rung, "Z", "Z")]
    if m == "tfim_nnn":
        return [(-job.J if t - s == 1 else -job.j2, "Z", "Z")]
    if m == "xxz":
        return [(0.25 * job.J, "X", "X"), (-0.25 * job.J, "T", "T"),
                (0.25 * job.J * job.delta, "Z", "Z")]
    if m == "rfheis":
        return [(0.25 * job.J, "X", "X"), (-0.25 * job.J, "T", "T"), (0.25 * job.J, "Z", "Z")]
    raise ValueError(m)


def _site_terms(job, s):
    if job.model in ("tfim", "tfim_ladder", "tfim_nnn"):
        return [(-job.h, "X")]
    if job.model == "rfheis":
        return [(0.5 * job.fields[s], "Z")]
    return []


def chain_terms(job) -> List[Term]:
    """Global canonical term list of a ChainJob."""
    out: List[Term] = []
    for s, t in _pairs(job):
        for c, a, b in _pair_terms(job, s, t):
            out.append((c, ((s, a), (t, b))))
    for s in range(job.n_sites):
        for c, o in _site_terms(job, s):
            out.append((c, ((s, o),)))
    return out


def block_terms(job, a, b) -> List[Term]:
    """Terms lying inside the sites [a, b), with sites shifted to 0..b-a-1."""
    out = []
    for c, ops in chain_terms(job):
        if all(a <= s < b for s, _ in ops):
            out.append((c, tuple((s - a, o) for s, o in ops)))
    return out
