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


def tree_from_spec(job, spec, k_of=None):
    """Module-tree nodes (the binding's rmc_recurse format) of the sites of `job` split
    and merged as `spec`: a leaf is a site range (a, b); a merge is a pair (left spec,
    right spec) of adjacent ranges, left first. A leaf carries the terms inside its
    range (sites from 0); a merge carries the two-site terms with one site in each
    child, as (coef, site in left, op, site in right, op), each child's sites from 0.
    k_of(width) gives a node's k (default 0: the tree's k)."""
    terms = chain_terms(job)
    nodes = []

    def go(s):
        if isinstance(s[0], int):
            a, b = s
            nodes.append(("leaf", b - a, block_terms(job, a, b), k_of(b - a) if k_of else 0))
            return len(nodes) - 1, a, b
        li, a, m = go(s[0])
        ri, m2, b = go(s[1])
        if m2 != m:
            raise ValueError("children of a merge must be adjacent, left first")
        cut = []
        for c, ops in terms:
            if len(ops) != 2:
                continue
            (s0, o0), (s1, o1) = ops
            if a <= s0 < m <= s1 < b:
                cut.append((c, s0 - a, o0, s1 - m, o1))
            elif a <= s1 < m <= s0 < b:
                cut.append((c, s1 - a, o1, s0 - m, o0))
        nodes.append(("merge", li, ri, cut, k_of(b - a) if k_of else 0))
        return len(nodes) - 1, a, b

    go(spec)
    return nodes


def chain_spec(n_sites, leaf_sites):
    """Spec of the default order on a chain: leaves of leaf_sites consecutive sites
    merged pairwise left to right, an odd module carried up."""
    mods = [(a, a + leaf_sites) for a in range(0, n_sites, leaf_sites)]
    while len(mods) > 1:
        nxt = [(mods[i], mods[i + 1]) for i in range(0, len(mods) - 1, 2)]
        if len(mods) % 2:
            nxt.append(mods[-1])
        mods = nxt
    return mods[0]
