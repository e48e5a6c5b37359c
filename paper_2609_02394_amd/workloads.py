"""Seeded synthetic workloads for the recursive module-coupling eigensolver.

This module only draws parameters: which spin model, how many sites, how many
sites per leaf module, the retained dimension k, the number of target states q,
coupling constants and random fields, and arrival times for the serving stream.
It holds none of the method's arithmetic and none of the models' Hamiltonian
construction; both the CPU oracle and the GPU path build their Hamiltonians from
these parameters independently.

The spin models are the open transverse-field Ising chain used throughout the
paper's classical section (Sec. III, block Hamiltonian and long-chain TFIM
equations), plus the XXZ chain, the random-field Heisenberg chain and the
transverse-field Ising ladder, which the paper does not treat but which share
its two-module coupling form (Sec. II, two-block Hamiltonian and general
coupling equations), and the TFIM with next-nearest-neighbour ZZ bonds, whose
cuts carry the longer-range terms of the coupling-geometry appendix (App. B).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

MODELS = ("tfim", "xxz", "rfheis", "tfim_ladder", "tfim_nnn")


@dataclass(frozen=True)
class ChainJob:
    """Parameters of one eigensolve job.

    model      : one of MODELS.
    n_sites    : total number of spins (for the ladder: 2 * number of columns).
    leaf_sites : spins per leaf module (for the ladder: 2 * columns per leaf).
    k          : retained dimension per module.
    q          : number of lowest eigenvalues wanted at the root.
    J          : chain / leg coupling.
    h          : transverse field (tfim, tfim_ladder).
    delta      : XXZ anisotropy.
    j_rung     : rung coupling (tfim_ladder).
    fields     : per-site longitudinal random fields (rfheis), length n_sites.
    j2         : next-nearest-neighbour ZZ coupling (tfim_nnn).
    """

    model: str
    n_sites: int
    leaf_sites: int
    k: int
    q: int
    J: float = 1.0
    h: float = 0.0
    delta: float = 1.0
    j_rung: float = 0.0
    fields: Tuple[float, ...] = field(default_factory=tuple)
    j2: float = 0.0

    def __post_init__(self):
        if self.model not in MODELS:
            raise ValueError(f"unknown model {self.model!r}")
        if self.n_sites <= 0 or self.leaf_sites <= 0:
            raise ValueError("n_sites and leaf_sites must be positive")
        if self.n_sites % self.leaf_sites != 0:
            raise ValueError("n_sites must be a multiple of leaf_sites")
        if self.model == "tfim_ladder" and (self.leaf_sites % 2 or self.n_sites % 2):
            raise ValueError("ladder sizes count both legs and must be even")
        if self.model == "rfheis" and len(self.fields) != self.n_sites:
            raise ValueError("rfheis needs one field per site")
        if self.k < 1 or self.q < 1:
            raise ValueError("k and q must be >= 1")

    @property
    def n_leaves(self) -> int:
        return self.n_sites // self.leaf_sites


def tfim_small() -> ChainJob:
    """Open TFIM, N=8, J=1, h=1, 2-site leaves (dim 4), k=8, lowest 4."""
    return ChainJob("tfim", n_sites=8, leaf_sites=2, k=8, q=4, J=1.0, h=1.0)


def xxz_chain64() -> ChainJob:
    """Open XXZ chain N=64, J=1, Delta=1, 8-site leaves, k=64, lowest 8."""
    return ChainJob("xxz", n_sites=64, leaf_sites=8, k=64, q=8, J=1.0, delta=1.0)


def rfheis_batch(n_chains: int = 512, W: float = 2.0) -> List[ChainJob]:
    """Random-field Heisenberg chains N=32, 8-site leaves, fields U[-W, W] seeded
    per chain, k drawn from {32, 48, 64, 96}, lowest 8."""
    ks = np.random.default_rng([2609, 3, 999]).choice([32, 48, 64, 96], size=n_chains)
    jobs = []
    for i in range(n_chains):
        hs = np.random.default_rng([2609, 3, i]).uniform(-W, W, size=32)
        jobs.append(ChainJob("rfheis", n_sites=32, leaf_sites=8, k=int(ks[i]), q=8,
                             J=1.0, fields=tuple(float(x) for x in hs)))
    return jobs


def tfim_nnn(n_sites: int = 24, leaf_sites: int = 4, k: int = 16, q: int = 4,
             J: float = 1.0, h: float = 0.7, gamma: float = 0.2) -> ChainJob:
    """TFIM with next-nearest ZZ bonds of strength gamma*J on every pair (s, s+2):
    each cut carries one nearest and two next-nearest terms, two of them on the
    sites next to the module edges (the longer-range coupling of App. B)."""
    return ChainJob("tfim_nnn", n_sites=n_sites, leaf_sites=leaf_sites, k=k, q=q, J=J, h=h,
                    j2=gamma * J)


def tfim_ladder96() -> ChainJob:
    """TFIM ladder 2x48 (96 spins), J_leg=1, J_rung=0.5, h=0.9, 2x4 leaves,
    k=128, lowest 8."""
    return ChainJob("tfim_ladder", n_sites=96, leaf_sites=8, k=128, q=8,
                    J=1.0, h=0.9, j_rung=0.5)


def serving_stream(n_jobs: int, rate: float = 200.0, seed=(2609, 5)):
    """Poisson arrivals at `rate` jobs/s. Each job is an open XXZ or TFIM chain with
    N in {16, 32, 64, 128}, 8-site leaves, Delta or h ~ U[0.5, 1.5], J=1,
    k in {32, 64, 128}, q in {4..8}. Returns a list of (arrival_seconds, job)."""
    rng = np.random.default_rng(list(seed))
    t = 0.0
    out = []
    for _ in range(n_jobs):
        t += float(rng.exponential(1.0 / rate))
        model = "xxz" if rng.integers(0, 2) == 0 else "tfim"
        n = int(rng.choice([16, 32, 64, 128]))
        par = float(rng.uniform(0.5, 1.5))
        k = int(rng.choice([32, 64, 128]))
        q = int(rng.integers(4, 9))
        if model == "xxz":
            job = ChainJob("xxz", n_sites=n, leaf_sites=8, k=k, q=q, J=1.0, delta=par)
        else:
            job = ChainJob("tfim", n_sites=n, leaf_sites=8, k=k, q=q, J=1.0, h=par)
        out.append((t, job))
    return out


def random_matrix(shape, seed, scale=1.0):
    """Seeded standard-normal test data (used only to feed kernels in tests)."""
    return scale * np.random.default_rng(seed).standard_normal(shape)
