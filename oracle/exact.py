"""Independent exact references for the oracle (not the recursion itself).

* brute-force ED of the whole system (the paper's ED reference for L=10, Sec. III);
* open transverse-field Ising chain by Jordan-Wigner free fermions (the "exact
  free-fermion reference" of Secs. III-IV; textbook Lieb-Schultz-Mattis / Pfeuty
  solution): H = -J sum Z_i Z_{i+1} - h sum X_i has single-particle energies
  eps_m = singular values of the N x N lower-bidiagonal matrix with diagonal 2h
  and subdiagonal 2J; E(n) = sum_m eps_m (n_m - 1/2) over every occupation
  n in {0,1}^N (no parity constraint for the open chain);
* open XX chain H = J sum (Sx Sx + Sy Sy): hopping J/2, eps_m = J cos(m pi/(N+1)),
  m = 1..N, E(n) = sum_m n_m eps_m.
"""
from __future__ import annotations

import heapq

import numpy as np

from . import hamiltonian as ham


def brute_energies(job, q):
    """Lowest q eigenvalues of the dense 2^N Hamiltonian (N <= 14)."""
    if job.n_sites > 14:
        raise ValueError("brute-force ED limited to N <= 14")
    return np.linalg.eigvalsh(ham.full_hamiltonian(job))[:q]


def lowest_subset_sums(costs, q):
    """The q smallest values of sum_{m in S} costs[m] over all subsets S, for
    non-negative costs, ascending (best-first enumeration)."""
    c = np.sort(np.asarray(costs, dtype=float))
    if np.any(c < 0):
        raise ValueError("costs must be non-negative")
    out = [0.0]
    if len(c) == 0:
        return np.array(out[:q])
    heap = [(c[0], 0, 0)]  # (sum, largest index, tiebreak)
    tie = 1
    while len(out) < q and heap:
        s, i, _ = heapq.heappop(heap)
        out.append(s)
        if i + 1 < len(c):
            heapq.heappush(heap, (s + c[i + 1], i + 1, tie)); tie += 1
            heapq.heappush(heap, (s - c[i] + c[i + 1], i + 1, tie)); tie += 1
    return np.array(out[:q])


def tfim_single_particle(N, J, h):
    B = np.diag(np.full(N, 2.0 * h)) + np.diag(np.full(N - 1, 2.0 * J), -1)
    return np.linalg.svd(B, compute_uv=False)


def tfim_free_fermion(N, J, h, q):
    """Lowest q energies of the open TFIM chain -J sum ZZ - h sum X."""
    eps = tfim_single_particle(N, J, h)
    return -0.5 * eps.sum() + lowest_subset_sums(eps, q)


def xx_free_fermion(N, J, q):
    """Lowest q energies of the open XX chain J sum (Sx Sx + Sy Sy)."""
    m = np.arange(1, N + 1)
    eps = J * np.cos(m * np.pi / (N + 1))
    e0 = np.minimum(eps, 0.0).sum()
    return e0 + lowest_subset_sums(np.abs(eps), q)
