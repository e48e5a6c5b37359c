"""Single-merge truncation diagnostics (Sec. IV, single-merge bound; App. on the
error bounds: block form of H, the discarded-sector gap, the bound r(b, gamma)).

TEST INFRASTRUCTURE ONLY (see the package header).

One merge of two leaf blocks, A = sites [0, nA) and B = [nA, L), each reduced to
its lowest k eigenstates by dense ED with the gap rule:

    W = V_A (x) V_B            retained product states (orthonormal columns)
    P = W W^T,  Q = I - P
    a = lambda_min(P H P)      on range(P)  (the merged module's lowest energy)
    b = || P H Q ||_2
    c = lambda_min(Q H Q)      on range(Q)
    gamma = c - a
    r(b, gamma) = (sqrt(gamma^2 + 4 b^2) - gamma) / 2      (<= b^2 / gamma)
    E0 = lambda_min(H)

The paper's bound is 0 <= a - E0 <= r(b, gamma) whenever gamma > 0.

Three routes, each written from the definitions:

* ``merge_bound_dense``: everything in the full 2^L space with dense matrices
  (range(Q) from the eigenvectors of P with eigenvalue 0); L <= 12.
* ``merge_bound_retained``: a from the effective Hamiltonian of the merge and b from
  b^2 = lambda_max(W^T V Q V W) = lambda_max(W^T V^2 W - (W^T V W)^2), which holds
  because the uncoupled blocks do not connect P and Q, so P H Q = P V Q (App.). No
  full-space object; the leaves set the size limit.
* ``merge_bound_sparse``: E0 and c by Lanczos (ARPACK) on the full-space sparse H,
  c as the lowest eigenvalue of Q H Q + sigma P with sigma = sum |coef| >= ||H||,
  which leaves range(Q)'s spectrum in place and moves range(P) to sigma; L <= ~22.
"""
from __future__ import annotations

from dataclasses import dataclass
from functools import reduce

import numpy as np

from . import hamiltonian as ham
from .recursion import TAU_GAP, couple_solve, leaf_ed, project


@dataclass
class MergeBound:
    a: float
    b: float
    c: float
    gamma: float
    r: float
    b2_over_gamma: float
    E0: float
    kA: int
    kB: int


def r_bound(b, gamma):
    """r(b, gamma) = (sqrt(gamma^2 + 4 b^2) - gamma) / 2, the smaller root's
    distance below a of the 2x2 form [[0, -b], [-b, gamma]] (App., single-merge
    bound equation)."""
    return 0.5 * (np.sqrt(gamma * gamma + 4.0 * b * b) - gamma)


def _finish(a, b, c, E0, kA, kB):
    """range(Q) empty (k covers both leaves): b = 0, c = gamma = inf, r = 0."""
    g = c - a
    if b == 0.0:
        return MergeBound(float(a), 0.0, float(c), float(g), 0.0, 0.0, float(E0), kA, kB)
    return MergeBound(float(a), float(b), float(c), float(g), float(r_bound(b, g)),
                      float(b * b / g) if g > 0 else float("inf"), float(E0), kA, kB)


def leaves(job, nA, k, tau_gap=TAU_GAP):
    """Leaf ED of both blocks: (E_A, V_A, E_B, V_B)."""
    L = job.n_sites
    E_A, V_A, _, _, _ = leaf_ed(ham.block_hamiltonian(job, 0, nA), k, tau_gap)
    E_B, V_B, _, _, _ = leaf_ed(ham.block_hamiltonian(job, nA, L), k, tau_gap)
    return E_A, V_A, E_B, V_B


def coupling_dense(job, nA):
    """V = sum over the bonds cut at nA of coef * (op at s) (op at t), dense 2^L."""
    L = job.n_sites
    V = np.zeros((2 ** L, 2 ** L))
    for c, s, oa, t, ob in ham.cut_terms(job, 0, nA, L):
        V = V + c * ham.term_matrix(L, {s: oa, t: ob})
    return V


def merge_bound_dense(job, nA, k, tau_gap=TAU_GAP):
    """All quantities from their definitions in the full space (dense, L <= 12)."""
    L = job.n_sites
    if L > 12:
        raise ValueError("dense route limited to L <= 12")
    _, V_A, _, V_B = leaves(job, nA, k, tau_gap)
    H = ham.full_hamiltonian(job)
    W = np.kron(V_A, V_B)
    P = W @ W.T
    w, U = np.linalg.eigh(P)
    Wq = U[:, w < 0.5]                       # orthonormal basis of range(Q)
    a = np.linalg.eigvalsh(W.T @ H @ W)[0]
    if Wq.shape[1] == 0:
        b, c = 0.0, float("inf")
    else:
        b = np.linalg.svd(W.T @ H @ Wq, compute_uv=False)[0]
        c = np.linalg.eigvalsh(Wq.T @ H @ Wq)[0]
    E0 = np.linalg.eigvalsh(H)[0]
    return _finish(a, b, c, E0, V_A.shape[1], V_B.shape[1])


def uncoupled_leak(job, nA, k, tau_gap=TAU_GAP):
    """|| P (H_A (x) I + I (x) H_B) Q ||_2 (dense, L <= 12); zero by the App.'s
    argument that the uncoupled blocks keep P and Q apart."""
    L = job.n_sites
    _, V_A, _, V_B = leaves(job, nA, k, tau_gap)
    H0 = (np.kron(ham.block_hamiltonian(job, 0, nA), np.eye(2 ** (L - nA))) +
          np.kron(np.eye(2 ** nA), ham.block_hamiltonian(job, nA, L)))
    W = np.kron(V_A, V_B)
    w, U = np.linalg.eigh(W @ W.T)
    Wq = U[:, w < 0.5]
    return float(np.linalg.svd(W.T @ H0 @ Wq, compute_uv=False)[0])


def retained_b2_matrix(job, nA, V_A, V_B):
    """W^T V Q V W = W^T V^2 W - (W^T V W)^2 in the retained product basis (index
    a * kB + b), from leaf-space operators only."""
    L = job.n_sites
    nB = L - nA
    cut = ham.cut_terms(job, 0, nA, L)
    kA, kB = V_A.shape[1], V_B.shape[1]
    V1 = np.zeros((kA * kB, kA * kB))
    V2 = np.zeros((kA * kB, kA * kB))
    opsA = [ham.site_operator(nA, s, oa) for _, s, oa, _, _ in cut]
    opsB = [ham.site_operator(nB, t - nA, ob) for _, _, _, t, ob in cut]
    for i, (ci, *_r) in enumerate(cut):
        V1 = V1 + ci * np.kron(project(V_A, opsA[i]), project(V_B, opsB[i]))
        for j, (cj, *_s) in enumerate(cut):
            V2 = V2 + ci * cj * np.kron(project(V_A, opsA[i] @ opsA[j]),
                                        project(V_B, opsB[i] @ opsB[j]))
    return V2 - V1 @ V1


def merge_bound_retained(job, nA, k, tau_gap=TAU_GAP):
    """(a, b, kA, kB) without any full-space object."""
    L = job.n_sites
    E_A, V_A, E_B, V_B = leaves(job, nA, k, tau_gap)
    terms = [(c, project(V_A, ham.site_operator(nA, s, oa)),
              project(V_B, ham.site_operator(L - nA, t - nA, ob)))
             for c, s, oa, t, ob in ham.cut_terms(job, 0, nA, L)]
    w, *_ = couple_solve(E_A, E_B, terms, None)
    M = retained_b2_matrix(job, nA, V_A, V_B)
    b2 = max(float(np.linalg.eigvalsh(M)[-1]), 0.0)
    return float(w[0]), float(np.sqrt(b2)), V_A.shape[1], V_B.shape[1]


def sparse_hamiltonian(job):
    """Full-space H as a scipy CSR matrix, term by term as sparse Kronecker
    products of the 2x2 operators (same terms and order as the dense one)."""
    import scipy.sparse as sp
    L = job.n_sites
    I2 = sp.identity(2, format="csr")
    P2 = {o: sp.csr_matrix(m) for o, m in ham.PAULI.items()}
    H = sp.csr_matrix((2 ** L, 2 ** L))
    for c, ops in ham.block_terms(job, 0, L):
        d = dict(ops)
        H = H + c * reduce(lambda x, y: sp.kron(x, y, format="csr"),
                           [P2[d[i]] if i in d else I2 for i in range(L)])
    return H.tocsr()


def merge_bound_sparse(job, nA, k, tau_gap=TAU_GAP, tol=1e-13):
    """E0 and c by Lanczos in the full space; a and b as in merge_bound_retained."""
    import scipy.sparse.linalg as sla
    L = job.n_sites
    DA, DB = 2 ** nA, 2 ** (L - nA)
    a, b, kA, kB = merge_bound_retained(job, nA, k, tau_gap)
    _, V_A, _, V_B = leaves(job, nA, k, tau_gap)
    H = sparse_hamiltonian(job)
    sigma = sum(abs(c) for c, _ in ham.block_terms(job, 0, L))

    def proj(y):
        Y = y.reshape(DA, DB)
        return (V_A @ (V_A.T @ Y @ V_B) @ V_B.T).reshape(-1)

    def qhq(y):
        y = np.asarray(y).reshape(-1)
        py = proj(y)
        h = H @ (y - py)
        return h - proj(h) + sigma * py

    n = DA * DB
    rng = np.random.default_rng(7)
    v0 = rng.standard_normal(n)
    E0 = sla.eigsh(H, k=1, which="SA", tol=tol, v0=v0, ncv=40, maxiter=20000,
                   return_eigenvectors=False)[0]
    op = sla.LinearOperator((n, n), matvec=qhq, dtype=np.float64)
    c = sla.eigsh(op, k=1, which="SA", tol=tol, v0=v0, ncv=40, maxiter=20000,
                  return_eigenvectors=False)[0]
    return _finish(a, b, c, E0, kA, kB)
