"""Plain FP64 CPU oracle for the recursive module-coupling eigensolver.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call, link or
execute anything in this package: only the tests, the smoke check and the CPU
baseline leg of the benchmark do.

The oracle follows the paper's own construction literally: every module is
diagonalised densely, the coupled Hamiltonian of a merge is assembled as an
explicit Kronecker sum, and it is fully diagonalised with LAPACK (``eigh``).
It shares no code with the HIP path; the only thing both sides import is the
seeded parameter generator in ``paper_2609_02394_amd.workloads``, which holds
no arithmetic of the method.

Modules:
  hamiltonian -- spin models as term lists and dense matrices (np.kron).
  recursion   -- leaf ED, projection, merge, gap-rule cut, edge-operator
                 transform, the recursive tree (Sec. II, Algorithm 1).
  exact       -- independent references: brute-force ED of the whole chain and
                 free-fermion closed forms of the open TFIM and XX chains.
"""
from . import hamiltonian, recursion, exact  # noqa: F401
