// Internal launch wrappers of librmc's HIP kernels (gfx950). All matrices are
// row-major; a "block" of vectors is stored one vector per row.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rmc {

// C[b] = alpha * op(A[b]) op(B[b]) + beta * C[b], op(A): M x K, op(B): K x N.
// tA: A is stored K x M (A[k*lda+i]); tB: B is stored N x K (B[j*ldb+k]).
// ksplit > 1 splits K over workgroups; the partial sums go to `work`
// (ksplit*batch*M*N doubles) and are reduced in a fixed order.
void gemm_f64(hipStream_t s, bool tA, bool tB, int M, int N, int K, double alpha,
              const double* A, long lda, long sA, const double* B, long ldb, long sB,
              double beta, double* C, long ldc, long sC, int batch, int ksplit, double* work);
// Pick a split-K factor for an M x N x K product so the launch covers the chip.
int gemm_pick_ksplit(int M, int N, int K, int batch);
// Split-K product that leaves its ksplit partial sums (each M x N, batch-major)
// in `work` for a consumer that adds them; returns the split used.
int gemm_f64_partials(hipStream_t s, bool tA, bool tB, int M, int N, int K, const double* A,
                      long lda, const double* B, long ldb, int ksplit, double* work);

// Y_out = Y_out + s1 * diag .* Y + s2 * Y + s3 * Xprev over nv vectors of length n
// (diag may be null; Xprev may be null when s3 == 0).
void axpy_epilogue(hipStream_t s, int nv, int n, double* out, const double* Y,
                   const double* Xprev, const double* diag, double s1, double s2, double s3,
                   bool out_is_zero);

// norms[j] = ||Y_j||_2, then Y_j /= norms[j] (if normalize) for nv vectors.
void row_norms(hipStream_t s, int nv, int n, double* Y, double* norms, bool normalize);
// res[j] = ||HX_j - theta_j X_j||_2.
void residual_norms(hipStream_t s, int nv, int n, const double* HX, const double* X,
                    const double* theta, double* res);

// Cholesky G + shift*I = L L^T (m x m, m <= 192) and Linv = L^{-1} (lower, m x m).
// G is the sum of nparts split-K partials spaced pstride apart.
// info[0] = 0 on success, 1 if a pivot was not positive.
void chol_inv(hipStream_t s, int m, const double* G, int nparts, long pstride, double shift,
              double* Linv, int* info);

// Parallel cyclic Jacobi eigensolver of `batch` symmetric m x m matrices (m <= 192,
// symmetrised as (A + A^T)/2). evals ascending, V columns = eigenvectors.
// Vwork: batch*m*m scratch. info[b] = sweeps used, negative if not converged.
// A[b] is the sum of nparts partials spaced pstride apart.
void jacobi_eig(hipStream_t s, int batch, int m, const double* A, long sA, int nparts,
                long pstride, double* evals, long sE, double* V, long sV, double* Vwork, int* info);
int jacobi_max_m();

// Dense leaf Hamiltonian from a device term list (bit-index assembly).
struct DevTerm {
  double coef;
  int nsite;
  int bit[2];   // bit positions (n_sites-1-site)
  int op[2];
};
void leaf_assemble(hipStream_t s, int n_sites, int n_terms, const DevTerm* terms, double* H);

// Every leaf of a batch: H (assembled as leaf_assemble does), its diagonal D, Gershgorin
// row bounds rb and their maximum bmax[0]; three launches.
struct LeafSetDesc {
  int n_sites, n_terms;
  const DevTerm* terms;
  double* H;
  double* D;
  double* rb;
  double* bmax;
};
void leaf_setup_batched(hipStream_t s, const LeafSetDesc* d, int P, int n_sites_max);

// W_j = O_site v_j for nv vectors of a 2^n_sites space; op in {1:X, 2:T, 3:Z}.
void site_op_apply(hipStream_t s, int nv, int n_sites, int bit, int op, const double* V,
                   double* W);
// The same for several (V, W, site, op) at once, one descriptor each.
struct SiteOpDesc {
  int nv, n_sites, bit, op;
  const double* V;
  double* W;
};
void site_op_batched(hipStream_t s, const SiteOpDesc* d, int P, long total_max);

// Symmetric blocks of a leaf Hamiltonian: A[i][j] = H[idx[i]][idx[j]] (nb x nb, from the
// D x D matrix H), one descriptor per block.
struct BlockGatherDesc {
  int nb, D;
  const int* idx;
  const double* H;
  double* A;
};
void gather_blocks(hipStream_t s, const BlockGatherDesc* d, int P, int nbmax);
// Full-space rows from block eigenvectors: out[idx[r]] = V[r * nb + col], r < nb (the row
// is zero elsewhere and must be cleared first).
// Row `out` (n entries) of a leaf's retained basis: zero, then column col of the block
// eigenvector matrix V (nb x nb) scattered to the block's basis indices idx.
struct BlockScatterDesc {
  int nb, col, n, pad;
  const int* idx;
  const double* V;
  double* out;
};
void scatter_block_rows(hipStream_t s, const BlockScatterDesc* d, int P, int nbmax);
// Selection of a block-diagonal leaf's lowest ne eigenpairs from its blocks' spectra
// (each block's eigenvalues ascending, the leaf's blocks consecutive from b0 in the
// eigensolver and gather tables): the rank of an eigenvalue is its place in the order
// (value, block, column) over the whole leaf; rank mu < ne goes to evout[mu] and to the
// scatter descriptor sd[sdbase + mu], which fills row mu of X (n entries each).
struct EigDesc;
struct LeafSelDesc {
  int b0, nblk, ne, n;
  long sdbase;
  double* X;
  double* evout;
};
void leaf_select(hipStream_t s, const LeafSelDesc* d, int P, const EigDesc* ed, const BlockGatherDesc* gd,
                 BlockScatterDesc* sd);

// Diagonal of H_eff: D[a*kB+b] = EA[a] + EB[b] + sum_i c_i OA_i[a,a] OB_i[b,b];
// Ediag[a*kB+b] = EA[a] + EB[b].
void kron_diag(hipStream_t s, int kA, int kB, const double* EA, const double* EB, int T,
               const double* coef_dev, const double* OAcat, const double* OBcat, double* D,
               double* Ediag);
// D[i] = H[i,i]; bound[i] = H[i,i] + sum_{j != i} |H[i,j]| (Gershgorin row bound).
void dense_diag(hipStream_t s, int n, const double* H, double* D, double* rowbound);
// out[0] = max(v[0..n)).
void vec_max(hipStream_t s, int n, const double* v, double* out);

// Start block: the m smallest D entries (ties by index) as unit vectors plus eps
// times a counter-based uniform(-1,1) perturbation; X is m x n.
void start_block(hipStream_t s, int n, int m, const double* D, double eps,
                 unsigned long long seed, int* sel, double* X);

// out_j = asgn * a[j] * P_j + b * Q_j (Q may be null) for nv rows of length n.
void rows_scale_add(hipStream_t s, int nv, int n, double* out, const double* P, const double* a,
                    double asgn, double b, const double* Q);

// out = src (m x n), strided copy helpers.
void copy_rows(hipStream_t s, int nv, int n, const double* src, long ld_src, double* dst,
               long ld_dst);

}  // namespace rmc
