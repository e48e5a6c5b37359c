// Per-problem descriptors of the batched ("grouped") kernels: one launch covers
// every active problem of a level, blockIdx.z selecting the problem. All
// pointers are device pointers; descriptors live in device memory.
#pragma once
#include <hip/hip_runtime.h>

namespace rmc {

// out_j = s1 (sum_i c_i O_A^i Y_j O_B^iT + Ediag .* Y_j) + s2 Y_j + s3 Xprev_j
//         + s1 phi[j] E_j   (E, phi optional), j < nv.
// vbase: number of vectors in the launch's earlier descriptors (the problem's first
// vector in the launch-wide numbering). pack: the operators in the streaming
// kernel's layout for the launch precision (kron_pack), pkm its tile size.
struct KronDesc {
  int kA, kB, T, nv;
  long vbase;
  const void* pack;
  int pkm, pad_;
  const double* coef;
  const double* OA;
  const double* OB;
  const double* Ediag;
  const double* Y;
  const double* Xprev;
  const double* E;
  const double* phi;
  double* out;
  double s1, s2, s3;
};

// The whole Chebyshev filter of one problem in defect form, every vector carried
// through all its steps by one workgroup (steps = degree - 1 matvecs):
//   D_1 = r0 E_j;  D_{k+1} = s1_k (H_low D_k + Ediag .* D_k) + s2_k D_k + s3_k D_{k-1}
//                            + s1_k phi_k[j] E_j   (k = 1..steps, D_0 = 0)
//   out_j = phi_{steps+1}[j] X_j + D_{steps+1}
// sc: steps x {s1, s2, s3}; phi: (steps + 1) x nv, row k-1 = phi_k. pack: the
// operators in the streaming layout of the launch precision (tile KM = pkm).
struct FilterDesc {
  int kA, kB, T, nv;
  long vbase;
  const void* pack;
  int pkm, steps;
  const double* Ediag;
  const double* EA;  // the module energies: Ediag[a k_B + b] = EA[a] + EB[b]
  const double* EB;
  const double* E;
  const double* X;
  double* out;
  const double* sc;
  const double* phi;
  double r0;
};
// The phi_k rows of a fused filter (steps + 1 rows of cn): phi_0 = r0 t_j, then
// phi_k = (s1_k t_j) phi_{k-1} - b_k phi_{k-2} with phi_{-1} = 1, b_1 = b1 and
// b_k = -s3_k after (s1_k, s3_k from sc, 3 per step); t_j = theta_j - c. Each product
// and the difference are rounded separately, as the host computes the same rows.
struct PhiDesc {
  int cn, steps;
  double r0, b1;
  const double* t;
  const double* sc;
  double* phi;
};
void filter_phi_batched(hipStream_t s, const PhiDesc* d, int P);
bool kron_filter_fits(int precision, int kA, int kB, int T);
void kron_filter_batched(hipStream_t s, const FilterDesc* d, int P, long total_vecs, int precision,
                         int kmax, int Tmax);

// C = alpha op(A) op(B) + beta C (row-major); with `work` non-null the launch
// writes split-K partials to work (ksplit x M x N) instead of C.
struct GemmDesc {
  int M, N, K, pad;
  const double* A;
  const double* B;
  double* C;
  long lda, ldb, ldc;
  double alpha, beta;
  double* work;
};

// Gram partials of tall-skinny blocks: work[s][i][j] = sum over K-slice s of
// A[i][k] B[j][k] (A: ca x n, B: cb x n, row-major, ca, cb <= 192), ks slices.
struct GramDesc {
  int ca, cb, n, sym;  // sym: A B^T is symmetric; upper tiles formed and mirrored
  int ks, pad;         // K-slices of this product: partials ks x ca x cb in work
  const double* A;
  const double* B;
  double* work;
};

// Symmetric eigensolver / Cholesky on m x m given as nparts partials (pstride apart).
struct EigDesc {
  int m, nparts;
  const double* A;
  long pstride;
  double* evals;
  double* V;
  double* Vwork;
  int* info;
};
struct CholDesc {
  int m, nparts;
  const double* G;
  long pstride;
  double* Linv;
  int* info;
  double shift;  // added to the diagonal when info[1] == 1 on entry (retry)
};

// Row-block vector operations over nv rows of length n.
enum VecOp {
  VEC_NORMALIZE = 0,
  VEC_RESIDUAL = 1,
  VEC_SCALE_ADD = 2,
  VEC_COPY = 3,
  VEC_AXPY3 = 4,
  VEC_REDUCE = 5  // out[i] = sum_{j < nv} P[j n + i], i < n (split-K partial sums)
};
struct VecDesc {
  int nv, n;
  double* out;        // NORMALIZE: rows to normalise; RESIDUAL: the residual rows (nullable); others: output
  const double* P;    // RESIDUAL: HX; SCALE_ADD: P; COPY: src; AXPY3: Y
  const double* Q;    // RESIDUAL: X;  SCALE_ADD: Q (nullable); AXPY3: Xprev (nullable)
  const double* a;    // RESIDUAL: theta; SCALE_ADD: per-row scale
  double* norms;      // NORMALIZE / RESIDUAL output (nv)
  double asgn, b, c;  // SCALE_ADD: out = asgn a_j P + b Q; AXPY3: out += b Y + c Q
};

// Block transpose of a merged basis (k vectors of k_A x k_B blocks).
struct TrDesc {
  int k, kA, kB, pad;
  const double* C;
  double* Ct;
};

// Start block: the m smallest D entries as unit vectors plus eps * uniform(-1,1).
struct StartDesc {
  int n, m;
  const double* D;
  int* sel;
  double* X;
  double eps;
  unsigned long long seed;
};

// T: largest term count of the launch; total_vecs: vectors over all problems (both
// only key the tile-shape autotuner). may_tune = false never times candidates (no
// events, no synchronisation): an untuned shape takes the default variant. A variant
// forced with RMC_KRON_VARIANT runs where it takes the shape; elsewhere the launch takes
// the autotuner's choice, or, with strict = true, fails with RMC_ERR_ARG. Returns the
// variant launched (1, 2, 4: tiled kernel column sub-tiles; 8 to 11: streaming kernel).
int kron_batched(hipStream_t s, const KronDesc* d, int P, int kBmax, int nvmax, int kAmax,
                 int precision, int T, long total_vecs, bool may_tune = true, bool strict = false);
void kron_set_tuning(bool on);
// Per host thread: off while a stream is being captured into a graph (untuned shapes
// then take the default variant instead of timing candidates).
void kron_thread_tuning(bool on);
int kron_max_k();
// Operators of one coupling in the streaming kernel's layout: for term t, the
// pkm x pkm zero-padded tiles O_B^t and c_t O_A^t (in that order, row-major) in the
// element type of the precision (FP64, FP32, BF16). kron_pack_bytes is 0 where the
// streaming kernel does not take the size in that precision; null outputs are skipped.
// Batched set-up of the coupling operators of a level (one descriptor per problem):
// OAcat / OBcat (the T operators of each side, concatenated), the diagonal D and
// E_A[a] + E_B[b] (Ediag) of H_eff, and the streaming packs (nullable).
struct OpSetDesc {
  int T, kA, kB, pkm;
  const double* coef;          // T
  const double* const* opa;    // T device pointers, k_A x k_A each
  const double* const* opb;    // T device pointers, k_B x k_B each
  const double* EA;
  const double* EB;
  double* OAcat;
  double* OBcat;
  double* D;
  double* Ediag;
  double* p64;
  float* p32;
  void* p16;
};
void op_setup_batched(hipStream_t s, const OpSetDesc* d, int P, long work_max);
int kron_pack_km(int kA, int kB);
size_t kron_pack_bytes(int precision, int kA, int kB, int T);
void kron_pack(hipStream_t s, int T, int kA, int kB, const double* coef, const double* OA,
               const double* OB, void* p64, void* p32, void* p16);
void gemm_batched(hipStream_t s, bool tA, bool tB, const GemmDesc* d, int P, int Mmax, int Nmax,
                  int ksplit);
void gram_batched(hipStream_t s, const GramDesc* d, int P, int ks, int cmax);
// threads: 1024, or 512 when every m <= 56 (two workgroups share a CU; the m <= 80 body
// needs no more threads up to that size)
void jacobi_batched(hipStream_t s, const EigDesc* d, int P, int mmax, int threads = 1024);
void chol_batched(hipStream_t s, const CholDesc* d, int P, int mmax);
void vec_batched(hipStream_t s, VecOp op, const VecDesc* d, int P, int nvmax, long elems_max);
void start_batched(hipStream_t s, const StartDesc* d, int P, int nmax, int mmax);
void transpose_blocks_batched(hipStream_t s, const TrDesc* d, int P, int kmax, int nmax);

// ---- full-space operators (single-merge truncation diagnostics) -------------------
// One Pauli string of an n-site block in the real alphabet {X, T, Z}: for basis row r,
// (term y)[r] = coef * (-1)^{|r & zm| + |~r & tm|} * y[r ^ flip] (flip: X and T sites,
// zm: Z sites, tm: T sites; bit n-1-s is site s).
struct FullTerm {
  double coef;
  unsigned flip, zm, tm, pad;
};
// out = s1 H (Y - sub) + s2 Y0 + s3 Xprev for nv vectors of 2^n_sites (sub, Y0, Xprev
// nullable), H = sum of the terms; terms with equal flip masks must be consecutive
// (they share one gather).
struct PauliDesc {
  int n_sites, n_terms, nv, pad;
  const FullTerm* terms;
  const double* Y;
  const double* sub;
  const double* Y0;
  const double* Xprev;
  double* out;
  double s1, s2, s3;
};
void pauli_batched(hipStream_t s, const PauliDesc* d, int P, long elems_max);
// out = sum_{i<5} w[i] U[i] over n elements (null U[i] skipped).
struct LinDesc {
  long n;
  double* out;
  const double* U[5];
  double w[5];
};
void lincomb_batched(hipStream_t s, const LinDesc* d, int P, long nmax);
// D[r] = sum of the diagonal terms at r, plus sigma * pA[r >> nB] * pB[r & (2^nB - 1)]
// where pA, pB are given (null: no projector part).
void full_diag(hipStream_t s, int n_sites, int nB, int n_terms, const FullTerm* terms,
               const double* pA, const double* pB, double sigma, double* D);
// p[j] = sum_i Psi[i][j]^2 for a k x D row-major Psi.
void col_sumsq(hipStream_t s, int k, int D, const double* Psi, double* p);
// M[(a kB + b)(kA kB) + a' kB + b'] = sum_t w[t] A_t[a][a'] B_t[b][b'] (A_t: kA x kA,
// B_t: kB x kB, consecutive; w on the device).
void kron_dense(hipStream_t s, int T, int kA, int kB, const double* w, const double* Acat,
                const double* Bcat, double* M);

}  // namespace rmc
