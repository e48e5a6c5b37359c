/*
 * rmc.h -- C ABI of librmc, the MI355X (gfx950) recursive module-coupling
 * eigensolver.
 *
 * The method (Sec. II and Algorithm 1 of the paper): split a spin system into
 * modules; keep the lowest k eigenstates of each; project the boundary
 * operators onto those bases; couple two neighbouring modules through the
 * effective Hamiltonian
 *     H_eff = diag(E_a^A + E_b^B) + sum_i c_i o_A^i (x) o_B^i        (k_A k_B square)
 * (assembled effective-Hamiltonian equation, with the coupling
 * V = -sum J' O_A (x) O_B written as c_i = -J'_i); keep its lowest k
 * eigenvectors, stored through their coefficients in the product basis, as the
 * merged module's basis; repeat until the whole system is reached and return
 * the lowest q eigenvalues.
 *
 * Here H_eff is never formed: it is applied matrix-free as
 *     X -> E_A X + X E_B + sum_i c_i O_A^i X (O_B^i)^T
 * (X is the k_A x k_B coefficient matrix, row-major, product index a*k_B + b,
 * A = left module) inside a Chebyshev-filtered block subspace eigensolver with
 * Rayleigh-Ritz and CholeskyQR2, all in HIP kernels on one GPU.
 *
 * General conventions
 *  - Every call returns an rmc_status; nothing throws or aborts across the ABI.
 *    On error outputs are left untouched, except RMC_ERR_NOCONV, which still
 *    fills the report and, where the failed solve is the one that returns them,
 *    the energies (best Ritz values; see each call).
 *  - rmc_last_error() gives a message for the last non-OK status of the ctx.
 *  - Pointers named *_host are host memory owned by the caller; pointers named
 *    *_dev are device memory owned by the caller. Modules are owned by the ctx
 *    and live in its device arena; rmc_destroy frees all of them.
 *  - One ctx per host thread. All device work is enqueued on the ctx stream;
 *    calls that return host data synchronise that stream.
 *  - Matrices are row-major FP64 unless stated otherwise.
 *  - Spin operators use the real alphabet X = sigma^x, T = -i sigma^y
 *    ([[0,-1],[1,0]]), Z = sigma^z. Site j of an n-site block is bit (n-1-j)
 *    of the basis index (site 0 = most significant bit); bit 0 is Z = +1.
 */
#ifndef RMC_H
#define RMC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RMC_OK = 0,
  RMC_ERR_ARG = 1,    /* invalid argument or descriptor                        */
  RMC_ERR_OOM = 2,    /* device arena exhausted                                */
  RMC_ERR_NOCONV = 3, /* eigensolver hit max_iter; best values still returned  */
  RMC_ERR_HIP = 4,    /* HIP runtime error                                     */
  RMC_ERR_STATE = 5   /* object in the wrong state (e.g. basis already freed)  */
} rmc_status;

typedef enum {
  RMC_FP64 = 0, /* all arithmetic in FP64                                        */
  RMC_FP32 = 1, /* Kronecker matvecs of the filter in FP32 MFMA, FP64 correction  */
  RMC_BF16 = 2  /* filter matvecs BF16 in / FP32 accumulate MFMA, FP64 correction */
} rmc_precision;

typedef enum { RMC_OP_X = 1, RMC_OP_T = 2, RMC_OP_Z = 3 } rmc_op;

/* One Hamiltonian term coef * op[0]@site[0] (x) op[1]@site[1] (nsite = 1 or 2). */
typedef struct {
  double coef;
  int nsite;
  int site[2];
  int op[2];
} rmc_term;

/* A leaf module (the paper's initial block Hamiltonian H_b). Sites are local,
 * 0..n_sites-1 (1 <= n_sites <= 12). The dense Hamiltonian is accumulated term
 * by term in list order, starting from +0.0. */
typedef struct {
  int n_sites;
  int n_terms;
  const rmc_term* terms;
} rmc_leaf_desc;

/* Coupling terms of one merge: sum_i coef[i] * O_A[opA[i]] (x) O_B[opB[i]], the op ids
 * being those returned by rmc_project_ops on module A (left) and B (right). */
typedef struct {
  int n_terms;
  const double* coef;
  const int* opA;
  const int* opB;
} rmc_bond_desc;

/* A module tree for rmc_recurse (the inputs of Algorithm 1 over a caller-defined
 * hierarchy: the initial block Hamiltonians H_b, the couplings V_bb' between blocks, and
 * the order in which blocks are merged, Fig. 1's recursive block merging).
 *
 * A leaf node (left = right = -1) is a block of n_sites sites (1..12), numbered
 * 0..n_sites-1; its terms are its Hamiltonian H_b, accumulated in list order from +0.0.
 * A merge node couples its children left (module A) and right (module B); its merged
 * module numbers its sites A's first (0..w_A-1), then B's (w_A..w_A+w_B-1). Its terms
 * are the coupling V_AB: two-site terms (nsite = 2) with site[0] / op[0] on A (a site
 * of A, 0..w_A-1) and site[1] / op[1] on B (0..w_B-1); n_sites is ignored.
 * Children come before their parents (left, right < the node's index) and the last
 * node is the root. A node referenced by several parents (or as both children of one)
 * is one module computed once: a declared shared subtree. Independently of that,
 * modules with identical content (terms, k and children, up to a shift of sites) are
 * computed once (the paper's reuse of identical blocks).
 * k of a node is the number of states its module keeps (0: the tree's k); the root
 * keeps nothing and returns its lowest q eigenvalues. Every node must belong to the
 * tree (reachable from the root). */
typedef struct {
  int left, right;        /* child node indices; -1, -1 for a leaf            */
  int n_sites;            /* leaf: sites of the block                         */
  int n_terms;
  const rmc_term* terms;  /* leaf: H_b; merge: the coupling V_AB             */
  int k;                  /* retained states of this module (0 = tree's k)    */
} rmc_tree_node;

typedef struct {
  int n_nodes;
  const rmc_tree_node* nodes;
  int k; /* retained states per module, unless a node sets its own */
  int q; /* lowest eigenvalues returned, 1 <= q <= k                */
} rmc_tree_desc;

/* A chain (the default order of Algorithm 1): sites 0..n_sites-1 split into leaves of
 * leaf_sites consecutive sites; terms is the global term list. A leaf's Hamiltonian is
 * the terms lying in it, in list order; a merge of A = [a, m) with B = [m, b) couples
 * through the two-site terms with one site in A and one in B, in list order. Adjacent
 * modules are merged pairwise left to right; an odd module is carried up unchanged.
 * rmc_recurse_chain builds that tree and solves it as rmc_recurse does. */
typedef struct {
  int n_sites;
  int leaf_sites;
  int n_terms;
  const rmc_term* terms;
  int k; /* retained states per module */
  int q; /* lowest eigenvalues returned, 1 <= q <= k */
} rmc_chain_desc;

/* One job of a batch or of the serving queue: exactly one of tree / chain is set. */
typedef struct {
  const rmc_tree_desc* tree;
  const rmc_chain_desc* chain;
} rmc_job_desc;

typedef struct {
  int precision;          /* rmc_precision                                          */
  double tol;             /* residual tolerance relative to the spectral scale (1e-13) */
  double gap_tol;         /* gap-rule tolerance relative to the eigenvalue scale (1e-6) */
  int max_iter;           /* outer filter iterations before RMC_ERR_NOCONV (200)     */
  int guard;              /* extra block vectors beyond the wanted ones (0 = auto)    */
  int max_degree;         /* cap of the Chebyshev degree per outer iteration (0=auto) */
  unsigned long long seed;/* seed of the random component of the start block        */
} rmc_solve_opts;

typedef struct {
  int level;     /* 0 = leaf                                             */
  int width;     /* sites of the module                                  */
  int kind;      /* 0 leaf, 1 merge, 2 root                              */
  int k_req;     /* min(k, dimension)                                    */
  int k_eff;     /* kept after the gap rule                              */
  int iters;     /* outer iterations of the eigensolver                  */
  int matvecs;   /* block-vector operator applications                   */
  int reused;    /* 1 if an identical module was reused                  */
  int rr_sweeps; /* Jacobi sweeps summed over the Rayleigh-Ritz solves   */
  double gap;    /* eigenvalue gap at the cut (inf if nothing was cut)   */
  double max_res;/* largest relative residual among the wanted pairs     */
  double ms;     /* wall time of this module                             */
} rmc_level_report;

typedef struct {
  int capacity;               /* entries available in records (caller-set)  */
  int n_records;              /* entries written                           */
  rmc_level_report* records;  /* caller-owned host array                   */
  int n_leaf_ed;
  int n_merges;
  double total_ms;
} rmc_report;

typedef struct rmc_ctx rmc_ctx;
typedef struct rmc_module rmc_module;

/* Fills opts with the defaults given above. */
void rmc_default_opts(rmc_solve_opts* opts);

/* Create a context on `device`. arena_dev is device memory of arena_bytes bytes
 * that the library sub-allocates (e.g. a torch tensor; caller keeps it alive
 * until rmc_destroy). hip_stream is a hipStream_t (NULL = the null stream). */
rmc_status rmc_create(rmc_ctx** out, int device, void* arena_dev, size_t arena_bytes,
                      void* hip_stream);
rmc_status rmc_destroy(rmc_ctx* ctx);
const char* rmc_last_error(const rmc_ctx* ctx);
/* Bytes of the arena currently in use / high-water mark. */
rmc_status rmc_arena_usage(const rmc_ctx* ctx, size_t* in_use, size_t* peak);

/* (1) Leaf ED (Algorithm 1, first step): assemble the leaf Hamiltonian by bit
 * indexing, find its lowest min(k, 2^n)+1 eigenpairs and keep k_eff of them (gap
 * rule: if the cut falls inside a cluster of eigenvalues closer than
 * gap_tol * max(1, |E_0|, |E_k|), the cut moves down to the cluster start).
 * Errors: RMC_ERR_ARG for k < 1, n_sites outside 1..12, bad sites/ops. */
rmc_status rmc_module_ed(rmc_ctx* ctx, const rmc_leaf_desc* leaf, int k,
                         const rmc_solve_opts* opts, rmc_module** out);

/* (2) Project one-site operators onto a module's retained basis (intra-block
 * matrix elements o = <a|O|a'>). site[i] is local to the module; for a merged
 * module the operator is taken from the child holding the site and transformed
 * through the coefficients C (Algorithm 1, transform step). Returns one op id per
 * request (an existing id if already projected). The children of a merged module
 * must still hold their bases or the requested ops (else RMC_ERR_STATE). */
rmc_status rmc_project_ops(rmc_ctx* ctx, rmc_module* m, int n_ops, const int* site,
                           const int* op, int* op_ids_host);

/* (3) One coupling step of A (left) and B (right) (reduced eigenproblem). If out
 * is non-NULL the lowest k_keep states (gap rule) become a new module whose
 * basis is the coefficient matrix C (k_eff x k_A k_B). The lowest q eigenvalues
 * are written to energies_host (q <= k_keep when out is non-NULL). */
rmc_status rmc_couple_solve(rmc_ctx* ctx, rmc_module* A, rmc_module* B,
                            const rmc_bond_desc* bond, int k_keep, int q,
                            const rmc_solve_opts* opts, rmc_module** out,
                            double* energies_host, rmc_level_report* rep_host);

/* (4) The whole recursion over a module tree (Algorithm 1). Writes the lowest q
 * eigenvalues of the root to energies_host; report is optional (NULL). Errors:
 * RMC_ERR_ARG for a malformed tree (a child index not below its parent, a node not in
 * the tree, a leaf outside 1..12 sites, a coupling term not of the form site of A /
 * site of B, q outside 1..k); RMC_ERR_NOCONV when a solve does not converge: if it was
 * the root's, energies_host holds its best Ritz values, else NaN. */
rmc_status rmc_recurse(rmc_ctx* ctx, const rmc_tree_desc* tree, const rmc_solve_opts* opts,
                       double* energies_host, rmc_report* report);
/* The same over a chain (its default tree, see rmc_chain_desc). */
rmc_status rmc_recurse_chain(rmc_ctx* ctx, const rmc_chain_desc* chain,
                             const rmc_solve_opts* opts, double* energies_host,
                             rmc_report* report);

/* Batched recursion: n_jobs trees or chains solved level by level, each level's leaf
 * EDs and merges of all jobs in batched launches. energies_host is n_jobs x q_stride;
 * status_host (optional) gets one rmc_status per job. */
rmc_status rmc_recurse_batch(rmc_ctx* ctx, int n_jobs, const rmc_job_desc* jobs,
                             const rmc_solve_opts* opts, double* energies_host,
                             int q_stride, int* status_host);

/* Serving (continuous batching). rmc_serve_start starts a scheduler thread that
 * owns the ctx's stream and arena until rmc_serve_stop; other calls on the ctx
 * return RMC_ERR_STATE meanwhile. Each scheduler step admits queued jobs while
 * at most max_inflight are in flight and their estimated device memory fits in
 * mem_budget bytes (0 = half the arena), then advances every job in flight by
 * one tree level in one batched level solve, so jobs that arrive while others run
 * share the device with them. A step solves the merges first and the leaves last;
 * jobs that arrive during its merges are admitted (by the same rule) before its
 * leaf phase and have their leaves solved in that step. Module bases and projected
 * operators stay device-resident between a job's levels. */
rmc_status rmc_serve_start(rmc_ctx* ctx, const rmc_solve_opts* opts, int max_inflight,
                           size_t mem_budget);
/* Queue a job (the descriptor, its tree or chain and their terms are copied); never
 * blocks. A job that can never fit the budget completes at once with RMC_ERR_OOM. */
rmc_status rmc_submit(rmc_ctx* ctx, const rmc_job_desc* job, unsigned long long* job_id);
/* done = 1 once finished; then min(q, capacity) energies, the job's status and its
 * latency (submission to completion, ms) are written and the result is released.
 * energies_host may be NULL (capacity is then ignored). */
rmc_status rmc_poll(rmc_ctx* ctx, unsigned long long job_id, int* done, double* energies_host,
                    int capacity, int* job_status, double* latency_ms);
/* Finish every queued and in-flight job, then stop the scheduler thread. */
rmc_status rmc_serve_stop(rmc_ctx* ctx);

/* Module inspection and lifetime. */
rmc_status rmc_module_info(const rmc_module* m, int* k_eff, int* dim, int* n_sites,
                           double* energies_host /* k_eff, may be NULL */);
/* Copy the basis (k_eff x dim, row-major: row = retained state) to the host. */
rmc_status rmc_module_basis(rmc_ctx* ctx, const rmc_module* m, double* basis_host);
/* The retained states of a module as full-space vectors (Sec. II, states of the
 * combined system from the stored coefficients, read recursively down to the
 * leaves): out_dev (device, caller-owned, k_eff x 2^n_sites doubles, row-major)
 * row mu = the state mu in the site basis (site 0 = most significant bit). Needs
 * the bases of the module and of every module below it, all still owned by ctx:
 * modules from rmc_module_ed / rmc_couple_solve keep them; rmc_recurse releases
 * them. n_sites <= 24. RMC_ERR_STATE if a basis is missing. */
rmc_status rmc_module_lift(rmc_ctx* ctx, const rmc_module* m, double* out_dev);

/* Single-merge truncation diagnostics (Sec. IV, single-merge bound; App. on the error
 * bounds: block form of H, discarded-sector gap, r(b, gamma)). A and B are leaf
 * modules from rmc_module_ed built from leaf_A and leaf_B (bases kept); bond is the
 * coupling as for rmc_couple_solve. With H the Hamiltonian of the nA + nB sites
 * (A's sites first; nA + nB <= 24), P the projector on the retained product states
 * psi_A[a] (x) psi_B[b] and Q = I - P, writes out_host[7] =
 *   a = lambda_min(P H P) on range(P) (the merged module's lowest energy),
 *   b = ||P H Q||_2, c = lambda_min(Q H Q) on range(Q), gamma = c - a,
 *   r = (sqrt(gamma^2 + 4 b^2) - gamma) / 2, b^2 / gamma, E0 = lambda_min(H).
 * b comes from the retained states alone (b^2 = largest eigenvalue of
 * P V^2 P - (P V P)^2, V the coupling); c and E0 from the block eigensolver on the
 * full 2^(nA+nB) space with H applied matrix-free (and Q H Q + sigma P, sigma the sum
 * of |coef|, for c). If the leaves keep every state, range(Q) is empty: b = r = 0 and
 * c = gamma = +inf. gamma <= 0 (the bound's assumption fails) gives b^2/gamma = +inf.
 * Always FP64 (opts->precision is ignored). Needs about 10 (nev + guard) x 2^(nA+nB)
 * doubles of arena. RMC_ERR_NOCONV if a solve does not converge. */
rmc_status rmc_merge_bound(rmc_ctx* ctx, rmc_module* A, const rmc_leaf_desc* leaf_A,
                           rmc_module* B, const rmc_leaf_desc* leaf_B,
                           const rmc_bond_desc* bond, const rmc_solve_opts* opts,
                           double* out_host);
/* Copy a projected operator (k_eff x k_eff) to the host. */
rmc_status rmc_module_op(rmc_ctx* ctx, const rmc_module* m, int op_id, double* op_host);
rmc_status rmc_module_free(rmc_ctx* ctx, rmc_module* m);
/* Create a module from host data: a checkpoint of a computed module (energies,
 * projected operators, optionally its basis) or synthetic test input. E_host has
 * k entries (ascending); basis_host is k x dim or NULL; op_data_host holds n_ops
 * k x k matrices for (sites[i], ops[i]). The module has no children, so only the
 * operators given (or, for a leaf-sized basis with dim = 2^n_sites, newly
 * projected ones) are available. Projected Pauli operators have spectral norm
 * <= 1; the eigensolver's spectral bound assumes imported operators do too. */
rmc_status rmc_module_import(rmc_ctx* ctx, int n_sites, int k, int dim, const double* E_host,
                             const double* basis_host, int n_ops, const int* sites,
                             const int* ops, const double* op_data_host, rmc_module** out);

/* Kernel-level entry points (used by the parity tests and the benchmark). */
/* Dense leaf Hamiltonian (2^n x 2^n) into caller device memory (bit-index assembly). */
rmc_status rmc_leaf_hamiltonian(rmc_ctx* ctx, const rmc_leaf_desc* leaf, double* H_dev);
/* Y = H_eff X for n_vec vectors (X, Y: n_vec x k_A k_B, device, FP64), with the
 * matvec done in `precision` (inputs rounded to it, FP32 accumulation for BF16). */
rmc_status rmc_kron_apply(rmc_ctx* ctx, rmc_module* A, rmc_module* B,
                          const rmc_bond_desc* bond, int precision, int n_vec,
                          const double* X_dev, double* Y_dev);
/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): rmc_kron_apply with every piece of
 * its scratch (the coupling coefficients, the concatenated operators, the diagonal
 * E_A + E_B, the operator pack of the precision, the launch descriptor) carved from a
 * fixed device array of 4 MiB per GPU that the library holds until the process ends.
 * It calls no hipMalloc, hipFree or arena allocation, never times tile candidates
 * (an untuned shape takes the default variant) and does not synchronise: Y_dev is
 * ready when the ctx stream reaches this point. Enough for T <= 8 terms at
 * k_A = k_B <= 128; a coupling that needs more scratch fails with RMC_ERR_ARG. The
 * array is shared by every call on that GPU and keeps the last call's contents: calls
 * that overlap on one GPU (other streams or other contexts) race; calls in order on
 * one stream do not. Arguments, layout and results as rmc_kron_apply. */
rmc_status rmc_kron_apply_noalloc(rmc_ctx* ctx, rmc_module* A, rmc_module* B,
                                  const rmc_bond_desc* bond, int precision, int n_vec,
                                  const double* X_dev, double* Y_dev);
/* Symmetric eigendecomposition of `batch` m x m matrices (device, row-major,
 * stride m*m) by parallel cyclic Jacobi: eigenvalues ascending into evals_dev
 * (batch x m), eigenvectors as columns into V_dev (batch x m x m). m <= 192. */
rmc_status rmc_sym_eig(rmc_ctx* ctx, int batch, int m, const double* A_dev,
                       double* evals_dev, double* V_dev);

/* Measurement of the Kronecker matvec (the dominant kernel): with enable = 1
 * every launch on the ctx stream is bracketed by a pair of HIP events and its
 * algorithmic work is counted (flops 2 T n (k_A + k_B) + 4 n per vector, n =
 * k_A k_B; bytes 8 n per vector read and written, plus the previous iterate of
 * the Chebyshev recurrence, E_A + E_B and the operators, once per launch).
 * enable = 1 also clears the totals; 0 stops recording. */
rmc_status rmc_profile(rmc_ctx* ctx, int enable);
/* Totals since the last rmc_profile(ctx, 1); synchronises the stream. ms is the
 * sum over launches of the event-measured kernel time. */
rmc_status rmc_profile_read(rmc_ctx* ctx, long long* launches, double* flops, double* bytes,
                            double* ms);
/* The same totals restricted to the launches of one precision (rmc_precision): in
 * the FP32 / BF16 forms a problem whose filter reached that precision's noise floor
 * continues in FP64, so a run mixes launches of several precisions. */
rmc_status rmc_profile_read_precision(rmc_ctx* ctx, int precision, long long* launches,
                                      double* flops, double* bytes, double* ms);
/* Kernels whose launches are recorded while profiling is on:
 *   RMC_PROF_KRON_STEP   one Kronecker matvec step (streaming or tiled kernel), the
 *                        Rayleigh-Ritz applies and the per-step filter path;
 *   RMC_PROF_KRON_FILTER the whole-filter launch (every vector through all Chebyshev
 *                        steps: flops as above per vector and step; bytes 8 n per vector
 *                        for the defect, the Ritz block and the output, plus E_A + E_B
 *                        and the operators once per problem);
 *   RMC_PROF_PAULI       the full-space Pauli-sum apply of rmc_merge_bound (bytes 8 per
 *                        amplitude for each input vector read and the output written;
 *                        flops 2 per term and amplitude; precision FP64).
 * rmc_profile_read and rmc_profile_read_precision sum the two Kronecker kinds. */
typedef enum { RMC_PROF_KRON_STEP = 0, RMC_PROF_KRON_FILTER = 1, RMC_PROF_PAULI = 2 } rmc_profile_kernel;
/* The totals of one kernel kind and precision. */
rmc_status rmc_profile_read_kernel(rmc_ctx* ctx, int kernel, int precision, long long* launches,
                                   double* flops, double* bytes, double* ms);

#ifdef __cplusplus
}
#endif
#endif /* RMC_H */
