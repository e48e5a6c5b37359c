// Internal host-side structures of librmc: modules, the coupled operator and the
// eigensolver interface (the arena and error type are in host_util.h).
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <set>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/rmc.h"
#include "host_util.h"
#include "rmc_batch.h"
#include "rmc_kernels.h"

namespace rmc {

#define RMC_HIP(x)                                                                      \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess)                                                               \
      throw ::rmc::Error(RMC_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

}  // namespace rmc

struct rmc_module {
  int kind = 0;        // 0 leaf, 1 merged
  int n_sites = 0;
  int dim = 0;         // leaf: 2^n_sites; merged: kA * kB
  int k_eff = 0;
  int kA = 0, kB = 0;  // merged: child dimensions
  double gap = 0.0;
  double* E = nullptr;          // device, k_eff
  std::vector<double> E_host;   // host copy
  double* basis = nullptr;      // device, k_eff x dim (row = retained state); null once freed
  rmc_module* A = nullptr;      // merged: children (not owned)
  rmc_module* B = nullptr;
  struct Op {
    int site, op;
    double* data;  // device k_eff x k_eff
  };
  std::vector<Op> ops;
};

struct rmc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_arena = false;
  void* arena_mem = nullptr;
  rmc::Arena arena;
  std::string last_error;
  std::unordered_set<rmc_module*> modules;  // every live module of this context
  // measurement of the Kronecker matvec launches
  bool prof = false;
  struct ProfRec {
    hipEvent_t a, b;
    double flops, bytes;
    int prec;
    int kind = 0;  // rmc_profile_kernel
  };
  std::vector<ProfRec> prof_recs;
  std::vector<hipEvent_t> ev_pool;
  std::mutex prof_mu;  // guards prof_recs and ev_pool against the solver's second lane
  // totals per kernel (rmc_profile_kernel) and precision (rmc_precision)
  long long prof_launches[3][3] = {};
  double prof_flops[3][3] = {}, prof_bytes[3][3] = {}, prof_ms[3][3] = {};
  // pinned host staging of the batched solver's descriptor tables, one per lane
  static constexpr int kMaxLanes = 4;
  char* pinned[kMaxLanes] = {};
  size_t pinned_cap[kMaxLanes] = {};
  // the batched solver's extra lanes: library-owned streams (default priority) and
  // the events that order them against `stream` (lane_ev[0]: fork; lane_ev[l]: join of
  // lane l)
  hipStream_t lane_stream[kMaxLanes] = {};  // [0] unused: lane 0 runs on `stream`
  hipEvent_t lane_ev[kMaxLanes] = {};
  // whole-filter launches of all lanes in one chain on the device (filter_ev: the last
  // one's end), so that a filter has the CUs to itself rather than sharing them with
  // another lane's filter; guarded by filter_mu
  std::mutex filter_mu;
  hipEvent_t filter_ev = nullptr;
  bool filter_ev_set = false;
  // serving: scheduler state (owned by recurse.hip); other calls are refused while set
  void* serve = nullptr;
  bool serving = false;
};

namespace rmc {

// The operator whose lowest eigenpairs are sought: a dense symmetric matrix (leaf
// module) or the Kronecker-sum effective Hamiltonian of a merge.
struct CoupledOp {
  int kind = 0;  // 0 dense, 1 kron, 2 full-space Pauli sum
  int n = 0;
  const double* H = nullptr;  // dense n x n
  int kA = 0, kB = 0, T = 0;
  const double* EA = nullptr;
  const double* EB = nullptr;
  std::vector<double> coef;     // host
  double* coef_dev = nullptr;   // device T
  double* OAcat = nullptr;      // device T x kA x kA
  double* OBcat = nullptr;      // device T x kB x kB
  double* Ediag = nullptr;      // device n: EA[a] + EB[b]
  double* D = nullptr;          // device n: full diagonal
  double bup = 0.0;             // upper bound of the spectrum
  int precision = RMC_FP64;
  // operators in the streaming Kronecker kernel's layout per precision (null where
  // that kernel does not take the size), tile size pkm
  void* pack[3] = {nullptr, nullptr, nullptr};
  int pkm = 0;
  // kind 2: H = sum of n_fterms Pauli strings on nA + nB sites (n = 2^(nA+nB)); with
  // PsiA / PsiB set, the operator is Q H Q + sigma P instead, P the projector on the
  // retained product states PsiA[a] (x) PsiB[b] (rows of kA x 2^nA and kB x 2^nB)
  const FullTerm* fterms = nullptr;
  int n_fterms = 0, nA = 0, nB = 0;
  const double* PsiA = nullptr;
  const double* PsiB = nullptr;
  double sigma = 0.0;
};

struct SolveStats {
  int iters = 0;
  int matvecs = 0;
  int rr_sweeps = 0;
  double max_res = 0.0;
  int status = RMC_OK;
};

// Block apply: out = s1 * (H Y) + s2 * Y + s3 * Xprev for nv vectors (rows).
void op_apply(rmc_ctx* ctx, const CoupledOp& op, int nv, const double* Y, double* out,
              const double* Xprev, double s1, double s2, double s3, double* zwork,
              double* kwork, int precision, const double* Ecorr = nullptr,
              const double* phi = nullptr);
size_t op_zwork_doubles(const CoupledOp& op, int nv);

// Lowest nev eigenpairs of op. X_out: device nev x n (rows = eigenvectors);
// evals: host nev. Returns RMC_OK or RMC_ERR_NOCONV.
int eig_lowest(rmc_ctx* ctx, const CoupledOp& op, int nev, const rmc_solve_opts& o,
               double* X_out, std::vector<double>& evals, SolveStats& st);

// Batched form: lowest nevs[i] eigenpairs of each operator (all of one kind).
void eig_lowest_batch(rmc_ctx* ctx, const std::vector<const CoupledOp*>& ops,
                      const std::vector<int>& nevs, const rmc_solve_opts& o,
                      const std::vector<double*>& X_out, std::vector<std::vector<double>>& evals,
                      std::vector<SolveStats>& stats);

// Gap rule (k_req < len(w) required for a cut); returns k_eff, gap.
int gap_cut(const std::vector<double>& w, int k_req, double tau, double* gap);

}  // namespace rmc
