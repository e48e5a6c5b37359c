// Matrix-free eigensolver for the lowest eigenpairs of module-coupling steps,
// batched: every problem of a level (across jobs) advances in lockstep and each
// device step is one launch over all active problems (per-problem descriptors).
//
// The paper assembles the k_A k_B square effective Hamiltonian and diagonalises it
// fully (reduced eigenproblem; dense eigensolve of App. A). Here the operator is
// only applied to blocks of vectors, and the lowest nev eigenpairs come from a
// Chebyshev-filtered block subspace iteration with Rayleigh-Ritz (a block
// Davidson-type method whose correction step is a polynomial filter):
//   1. start block: the m lowest diagonal entries as unit vectors plus a small
//      seeded random component; CholeskyQR2; Rayleigh-Ritz;
//   2. repeat: filter the unconverged Ritz vectors with a scaled Chebyshev
//      polynomial damping [theta_{m-1}, upper bound] (degree from the residuals),
//      orthogonalise twice against the locked vectors, CholeskyQR2 (a shifted
//      first pass and a third pass if a pivot fails), Rayleigh-Ritz on the
//      filtered block (Jacobi), residual norms, lock the converged leading ones;
//   3. a final Rayleigh-Ritz over the whole block and the FP64 residual check.
// Coupling steps filter in the residual-driven (defect) form
//   Y_k = X phi_k(Theta) + D_k,  E = H X - X Theta (FP64),
//   D_1 = (sigma_1/e) E,  D_{k+1} = (2 sigma_{k+1}/e)[(H - c) D_k + E phi_k(Theta)]
//                                  - sigma_k sigma_{k+1} D_{k-1},
// in which only H D_k runs in the requested precision (FP64, FP32 or BF16 MFMA):
// its rounding error scales with the defect D, so the FP64 Rayleigh-Ritz and
// residual check recover full accuracy. A problem whose low-precision filter
// stops reducing the residual 10x per iteration moves up (BF16 -> FP32 -> FP64).
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <exception>
#include <functional>
#include <thread>
#include <vector>

#include "rmc_batch.h"
#include "rmc_internal.h"

namespace rmc {

int gap_cut(const std::vector<double>& w, int k_req, double tau, double* gap) {
  int n = (int)w.size();
  if (k_req >= n) {
    *gap = INFINITY;
    return n;
  }
  double scale = std::max(1.0, std::max(std::fabs(w[0]), std::fabs(w[k_req])));
  double tol = tau * scale;
  double g = w[k_req] - w[k_req - 1];
  if (g > tol) {
    *gap = g;
    return k_req;
  }
  int j = k_req - 1;
  while (j >= 1 && w[j] - w[j - 1] <= tol) --j;
  if (j >= 1) {
    *gap = w[j] - w[j - 1];
    return j;
  }
  *gap = g;
  return k_req;
}

namespace {

void sync(rmc_ctx* ctx) { RMC_HIP(hipStreamSynchronize(ctx->stream)); }

// Descriptor tables uploaded in one copy per phase: host staging (pinned, owned by
// the ctx) mirrored into a device region of the arena.
struct DescArena {
  rmc_ctx* ctx;
  hipStream_t st;
  char* host = nullptr;
  char* dev = nullptr;
  size_t cap = 0, used = 0, flushed = 0;
  DescArena(rmc_ctx* c, hipStream_t s, int lane, Scratch& sc, size_t bytes) : ctx(c), st(s) {
    cap = bytes;
    dev = sc.get<char>(bytes);
    if (ctx->pinned_cap[lane] < bytes) {
      if (ctx->pinned[lane]) RMC_HIP(hipHostFree(ctx->pinned[lane]));
      ctx->pinned[lane] = nullptr;
      ctx->pinned_cap[lane] = 0;
      RMC_HIP(hipHostMalloc((void**)&ctx->pinned[lane], bytes));
      ctx->pinned_cap[lane] = bytes;
    }
    host = ctx->pinned[lane];
  }
  template <class T>
  T* add(const T* p, size_t count) {
    size_t off = (used + 63) & ~(size_t)63;
    size_t b = count * sizeof(T);
    RMC_CHECK(off + b <= cap, RMC_ERR_OOM, "descriptor table overflow");
    if (b) memcpy(host + off, p, b);
    used = off + b;
    return reinterpret_cast<T*>(dev + off);
  }
  template <class T>
  T* add(const std::vector<T>& v) {
    return add(v.data(), v.size());
  }
  // Launches are queued and issued after one upload of everything added so far. While
  // `hold` is set (an iteration being built for graph replay) flushes wait for the one
  // at its end.
  std::vector<std::function<void()>> pending;
  bool hold = false;
  void defer(std::function<void()> f) { pending.push_back(std::move(f)); }
  void flush() {
    if (hold) return;
    if (used > flushed)
      RMC_HIP(hipMemcpyAsync(dev + flushed, host + flushed, used - flushed,
                             hipMemcpyHostToDevice, st));
    flushed = used;
    for (auto& f : pending) f();
    pending.clear();
  }
  // Replay of an already captured iteration: its graph copies the (rewritten, equally
  // laid out) host tables and runs the same launches, so the queued ones are dropped.
  void drop() {
    flushed = used;
    pending.clear();
  }
  void reset() { used = flushed = 0; }  // only after the stream has been synchronised
};

struct BP {
  const CoupledOp* op;
  double* Xout;
  int n, m, nev, guard;
  int ks = 1;  // K-slices of its Gram products (partials summed before use)
  double *X, *HX, *Y[3], *E, *S, *Linv, *Vwork, *Pm, *kwork;
  double *theta, *res;
  double *wPY = nullptr, *wH = nullptr, *wPH = nullptr, *wT = nullptr, *wU = nullptr;  // kind 2, projected
  int* info;
  int* sel;
  // host state
  std::vector<double> th, rs;
  int nlock = 0, nw = 0, prec = RMC_FP64, iters = 0, matvecs = 0, rr_sweeps = 0, cnt = 0;
  int state = 0;  // 0 active, 1 converged, 2 retry with more guard vectors, 3 out of iterations
  int deg = 2;
  double prev_worst = INFINITY, prev_expect = 1.0, scale = 1.0, a = 0, b = 0, c = 0, e = 1, sigma1 = 0;
  int shifted = 0;
  int slow = 0;  // consecutive filters far short of their damping, not rounding-limited
  // CholeskyQR flags to read with the next state: 1 after a two-pass orthonormalisation
  // (role ortho_r), 2 after a third pass
  int ortho_check = 0, ortho_r = 0;
};

struct Batch {
  rmc_ctx* ctx;
  hipStream_t st = nullptr;  // the lane's stream: every launch of this batch goes there
  int lane = 0;
  int kind;
  int mmax = 0, nmax = 0, kAmax = 0, kBmax = 0;
  DescArena* da;
  double* TR = nullptr;  // per-problem theta / res / info block
  long trs = 0;          // its stride (doubles)
  std::vector<double> TRh;
  double* phi_dev = nullptr;  // the fused filters' phi_k rows (device), phi_cap doubles
  size_t phi_cap = 0;
};

// Row-block roles: 0..2 = Y[i], 3 = X + nlock rows, 4 = HX + nlock rows, 5 = E,
// 6 = X (row 0), 7 = HX (row 0).
// defect rows E of the active block (E is kept for every row of the block)
const double* defect_of(const BP* p) { return p->E + (size_t)p->nlock * p->n; }

double* role_ptr(BP* p, int role) {
  switch (role) {
    case 0: case 1: case 2: return p->Y[role];
    case 3: return p->X + (size_t)p->nlock * p->n;
    case 4: return p->HX + (size_t)p->nlock * p->n;
    case 5: return p->E;
    case 6: return p->X;
    case 7: return p->HX;
  }
  return nullptr;
}

void vec_launch(Batch& B, VecOp op, const std::vector<VecDesc>& d) {
  if (d.empty()) return;
  int nvmax = 0;
  long emax = 0;
  for (auto& x : d) {
    nvmax = std::max(nvmax, x.nv);
    emax = std::max(emax, (long)x.nv * x.n);
  }
  const VecDesc* dd = B.da->add(d);
  hipStream_t st = B.st;
  const int P = (int)d.size();
  B.da->defer([=] { vec_batched(st, op, dd, P, nvmax, emax); });
}

void gemm_launch(Batch& B, bool tA, bool tB, const std::vector<GemmDesc>& d, int ksplit) {
  if (d.empty()) return;
  int Mmax = 0, Nmax = 0;
  for (auto& x : d) {
    Mmax = std::max(Mmax, x.M);
    Nmax = std::max(Nmax, x.N);
  }
  const GemmDesc* dd = B.da->add(d);
  hipStream_t st = B.st;
  const int P = (int)d.size();
  B.da->defer([=] { gemm_batched(st, tA, tB, dd, P, Mmax, Nmax, ksplit); });
}

// (caller holds ctx->prof_mu)
hipEvent_t take_event(rmc_ctx* ctx) {
  hipEvent_t e;
  if (!ctx->ev_pool.empty()) {
    e = ctx->ev_pool.back();
    ctx->ev_pool.pop_back();
  } else {
    RMC_HIP(hipEventCreate(&e));
  }
  return e;
}

struct Apply {
  std::vector<const double*> Y, prev, E, phi;
  std::vector<double*> out;
  std::vector<std::array<double, 3>> sc;
  std::vector<int> cnt;
};

// dst = P src for cnt rows of 2^(nA+nB) per problem, P = (PsiA^T PsiA) (x) (PsiB^T PsiB):
// each row as a 2^nA x 2^nB matrix Y, P Y = PsiA^T (PsiA Y PsiB^T) PsiB, in four
// grouped GEMMs (the outer two over all rows of a problem at once).
void proj_launch(Batch& B, const std::vector<BP*>& L, const std::vector<const double*>& src,
                 const std::vector<double*>& dst, const std::vector<int>& cnt) {
  std::vector<GemmDesc> g1, g2, g3, g4;
  for (size_t i = 0; i < L.size(); ++i) {
    const CoupledOp& op = *L[i]->op;
    const int DA = 1 << op.nA, DB = 1 << op.nB, kA = op.kA, kB = op.kB, c = cnt[i];
    double* T = L[i]->wT;
    double* U = L[i]->wU;
    GemmDesc d{};
    d.alpha = 1.0; d.beta = 0.0;
    // T (c DA x kB) = Y (c DA x DB) PsiB^T
    d.M = c * DA; d.N = kB; d.K = DB;
    d.A = src[i]; d.lda = DB; d.B = op.PsiB; d.ldb = DB; d.C = T; d.ldc = kB;
    g1.push_back(d);
    // Q = P Y = T2 (c DA x kB) PsiB with T2_v = PsiA^T U_v
    d.M = c * DA; d.N = DB; d.K = kB;
    d.A = T; d.lda = kB; d.B = op.PsiB; d.ldb = DB; d.C = dst[i]; d.ldc = DB;
    g4.push_back(d);
    for (int v = 0; v < c; ++v) {
      GemmDesc e{};
      e.alpha = 1.0; e.beta = 0.0;
      // U_v (kA x kB) = PsiA (kA x DA) T_v (DA x kB)
      e.M = kA; e.N = kB; e.K = DA;
      e.A = op.PsiA; e.lda = DA; e.B = T + (size_t)v * DA * kB; e.ldb = kB;
      e.C = U + (size_t)v * kA * kB; e.ldc = kB;
      g2.push_back(e);
      // T_v (DA x kB) = PsiA^T U_v
      e.M = DA; e.N = kB; e.K = kA;
      e.A = op.PsiA; e.lda = DA; e.B = U + (size_t)v * kA * kB; e.ldb = kB;
      e.C = T + (size_t)v * DA * kB; e.ldc = kB;
      g3.push_back(e);
    }
  }
  gemm_launch(B, false, true, g1, 1);
  gemm_launch(B, false, false, g2, 1);
  gemm_launch(B, true, false, g3, 1);
  gemm_launch(B, false, false, g4, 1);
}

void pauli_launch(Batch& B, const std::vector<PauliDesc>& d) {
  if (d.empty()) return;
  long emax = 0;
  double flops = 0.0, bytes = 0.0;
  for (auto& x : d) {
    const double amp = (double)((long)x.nv << x.n_sites);
    emax = std::max(emax, (long)x.nv << x.n_sites);
    flops += 2.0 * x.n_terms * amp;
    bytes += 8.0 * amp * (2.0 + (x.sub ? 1.0 : 0.0) + (x.Y0 ? 1.0 : 0.0) + (x.Xprev ? 1.0 : 0.0));
  }
  const PauliDesc* dd = B.da->add(d);
  hipStream_t st = B.st;
  const int P = (int)d.size();
  rmc_ctx* ctx = B.ctx;
  if (!ctx->prof) {
    B.da->defer([=] { pauli_batched(st, dd, P, emax); });
    return;
  }
  rmc_ctx::ProfRec r;
  {
    std::lock_guard<std::mutex> lk(ctx->prof_mu);
    r.a = take_event(ctx);
    r.b = take_event(ctx);
  }
  hipEvent_t ea = r.a, eb = r.b;
  B.da->defer([=] {
    RMC_HIP(hipEventRecord(ea, st));
    pauli_batched(st, dd, P, emax);
    RMC_HIP(hipEventRecord(eb, st));
  });
  r.flops = flops;
  r.bytes = bytes;
  r.prec = RMC_FP64;
  r.kind = RMC_PROF_PAULI;
  std::lock_guard<std::mutex> lk(ctx->prof_mu);
  ctx->prof_recs.push_back(r);
}

// Full-space operators: out = s1 Hsel Y + s2 Y + s3 Xprev, Hsel = H, or
// Q H Q + sigma P = (H q - P H q) + sigma P Y with q = Y - P Y.
void apply_full(Batch& B, const std::vector<BP*>& L, const Apply& a) {
  std::vector<PauliDesc> pd;
  std::vector<BP*> L1;
  std::vector<size_t> i1;
  std::vector<const double*> s1;
  std::vector<double*> d1;
  std::vector<int> c1;
  for (size_t i = 0; i < L.size(); ++i) {
    BP* p = L[i];
    const CoupledOp& op = *p->op;
    PauliDesc d{};
    d.n_sites = op.nA + op.nB; d.n_terms = op.n_fterms; d.nv = a.cnt[i]; d.terms = op.fterms;
    d.Y = a.Y[i];
    if (!op.PsiA) {
      d.out = a.out[i]; d.Y0 = a.Y[i]; d.Xprev = a.prev[i];
      d.s1 = a.sc[i][0]; d.s2 = a.sc[i][1]; d.s3 = a.sc[i][2];
    } else {
      d.Y = p->wPH; d.out = p->wH; d.s1 = 1.0;  // q = Y - P Y, staged in wPH
      L1.push_back(p); i1.push_back(i);
      s1.push_back(a.Y[i]); d1.push_back(p->wPY); c1.push_back(a.cnt[i]);
    }
    pd.push_back(d);
  }
  proj_launch(B, L1, s1, d1, c1);  // P Y
  if (!L1.empty()) {
    std::vector<LinDesc> qd;
    long qmax = 0;
    for (size_t t = 0; t < L1.size(); ++t) {
      LinDesc d{};
      d.n = (long)c1[t] * L1[t]->n; d.out = L1[t]->wPH;
      d.U[0] = s1[t]; d.w[0] = 1.0;
      d.U[1] = L1[t]->wPY; d.w[1] = -1.0;
      qd.push_back(d);
      qmax = std::max(qmax, d.n);
    }
    const LinDesc* qq = B.da->add(qd);
    hipStream_t st = B.st;
    const int nq = (int)qd.size();
    B.da->defer([=] { lincomb_batched(st, qq, nq, qmax); });
  }
  pauli_launch(B, pd);             // plain problems done; H q for the others
  if (L1.empty()) return;
  for (size_t t = 0; t < L1.size(); ++t) s1[t] = L1[t]->wH, d1[t] = L1[t]->wPH;
  proj_launch(B, L1, s1, d1, c1);  // P H q
  std::vector<LinDesc> ld;
  long nmax = 0;
  for (size_t t = 0; t < L1.size(); ++t) {
    BP* p = L1[t];
    const size_t i = i1[t];
    const double sA = a.sc[i][0];
    LinDesc d{};
    d.n = (long)a.cnt[i] * p->n; d.out = a.out[i];
    d.U[0] = p->wH; d.w[0] = sA;
    d.U[1] = p->wPH; d.w[1] = -sA;
    d.U[2] = p->wPY; d.w[2] = sA * p->op->sigma;
    d.U[3] = a.Y[i]; d.w[3] = a.sc[i][1];
    d.U[4] = a.prev[i]; d.w[4] = a.sc[i][2];
    ld.push_back(d);
    nmax = std::max(nmax, d.n);
  }
  const LinDesc* dd = B.da->add(ld);
  hipStream_t st = B.st;
  const int P = (int)ld.size();
  B.da->defer([=] { lincomb_batched(st, dd, P, nmax); });
}

// out = s1 H Y + s2 Y + s3 Xprev (+ s1 phi E) for every problem of L.
void apply_launch(Batch& B, const std::vector<BP*>& L, const Apply& a, bool use_prec) {
  if (L.empty()) return;
  rmc_ctx* ctx = B.ctx;
  if (B.kind == 2) {
    apply_full(B, L, a);
    return;
  }
  if (B.kind == 0) {  // dense leaf: GEMM then axpy
    std::vector<GemmDesc> g;
    std::vector<VecDesc> v;
    for (size_t i = 0; i < L.size(); ++i) {
      BP* p = L[i];
      GemmDesc d{};
      d.M = a.cnt[i]; d.N = p->n; d.K = p->n;
      d.A = a.Y[i]; d.lda = p->n;
      d.B = p->op->H; d.ldb = p->n;
      d.C = a.out[i]; d.ldc = p->n;
      d.alpha = a.sc[i][0]; d.beta = 0.0; d.work = nullptr;
      g.push_back(d);
      VecDesc w{};
      w.nv = a.cnt[i]; w.n = p->n; w.out = a.out[i]; w.P = a.Y[i]; w.Q = a.prev[i];
      w.b = a.sc[i][1]; w.c = a.sc[i][2];
      v.push_back(w);
    }
    gemm_launch(B, false, true, g, 1);
    vec_launch(B, VEC_AXPY3, v);
    return;
  }
  // one launch per precision and tile class (the padded tile of the streaming
  // kernel, 32 / 64 / 96 / 128, or wider): each problem gets the kernel of its own size
  // rather than that of the largest problem of the batch
  auto tile_class = [](const CoupledOp* op) {
    const int k = std::max(op->kA, op->kB);
    return k <= 32 ? 0 : (k <= 64 ? 1 : (k <= 96 ? 2 : (k <= 128 ? 3 : 4)));
  };
  for (int pc = 0; pc < 15; ++pc) {
    const int prec = pc / 5, cls = pc % 5;
    std::vector<KronDesc> kd;
    int nvmax = 0, Tm = 0, kAm = 0, kBm = 0;
    long tv = 0;
    for (size_t i = 0; i < L.size(); ++i) {
      BP* p = L[i];
      int pr = use_prec ? p->prec : RMC_FP64;
      if (pr != prec || tile_class(p->op) != cls) continue;
      kAm = std::max(kAm, p->op->kA);
      kBm = std::max(kBm, p->op->kB);
      KronDesc d{};
      d.kA = p->op->kA; d.kB = p->op->kB; d.T = p->op->T; d.nv = a.cnt[i];
      d.coef = p->op->coef_dev; d.OA = p->op->OAcat; d.OB = p->op->OBcat; d.Ediag = p->op->Ediag;
      d.Y = a.Y[i]; d.Xprev = a.prev[i]; d.E = a.E[i]; d.phi = a.phi[i]; d.out = a.out[i];
      d.s1 = a.sc[i][0]; d.s2 = a.sc[i][1]; d.s3 = a.sc[i][2];
      d.vbase = tv;
      d.pack = p->op->pack[prec];
      d.pkm = p->op->pkm;
      kd.push_back(d);
      nvmax = std::max(nvmax, a.cnt[i]);
      Tm = std::max(Tm, d.T);
      tv += a.cnt[i];
    }
    if (kd.empty()) continue;
    const KronDesc* dd = B.da->add(kd);
    hipStream_t st = B.st;
    const int P = (int)kd.size();
    if (!ctx->prof) {
      B.da->defer([=] { kron_batched(st, dd, P, kBm, nvmax, kAm, prec, Tm, tv); });
      continue;
    }
    rmc_ctx::ProfRec r;
    {
      std::lock_guard<std::mutex> lk(ctx->prof_mu);
      r.a = take_event(ctx);
      r.b = take_event(ctx);
    }
    hipEvent_t ea = r.a, eb = r.b;
    B.da->defer([=] {
      RMC_HIP(hipEventRecord(ea, st));
      kron_batched(st, dd, P, kBm, nvmax, kAm, prec, Tm, tv);
      RMC_HIP(hipEventRecord(eb, st));
    });
    r.flops = r.bytes = 0.0;
    r.prec = prec;
    for (auto& d : kd) {
      const double nn = (double)d.kA * d.kB;
      r.flops += (double)d.nv * (2.0 * d.T * nn * (d.kA + d.kB) + 4.0 * nn);
      r.bytes += 8.0 * nn * ((double)d.nv * (2.0 + (d.Xprev ? 1.0 : 0.0) + (d.E ? 1.0 : 0.0)) + 1.0) +
                 8.0 * d.T * ((double)d.kA * d.kA + (double)d.kB * d.kB);
    }
    std::lock_guard<std::mutex> lk(ctx->prof_mu);
    ctx->prof_recs.push_back(r);
  }
}

// Gram partials A B^T (ca x cb per problem) into p->kwork. `sym`: the product is
// symmetric (Q^T H Q), so only the tiles on and above the diagonal are formed and
// mirrored (the consumer symmetrises the diagonal tiles).
void gram_launch(Batch& B, const std::vector<BP*>& L, const std::vector<const double*>& Ap,
                 const std::vector<const double*>& Bp, const std::vector<int>& ca,
                 const std::vector<int>& cb, bool sym = false) {
  if (L.empty()) return;
  std::vector<GramDesc> g;
  int cmax = 0, ksmax = 1;
  for (size_t i = 0; i < L.size(); ++i) {
    BP* p = L[i];
    GramDesc d{};
    d.ca = ca[i]; d.cb = cb[i]; d.n = p->n; d.sym = sym && ca[i] == cb[i] ? 1 : 0;
    d.ks = p->ks;
    d.A = Ap[i]; d.B = Bp[i]; d.work = p->kwork;
    g.push_back(d);
    cmax = std::max(cmax, std::max(ca[i], cb[i]));
    ksmax = std::max(ksmax, p->ks);
  }
  const GramDesc* dd = B.da->add(g);
  hipStream_t st = B.st;
  const int P = (int)g.size();
  B.da->defer([=] { gram_batched(st, dd, P, ksmax, cmax); });
}

void read_state(Batch& B) {
  B.da->flush();
  RMC_HIP(hipMemcpyAsync(B.TRh.data(), B.TR, B.TRh.size() * sizeof(double), hipMemcpyDeviceToHost,
                         B.st));
  RMC_HOST_SCOPE("solve.state_wait");
  RMC_HIP(hipStreamSynchronize(B.st));
  B.da->reset();
}

int info_of(const Batch& B, int idx, int k) {
  const int* ip = reinterpret_cast<const int*>(B.TRh.data() + (size_t)idx * B.trs + 2 * B.mmax);
  return ip[k];
}

// Sum of the Gram's split-K partials (cnt x cnt each, in p->kwork) into p->Pm with one
// chip-wide launch, so that the one-workgroup Cholesky and Jacobi kernels read a single
// matrix instead of every partial; returns null when there is one partial only.
const double* reduce_parts(Batch& B, const std::vector<BP*>& L) {
  bool any = false;
  for (BP* p : L) any = any || p->ks > 1;
  if (!any) return nullptr;
  std::vector<VecDesc> rd;
  for (BP* p : L) {
    VecDesc v{};
    v.nv = p->ks; v.n = p->cnt * p->cnt; v.out = p->Pm; v.P = p->kwork;
    rd.push_back(v);
  }
  vec_launch(B, VEC_REDUCE, rd);
  return L[0]->Pm;  // non-null marker: every problem's sum is in its own Pm
}

// One CholeskyQR pass from role src to role dst for the problems of L; the Cholesky
// kernel leaves its failure flag in info[slot] and its shift flag in info[slot + 1].
void cholqr_pass(Batch& B, const std::vector<BP*>& L, int src, int dst, int slot) {
  const double u = 1.1102230246251565e-16;
  std::vector<const double*> A;
  std::vector<int> ca;
  for (BP* p : L) {
    A.push_back(role_ptr(p, src));
    ca.push_back(p->cnt);
  }
  gram_launch(B, L, A, A, ca, ca);
  const double* G = reduce_parts(B, L);
  std::vector<CholDesc> cd;
  int mm = 0;
  for (BP* p : L) {
    CholDesc c{};
    c.m = p->cnt; c.nparts = G ? 1 : p->ks; c.G = G ? p->Pm : p->kwork; c.pstride = (long)p->cnt * p->cnt;
    c.Linv = p->Linv; c.info = p->info + slot;
    c.shift = 11.0 * ((double)p->n * p->cnt + (double)p->cnt * (p->cnt + 1)) * u * p->cnt;
    cd.push_back(c);
    mm = std::max(mm, p->cnt);
  }
  const CholDesc* dd = B.da->add(cd);
  {
    hipStream_t st = B.st;
    const int P = (int)cd.size();
    B.da->defer([=] { chol_batched(st, dd, P, mm); });
  }
  std::vector<GemmDesc> g;
  for (BP* p : L) {
    GemmDesc d{};
    d.M = p->cnt; d.N = p->n; d.K = p->cnt;
    d.A = p->Linv; d.lda = p->cnt; d.B = role_ptr(p, src); d.ldb = p->n;
    d.C = role_ptr(p, dst); d.ldc = p->n; d.alpha = 1.0; d.beta = 0.0;
    g.push_back(d);
  }
  gemm_launch(B, false, false, g, 1);
}

// Orthonormalise the cnt rows at Y[r] of each problem against its locked rows
// X[0..nlock), then among themselves. The result ends in Y[r].
void orthonormalize(Batch& B, const std::vector<BP*>& L, int r) {
  std::vector<BP*> LL;
  for (BP* p : L)
    if (p->nlock > 0) LL.push_back(p);
  if (!LL.empty()) {
    // Y -= (Y X_lock^T) X_lock twice (invariant to the scale of Y's rows, so it runs
    // before the normalisation)
    for (int pass = 0; pass < 2; ++pass) {
      // P = Y X_lock^T as split-K partials, reduced, then Y -= P X_lock
      std::vector<const double*> A, Bl;
      std::vector<int> ca, cb;
      for (BP* p : LL) {
        A.push_back(role_ptr(p, r));
        Bl.push_back(p->X);
        ca.push_back(p->cnt);
        cb.push_back(p->nlock);
      }
      gram_launch(B, LL, A, Bl, ca, cb);
      std::vector<VecDesc> rd;
      std::vector<GemmDesc> g2;
      for (BP* p : LL) {
        VecDesc v{};
        v.nv = p->ks; v.n = p->cnt * p->nlock; v.out = p->Pm; v.P = p->kwork;
        rd.push_back(v);
        GemmDesc e{};
        e.M = p->cnt; e.N = p->n; e.K = p->nlock;
        e.A = p->Pm; e.lda = p->nlock; e.B = p->X; e.ldb = p->n;
        e.C = role_ptr(p, r); e.ldc = p->n; e.alpha = -1.0; e.beta = 1.0;
        g2.push_back(e);
      }
      vec_launch(B, VEC_REDUCE, rd);
      gemm_launch(B, false, false, g2, 1);
    }
  }
  // unit rows into CholeskyQR
  std::vector<VecDesc> nd;
  for (BP* p : L) {
    VecDesc v{};
    v.nv = p->cnt; v.n = p->n; v.out = role_ptr(p, r);
    nd.push_back(v);
  }
  vec_launch(B, VEC_NORMALIZE, nd);
  // CholeskyQR2; its flags are read with the next state (ortho_fixup), so that the
  // common case costs no host round trip
  const int sp = (r == 0) ? 1 : 0;
  cholqr_pass(B, L, r, sp, 2);
  cholqr_pass(B, L, sp, r, 4);
  for (BP* p : L) {
    p->ortho_check = 1;
    p->ortho_r = r;
  }
}

// Rayleigh-Ritz of the orthonormal rows at role q (cnt rows), W = H Q into role w
// (already there when `full`); Ritz pairs into X/HX/theta/res at row offset nlock,
// or, when `full`, into Y[2]/E/theta/res from row 0.
void rayleigh_ritz(Batch& B, const std::vector<BP*>& L, int q, int w, bool full) {
  if (!full) {
    Apply a;
    for (BP* p : L) {
      a.Y.push_back(role_ptr(p, q));
      a.out.push_back(role_ptr(p, w));
      a.prev.push_back(nullptr);
      a.E.push_back(nullptr);
      a.phi.push_back(nullptr);
      a.sc.push_back({1.0, 0.0, 0.0});
      a.cnt.push_back(p->cnt);
    }
    apply_launch(B, L, a, false);
    for (BP* p : L) p->matvecs += p->cnt;
  }
  std::vector<const double*> A, Bm;
  std::vector<int> cnt;
  for (BP* p : L) {
    A.push_back(role_ptr(p, q));
    Bm.push_back(role_ptr(p, w));
    cnt.push_back(p->cnt);
  }
  gram_launch(B, L, A, Bm, cnt, cnt, true);
  const double* G = reduce_parts(B, L);
  std::vector<EigDesc> ed;
  int mm = 0;
  for (BP* p : L) {
    EigDesc d{};
    d.m = p->cnt; d.nparts = G ? 1 : p->ks; d.A = G ? p->Pm : p->kwork; d.pstride = (long)p->cnt * p->cnt;
    d.evals = p->theta + (full ? 0 : p->nlock); d.V = p->S; d.Vwork = p->Vwork; d.info = p->info + 1;
    ed.push_back(d);
    mm = std::max(mm, p->cnt);
  }
  const EigDesc* dd = B.da->add(ed);
  {
    hipStream_t st = B.st;
    const int P = (int)ed.size();
    B.da->defer([=] { jacobi_batched(st, dd, P, mm); });
  }
  std::vector<GemmDesc> g1, g2;
  for (BP* p : L) {
    const size_t off = full ? 0 : (size_t)p->nlock * p->n;
    GemmDesc d{};
    d.M = p->cnt; d.N = p->n; d.K = p->cnt;
    d.A = p->S; d.lda = p->cnt; d.B = role_ptr(p, q); d.ldb = p->n;
    d.C = full ? p->Y[2] : p->X + off; d.ldc = p->n; d.alpha = 1.0; d.beta = 0.0;
    g1.push_back(d);
    d.B = role_ptr(p, w);
    d.C = full ? p->E : p->HX + off;
    g2.push_back(d);
  }
  g1.insert(g1.end(), g2.begin(), g2.end());  // X and H X in one launch
  gemm_launch(B, true, false, g1, 1);
  std::vector<VecDesc> rd;
  for (BP* p : L) {
    const size_t off = full ? 0 : (size_t)p->nlock * p->n;
    VecDesc v{};
    v.nv = p->cnt; v.n = p->n;
    v.P = full ? p->E : p->HX + off;
    v.Q = full ? p->Y[2] : p->X + off;
    v.a = p->theta + (full ? 0 : p->nlock);
    v.norms = p->res + (full ? 0 : p->nlock);
    // inside the iteration the residual rows are the next filter's defect E = HX - X Theta
    // (E holds every row of the block; the filter starts at its own lock count)
    v.out = full ? nullptr : p->E + off;
    rd.push_back(v);
  }
  vec_launch(B, VEC_RESIDUAL, rd);
}

// After a state read: a failed Cholesky (even with its shift) is an error; problems
// whose first CholeskyQR pass needed the shift (shifted CholeskyQR) get the third pass
// and their Rayleigh-Ritz again. Returns true when the state must be read again.
bool ortho_fixup(Batch& B, const std::vector<BP*>& probs) {
  std::vector<BP*> L3;
  for (size_t i = 0; i < probs.size(); ++i) {
    BP* p = probs[i];
    const int chk = p->ortho_check;
    p->ortho_check = 0;
    if (chk == 1) {
      RMC_CHECK(info_of(B, (int)i, 2) == 0 && info_of(B, (int)i, 4) == 0, RMC_ERR_NOCONV,
                "CholeskyQR failed even with a shift");
      if (info_of(B, (int)i, 3)) L3.push_back(p);
    } else if (chk == 2) {
      RMC_CHECK(info_of(B, (int)i, 6) == 0, RMC_ERR_NOCONV, "CholeskyQR failed even with a shift");
    }
  }
  if (L3.empty()) return false;
  for (int r = 0; r < 2; ++r) {
    std::vector<BP*> Lr;
    for (BP* p : L3)
      if (p->ortho_r == r) Lr.push_back(p);
    if (Lr.empty()) continue;
    const int sp = r == 0 ? 1 : 0;
    cholqr_pass(B, Lr, r, sp, 6);
    std::vector<VecDesc> cp;
    for (BP* p : Lr) {
      VecDesc v{};
      v.nv = p->cnt; v.n = p->n; v.out = role_ptr(p, r); v.P = role_ptr(p, sp);
      cp.push_back(v);
      p->shifted++;
      p->ortho_check = 2;
      if (getenv("RMC_TRACE_SOLVER"))
        fprintf(stderr, "[rmc] n=%d it=%d third CholeskyQR pass\n", p->n, p->iters);
    }
    vec_launch(B, VEC_COPY, cp);
    rayleigh_ritz(B, Lr, r, sp, false);
  }
  return true;
}

// Convergence bookkeeping after a state read; returns true if the problem goes on.
bool update_problem(Batch& B, BP* p, int idx, int max_iter, double tol, int pmax, bool last_attempt) {
  const int m = p->m, n = p->n, nev = p->nev;
  const double* t = B.TRh.data() + (size_t)idx * B.trs;
  p->th.assign(t, t + m);
  p->rs.assign(t + B.mmax, t + B.mmax + m);
  p->rr_sweeps += std::abs(info_of(B, idx, 1));
  const auto& th = p->th;
  const auto& rs = p->rs;
  p->scale = std::max({1.0, std::fabs(p->op->bup), std::fabs(th[0])});
  const double scale = p->scale;
  // wanted set: the nev lowest plus the rest of the cluster holding theta[nev-1]
  int nw = nev;
  while (nw < m && th[nw] - th[nw - 1] <= 1e-6 * scale) ++nw;
  if (nw >= m && m < n) {
    // the cluster runs to the end of the block: the filter cannot separate it
    if (!last_attempt) {
      p->state = 2;
      return false;
    }
    nw = m;
  }
  p->nw = nw;
  int first_bad = nw;
  for (int j = 0; j < nw; ++j)
    if (!(rs[j] <= tol * scale)) {
      first_bad = j;
      break;
    }
  if (first_bad == nw || m == n) {
    p->state = 1;
    return false;
  }
  if (p->iters >= max_iter) {
    p->state = last_attempt ? 3 : 2;
    return false;
  }
  p->nlock = std::max(p->nlock, first_bad);
  double worst = 0.0;
  for (int j = p->nlock; j < nw; ++j) worst = std::max(worst, rs[j]);
  // At the rounding floor of the residual (every unlocked wanted residual within the
  // final acceptance bound of 10 tol and no longer halving per filter): done. The
  // residuals come from rotated products H Q, whose FP64 rounding can sit just above
  // tol on some spectra; iterating on would only spin to the iteration cap.
  if (p->iters > 1 && worst <= 10.0 * tol * scale && worst > 0.5 * p->prev_worst) {
    p->state = 1;
    return false;
  }
  // Per-iteration residual reduction the low-precision filter can deliver (its
  // rounding noise relative to the filtered defect); the filter does not aim below it.
  const double floor_red = p->prec == RMC_BF16 ? 3e-2 : (p->prec == RMC_FP32 ? 1e-5 : 0.0);
  // escalate when the last filter fell well short of both its Chebyshev damping and
  // that floor by a margin rounding noise explains (a reduction within 1e3 of the
  // floor): the noise of this precision now dominates. A far weaker reduction comes
  // from the spectrum (a cluster at the cut, Ritz values still rough), which more
  // precision does not cure; it escalates only after three such filters in a row.
  // The first filter is not judged: its Ritz values and bounds come from the start block.
  static const bool no_ladder = getenv("RMC_NO_LADDER") != nullptr;
  if (p->prec != RMC_FP64 && p->iters > 1 && !no_ladder) {
    if (worst > std::max(floor_red, 100.0 * p->prev_expect) * p->prev_worst) {
      if (worst < 1e3 * floor_red * p->prev_worst || ++p->slow >= 3) {
        p->prec = p->prec == RMC_BF16 ? RMC_FP32 : RMC_FP64;
        p->slow = 0;
      }
    } else {
      p->slow = 0;
    }
  }
  p->prev_worst = worst;
  p->cnt = m - p->nlock;
  double a = th[m - 1], b = p->op->bup, a0 = th[0];
  if (!(b > a)) b = a + std::max(1e-3 * std::fabs(a), 1e-6);
  if (!(a0 < a)) a0 = a - 1e-3 * (b - a);
  p->a = a;
  p->b = b;
  p->e = 0.5 * (b - a);
  p->c = 0.5 * (b + a);
  p->sigma1 = p->e / (a0 - p->c);
  const double fl = p->prec == RMC_BF16 ? 3e-2 : (p->prec == RMC_FP32 ? 1e-5 : 0.0);
  int deg = 2;
  for (int j = p->nlock; j < nw; ++j) {
    if (rs[j] <= tol * scale) continue;
    double x = std::fabs((th[j] - p->c) / p->e);
    double rho = x > 1.0 ? std::acosh(x) : 1e-3;
    double target = 2.0 * rs[j] / (tol * scale);
    if (fl > 0.0) target = std::min(target, 1.0 / fl);
    double need = std::log(target) / rho;
    deg = std::max(deg, (int)std::ceil(need));
  }
  // FP32 filters above degree ~24 stall at a noise floor on these spectra (rounding
  // noise grows with the spread of T_deg over the wanted set); with each problem at its
  // own degree, a cap of 22 balances filter length against outer iterations best on the
  // random-field batch (caps 16-24 measured); BF16 is held lower by its reduction target
  static const int fp32_cap = [] {
    const char* e = getenv("RMC_FP32_MAXDEG");
    return e ? std::max(2, atoi(e)) : 22;
  }();
  if (p->prec == RMC_FP32) deg = std::min(deg, fp32_cap);
  p->deg = std::min(std::max(deg, 2), pmax);
  // damping 1 / T_deg(x) of the slowest active wanted vector
  double expect = 0.0;
  for (int j = p->nlock; j < nw; ++j) {
    if (rs[j] <= tol * scale) continue;
    double x = std::fabs((th[j] - p->c) / p->e);
    double rho = x > 1.0 ? std::acosh(x) : 0.0;
    expect = std::max(expect, rho * p->deg > 700.0 ? 0.0 : 1.0 / std::cosh(rho * p->deg));
  }
  p->prev_expect = expect;
  return true;
}

int filter_steps(Batch& B, const std::vector<BP*>& L, int P, int outr);

// Whole-filter launches (kron_filter_batched), one per precision: the step scalars
// and the phi_k rows of every problem are computed on the host up front (the same
// recurrences as the per-step path) and travel in the descriptor tables. Each problem
// is filtered to its own degree (the kernel takes the step count per descriptor).
// A whole-filter launch (launch()) placed in the lanes' common chain: it starts once
// the previous chained filter of any lane has ended. RMC_FILTER_CHAIN=0: no chain; 2:
// only the 96-wide launches (one workgroup a CU), so that 64-wide launches of lanes in
// lockstep (a batch of identical jobs) may still share the CUs
template <class F>
void filter_in_chain(rmc_ctx* ctx, hipStream_t st, bool wide, F&& launch) {
  static const int mode = [] {
    const char* e = getenv("RMC_FILTER_CHAIN");
    return e ? atoi(e) : 1;
  }();
  const bool on = mode == 1 || (mode == 2 && wide);
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  RMC_HIP(hipStreamIsCapturing(st, &cs));
  if (!on || cs != hipStreamCaptureStatusNone) {  // (a captured iteration keeps its own order)
    launch();
    return;
  }
  std::lock_guard<std::mutex> lk(ctx->filter_mu);
  if (!ctx->filter_ev) RMC_HIP(hipEventCreateWithFlags(&ctx->filter_ev, hipEventDisableTiming));
  if (ctx->filter_ev_set) RMC_HIP(hipStreamWaitEvent(st, ctx->filter_ev, 0));
  launch();
  RMC_HIP(hipEventRecord(ctx->filter_ev, st));
  ctx->filter_ev_set = true;
}

void fused_filter(Batch& B, const std::vector<BP*>& L, int outr) {
  rmc_ctx* ctx = B.ctx;
  // the step scalars of every problem (host) and its phi_k rows, computed by one device
  // launch ahead of the filters from theta_j - c (the same recurrence, in the same
  // operation order, as the per-step path's host rows)
  std::vector<const double*> scp(L.size());
  std::vector<double*> php(L.size());
  {
    std::vector<PhiDesc> phd;
    size_t off = 0;
    for (size_t i = 0; i < L.size(); ++i) {
      BP* p = L[i];
      const int cn = p->cnt, steps = p->deg - 1;
      std::vector<double> sc(3 * (size_t)std::max(steps, 1)), t(std::max(cn, 1));
      for (int j = 0; j < cn; ++j) t[j] = p->th[p->nlock + j] - p->c;
      double sg = p->sigma1, b1 = 0.0;
      const double tau2 = 2.0 / p->sigma1;
      for (int k = 1; k <= steps; ++k) {
        const double sk1 = 1.0 / (tau2 - sg);
        sc[3 * (k - 1)] = 2.0 * sk1 / p->e;
        sc[3 * (k - 1) + 1] = -2.0 * p->c * sk1 / p->e;
        sc[3 * (k - 1) + 2] = k > 1 ? -sg * sk1 : 0.0;
        if (k == 1) b1 = sg * sk1;
        sg = sk1;
      }
      const size_t need = (size_t)(steps + 1) * cn;
      RMC_CHECK(off + need <= B.phi_cap, RMC_ERR_OOM, "filter scalar table overflow");
      php[i] = B.phi_dev + off;
      off += need;
      scp[i] = B.da->add(sc);
      phd.push_back(PhiDesc{cn, steps, p->sigma1 / p->e, b1, B.da->add(t), scp[i], php[i]});
    }
    if (!phd.empty()) {
      const PhiDesc* dd = B.da->add(phd);
      const int np = (int)phd.size();
      hipStream_t st = B.st;
      B.da->defer([=] { filter_phi_batched(st, dd, np); });
    }
  }
  // one launch per precision and tile class: problems up to 64 share the 64-wide kernel
  // (smaller operators padded inside its tiles), 96-wide problems take the wide kernel
  auto wide = [](const CoupledOp& op) { return std::max(op.kA, op.kB) > 64; };
  for (int pc = 0; pc < 6; ++pc) {
    const int prec = pc / 2;
    const bool cls_wide = pc % 2 == 1;
    std::vector<FilterDesc> fd;
    int kmax = 0, Tm = 0;
    long tv = 0;
    double flops = 0.0, bytes = 0.0;
    for (size_t i = 0; i < L.size(); ++i) {
      BP* p = L[i];
      if (p->prec != prec || wide(*p->op) != cls_wide) continue;
      const CoupledOp& op = *p->op;
      const int cn = p->cnt, steps = p->deg - 1;
      FilterDesc d{};
      d.kA = op.kA; d.kB = op.kB; d.T = op.T; d.nv = cn; d.vbase = tv;
      d.pack = op.pack[prec]; d.pkm = op.pkm; d.steps = steps;
      d.Ediag = op.Ediag; d.EA = op.EA; d.EB = op.EB;
      d.E = defect_of(p); d.X = role_ptr(p, 3); d.out = p->Y[outr];
      d.sc = scp[i];
      d.phi = php[i];
      d.r0 = p->sigma1 / p->e;
      fd.push_back(d);
      kmax = std::max(kmax, std::max(op.kA, op.kB));
      Tm = std::max(Tm, op.T);
      tv += cn;
      const double nn = (double)op.kA * op.kB;
      flops += (double)cn * steps * (2.0 * op.T * nn * (op.kA + op.kB) + 4.0 * nn);
      bytes += 8.0 * nn * (3.0 * cn + 1.0) + 8.0 * op.T * ((double)op.kA * op.kA + (double)op.kB * op.kB);
    }
    if (fd.empty()) continue;
    const FilterDesc* dd = B.da->add(fd);
    hipStream_t st = B.st;
    const int nd = (int)fd.size();
    if (!ctx->prof) {
      B.da->defer([=] { filter_in_chain(ctx, st, cls_wide, [&] { kron_filter_batched(st, dd, nd, tv, prec, kmax, Tm); }); });
      continue;
    }
    rmc_ctx::ProfRec r;
    {
      std::lock_guard<std::mutex> lk(ctx->prof_mu);
      r.a = take_event(ctx);
      r.b = take_event(ctx);
    }
    hipEvent_t ea = r.a, eb = r.b;
    B.da->defer([=] {
      filter_in_chain(ctx, st, cls_wide, [&] {
        RMC_HIP(hipEventRecord(ea, st));
        kron_filter_batched(st, dd, nd, tv, prec, kmax, Tm);
        RMC_HIP(hipEventRecord(eb, st));
      });
    });
    r.flops = flops;
    r.bytes = bytes;
    r.prec = prec;
    r.kind = RMC_PROF_KRON_FILTER;
    std::lock_guard<std::mutex> lk(ctx->prof_mu);
    ctx->prof_recs.push_back(r);
  }
}

// One filter application on the problems of L; returns the Y buffer holding it.
int filter(Batch& B, const std::vector<BP*>& L) {
  int P = 0;
  for (BP* p : L) P = std::max(P, p->deg);
  if (B.kind != 1) {
    // dense (leaf): direct scaled recurrence Y_{k+1} = (2s'/e)(H-c)Y_k - s s' Y_{k-1}
    std::vector<double> sig(L.size());
    Apply a;
    for (size_t i = 0; i < L.size(); ++i) {
      BP* p = L[i];
      sig[i] = p->sigma1;
      a.Y.push_back(role_ptr(p, 3));
      a.out.push_back(role_ptr(p, 0));
      a.prev.push_back(nullptr);
      a.E.push_back(nullptr);
      a.phi.push_back(nullptr);
      a.sc.push_back({sig[i] / p->e, -p->c * sig[i] / p->e, 0.0});
      a.cnt.push_back(p->cnt);
    }
    apply_launch(B, L, a, false);
    int prev = 3, cur = 0;
    for (int k = 2; k <= P; ++k) {
      int nw = -1;
      for (int q = 0; q < 3; ++q)
        if (q != cur && q != prev) {
          nw = q;
          break;
        }
      a.Y.clear(); a.out.clear(); a.prev.clear(); a.sc.clear();
      for (size_t i = 0; i < L.size(); ++i) {
        BP* p = L[i];
        const double tau2 = 2.0 / p->sigma1;
        const double s2 = 1.0 / (tau2 - sig[i]);
        a.Y.push_back(role_ptr(p, cur));
        a.out.push_back(role_ptr(p, nw));
        a.prev.push_back(role_ptr(p, prev));
        a.sc.push_back({2.0 * s2 / p->e, -2.0 * p->c * s2 / p->e, -sig[i] * s2});
        sig[i] = s2;
      }
      apply_launch(B, L, a, false);
      prev = cur;
      cur = nw;
    }
    for (BP* p : L) p->matvecs += p->cnt * P;
    return cur;
  }
  // Kronecker problems, defect form: E = HX - X Theta on the active rows was written by
  // the last Rayleigh-Ritz step's residual pass (rows from the lock count on: defect_of)
  // buffer that holds the result: the per-step path rotates three buffers
  int outr;
  {
    int pv = -1, cu = 0;
    for (int k = 1; k < P; ++k) {
      int nw = 0;
      while (nw == cu || nw == pv) ++nw;
      pv = cu;
      cu = nw;
    }
    outr = (cu == 0) ? 1 : 0;
  }
  // problems whose operators fit the fused kernel's LDS run the whole filter in one
  // launch per precision (RMC_FUSED_FILTER=0 keeps every problem on the per-step path)
  std::vector<BP*> Lf, Ls;
  {
    const char* f = getenv("RMC_FUSED_FILTER");
    const bool fused = !(f && atoi(f) == 0);
    for (BP* p : L) {
      const CoupledOp& op = *p->op;
      const bool ok = fused && op.pack[p->prec] && kron_filter_fits(p->prec, op.kA, op.kB, op.T);
      (ok ? Lf : Ls).push_back(p);
    }
  }
  if (!Lf.empty()) fused_filter(B, Lf, outr);
  for (BP* p : Lf) p->matvecs += p->cnt * (p->deg - 1);
  if (Ls.empty()) return outr;
  return filter_steps(B, Ls, P, outr);
}

// The per-step path of the defect-form filter (one Kronecker launch per step for the
// problems of L that still have steps to go: each is filtered to its own degree); the
// result ends in Y[outr].
int filter_steps(Batch& B, const std::vector<BP*>& L, int P, int outr) {
  // phi_k at the active Ritz values, one row per filter step, computed on the host just
  // before the step that uses it (so the device starts on the first steps while later
  // rows are still being computed); row 0 holds sigma_1/e
  const size_t NL = L.size();
  std::vector<std::vector<double>> pm1(NL), pk(NL);
  std::vector<double> sgp(NL), tau2(NL);
  std::vector<const double*> rowk(NL);
  {
    std::vector<VecDesc> dd;
    for (size_t i = 0; i < NL; ++i) {
      BP* p = L[i];
      const int cn = p->cnt;
      std::vector<double> r0(cn, p->sigma1 / p->e);
      const double* row0 = B.da->add(r0);
      pk[i].resize(cn);
      for (int j = 0; j < cn; ++j) pk[i][j] = (p->sigma1 / p->e) * (p->th[p->nlock + j] - p->c);
      pm1[i].assign(cn, 1.0);
      rowk[i] = B.da->add(pk[i]);
      sgp[i] = p->sigma1;
      tau2[i] = 2.0 / p->sigma1;
      VecDesc v{};
      v.nv = p->cnt; v.n = p->n; v.out = p->Y[0]; v.P = defect_of(p); v.a = row0; v.asgn = 1.0;
      v.b = 0.0; v.Q = nullptr;
      dd.push_back(v);
    }
    vec_launch(B, VEC_SCALE_ADD, dd);  // D_1
  }
  int prev = -1, cur = 0;
  std::vector<int> last(NL, 0);  // buffer holding a problem's D at its own degree
  for (int k = 1; k < P; ++k) {
    int nw = -1;
    for (int q = 0; q < 3; ++q)
      if (q != cur && q != prev) {
        nw = q;
        break;
      }
    Apply a;
    std::vector<BP*> Lk;
    std::vector<double> sk1v(NL);
    for (size_t i = 0; i < NL; ++i) {
      BP* p = L[i];
      if (k >= p->deg) continue;  // done: D at its degree sits in Y[last[i]]
      Lk.push_back(p);
      const double sk = sgp[i], sk1 = 1.0 / (tau2[i] - sk);
      sk1v[i] = sk1;
      a.Y.push_back(role_ptr(p, cur));
      a.out.push_back(role_ptr(p, nw));
      a.prev.push_back(prev >= 0 ? role_ptr(p, prev) : nullptr);
      a.E.push_back(defect_of(p));
      a.phi.push_back(rowk[i]);
      a.sc.push_back({2.0 * sk1 / p->e, -2.0 * p->c * sk1 / p->e, prev >= 0 ? -sk * sk1 : 0.0});
      a.cnt.push_back(p->cnt);
    }
    apply_launch(B, Lk, a, true);
    if (k % 8 == 1) B.da->flush();
    // row k+1 of every problem still filtering
    for (size_t i = 0; i < NL; ++i) {
      BP* p = L[i];
      if (k >= p->deg) continue;
      last[i] = nw;
      const int cn = p->cnt;
      const double sg = sgp[i], sg2 = sk1v[i];
      for (int j = 0; j < cn; ++j) {
        const double nx = (2.0 * sg2 / p->e) * (p->th[p->nlock + j] - p->c) * pk[i][j] - sg * sg2 * pm1[i][j];
        pm1[i][j] = pk[i][j];
        pk[i][j] = nx;
      }
      rowk[i] = B.da->add(pk[i]);
      sgp[i] = sg2;
    }
    prev = cur;
    cur = nw;
  }
  RMC_CHECK(outr == ((cur == 0) ? 1 : 0), RMC_ERR_STATE, "filter buffer rotation");
  {
    // (elementwise, so a problem whose D already sits in Y[outr] is combined in place)
    std::vector<VecDesc> dd;
    for (size_t i = 0; i < L.size(); ++i) {
      BP* p = L[i];
      VecDesc v{};
      v.nv = p->cnt; v.n = p->n; v.out = p->Y[outr]; v.P = role_ptr(p, 3);
      v.a = rowk[i]; v.asgn = 1.0; v.b = 1.0; v.Q = p->Y[last[i]];
      dd.push_back(v);
    }
    vec_launch(B, VEC_SCALE_ADD, dd);  // Y_deg = X phi_deg + D_deg
  }
  for (BP* p : L) p->matvecs += p->cnt * (p->deg - 1);
  return outr;
}

// One attempt at all problems with their current guard sizes.
void solve_attempt(rmc_ctx* ctx, std::vector<BP*>& probs, const rmc_solve_opts& o, bool last,
                   hipStream_t stream, int lane) {
  const int JM = jacobi_max_m();
  Scratch sc(&ctx->arena);
  Batch B;
  B.ctx = ctx;
  B.st = stream;
  B.lane = lane;
  B.kind = probs[0]->op->kind;
  for (BP* p : probs) {
    p->m = std::min(p->n, p->nev + p->guard);
    if (p->m > JM) p->m = JM;
    RMC_CHECK(p->m >= p->nev, RMC_ERR_ARG, "too many eigenpairs requested for the Rayleigh-Ritz size");
    B.mmax = std::max(B.mmax, p->m);
    B.nmax = std::max(B.nmax, p->n);
    B.kAmax = std::max(B.kAmax, p->op->kA);
    B.kBmax = std::max(B.kBmax, p->op->kB);
    p->nlock = 0;
    p->iters = 0;
    p->state = 0;
    p->prec = o.precision;
    p->prev_worst = INFINITY;
    p->prev_expect = 1.0;
    p->slow = 0;
    p->matvecs = 0;
  }
  const int P = (int)probs.size();
  std::unique_ptr<HostScope> alloc_scope(new HostScope("solve.alloc"));
  // K-slices of the Gram products, per problem and in proportion to its length, so that
  // every workgroup of a launch gets about the same columns: about 1024 slices over the
  // call (four workgroups a CU), each at least 128 columns wide, at most 64 a problem
  {
    long ntot = 0;
    for (BP* p : probs) ntot += p->n;
    const long w = std::max(128L, (ntot + 1023) / 1024);
    for (BP* p : probs) p->ks = (int)std::max(1L, std::min(64L, ((long)p->n + w - 1) / w));
  }
  B.trs = 2 * B.mmax + 4;  // theta, res, then room for 8 ints
  B.TR = sc.get<double>((size_t)P * B.trs);
  B.TRh.assign((size_t)P * B.trs, 0.0);
  // each problem's buffers carved from one arena block (256-byte aligned pieces), so a
  // call costs one allocation per problem rather than a dozen (the lanes share the arena)
  for (int i = 0; i < P; ++i) {
    BP* p = probs[i];
    const size_t mn = (size_t)p->m * p->n, mm = (size_t)p->m * p->m;
    const bool full = p->op->kind == 2 && p->op->PsiA;
    const size_t DA = full ? (size_t)1 << p->op->nA : 0;
    auto al = [](size_t doubles) { return (doubles + 31) / 32 * 32; };
    size_t total = 6 * al(mn) + 4 * al(mm) + al((size_t)p->ks * mm) + al(((size_t)p->m + 1) / 2);
    if (full) total += 3 * al(mn) + al((size_t)p->m * DA * p->op->kB) + al((size_t)p->m * p->op->kA * p->op->kB);
    double* blk = sc.get<double>(total);
    auto take = [&](size_t doubles) {
      double* q = blk;
      blk += al(doubles);
      return q;
    };
    p->X = take(mn);
    p->HX = take(mn);
    for (int q = 0; q < 3; ++q) p->Y[q] = take(mn);
    p->E = take(mn);
    p->S = take(mm);
    p->Linv = take(mm);
    p->Vwork = take(mm);
    p->Pm = take(mm);
    p->kwork = take((size_t)p->ks * mm);
    p->theta = B.TR + (size_t)i * B.trs;
    p->res = p->theta + B.mmax;
    p->info = reinterpret_cast<int*>(p->res + B.mmax);
    p->sel = reinterpret_cast<int*>(take(((size_t)p->m + 1) / 2));
    if (full) {
      p->wPY = take(mn);
      p->wH = take(mn);
      p->wPH = take(mn);
      p->wT = take((size_t)p->m * DA * p->op->kB);
      p->wU = take((size_t)p->m * p->op->kA * p->op->kB);
    }
  }
  RMC_HIP(hipMemsetAsync(B.TR, 0, (size_t)P * B.trs * sizeof(double), B.st));
  const int pmax = o.max_degree > 0 ? o.max_degree : 40;
  B.phi_cap = (size_t)P * pmax * B.mmax;  // (deg <= pmax rows of at most m entries each)
  B.phi_dev = sc.get<double>(B.phi_cap);
  const size_t da_bytes =
      (size_t)P * ((size_t)(pmax + 4) * B.mmax * 8 + (size_t)(pmax + 48) * 4 * 256) + (1 << 20);
  DescArena da(ctx, B.st, lane, sc, da_bytes);
  B.da = &da;
  alloc_scope.reset();

  {
    std::vector<StartDesc> sd;
    for (BP* p : probs) {
      StartDesc d{};
      d.n = p->n; d.m = p->m; d.D = p->op->D; d.sel = p->sel; d.X = p->Y[0];
      d.eps = (p->m == p->n) ? 0.0 : 1e-3; d.seed = o.seed;
      sd.push_back(d);
    }
    const StartDesc* dd = da.add(sd);
    hipStream_t st = B.st;
    const int nm = B.nmax, mm = B.mmax;
    da.defer([=] { start_batched(st, dd, P, nm, mm); });
  }
  for (BP* p : probs) p->cnt = p->m;
  orthonormalize(B, probs, 0);
  rayleigh_ritz(B, probs, 0, 1, false);

  const double tol = o.tol > 0 ? o.tol : 1e-13;
  const int max_iter = o.max_iter > 0 ? o.max_iter : 200;
  // RMC_GRAPHS=1: each outer iteration's launch sequence (filter, orthonormalisation,
  // Rayleigh-Ritz, with the upload of their tables) is captured once per shape (every
  // active problem's index, row count, lock count, precision, and the filter degree) and
  // replayed when the shape repeats; the tables are rebuilt on the host each iteration
  // in the same layout and the graph's copy node uploads them. No memset is captured.
  static const bool use_graphs = [] {
    const char* e = getenv("RMC_GRAPHS");
    return e && atoi(e) != 0;
  }();
  std::map<std::string, hipGraphExec_t> graphs;
  struct GraphsGuard {
    std::map<std::string, hipGraphExec_t>& g;
    ~GraphsGuard() {
      for (auto& kv : g) (void)hipGraphExecDestroy(kv.second);
    }
  } graphs_guard{graphs};
  long graph_hits = 0, graph_misses = 0;
  for (;;) {
    read_state(B);
    if (ortho_fixup(B, probs)) read_state(B);
    std::vector<BP*> act;
    std::vector<int> ai;
    static const bool trace = getenv("RMC_TRACE_SOLVER") != nullptr;
    std::unique_ptr<HostScope> upd(new HostScope("solve.update"));
    for (int i = 0; i < P; ++i) {
      BP* p = probs[i];
      if (p->state != 0) continue;
      if (update_problem(B, p, i, max_iter, tol, pmax, last)) {
        act.push_back(p);
        ai.push_back(i);
        if (trace)
          fprintf(stderr, "[rmc] n=%d it=%d prec=%d deg=%d nlock=%d worst=%.3e expect=%.3e sweeps=%d\n",
                  p->n, p->iters, p->prec, p->deg, p->nlock, p->prev_worst, p->prev_expect,
                  p->rr_sweeps);
      }
    }
    upd.reset();
    if (act.empty()) break;
    // (not on the legacy null stream, which cannot be captured)
    const bool graph_iter = use_graphs && !ctx->prof && B.st != nullptr;
    std::string sig;
    if (graph_iter) {
      sig.reserve(act.size() * 24);
      for (size_t t = 0; t < act.size(); ++t) {
        const BP* p = act[t];
        int v[6] = {ai[t], p->cnt, p->nlock, p->prec, p->deg, p->m};
        sig.append(reinterpret_cast<const char*>(v), sizeof(v));
      }
      B.da->hold = true;
    }
    // each phase's launches go out as soon as their tables are built, so the host
    // prepares the next phase while the device runs this one
    int r;
    {
      RMC_HOST_SCOPE("solve.filter_host");
      r = filter(B, act);
      B.da->flush();
    }
    {
      RMC_HOST_SCOPE("solve.ortho_host");
      orthonormalize(B, act, r);
      B.da->flush();
    }
    {
      RMC_HOST_SCOPE("solve.rr_host");
      rayleigh_ritz(B, act, r, r == 0 ? 1 : 0, false);
    }
    if (graph_iter) {
      RMC_HOST_SCOPE("solve.graph");
      B.da->hold = false;
      auto it = graphs.find(sig);
      if (it == graphs.end()) {
        ++graph_misses;
        kron_thread_tuning(false);  // no timed candidates while the stream is captured
        hipGraph_t g = nullptr;
        // relaxed: the other lanes' threads synchronise their own streams meanwhile
        hipError_t e = hipStreamBeginCapture(B.st, hipStreamCaptureModeRelaxed);
        if (e == hipSuccess) {
          try {
            B.da->flush();
          } catch (...) {
            (void)hipStreamEndCapture(B.st, &g);
            if (g) (void)hipGraphDestroy(g);
            kron_thread_tuning(true);
            throw;
          }
          e = hipStreamEndCapture(B.st, &g);
        }
        kron_thread_tuning(true);
        RMC_HIP(e);
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        RMC_HIP(e);
        it = graphs.emplace(sig, ex).first;
      } else {
        ++graph_hits;
        B.da->drop();
      }
      RMC_HIP(hipGraphLaunch(it->second, B.st));
    }
    for (BP* p : act) p->iters++;
  }
  if (use_graphs && getenv("RMC_TRACE_SOLVER"))
    fprintf(stderr, "[rmc] lane %d: %ld iterations replayed from %zu graphs, %ld captured\n", lane,
            graph_hits, graphs.size(), graph_misses);
  // final Rayleigh-Ritz over whole blocks (with the stored H X) and FP64 residual check
  std::vector<BP*> fin;
  std::vector<int> fi;
  for (int i = 0; i < P; ++i)
    if (probs[i]->state == 1 || probs[i]->state == 3) {
      fin.push_back(probs[i]);
      fi.push_back(i);
    }
  if (!fin.empty()) {
    // converged problems: the wanted set only (every row of it met the tolerance); the
    // unconverged guard rows would otherwise mix into it at residual / gap
    for (BP* p : fin) p->cnt = p->state == 1 ? std::max(p->nev, std::min(p->nw, p->m)) : p->m;
    rayleigh_ritz(B, fin, 6, 7, true);
    std::vector<VecDesc> cp;
    for (BP* p : fin) {
      VecDesc v{};
      v.nv = p->nev; v.n = p->n; v.out = p->Xout; v.P = p->Y[2];
      cp.push_back(v);
    }
    vec_launch(B, VEC_COPY, cp);
    read_state(B);
    for (size_t t = 0; t < fin.size(); ++t) {
      BP* p = fin[t];
      const double* tt = B.TRh.data() + (size_t)fi[t] * B.trs;
      p->th.assign(tt, tt + p->m);
      p->rs.assign(tt + B.mmax, tt + B.mmax + p->m);
      p->rr_sweeps += std::abs(info_of(B, fi[t], 1));
    }
  }
}

// Solver lanes (RMC_LANES = 1..4, default 2). With L > 1, a batch of at least 4 L
// problems is split into L parts that run the same lockstep iteration on L streams
// from L host threads: the Rayleigh-Ritz, Cholesky and Gram kernels of one part (one
// or a few workgroups per problem, far fewer than the chip holds) then run beside the
// other parts' Kronecker filters, and each part's host-side bookkeeping overlaps the
// others' device work. The parts share nothing but the arena and the profiling
// records, both locked.
int solver_lanes() {
  static const int n = [] {
    const char* e = getenv("RMC_LANES");
    const int v = e ? atoi(e) : 2;
    return std::max(1, std::min(v, (int)rmc_ctx::kMaxLanes));
  }();
  return n;
}

void run_attempt(rmc_ctx* ctx, std::vector<BP*>& L, const rmc_solve_opts& o, bool last) {
  int nl = solver_lanes();
  while (nl > 1 && L.size() < (size_t)(4 * nl)) --nl;
  if (nl < 2) {
    solve_attempt(ctx, L, o, last, ctx->stream, 0);
    return;
  }
  if (!ctx->lane_ev[0]) RMC_HIP(hipEventCreateWithFlags(&ctx->lane_ev[0], hipEventDisableTiming));
  for (int l = 1; l < nl; ++l)
    if (!ctx->lane_stream[l]) {
      RMC_HIP(hipStreamCreateWithFlags(&ctx->lane_stream[l], hipStreamNonBlocking));
      RMC_HIP(hipEventCreateWithFlags(&ctx->lane_ev[l], hipEventDisableTiming));
    }
  // deal the problems out by size so every part carries a similar load
  std::vector<BP*> srt(L);
  std::vector<std::vector<BP*>> part(nl);
  std::stable_sort(srt.begin(), srt.end(), [](const BP* a, const BP* b) {
    return (long)a->n * (a->nev + a->guard) > (long)b->n * (b->nev + b->guard);
  });
  for (size_t i = 0; i < srt.size(); ++i) part[i % nl].push_back(srt[i]);
  // the extra lanes start once everything queued on the ctx stream so far has run
  RMC_HIP(hipEventRecord(ctx->lane_ev[0], ctx->stream));
  for (int l = 1; l < nl; ++l) RMC_HIP(hipStreamWaitEvent(ctx->lane_stream[l], ctx->lane_ev[0], 0));
  std::vector<std::exception_ptr> err(nl);
  std::vector<std::thread> th;
  for (int l = 1; l < nl; ++l)
    th.emplace_back([&, l] {
      try {
        RMC_HIP(hipSetDevice(ctx->device));
        solve_attempt(ctx, part[l], o, last, ctx->lane_stream[l], l);
      } catch (...) {
        err[l] = std::current_exception();
      }
    });
  try {
    solve_attempt(ctx, part[0], o, last, ctx->stream, 0);
  } catch (...) {
    err[0] = std::current_exception();
  }
  for (auto& t : th) t.join();
  // later work on the ctx stream runs after every lane (each lane has already drained
  // its stream before returning; this keeps the order explicit)
  hipError_t e = hipSuccess;
  for (int l = 1; l < nl && e == hipSuccess; ++l) {
    e = hipEventRecord(ctx->lane_ev[l], ctx->lane_stream[l]);
    if (e == hipSuccess) e = hipStreamWaitEvent(ctx->stream, ctx->lane_ev[l], 0);
  }
  for (auto& x : err)
    if (x) std::rethrow_exception(x);
  RMC_HIP(e);
}

}  // namespace

// Lowest nevs[i] eigenpairs of several operators of one kind, in lockstep.
void eig_lowest_batch(rmc_ctx* ctx, const std::vector<const CoupledOp*>& ops,
                      const std::vector<int>& nevs, const rmc_solve_opts& o,
                      const std::vector<double*>& X_out, std::vector<std::vector<double>>& evals,
                      std::vector<SolveStats>& stats) {
  const int P = (int)ops.size();
  evals.assign(P, {});
  stats.assign(P, SolveStats());
  if (P == 0) return;
  const int JM = jacobi_max_m();
  std::vector<BP> bp(P);
  std::vector<BP*> todo;
  for (int i = 0; i < P; ++i) {
    RMC_CHECK(ops[i]->n >= 1, RMC_ERR_ARG, "empty operator");
    RMC_CHECK(ops[i]->kind == ops[0]->kind, RMC_ERR_ARG, "mixed operator kinds in one batch");
    bp[i].op = ops[i];
    bp[i].n = ops[i]->n;
    bp[i].nev = std::max(1, std::min(nevs[i], ops[i]->n));
    bp[i].guard = o.guard > 0 ? o.guard : std::max(8, (bp[i].nev + 7) / 8);
    bp[i].Xout = X_out[i];
    todo.push_back(&bp[i]);
  }
  for (int attempt = 0; !todo.empty(); ++attempt) {
    std::vector<BP*> last, more, next;
    for (BP* p : todo) {
      const bool is_last = (p->nev + p->guard >= std::min(p->n, JM)) || attempt >= 3;
      (is_last ? last : more).push_back(p);
    }
    for (int pass = 0; pass < 2; ++pass) {
      auto& L = pass == 0 ? more : last;
      if (L.empty()) continue;
      run_attempt(ctx, L, o, pass == 1);
      for (BP* p : L) {
        const int i = (int)(p - bp.data());
        stats[i].iters += p->iters;
        stats[i].matvecs += p->matvecs;
        stats[i].rr_sweeps += p->rr_sweeps;
        p->rr_sweeps = 0;
        if (p->state == 2) {
          p->guard = 2 * p->guard + 8;  // a degenerate cluster reaches past the guard vectors
          next.push_back(p);
        }
      }
    }
    todo.swap(next);
  }
  const double tol = o.tol > 0 ? o.tol : 1e-13;
  for (int i = 0; i < P; ++i) {
    BP* p = &bp[i];
    evals[i].assign(p->th.begin(), p->th.begin() + p->nev);
    int nwf = p->nev;
    const double scale = std::max({1.0, std::fabs(p->op->bup), std::fabs(p->th[0])});
    const int lim = std::min(p->cnt > 0 ? p->cnt : p->m, p->m);  // rows of the final Rayleigh-Ritz
    while (nwf < lim && p->th[nwf] - p->th[nwf - 1] <= 1e-6 * scale) ++nwf;
    double mr = 0.0;
    for (int j = 0; j < std::min(nwf, lim); ++j) mr = std::max(mr, p->rs[j] / scale);
    stats[i].max_res = mr;
    stats[i].status = (p->state == 1 && mr <= 10.0 * tol) ? RMC_OK : RMC_ERR_NOCONV;
    if (stats[i].status != RMC_OK && getenv("RMC_TRACE_SOLVER"))
      fprintf(stderr, "[rmc] problem %d of %d not converged: n=%d nev=%d m=%d guard=%d state=%d iters=%d "
              "th0=%.6e res0=%.3e nlock=%d\n", i, P, p->n, p->nev, p->m, p->guard, p->state, p->iters,
              p->th.empty() ? 0.0 : p->th[0], p->rs.empty() ? 0.0 : p->rs[0], p->nlock);
  }
}

int eig_lowest(rmc_ctx* ctx, const CoupledOp& op, int nev, const rmc_solve_opts& o, double* X_out,
               std::vector<double>& evals, SolveStats& st) {
  std::vector<std::vector<double>> ev;
  std::vector<SolveStats> ss;
  eig_lowest_batch(ctx, {&op}, {nev}, o, {X_out}, ev, ss);
  evals = ev[0];
  st = ss[0];
  return st.status;
}

// One block apply through the batched kernel (used by rmc_kron_apply).
void op_apply(rmc_ctx* ctx, const CoupledOp& op, int nv, const double* Y, double* out,
              const double* Xprev, double s1, double s2, double s3, double*, double*, int precision,
              const double* Ecorr, const double* phi) {
  RMC_CHECK(op.kind == 1, RMC_ERR_ARG, "op_apply supports Kronecker operators");
  Scratch sc(&ctx->arena);
  KronDesc d{};
  d.kA = op.kA; d.kB = op.kB; d.T = op.T; d.nv = nv; d.vbase = 0;
  d.pack = op.pack[precision]; d.pkm = op.pkm;
  d.coef = op.coef_dev; d.OA = op.OAcat; d.OB = op.OBcat; d.Ediag = op.Ediag;
  d.Y = Y; d.Xprev = s3 != 0.0 ? Xprev : nullptr; d.E = Ecorr; d.phi = phi; d.out = out;
  d.s1 = s1; d.s2 = s2; d.s3 = s3;
  KronDesc* dd = sc.get<KronDesc>(1);
  RMC_HIP(hipMemcpyAsync(dd, &d, sizeof(d), hipMemcpyHostToDevice, ctx->stream));
  // a variant forced for this one apply must take the shape (no silent substitute)
  kron_batched(ctx->stream, dd, 1, op.kB, nv, op.kA, precision, op.T, nv, true, /*strict=*/true);
  sync(ctx);
}

size_t op_zwork_doubles(const CoupledOp&, int) { return 1; }

}  // namespace rmc
