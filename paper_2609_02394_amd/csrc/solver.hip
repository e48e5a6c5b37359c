// Matrix-free eigensolver for the lowest eigenpairs of a module-coupling step.
//
// The paper assembles the k_A k_B square effective Hamiltonian and diagonalises it
// fully (reduced eigenproblem; dense eigensolve of App. A). Here the operator is
// only applied to blocks of vectors, and the lowest nev eigenpairs are found by a
// Chebyshev-filtered block subspace iteration with Rayleigh-Ritz (a block
// Davidson-type method in which the Chebyshev filter plays the role of the
// correction step):
//   1. start block: the m lowest diagonal product states plus a small seeded
//      random component; CholeskyQR2; Rayleigh-Ritz;
//   2. repeat: filter the unconverged Ritz vectors with a scaled Chebyshev
//      polynomial that damps [theta_{m-1}, upper bound] (degree chosen from the
//      residuals), orthogonalise against the locked vectors (twice), CholeskyQR2,
//      Rayleigh-Ritz on the filtered block, residual norms, lock converged ones;
//   3. a final Rayleigh-Ritz over the whole block and a final FP64 residual check.
// Everything on the device is FP64 except, in the FP32/BF16 forms, the operator
// applications inside the filter.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "rmc_internal.h"

namespace rmc {

void kron_apply_fused(hipStream_t s, const CoupledOp& op, int nv, const double* Y, double* out,
                      const double* Xprev, double s1, double s2, double s3, int precision);

size_t op_zwork_doubles(const CoupledOp& op, int nv) { return 1; }

void op_apply(rmc_ctx* ctx, const CoupledOp& op, int nv, const double* Y, double* out,
              const double* Xprev, double s1, double s2, double s3, double* zwork, double* kwork,
              int precision) {
  hipStream_t s = ctx->stream;
  const int n = op.n;
  if (op.kind == 0) {
    gemm_f64(s, false, true, nv, n, n, s1, Y, n, 0, op.H, n, 0, 0.0, out, n, 0, 1,
             gemm_pick_ksplit(nv, n, n, 1), kwork);
    axpy_epilogue(s, nv, n, out, Y, Xprev, nullptr, s1, s2, s3, false);
    return;
  }
  if (!ctx->prof) {
    kron_apply_fused(s, op, nv, Y, out, Xprev, s1, s2, s3, precision);
    return;
  }
  auto take = [&]() {
    hipEvent_t e;
    if (!ctx->ev_pool.empty()) {
      e = ctx->ev_pool.back();
      ctx->ev_pool.pop_back();
    } else {
      RMC_HIP(hipEventCreate(&e));
    }
    return e;
  };
  rmc_ctx::ProfRec r;
  r.a = take();
  r.b = take();
  RMC_HIP(hipEventRecord(r.a, s));
  kron_apply_fused(s, op, nv, Y, out, Xprev, s1, s2, s3, precision);
  RMC_HIP(hipEventRecord(r.b, s));
  const double nn = (double)n;
  r.flops = (double)nv * (2.0 * op.T * nn * (op.kA + op.kB) + 4.0 * nn);
  r.bytes = 8.0 * nn * ((double)nv * (s3 != 0.0 ? 3.0 : 2.0) + 1.0) +
            8.0 * op.T * ((double)op.kA * op.kA + (double)op.kB * op.kB);
  ctx->prof_recs.push_back(r);
}

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

struct Work {
  int n, m;
  double *X, *HX, *Yb[3], *Z, *G, *S, *Linv, *Vwork, *theta, *res, *norms, *P, *kwork, *scal;
  int *sel, *info;
};

void sync(rmc_ctx* ctx) { RMC_HIP(hipStreamSynchronize(ctx->stream)); }

// Orthonormalise rows Y[0..cnt) against the locked rows L[0..nlock) and among
// themselves (two projection passes, then CholeskyQR2, a third pass if the first
// Cholesky needed a shift).
void orthonormalize(rmc_ctx* ctx, Work& w, double*& Y, double* spare, int cnt, const double* L,
                    int nlock) {
  hipStream_t s = ctx->stream;
  const int n = w.n;
  row_norms(s, cnt, n, Y, w.norms, true);
  if (nlock > 0) {
    for (int pass = 0; pass < 2; ++pass) {
      gemm_f64(s, false, true, cnt, nlock, n, 1.0, Y, n, 0, L, n, 0, 0.0, w.P, nlock, 0, 1,
               gemm_pick_ksplit(cnt, nlock, n, 1), w.kwork);
      gemm_f64(s, false, false, cnt, n, nlock, -1.0, w.P, nlock, 0, L, n, 0, 1.0, Y, n, 0, 1, 1,
               nullptr);
    }
    row_norms(s, cnt, n, Y, w.norms, true);
  }
  int passes = 2;
  for (int pass = 0; pass < passes; ++pass) {
    gemm_f64(s, false, true, cnt, cnt, n, 1.0, Y, n, 0, Y, n, 0, 0.0, w.G, cnt, 0, 1,
             gemm_pick_ksplit(cnt, cnt, n, 1), w.kwork);
    chol_inv(s, cnt, w.G, 0.0, w.Linv, w.info);
    int info = 0;
    RMC_HIP(hipMemcpyAsync(&info, w.info, sizeof(int), hipMemcpyDeviceToHost, s));
    sync(ctx);
    if (info != 0) {
      // shifted CholeskyQR (trace(G) = cnt for normalised rows)
      double u = 1.1102230246251565e-16;
      double shift = 11.0 * ((double)n * cnt + (double)cnt * (cnt + 1)) * u * (double)cnt;
      chol_inv(s, cnt, w.G, shift, w.Linv, w.info);
      RMC_HIP(hipMemcpyAsync(&info, w.info, sizeof(int), hipMemcpyDeviceToHost, s));
      sync(ctx);
      RMC_CHECK(info == 0, RMC_ERR_NOCONV, "CholeskyQR failed even with a shift");
      if (passes < 3) passes = 3;
    }
    gemm_f64(s, false, false, cnt, n, cnt, 1.0, w.Linv, cnt, 0, Y, n, 0, 0.0, spare, n, 0, 1, 1,
             nullptr);
    std::swap(Y, spare);
  }
}

// Rayleigh-Ritz of the orthonormal rows Q[0..cnt): W = H Q, G = Q W^T, G = S diag S^T,
// Xdst = S^T Q, HXdst = S^T W, theta_dst, residuals.
void rayleigh_ritz(rmc_ctx* ctx, const CoupledOp& op, Work& w, const double* Q, double* Wtmp,
                   int cnt, double* Xdst, double* HXdst, double* theta_dst, double* res_dst,
                   bool have_W) {
  hipStream_t s = ctx->stream;
  const int n = w.n;
  if (!have_W) op_apply(ctx, op, cnt, Q, Wtmp, nullptr, 1.0, 0.0, 0.0, w.Z, w.kwork, RMC_FP64);
  gemm_f64(s, false, true, cnt, cnt, n, 1.0, Q, n, 0, Wtmp, n, 0, 0.0, w.G, cnt, 0, 1,
           gemm_pick_ksplit(cnt, cnt, n, 1), w.kwork);
  jacobi_eig(s, 1, cnt, w.G, 0, theta_dst, 0, w.S, 0, w.Vwork, w.info + 1);
  gemm_f64(s, true, false, cnt, n, cnt, 1.0, w.S, cnt, 0, Q, n, 0, 0.0, Xdst, n, 0, 1, 1, nullptr);
  gemm_f64(s, true, false, cnt, n, cnt, 1.0, w.S, cnt, 0, Wtmp, n, 0, 0.0, HXdst, n, 0, 1, 1,
           nullptr);
  residual_norms(s, cnt, n, HXdst, Xdst, theta_dst, res_dst);
}

}  // namespace

int eig_lowest(rmc_ctx* ctx, const CoupledOp& op, int nev, const rmc_solve_opts& o, double* X_out,
               std::vector<double>& evals, SolveStats& st) {
  hipStream_t s = ctx->stream;
  const int n = op.n;
  RMC_CHECK(n >= 1, RMC_ERR_ARG, "empty operator");
  if (nev > n) nev = n;
  RMC_CHECK(nev >= 1, RMC_ERR_ARG, "nev < 1");
  const int JM = jacobi_max_m();
  int guard = o.guard > 0 ? o.guard : std::max(8, (nev + 7) / 8);
  int m = std::min(n, nev + guard);
  if (m > JM) m = JM;
  RMC_CHECK(m >= nev, RMC_ERR_ARG, "too many eigenpairs requested for the Rayleigh-Ritz size");
  RMC_CHECK(m == n || m > nev, RMC_ERR_ARG, "no guard vectors left");

  Scratch sc(&ctx->arena);
  Work w;
  w.n = n;
  w.m = m;
  w.X = sc.get<double>((size_t)m * n);
  w.HX = sc.get<double>((size_t)m * n);
  for (int i = 0; i < 3; ++i) w.Yb[i] = sc.get<double>((size_t)m * n);
  w.Z = sc.get<double>(op_zwork_doubles(op, m));
  w.G = sc.get<double>((size_t)m * m);
  w.S = sc.get<double>((size_t)m * m);
  w.Linv = sc.get<double>((size_t)m * m);
  w.Vwork = sc.get<double>((size_t)m * m);
  w.theta = sc.get<double>(m);
  w.res = sc.get<double>(m);
  w.norms = sc.get<double>(m);
  w.P = sc.get<double>((size_t)m * m);
  size_t kw = 64 * (size_t)m * std::max(m, 1) + 64 * (size_t)std::max(m, 64) * 64;
  if (op.kind == 0) kw = std::max(kw, (size_t)64 * m * n);
  w.kwork = sc.get<double>(kw);
  w.scal = sc.get<double>(4);
  w.sel = sc.get<int>(m);
  w.info = sc.get<int>(4);
  double* D = op.D;

  // start block
  double eps0 = (m == n) ? 0.0 : 1e-3;
  start_block(s, n, m, D, eps0, o.seed, w.sel, w.X);
  double* Y = w.Yb[0];
  double* spare = w.Yb[1];
  copy_rows(s, m, n, w.X, n, Y, n);
  orthonormalize(ctx, w, Y, spare, m, nullptr, 0);
  double* Wt = (Y == w.Yb[0]) ? w.Yb[1] : w.Yb[0];
  rayleigh_ritz(ctx, op, w, Y, Wt, m, w.X, w.HX, w.theta, w.res, false);
  st.matvecs = m;

  std::vector<double> th(m), rs(m);
  const double tol = o.tol > 0 ? o.tol : 1e-13;
  const int max_iter = o.max_iter > 0 ? o.max_iter : 200;
  const int pmax = o.max_degree > 0 ? o.max_degree : 40;
  const int prec = o.precision;
  int nlock = 0;
  int status = RMC_ERR_NOCONV;
  double scale = 1.0;
  int it = 0;
  for (;; ++it) {
    RMC_HIP(hipMemcpyAsync(th.data(), w.theta, m * sizeof(double), hipMemcpyDeviceToHost, s));
    RMC_HIP(hipMemcpyAsync(rs.data(), w.res, m * sizeof(double), hipMemcpyDeviceToHost, s));
    sync(ctx);
    scale = std::max({1.0, std::fabs(op.bup), std::fabs(th[0])});
    int first_bad = nev;
    for (int j = 0; j < nev; ++j)
      if (!(rs[j] <= tol * scale)) {
        first_bad = j;
        break;
      }
    if (first_bad == nev || m == n) {
      status = RMC_OK;
      break;
    }
    if (it >= max_iter) break;
    nlock = std::max(nlock, first_bad);
    const int cnt = m - nlock;
    double a = th[m - 1], b = op.bup, a0 = th[0];
    if (!(b > a)) b = a + std::max(1e-3 * std::fabs(a), 1e-6);
    if (!(a0 < a)) a0 = a - 1e-3 * (b - a);
    const double e = 0.5 * (b - a), c = 0.5 * (b + a);
    // degree from the slowest unconverged wanted pair
    int p = 2;
    for (int j = nlock; j < nev; ++j) {
      if (rs[j] <= tol * scale) continue;
      double x = std::fabs((th[j] - c) / e);
      double rho = x > 1.0 ? std::acosh(x) : 1e-3;
      double need = std::log(2.0 * rs[j] / (tol * scale)) / rho;
      p = std::max(p, (int)std::ceil(need));
    }
    p = std::min(std::max(p, 2), pmax);
    // scaled Chebyshev filter on X[nlock..m)
    const double* Xa = w.X + (size_t)nlock * n;
    double sigma = e / (a0 - c);
    const double tau2 = 2.0 / sigma;
    op_apply(ctx, op, cnt, Xa, w.Yb[0], nullptr, sigma / e, -c * sigma / e, 0.0, w.Z, w.kwork,
             prec);
    const double* prev = Xa;
    double* cur = w.Yb[0];
    for (int i = 2; i <= p; ++i) {
      double sig2 = 1.0 / (tau2 - sigma);
      double* nw = nullptr;
      for (int q = 0; q < 3 && !nw; ++q)
        if (w.Yb[q] != cur && w.Yb[q] != prev) nw = w.Yb[q];
      op_apply(ctx, op, cnt, cur, nw, prev, 2.0 * sig2 / e, -2.0 * c * sig2 / e, -sigma * sig2,
               w.Z, w.kwork, prec);
      prev = cur;
      cur = nw;
      sigma = sig2;
    }
    double* Ycur = cur;
    st.matvecs += cnt * p;
    // buffers: Ycur holds the filtered block; pick a spare among Yb not equal to Ycur/Xp
    double* sp = nullptr;
    for (int i = 0; i < 3; ++i)
      if (w.Yb[i] != Ycur) { sp = w.Yb[i]; break; }
    double* Q = Ycur;
    orthonormalize(ctx, w, Q, sp, cnt, w.X, nlock);
    double* Wt2 = nullptr;
    for (int i = 0; i < 3; ++i)
      if (w.Yb[i] != Q) { Wt2 = w.Yb[i]; break; }
    rayleigh_ritz(ctx, op, w, Q, Wt2, cnt, w.X + (size_t)nlock * n, w.HX + (size_t)nlock * n,
                  w.theta + nlock, w.res + nlock, false);
    st.matvecs += cnt;
  }
  st.iters = it;
  // final Rayleigh-Ritz over the whole block with the stored H X, and residual check
  {
    gemm_f64(s, false, true, m, m, n, 1.0, w.X, n, 0, w.HX, n, 0, 0.0, w.G, m, 0, 1,
             gemm_pick_ksplit(m, m, n, 1), w.kwork);
    jacobi_eig(s, 1, m, w.G, 0, w.theta, 0, w.S, 0, w.Vwork, w.info + 1);
    gemm_f64(s, true, false, m, n, m, 1.0, w.S, m, 0, w.X, n, 0, 0.0, w.Yb[0], n, 0, 1, 1, nullptr);
    gemm_f64(s, true, false, m, n, m, 1.0, w.S, m, 0, w.HX, n, 0, 0.0, w.Yb[1], n, 0, 1, 1,
             nullptr);
    residual_norms(s, m, n, w.Yb[1], w.Yb[0], w.theta, w.res);
    copy_rows(s, nev, n, w.Yb[0], n, X_out, n);
  }
  RMC_HIP(hipMemcpyAsync(th.data(), w.theta, m * sizeof(double), hipMemcpyDeviceToHost, s));
  RMC_HIP(hipMemcpyAsync(rs.data(), w.res, m * sizeof(double), hipMemcpyDeviceToHost, s));
  sync(ctx);
  evals.assign(th.begin(), th.begin() + nev);
  double mr = 0.0;
  for (int j = 0; j < nev; ++j) mr = std::max(mr, rs[j] / scale);
  st.max_res = mr;
  if (status == RMC_OK && mr > 10.0 * tol) status = RMC_ERR_NOCONV;
  st.status = status;
  return status;
}

}  // namespace rmc
