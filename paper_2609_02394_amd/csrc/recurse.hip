// Recursion over a chain (Algorithm 1): leaves of consecutive sites, pairwise
// merges of neighbouring modules left to right (an odd module is carried up),
// boundary operators projected and transformed as later merges require, identical
// modules computed once (the paper's reuse of identical blocks), the lowest q
// eigenvalues of the final merge returned.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <map>
#include <set>
#include <string>
#include <vector>

#include "rmc_internal.h"

namespace rmc {
// defined in api.hip
rmc_module* api_leaf_solve(rmc_ctx* ctx, const rmc_leaf_desc* leaf, int k, int q_only,
                           const rmc_solve_opts& o, std::vector<double>& evals, rmc_level_report* rep);
int api_project_op(rmc_ctx* ctx, rmc_module* m, int site, int op);
rmc_module* api_couple(rmc_ctx* ctx, rmc_module* A, rmc_module* B, const rmc_bond_desc* bond,
                       int k_keep, int q, const rmc_solve_opts& o, bool want_module,
                       std::vector<double>& evals, rmc_level_report* rep);
void api_release_basis(rmc_ctx* ctx, rmc_module* m);
void api_free_module(rmc_ctx* ctx, rmc_module* m);
}  // namespace rmc

using namespace rmc;

namespace {

struct CutTerm {
  double coef;
  int sa, oa, sb, ob;
};

struct Node {
  int kind = 0;  // 0 leaf, 1 merge
  int a = 0, b = 0;
  int left = -1, right = -1;
  int level = 0;
  bool root = false;
  int key = -1;
  std::vector<rmc_term> terms;  // leaf: local sites
  std::vector<CutTerm> cut;
};

struct Plan {
  std::vector<Node> nodes;
  int root = -1;
  int n_keys = 0;
  std::vector<std::set<std::pair<int, int>>> need;  // per key: (site, op)
};

std::string term_bytes(const rmc_term& t, int shift) {
  std::string s;
  s.append((const char*)&t.coef, sizeof(double));
  int v[5] = {t.nsite, t.site[0] - shift, t.nsite > 1 ? t.site[1] - shift : -1, t.op[0],
              t.nsite > 1 ? t.op[1] : 0};
  s.append((const char*)v, sizeof(v));
  return s;
}

void validate_chain(const rmc_chain_desc* c) {
  RMC_CHECK(c != nullptr, RMC_ERR_ARG, "null chain");
  RMC_CHECK(c->n_sites >= 1 && c->leaf_sites >= 1 && c->leaf_sites <= 12, RMC_ERR_ARG,
            "leaf_sites must be 1..12");
  RMC_CHECK(c->n_sites % c->leaf_sites == 0, RMC_ERR_ARG, "n_sites must be a multiple of leaf_sites");
  RMC_CHECK(c->k >= 1, RMC_ERR_ARG, "k must be >= 1");
  RMC_CHECK(c->q >= 1 && c->q <= c->k, RMC_ERR_ARG, "need 1 <= q <= k");
  RMC_CHECK(c->n_terms >= 0 && (c->n_terms == 0 || c->terms), RMC_ERR_ARG, "bad term list");
  for (int t = 0; t < c->n_terms; ++t) {
    const rmc_term& tm = c->terms[t];
    RMC_CHECK(tm.nsite == 1 || tm.nsite == 2, RMC_ERR_ARG, "term nsite must be 1 or 2");
    for (int u = 0; u < tm.nsite; ++u) {
      RMC_CHECK(tm.site[u] >= 0 && tm.site[u] < c->n_sites, RMC_ERR_ARG, "term site out of range");
      RMC_CHECK(tm.op[u] >= RMC_OP_X && tm.op[u] <= RMC_OP_Z, RMC_ERR_ARG, "unknown operator");
    }
    if (tm.nsite == 2) RMC_CHECK(tm.site[0] != tm.site[1], RMC_ERR_ARG, "two-site term on one site");
  }
}

Plan make_plan(const rmc_chain_desc* c) {
  Plan P;
  std::map<std::string, int> keys;
  auto intern = [&](const std::string& s) {
    auto it = keys.find(s);
    if (it != keys.end()) return it->second;
    int id = (int)keys.size();
    keys[s] = id;
    return id;
  };
  const int L0 = c->leaf_sites;
  std::vector<int> cur;
  for (int a = 0; a < c->n_sites; a += L0) {
    Node nd;
    nd.kind = 0;
    nd.a = a;
    nd.b = a + L0;
    std::string ks = "L" + std::to_string(L0) + ":";
    for (int t = 0; t < c->n_terms; ++t) {
      const rmc_term& tm = c->terms[t];
      bool in = true;
      for (int u = 0; u < tm.nsite; ++u) in = in && tm.site[u] >= a && tm.site[u] < a + L0;
      if (!in) continue;
      rmc_term lt = tm;
      for (int u = 0; u < tm.nsite; ++u) lt.site[u] -= a;
      nd.terms.push_back(lt);
      ks += term_bytes(tm, a);
    }
    nd.key = intern(ks);
    P.nodes.push_back(nd);
    cur.push_back((int)P.nodes.size() - 1);
  }
  int level = 0;
  while (cur.size() > 1) {
    ++level;
    std::vector<int> nxt;
    const bool last = cur.size() == 2;
    for (size_t i = 0; i + 1 < cur.size(); i += 2) {
      const Node& L = P.nodes[cur[i]];
      const Node& R = P.nodes[cur[i + 1]];
      Node nd;
      nd.kind = 1;
      nd.a = L.a;
      nd.b = R.b;
      nd.left = cur[i];
      nd.right = cur[i + 1];
      nd.level = level;
      nd.root = last;
      const int a = L.a, m = L.b, b = R.b;
      std::string ks = "M" + std::to_string(L.key) + "," + std::to_string(R.key) + (last ? "R:" : ":");
      for (int t = 0; t < c->n_terms; ++t) {
        const rmc_term& tm = c->terms[t];
        if (tm.nsite != 2) continue;
        int s0 = tm.site[0], s1 = tm.site[1];
        bool f = s0 >= a && s0 < m && s1 >= m && s1 < b;
        bool r = s1 >= a && s1 < m && s0 >= m && s0 < b;
        if (!f && !r) continue;
        CutTerm ct;
        ct.coef = tm.coef;
        if (f) {
          ct.sa = s0 - a; ct.oa = tm.op[0]; ct.sb = s1 - m; ct.ob = tm.op[1];
        } else {
          ct.sa = s1 - a; ct.oa = tm.op[1]; ct.sb = s0 - m; ct.ob = tm.op[0];
        }
        nd.cut.push_back(ct);
        int v[4] = {ct.sa, ct.oa, ct.sb, ct.ob};
        ks.append((const char*)&ct.coef, sizeof(double));
        ks.append((const char*)v, sizeof(v));
      }
      nd.key = intern(ks);
      P.nodes.push_back(nd);
      nxt.push_back((int)P.nodes.size() - 1);
    }
    if (cur.size() % 2) nxt.push_back(cur.back());
    cur.swap(nxt);
  }
  P.root = cur[0];
  P.n_keys = (int)keys.size();
  // operator requirements: top-down per node, then per key
  std::vector<std::set<std::pair<int, int>>> nneed(P.nodes.size());
  for (int i = (int)P.nodes.size() - 1; i >= 0; --i) {
    const Node& nd = P.nodes[i];
    if (nd.kind != 1) continue;
    for (const CutTerm& ct : nd.cut) {
      nneed[nd.left].insert({ct.sa, ct.oa});
      nneed[nd.right].insert({ct.sb, ct.ob});
    }
    const int wA = P.nodes[nd.left].b - P.nodes[nd.left].a;
    for (auto& so : nneed[i]) {
      if (so.first < wA) nneed[nd.left].insert(so);
      else nneed[nd.right].insert({so.first - wA, so.second});
    }
  }
  P.need.assign(P.n_keys, {});
  for (size_t i = 0; i < P.nodes.size(); ++i)
    for (auto& so : nneed[i]) P.need[P.nodes[i].key].insert(so);
  return P;
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

void add_record(rmc_report* rep, const rmc_level_report& r) {
  if (!rep) return;
  if (rep->records && rep->n_records < rep->capacity) rep->records[rep->n_records] = r;
  rep->n_records++;
}

// Runs the plan; fills energies (q). Modules created are freed before return.
void run_plan(rmc_ctx* ctx, const rmc_chain_desc* c, const Plan& P, const rmc_solve_opts& o,
              double* energies, rmc_report* rep) {
  std::vector<rmc_module*> by_key(P.n_keys, nullptr);
  std::vector<rmc_module*> created;
  double t0 = now_ms();
  if (rep) {
    rep->n_records = 0;
    rep->n_leaf_ed = 0;
    rep->n_merges = 0;
  }
  try {
    const Node& root = P.nodes[P.root];
    if (root.kind == 0) {  // a single leaf: its lowest q eigenvalues
      rmc_leaf_desc ld{root.b - root.a, (int)root.terms.size(), root.terms.data()};
      std::vector<double> ev;
      rmc_level_report r{};
      api_leaf_solve(ctx, &ld, c->k, c->q, o, ev, &r);
      r.kind = 2;
      r.width = ld.n_sites;
      add_record(rep, r);
      if (rep) rep->n_leaf_ed++;
      for (int i = 0; i < c->q; ++i) energies[i] = ev[i];
    } else {
      for (size_t i = 0; i < P.nodes.size(); ++i) {
        const Node& nd = P.nodes[i];
        rmc_level_report r{};
        r.level = nd.level;
        r.width = nd.b - nd.a;
        r.kind = nd.kind == 0 ? 0 : (nd.root ? 2 : 1);
        if (!nd.root && by_key[nd.key]) {
          r.reused = 1;
          r.k_eff = by_key[nd.key]->k_eff;
          r.gap = by_key[nd.key]->gap;
          add_record(rep, r);
          continue;
        }
        rmc_module* m = nullptr;
        std::vector<double> ev;
        if (nd.kind == 0) {
          rmc_leaf_desc ld{nd.b - nd.a, (int)nd.terms.size(), nd.terms.data()};
          m = api_leaf_solve(ctx, &ld, c->k, 0, o, ev, &r);
          if (rep) rep->n_leaf_ed++;
        } else {
          rmc_module* A = by_key[P.nodes[nd.left].key];
          rmc_module* B = by_key[P.nodes[nd.right].key];
          RMC_CHECK(A && B, RMC_ERR_STATE, "child module missing");
          std::vector<double> coef;
          std::vector<int> ia, ib;
          for (const CutTerm& ct : nd.cut) {
            coef.push_back(ct.coef);
            ia.push_back(api_project_op(ctx, A, ct.sa, ct.oa));
            ib.push_back(api_project_op(ctx, B, ct.sb, ct.ob));
          }
          rmc_bond_desc bd{(int)coef.size(), coef.data(), ia.data(), ib.data()};
          if (nd.root) {
            api_couple(ctx, A, B, &bd, c->k, c->q, o, false, ev, &r);
            for (int q = 0; q < c->q; ++q) energies[q] = ev[q];
          } else {
            m = api_couple(ctx, A, B, &bd, c->k, std::min(c->q, c->k), o, true, ev, &r);
          }
          if (rep) rep->n_merges++;
        }
        if (m) {
          created.push_back(m);
          for (auto& so : P.need[nd.key]) api_project_op(ctx, m, so.first, so.second);
          api_release_basis(ctx, m);
          by_key[nd.key] = m;
        }
        add_record(rep, r);
      }
    }
  } catch (...) {
    for (rmc_module* m : created) api_free_module(ctx, m);
    throw;
  }
  for (rmc_module* m : created) api_free_module(ctx, m);
  if (rep) rep->total_ms = now_ms() - t0;
}

template <class F>
rmc_status guard(rmc_ctx* ctx, F&& f) {
  try {
    f();
    return RMC_OK;
  } catch (const rmc::Error& e) {
    if (ctx) ctx->last_error = e.what();
    return e.code;
  } catch (const std::exception& e) {
    if (ctx) ctx->last_error = e.what();
    return RMC_ERR_STATE;
  }
}

}  // namespace

extern "C" {

rmc_status rmc_recurse(rmc_ctx* ctx, const rmc_chain_desc* chain, const rmc_solve_opts* opts,
                       double* energies, rmc_report* report) {
  if (!ctx) return RMC_ERR_ARG;
  return guard(ctx, [&] {
    validate_chain(chain);
    RMC_CHECK(energies != nullptr, RMC_ERR_ARG, "null energies");
    rmc_solve_opts o;
    rmc_default_opts(&o);
    if (opts) o = *opts;
    RMC_CHECK(o.precision >= RMC_FP64 && o.precision <= RMC_BF16, RMC_ERR_ARG, "bad precision");
    Plan P = make_plan(chain);
    std::vector<double> e(chain->q);
    run_plan(ctx, chain, P, o, e.data(), report);
    for (int i = 0; i < chain->q; ++i) energies[i] = e[i];
  });
}

rmc_status rmc_recurse_batch(rmc_ctx* ctx, int n_jobs, const rmc_chain_desc* chains,
                             const rmc_solve_opts* opts, double* energies, int q_stride,
                             int* status_host) {
  if (!ctx) return RMC_ERR_ARG;
  if (n_jobs < 0 || (n_jobs > 0 && (!chains || !energies))) return RMC_ERR_ARG;
  rmc_status worst = RMC_OK;
  for (int j = 0; j < n_jobs; ++j) {
    if (chains[j].q > q_stride) {
      if (status_host) status_host[j] = RMC_ERR_ARG;
      worst = RMC_ERR_ARG;
      continue;
    }
    rmc_status st = rmc_recurse(ctx, &chains[j], opts, energies + (size_t)j * q_stride, nullptr);
    if (status_host) status_host[j] = st;
    if (st != RMC_OK) worst = st;
  }
  return worst;
}

}  // extern "C"
