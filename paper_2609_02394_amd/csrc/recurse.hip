// Recursion over a module tree (Algorithm 1 with a caller-defined hierarchy, Fig. 1's
// recursive block merging): leaf blocks with their own Hamiltonians, merges with
// their children and coupling terms, run level by level (a merge one level above its
// deeper child); boundary operators projected and transformed as later merges
// require; identical modules computed once (the paper's reuse of identical blocks);
// the lowest q eigenvalues of the root returned. A chain is one such tree: leaves of
// consecutive sites merged pairwise left to right, an odd module carried up.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "rmc_batch.h"
#include "rmc_internal.h"

namespace rmc {
// defined in api.hip
rmc_module* api_leaf_solve(rmc_ctx* ctx, const rmc_leaf_desc* leaf, int k, int q_only,
                           const rmc_solve_opts& o, std::vector<double>& evals, rmc_level_report* rep);
int api_project_op(rmc_ctx* ctx, rmc_module* m, int site, int op);
void api_project_ops_batch(rmc_ctx* ctx, const std::vector<rmc_module*>& ms,
                           const std::vector<std::pair<int, int>>& so);
rmc_module* api_couple(rmc_ctx* ctx, rmc_module* A, rmc_module* B, const rmc_bond_desc* bond,
                       int k_keep, int q, const rmc_solve_opts& o, bool want_module,
                       std::vector<double>& evals, rmc_level_report* rep);
void api_release_basis(rmc_ctx* ctx, rmc_module* m);
void api_free_module(rmc_ctx* ctx, rmc_module* m);
std::vector<rmc_module*> api_leaf_solve_batch(rmc_ctx* ctx,
                                              const std::vector<const rmc_leaf_desc*>& leaves,
                                              const std::vector<int>& ks,
                                              const std::vector<int>& q_only,
                                              const rmc_solve_opts& o,
                                              std::vector<std::vector<double>>& evals,
                                              std::vector<rmc_level_report>* reps);
std::vector<rmc_module*> api_couple_batch(rmc_ctx* ctx, const std::vector<rmc_module*>& As,
                                          const std::vector<rmc_module*>& Bs,
                                          const std::vector<const rmc_bond_desc*>& bonds,
                                          const std::vector<char>& want,
                                          const std::vector<int>& k_keep, const std::vector<int>& q,
                                          const rmc_solve_opts& o,
                                          std::vector<std::vector<double>>& evals,
                                          std::vector<rmc_level_report>* reps);
size_t api_arena_free(rmc_ctx* ctx);
}  // namespace rmc

using namespace rmc;

namespace {

struct CutTerm {
  double coef;
  int sa, oa, sb, ob;
};

// An owned copy of a module tree (the caller's descriptor, or the tree of a chain).
struct TreeStore {
  std::vector<rmc_tree_node> nodes;
  std::vector<std::vector<rmc_term>> terms;  // per node
  int k = 0, q = 0;
  void fix() {  // point the nodes at their own term storage
    for (size_t i = 0; i < nodes.size(); ++i) {
      nodes[i].n_terms = (int)terms[i].size();
      nodes[i].terms = terms[i].empty() ? nullptr : terms[i].data();
    }
  }
};

struct Node {
  int kind = 0;  // 0 leaf, 1 merge
  int width = 0;
  int left = -1, right = -1;
  int level = 0;
  int k = 0;     // retained states
  bool root = false;
  int key = -1;
  std::vector<rmc_term> terms;  // leaf: local sites
  std::vector<CutTerm> cut;
};

struct Plan {
  std::vector<Node> nodes;
  int root = -1;
  int n_keys = 0;
  int q = 0;
  std::vector<std::set<std::pair<int, int>>> need;  // per key: (site, op)
};

std::string term_bytes(const rmc_term& t) {
  std::string s;
  s.append((const char*)&t.coef, sizeof(double));
  int v[5] = {t.nsite, t.site[0], t.nsite > 1 ? t.site[1] : -1, t.op[0], t.nsite > 1 ? t.op[1] : 0};
  s.append((const char*)v, sizeof(v));
  return s;
}

void validate_term(const rmc_term& tm, int n_sites) {
  RMC_CHECK(tm.nsite == 1 || tm.nsite == 2, RMC_ERR_ARG, "term nsite must be 1 or 2");
  for (int u = 0; u < tm.nsite; ++u) {
    RMC_CHECK(tm.site[u] >= 0 && tm.site[u] < n_sites, RMC_ERR_ARG, "term site out of range");
    RMC_CHECK(tm.op[u] >= RMC_OP_X && tm.op[u] <= RMC_OP_Z, RMC_ERR_ARG, "unknown operator");
  }
  if (tm.nsite == 2) RMC_CHECK(tm.site[0] != tm.site[1], RMC_ERR_ARG, "two-site term on one site");
}

void validate_chain(const rmc_chain_desc* c) {
  RMC_CHECK(c != nullptr, RMC_ERR_ARG, "null chain");
  RMC_CHECK(c->n_sites >= 1 && c->leaf_sites >= 1 && c->leaf_sites <= 12, RMC_ERR_ARG,
            "leaf_sites must be 1..12");
  RMC_CHECK(c->n_sites % c->leaf_sites == 0, RMC_ERR_ARG, "n_sites must be a multiple of leaf_sites");
  RMC_CHECK(c->k >= 1, RMC_ERR_ARG, "k must be >= 1");
  RMC_CHECK(c->q >= 1 && c->q <= c->k, RMC_ERR_ARG, "need 1 <= q <= k");
  RMC_CHECK(c->n_terms >= 0 && (c->n_terms == 0 || c->terms), RMC_ERR_ARG, "bad term list");
  for (int t = 0; t < c->n_terms; ++t) validate_term(c->terms[t], c->n_sites);
}

// The tree of a chain: leaves of leaf_sites consecutive sites, pairwise merges of
// adjacent modules left to right, an odd module carried up. A leaf takes the terms
// lying in it, a merge the two-site terms with one site in each child (in list order,
// oriented A first, sites local to each child).
TreeStore tree_of_chain(const rmc_chain_desc* c) {
  validate_chain(c);
  TreeStore T;
  T.k = c->k;
  T.q = c->q;
  struct Span { int node, a, b; };
  std::vector<Span> cur;
  const int L0 = c->leaf_sites;
  for (int a = 0; a < c->n_sites; a += L0) {
    rmc_tree_node nd{-1, -1, L0, 0, nullptr, 0};
    std::vector<rmc_term> ts;
    for (int t = 0; t < c->n_terms; ++t) {
      const rmc_term& tm = c->terms[t];
      bool in = true;
      for (int u = 0; u < tm.nsite; ++u) in = in && tm.site[u] >= a && tm.site[u] < a + L0;
      if (!in) continue;
      rmc_term lt = tm;
      for (int u = 0; u < tm.nsite; ++u) lt.site[u] -= a;
      ts.push_back(lt);
    }
    T.nodes.push_back(nd);
    T.terms.push_back(std::move(ts));
    cur.push_back({(int)T.nodes.size() - 1, a, a + L0});
  }
  while (cur.size() > 1) {
    std::vector<Span> nxt;
    for (size_t i = 0; i + 1 < cur.size(); i += 2) {
      const int a = cur[i].a, m = cur[i].b, b = cur[i + 1].b;
      rmc_tree_node nd{cur[i].node, cur[i + 1].node, 0, 0, nullptr, 0};
      std::vector<rmc_term> ts;
      for (int t = 0; t < c->n_terms; ++t) {
        const rmc_term& tm = c->terms[t];
        if (tm.nsite != 2) continue;
        const int s0 = tm.site[0], s1 = tm.site[1];
        const bool f = s0 >= a && s0 < m && s1 >= m && s1 < b;
        const bool r = s1 >= a && s1 < m && s0 >= m && s0 < b;
        if (!f && !r) continue;
        rmc_term ct = tm;
        ct.site[0] = (f ? s0 : s1) - a;
        ct.op[0] = f ? tm.op[0] : tm.op[1];
        ct.site[1] = (f ? s1 : s0) - m;
        ct.op[1] = f ? tm.op[1] : tm.op[0];
        ts.push_back(ct);
      }
      T.nodes.push_back(nd);
      T.terms.push_back(std::move(ts));
      nxt.push_back({(int)T.nodes.size() - 1, a, b});
    }
    if (cur.size() % 2) nxt.push_back(cur.back());
    cur.swap(nxt);
  }
  T.fix();
  return T;
}

// A validated copy of a caller's tree.
TreeStore tree_copy(const rmc_tree_desc* t) {
  RMC_CHECK(t != nullptr, RMC_ERR_ARG, "null tree");
  RMC_CHECK(t->n_nodes >= 1 && t->nodes, RMC_ERR_ARG, "a tree needs at least one node");
  RMC_CHECK(t->k >= 1, RMC_ERR_ARG, "k must be >= 1");
  RMC_CHECK(t->q >= 1 && t->q <= t->k, RMC_ERR_ARG, "need 1 <= q <= k");
  const int n = t->n_nodes;
  TreeStore T;
  T.k = t->k;
  T.q = t->q;
  std::vector<int> width(n, 0);
  std::vector<char> reached(n, 0);
  reached[n - 1] = 1;
  for (int i = 0; i < n; ++i) {
    const rmc_tree_node& nd = t->nodes[i];
    RMC_CHECK(nd.n_terms >= 0 && (nd.n_terms == 0 || nd.terms), RMC_ERR_ARG, "bad term list");
    RMC_CHECK(nd.k >= 0, RMC_ERR_ARG, "a node's k must be >= 0");
    const bool leaf = nd.left < 0 && nd.right < 0;
    if (leaf) {
      RMC_CHECK(nd.left == -1 && nd.right == -1, RMC_ERR_ARG, "a leaf has left = right = -1");
      RMC_CHECK(nd.n_sites >= 1 && nd.n_sites <= 12, RMC_ERR_ARG, "a leaf has 1..12 sites");
      width[i] = nd.n_sites;
      for (int u = 0; u < nd.n_terms; ++u) validate_term(nd.terms[u], nd.n_sites);
    } else {
      RMC_CHECK(nd.left >= 0 && nd.left < i && nd.right >= 0 && nd.right < i, RMC_ERR_ARG,
                "a merge's children must come before it");
      const int wA = width[nd.left], wB = width[nd.right];
      RMC_CHECK(wA + wB <= (1 << 24), RMC_ERR_ARG, "tree too wide");
      width[i] = wA + wB;
      for (int u = 0; u < nd.n_terms; ++u) {
        const rmc_term& tm = nd.terms[u];
        RMC_CHECK(tm.nsite == 2, RMC_ERR_ARG, "a coupling term acts on one site of each child");
        RMC_CHECK(tm.site[0] >= 0 && tm.site[0] < wA && tm.site[1] >= 0 && tm.site[1] < wB,
                  RMC_ERR_ARG, "coupling term site outside its child");
        for (int v = 0; v < 2; ++v)
          RMC_CHECK(tm.op[v] >= RMC_OP_X && tm.op[v] <= RMC_OP_Z, RMC_ERR_ARG, "unknown operator");
      }
    }
    T.nodes.push_back(nd);
    T.terms.emplace_back(nd.terms, nd.terms + nd.n_terms);
  }
  for (int i = n - 1; i >= 0; --i)
    if (reached[i] && t->nodes[i].left >= 0) reached[t->nodes[i].left] = reached[t->nodes[i].right] = 1;
  for (int i = 0; i < n; ++i) RMC_CHECK(reached[i], RMC_ERR_ARG, "a node is not part of the tree");
  T.fix();
  return T;
}

// Plan of a tree: levels (leaf 0, merge 1 + deeper child), structural keys (modules
// with equal content are computed once), and the operators each module must project
// for the merges above it.
Plan make_plan(const TreeStore& T) {
  Plan P;
  std::map<std::string, int> keys;
  auto intern = [&](const std::string& s) {
    auto it = keys.find(s);
    if (it != keys.end()) return it->second;
    int id = (int)keys.size();
    keys[s] = id;
    return id;
  };
  const int n = (int)T.nodes.size();
  P.nodes.resize(n);
  P.root = n - 1;
  P.q = T.q;
  for (int i = 0; i < n; ++i) {
    const rmc_tree_node& tn = T.nodes[i];
    Node& nd = P.nodes[i];
    nd.k = tn.k > 0 ? tn.k : T.k;
    nd.root = i == n - 1;
    if (tn.left < 0) {
      nd.kind = 0;
      nd.width = tn.n_sites;
      std::string ks = "L" + std::to_string(nd.width) + "k" + std::to_string(nd.k) + ":";
      for (int u = 0; u < tn.n_terms; ++u) {
        nd.terms.push_back(tn.terms[u]);
        ks += term_bytes(tn.terms[u]);
      }
      nd.key = intern(ks);
      continue;
    }
    const Node& L = P.nodes[tn.left];
    const Node& R = P.nodes[tn.right];
    nd.kind = 1;
    nd.left = tn.left;
    nd.right = tn.right;
    nd.width = L.width + R.width;
    nd.level = 1 + std::max(L.level, R.level);
    std::string ks = "M" + std::to_string(L.key) + "," + std::to_string(R.key) + "k" +
                     std::to_string(nd.k) + (nd.root ? "R:" : ":");
    for (int u = 0; u < tn.n_terms; ++u) {
      const rmc_term& tm = tn.terms[u];
      CutTerm ct{tm.coef, tm.site[0], tm.op[0], tm.site[1], tm.op[1]};
      nd.cut.push_back(ct);
      int v[4] = {ct.sa, ct.oa, ct.sb, ct.ob};
      ks.append((const char*)&ct.coef, sizeof(double));
      ks.append((const char*)v, sizeof(v));
    }
    nd.key = intern(ks);
  }
  P.n_keys = (int)keys.size();
  // operator requirements: top-down (parents have larger indices), then per key
  std::vector<std::set<std::pair<int, int>>> nneed(n);
  for (int i = n - 1; i >= 0; --i) {
    const Node& nd = P.nodes[i];
    if (nd.kind != 1) continue;
    for (const CutTerm& ct : nd.cut) {
      nneed[nd.left].insert({ct.sa, ct.oa});
      nneed[nd.right].insert({ct.sb, ct.ob});
    }
    const int wA = P.nodes[nd.left].width;
    for (auto& so : nneed[i]) {
      if (so.first < wA) nneed[nd.left].insert(so);
      else nneed[nd.right].insert({so.first - wA, so.second});
    }
  }
  P.need.assign(P.n_keys, {});
  for (int i = 0; i < n; ++i)
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

// One job in flight: its tree, plan, modules (by structural key) and results.
struct JobRun {
  TreeStore tree;
  Plan P;
  std::vector<rmc_module*> by_key;
  std::vector<rmc_module*> created;
  std::vector<double> e;
  rmc_report* rep = nullptr;
  rmc_status status = RMC_OK;
  std::string err;
  double t0 = 0.0;
  int level = 0;  // next level to run
  int max_level = 0;
  bool done = false;
};

void job_init(JobRun& J, TreeStore&& T, rmc_report* rep) {
  J.tree = std::move(T);
  J.tree.fix();
  J.P = make_plan(J.tree);
  J.by_key.assign(J.P.n_keys, nullptr);
  J.e.assign(J.P.q, NAN);
  J.rep = rep;
  J.t0 = now_ms();
  J.level = 0;
  J.max_level = 0;
  for (const Node& nd : J.P.nodes) J.max_level = std::max(J.max_level, nd.level);
  if (rep) {
    rep->n_records = 0;
    rep->n_leaf_ed = 0;
    rep->n_merges = 0;
  }
}

TreeStore tree_of_job(const rmc_job_desc* j) {
  RMC_CHECK(j != nullptr, RMC_ERR_ARG, "null job");
  RMC_CHECK((j->tree != nullptr) != (j->chain != nullptr), RMC_ERR_ARG,
            "a job sets exactly one of tree and chain");
  return j->tree ? tree_copy(j->tree) : tree_of_chain(j->chain);
}

void job_release(rmc_ctx* ctx, JobRun& J) {
  for (rmc_module* m : J.created) api_free_module(ctx, m);
  J.created.clear();
  std::fill(J.by_key.begin(), J.by_key.end(), nullptr);
}

void job_fail(rmc_ctx* ctx, JobRun& J, rmc_status st, const std::string& msg) {
  J.status = st;
  J.err = msg;
  J.done = true;
  job_release(ctx, J);
}

// Bytes one coupling step (or leaf solve) of dimension n, nev wanted, needs.
size_t task_bytes(int n, int nev) {
  const size_t m = (size_t)std::min(n, nev + std::max(8, (nev + 7) / 8) + 8);
  return (7 * m * n + 6 * m * m + 64 * m * m) * sizeof(double) + (size_t)n * 64 + (1 << 16);
}

struct Task {
  JobRun* J;
  int node;
};

// Runs one level (the next level of every job in `jobs`) as batched solves: the merges
// first, then the leaves. `admit`, if set, is called between the two and may append
// jobs that have not started; their leaves join this round's leaf solve.
void run_level(rmc_ctx* ctx, std::vector<JobRun*>& jobs, const rmc_solve_opts& o,
               const std::function<void(std::vector<JobRun*>&)>& admit = {}) {
  std::unique_ptr<HostScope> tasks_scope(new HostScope("level.tasks"));
  std::vector<Task> leaf_t, merge_t, reused;
  auto collect = [&](size_t from) {
    for (size_t ji = from; ji < jobs.size(); ++ji) {
      JobRun* J = jobs[ji];
      if (J->done) continue;
      const int L = J->level;
      std::vector<char> seen(J->P.n_keys, 0);
      for (size_t i = 0; i < J->P.nodes.size(); ++i) {
        const Node& nd = J->P.nodes[i];
        if (nd.level != L) continue;
        const bool single = (int)i == J->P.root && nd.kind == 0;
        if (!nd.root && !single && (J->by_key[nd.key] || seen[nd.key])) {
          reused.push_back(Task{J, (int)i});
          continue;
        }
        seen[nd.key] = 1;
        (nd.kind == 0 ? leaf_t : merge_t).push_back(Task{J, (int)i});
      }
    }
  };
  collect(0);
  // memory-admitted chunks
  auto chunks = [&](std::vector<Task>& T, auto size_of) {
    std::vector<std::vector<Task>> out;
    const size_t budget = api_arena_free(ctx) / 2;
    size_t acc = 0;
    for (const Task& t : T) {
      size_t b = size_of(t);
      if (!out.empty() && acc + b <= budget) {
        out.back().push_back(t);
        acc += b;
      } else {
        out.push_back({t});
        acc = b;
      }
    }
    return out;
  };
  tasks_scope.reset();
  auto after_module = [&](JobRun* J, int node, rmc_module* m, rmc_level_report r,
                          const std::vector<double>& ev) {
    RMC_HOST_SCOPE("level.after_module");
    const Node& nd = J->P.nodes[node];
    r.level = nd.level;
    r.width = nd.width;
    if (m) {
      J->created.push_back(m);
      for (auto& so : J->P.need[nd.key]) api_project_op(ctx, m, so.first, so.second);  // already batched
      api_release_basis(ctx, m);
      J->by_key[nd.key] = m;
    } else {  // root: energies
      for (int q = 0; q < J->P.q; ++q) J->e[q] = ev[q];
    }
    add_record(J->rep, r);
    if (J->rep) (nd.kind == 0 ? J->rep->n_leaf_ed : J->rep->n_merges)++;
  };
  // the operators later steps need from the new modules, in one batch
  auto project_new = [&](const std::vector<Task>& C, const std::vector<rmc_module*>& mods) {
    RMC_HOST_SCOPE("level.project_new");
    std::vector<rmc_module*> ms;
    std::vector<std::pair<int, int>> so;
    for (size_t i = 0; i < C.size() && i < mods.size(); ++i) {
      if (!mods[i]) continue;
      const Node& nd = C[i].J->P.nodes[C[i].node];
      for (auto& x : C[i].J->P.need[nd.key]) {
        ms.push_back(mods[i]);
        so.push_back(x);
      }
    }
    api_project_ops_batch(ctx, ms, so);
  };
  // merges
  for (auto& ch : chunks(merge_t, [&](const Task& t) {
         const Node& nd = t.J->P.nodes[t.node];
         rmc_module* A = t.J->by_key[t.J->P.nodes[nd.left].key];
         rmc_module* B = t.J->by_key[t.J->P.nodes[nd.right].key];
         const int n = (A && B) ? A->k_eff * B->k_eff : 1;
         size_t packs = 0;
         if (A && B)
           for (int pr = 0; pr < 3; ++pr)
             packs += kron_pack_bytes(pr, A->k_eff, B->k_eff, (int)nd.cut.size()) + 256;
         return task_bytes(n, nd.root ? t.J->P.q : nd.k + 1) + packs;
       })) {
    auto solve = [&](std::vector<Task>& C) {
      std::vector<rmc_module*> As, Bs;
      std::vector<std::vector<double>> coefs(C.size());
      std::vector<std::vector<int>> ia(C.size()), ib(C.size());
      std::vector<rmc_bond_desc> bds(C.size());
      std::vector<const rmc_bond_desc*> bp;
      std::vector<char> want;
      std::vector<int> kk, qq;
      std::vector<Task> live;
      for (size_t i = 0; i < C.size(); ++i) {
        JobRun* J = C[i].J;
        if (J->done) continue;
        const Node& nd = J->P.nodes[C[i].node];
        rmc_module* A = J->by_key[J->P.nodes[nd.left].key];
        rmc_module* B = J->by_key[J->P.nodes[nd.right].key];
        RMC_CHECK(A && B, RMC_ERR_STATE, "child module missing");
        const size_t w = live.size();
        for (const CutTerm& ct : nd.cut) {
          coefs[w].push_back(ct.coef);
          ia[w].push_back(api_project_op(ctx, A, ct.sa, ct.oa));
          ib[w].push_back(api_project_op(ctx, B, ct.sb, ct.ob));
        }
        bds[w] = rmc_bond_desc{(int)coefs[w].size(), coefs[w].data(), ia[w].data(), ib[w].data()};
        As.push_back(A);
        Bs.push_back(B);
        want.push_back(nd.root ? 0 : 1);
        kk.push_back(nd.k);
        qq.push_back(nd.root ? J->P.q : std::min(J->P.q, nd.k));
        live.push_back(C[i]);
      }
      for (size_t w = 0; w < live.size(); ++w) bp.push_back(&bds[w]);
      if (live.empty()) return;
      std::vector<std::vector<double>> ev;
      std::vector<rmc_level_report> reps;
      std::vector<rmc_module*> mods;
      try {
        mods = api_couple_batch(ctx, As, Bs, bp, want, kk, qq, o, ev, &reps);
      } catch (const Error& e) {
        // a root that did not converge keeps its best Ritz values (the error still
        // ends the job)
        if (e.code == RMC_ERR_NOCONV)
          for (size_t i = 0; i < live.size() && i < ev.size(); ++i)
            if (!want[i] && (int)ev[i].size() >= live[i].J->P.q)
              for (int q = 0; q < live[i].J->P.q; ++q) live[i].J->e[q] = ev[i][q];
        throw;
      }
      project_new(live, mods);
      for (size_t i = 0; i < live.size(); ++i) after_module(live[i].J, live[i].node, mods[i], reps[i], ev[i]);
    };
    try {
      solve(ch);
    } catch (const Error& e) {
      if (getenv("RMC_TRACE_SOLVER"))
        fprintf(stderr, "[rmc] level chunk of %zu tasks failed: %s\n", ch.size(), e.what());
      if (ch.size() == 1) {
        job_fail(ctx, *ch[0].J, e.code, e.what());
        continue;
      }
      for (Task& t : ch) {
        if (t.J->done) continue;
        std::vector<Task> one{t};
        try {
          solve(one);
        } catch (const Error& e2) {
          job_fail(ctx, *t.J, e2.code, e2.what());
        }
      }
    }
  }
  // jobs admitted between the merge and leaf phases start with this round's leaves
  if (admit) {
    const size_t before = jobs.size();
    admit(jobs);
    collect(before);
  }
  // leaves
  for (auto& ch : chunks(leaf_t, [&](const Task& t) {
         const Node& nd = t.J->P.nodes[t.node];
         const int D = 1 << nd.width;
         return task_bytes(D, std::min(D, nd.k + 1)) + (size_t)D * D * 8;
       })) {
    auto solve = [&](std::vector<Task>& C) {
      std::vector<rmc_leaf_desc> lds(C.size());
      std::vector<const rmc_leaf_desc*> lp;
      std::vector<int> ks, qo;
      for (size_t i = 0; i < C.size(); ++i) {
        const Node& nd = C[i].J->P.nodes[C[i].node];
        lds[i] = rmc_leaf_desc{nd.width, (int)nd.terms.size(), nd.terms.data()};
        lp.push_back(&lds[i]);
        ks.push_back(nd.k);
        const bool single = C[i].node == C[i].J->P.root;
        qo.push_back(single ? C[i].J->P.q : 0);
      }
      std::vector<std::vector<double>> ev;
      std::vector<rmc_level_report> reps;
      std::vector<rmc_module*> mods;
      try {
        mods = api_leaf_solve_batch(ctx, lp, ks, qo, o, ev, &reps);
      } catch (const Error& e) {
        if (e.code == RMC_ERR_NOCONV)  // a single-leaf job's best Ritz values
          for (size_t i = 0; i < C.size() && i < ev.size(); ++i)
            if (qo[i] > 0 && (int)ev[i].size() >= qo[i])
              for (int q = 0; q < qo[i]; ++q) C[i].J->e[q] = ev[i][q];
        throw;
      }
      project_new(C, mods);
      for (size_t i = 0; i < C.size(); ++i) {
        reps[i].kind = qo[i] > 0 ? 2 : 0;
        after_module(C[i].J, C[i].node, mods[i], reps[i], ev[i]);
      }
    };
    try {
      solve(ch);
    } catch (const Error& e) {
      if (getenv("RMC_TRACE_SOLVER"))
        fprintf(stderr, "[rmc] level chunk of %zu tasks failed: %s\n", ch.size(), e.what());
      if (ch.size() == 1) {
        job_fail(ctx, *ch[0].J, e.code, e.what());
        continue;
      }
      for (Task& t : ch) {  // isolate the failing job(s)
        if (t.J->done) continue;
        std::vector<Task> one{t};
        try {
          solve(one);
        } catch (const Error& e2) {
          job_fail(ctx, *t.J, e2.code, e2.what());
        }
      }
    }
  }
  for (const Task& t : reused) {  // records of modules computed once and reused
    if (t.J->done) continue;
    const Node& nd = t.J->P.nodes[t.node];
    rmc_level_report r{};
    r.level = nd.level;
    r.width = nd.width;
    r.kind = nd.kind;
    r.reused = 1;
    if (rmc_module* m = t.J->by_key[nd.key]) {
      r.k_eff = m->k_eff;
      r.gap = m->gap;
    }
    add_record(t.J->rep, r);
  }
  RMC_HOST_SCOPE("level.finish");
  for (JobRun* J : jobs) {
    if (J->done) continue;
    if (J->level >= J->max_level) {
      J->done = true;
      if (J->rep) J->rep->total_ms = now_ms() - J->t0;
      job_release(ctx, *J);
    } else {
      J->level++;
    }
  }
}

void run_jobs(rmc_ctx* ctx, std::vector<JobRun*>& jobs, const rmc_solve_opts& o) {
  for (;;) {
    bool any = false;
    for (JobRun* J : jobs) any = any || !J->done;
    if (!any) break;
    run_level(ctx, jobs, o);
  }
}

// ---- serving (continuous batching) ------------------------------------------------

struct ServeJob {
  unsigned long long id = 0;
  double t_submit = 0.0;
  size_t mem = 0;
  JobRun run;
};

struct ServeResult {
  std::vector<double> e;
  int status = RMC_OK;
  double latency_ms = 0.0;
};

struct ServeState {
  rmc_ctx* ctx = nullptr;
  std::thread th;
  std::mutex mu;
  std::condition_variable cv;
  bool stop = false;
  rmc_solve_opts opts{};
  int max_inflight = 64;
  size_t budget = 0;
  std::deque<std::unique_ptr<ServeJob>> queue;
  std::vector<std::unique_ptr<ServeJob>> inflight;  // scheduler thread only
  std::set<unsigned long long> pending;             // queued or in flight
  std::map<unsigned long long, ServeResult> done;
  unsigned long long next_id = 1;
  size_t inflight_mem = 0;
  std::string fatal;
};

// Device memory a job needs at its widest level (solver workspace of the distinct
// modules of that level) plus the projected operators its modules keep, from its plan.
size_t job_memory(const Plan& P) {
  const int n = (int)P.nodes.size();
  std::vector<long> kept(n, 1);
  std::map<int, std::map<int, size_t>> by_level;  // level -> key -> bytes
  std::set<int> seen;
  size_t keep_bytes = 0;
  for (int i = 0; i < n; ++i) {
    const Node& nd = P.nodes[i];
    long dim, nev;
    size_t b;
    if (nd.kind == 0) {
      dim = 1L << nd.width;
      kept[i] = nd.root ? std::min<long>(P.q, dim) : std::min<long>(nd.k, dim);
      nev = nd.root ? std::min<long>(P.q, dim) : std::min<long>(dim, nd.k + 1);
      b = task_bytes((int)dim, (int)nev) + (size_t)dim * dim * 8;
    } else {
      const long kA = kept[nd.left], kB = kept[nd.right];
      dim = kA * kB;
      kept[i] = nd.root ? std::min<long>(P.q, dim) : std::min<long>(nd.k, dim);
      nev = nd.root ? std::min<long>(P.q, dim) : std::min<long>(dim, nd.k + 1);
      size_t packs = 0;
      for (int pr = 0; pr < 3; ++pr) packs += kron_pack_bytes(pr, (int)kA, (int)kB, (int)nd.cut.size()) + 256;
      b = task_bytes((int)dim, (int)nev) + (size_t)dim * 64 + packs;
    }
    size_t& slot = by_level[nd.level][nd.key];
    slot = std::max(slot, b);
    if (seen.insert(nd.key).second)
      keep_bytes += (P.need[nd.key].size() * kept[i] * kept[i] + kept[i]) * sizeof(double) +
                    (size_t)kept[i] * dim * sizeof(double);  // basis until its projections
  }
  size_t best = 0;
  for (auto& lv : by_level) {
    size_t sum = 0;
    for (auto& kv : lv.second) sum += kv.second;
    best = std::max(best, sum);
  }
  return best + keep_bytes;
}

// Admission (S->mu held): queued jobs go into flight, in arrival order, while a slot is
// free and their memory estimate fits beside the jobs in flight; a job that could never
// fit finishes with RMC_ERR_OOM. Returns the admitted jobs.
std::vector<JobRun*> admit_locked(ServeState* S) {
  std::vector<size_t> mem;
  mem.reserve(S->queue.size());
  for (const auto& j : S->queue) mem.push_back(j->mem);
  const std::string d = admit_pass(mem, S->inflight_mem, (int)S->inflight.size(), S->max_inflight, S->budget);
  std::vector<JobRun*> out;
  for (char c : d) {
    ServeJob* j = S->queue.front().get();
    if (c == 'r') {  // can never fit: finished with RMC_ERR_OOM
      ServeResult r;
      r.status = RMC_ERR_OOM;
      r.latency_ms = now_ms() - j->t_submit;
      S->done[j->id] = r;
      S->pending.erase(j->id);
      S->queue.pop_front();
      continue;
    }
    S->inflight_mem += j->mem;
    S->inflight.push_back(std::move(S->queue.front()));
    S->queue.pop_front();
    out.push_back(&S->inflight.back()->run);
  }
  return out;
}

void serve_loop(ServeState* S) {
  rmc_ctx* ctx = S->ctx;
  (void)hipSetDevice(ctx->device);
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv.wait(lk, [&] { return S->stop || !S->queue.empty() || !S->inflight.empty(); });
      if (S->stop && S->queue.empty() && S->inflight.empty()) break;
      admit_locked(S);
    }
    std::vector<JobRun*> runs;
    for (auto& j : S->inflight) runs.push_back(&j->run);
    // jobs that arrive while this round's merges run are admitted before its leaf phase
    auto admit_more = [S](std::vector<JobRun*>& js) {
      std::lock_guard<std::mutex> lk(S->mu);
      for (JobRun* J : admit_locked(S)) js.push_back(J);
    };
    try {
      run_level(ctx, runs, S->opts, admit_more);
    } catch (const Error& e) {
      for (JobRun* J : runs)
        if (!J->done) job_fail(ctx, *J, e.code, e.what());
    } catch (const std::exception& e) {
      for (JobRun* J : runs)
        if (!J->done) job_fail(ctx, *J, RMC_ERR_STATE, e.what());
    }
    std::lock_guard<std::mutex> lk(S->mu);
    for (size_t i = 0; i < S->inflight.size();) {
      ServeJob* j = S->inflight[i].get();
      if (!j->run.done) {
        ++i;
        continue;
      }
      ServeResult r;
      r.e = j->run.e;
      r.status = j->run.status;
      r.latency_ms = now_ms() - j->t_submit;
      S->done[j->id] = std::move(r);
      S->pending.erase(j->id);
      S->inflight_mem -= j->mem;
      S->inflight.erase(S->inflight.begin() + i);
    }
  }
}

template <class F>
rmc_status guard(rmc_ctx* ctx, F&& f) {
  try {
    RMC_CHECK(!ctx || !ctx->serving, RMC_ERR_STATE, "the context is serving; stop it first");
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

namespace {
rmc_status recurse_one(rmc_ctx* ctx, const rmc_job_desc* job, const rmc_solve_opts* opts,
                       double* energies, rmc_report* report) {
  if (!ctx) return RMC_ERR_ARG;
  JobRun J;
  rmc_status st = guard(ctx, [&] {
    RMC_CHECK(energies != nullptr, RMC_ERR_ARG, "null energies");
    rmc_solve_opts o;
    rmc_default_opts(&o);
    if (opts) o = *opts;
    RMC_CHECK(o.precision >= RMC_FP64 && o.precision <= RMC_BF16, RMC_ERR_ARG, "bad precision");
    job_init(J, tree_of_job(job), report);
    std::vector<JobRun*> jobs{&J};
    run_jobs(ctx, jobs, o);
    if (J.status != RMC_OK) throw Error(J.status, J.err);
    for (int i = 0; i < J.P.q; ++i) energies[i] = J.e[i];
  });
  // a solve that did not converge: the root's best Ritz values where it was the root's
  // (NaN otherwise), and the report as far as it got
  if (st == RMC_ERR_NOCONV && J.status == RMC_ERR_NOCONV)
    for (int i = 0; i < J.P.q; ++i) energies[i] = J.e[i];
  return st;
}
}  // namespace

rmc_status rmc_recurse(rmc_ctx* ctx, const rmc_tree_desc* tree, const rmc_solve_opts* opts,
                       double* energies, rmc_report* report) {
  rmc_job_desc j{tree, nullptr};
  if (!tree) return RMC_ERR_ARG;
  return recurse_one(ctx, &j, opts, energies, report);
}

rmc_status rmc_recurse_chain(rmc_ctx* ctx, const rmc_chain_desc* chain, const rmc_solve_opts* opts,
                             double* energies, rmc_report* report) {
  rmc_job_desc j{nullptr, chain};
  if (!chain) return RMC_ERR_ARG;
  return recurse_one(ctx, &j, opts, energies, report);
}

rmc_status rmc_recurse_batch(rmc_ctx* ctx, int n_jobs, const rmc_job_desc* jobs,
                             const rmc_solve_opts* opts, double* energies, int q_stride,
                             int* status_host) {
  if (!ctx) return RMC_ERR_ARG;
  if (n_jobs < 0 || (n_jobs > 0 && (!jobs || !energies))) return RMC_ERR_ARG;
  std::vector<JobRun> runs(n_jobs);
  std::vector<int> st(n_jobs, RMC_OK);
  rmc_status top = guard(ctx, [&] {
    rmc_solve_opts o;
    rmc_default_opts(&o);
    if (opts) o = *opts;
    RMC_CHECK(o.precision >= RMC_FP64 && o.precision <= RMC_BF16, RMC_ERR_ARG, "bad precision");
    std::vector<JobRun*> live;
    std::unique_ptr<HostScope> plans(new HostScope("batch.plans"));
    for (int j = 0; j < n_jobs; ++j) {
      try {
        TreeStore T = tree_of_job(&jobs[j]);
        RMC_CHECK(T.q <= q_stride, RMC_ERR_ARG, "q above q_stride");
        job_init(runs[j], std::move(T), nullptr);
        live.push_back(&runs[j]);
      } catch (const Error& e) {
        st[j] = e.code;
      }
    }
    plans.reset();
    RMC_HOST_SCOPE("batch.run");
    run_jobs(ctx, live, o);
  });
  host_trace_dump("rmc_recurse_batch");
  rmc_status worst = top;
  for (int j = 0; j < n_jobs; ++j) {
    if (st[j] == RMC_OK) st[j] = runs[j].status;
    if (st[j] == RMC_OK && top == RMC_OK)
      for (int i = 0; i < runs[j].P.q; ++i) energies[(size_t)j * q_stride + i] = runs[j].e[i];
    if (status_host) status_host[j] = top != RMC_OK ? top : st[j];
    if (st[j] != RMC_OK && worst == RMC_OK) worst = (rmc_status)st[j];
  }
  return worst;
}

rmc_status rmc_serve_start(rmc_ctx* ctx, const rmc_solve_opts* opts, int max_inflight,
                           size_t mem_budget) {
  if (!ctx) return RMC_ERR_ARG;
  return guard(ctx, [&] {
    RMC_CHECK(max_inflight >= 1, RMC_ERR_ARG, "max_inflight must be >= 1");
    auto* S = new ServeState();
    S->ctx = ctx;
    rmc_default_opts(&S->opts);
    if (opts) S->opts = *opts;
    RMC_CHECK(S->opts.precision >= RMC_FP64 && S->opts.precision <= RMC_BF16, RMC_ERR_ARG,
              "bad precision");
    S->max_inflight = max_inflight;
    S->budget = mem_budget ? mem_budget : ctx->arena.size() / 2;
    RMC_HIP(hipStreamSynchronize(ctx->stream));
    ctx->serve = S;
    ctx->serving = true;
    S->th = std::thread(serve_loop, S);
  });
}

rmc_status rmc_submit(rmc_ctx* ctx, const rmc_job_desc* job, unsigned long long* job_id) {
  if (!ctx || !ctx->serving || !job_id) return !ctx ? RMC_ERR_ARG : (!job_id ? RMC_ERR_ARG : RMC_ERR_STATE);
  ServeState* S = (ServeState*)ctx->serve;
  try {
    auto j = std::make_unique<ServeJob>();
    j->t_submit = now_ms();
    job_init(j->run, tree_of_job(job), nullptr);
    j->mem = job_memory(j->run.P);
    std::lock_guard<std::mutex> lk(S->mu);
    j->id = S->next_id++;
    *job_id = j->id;
    S->pending.insert(j->id);
    S->queue.push_back(std::move(j));
  } catch (const Error& e) {
    std::lock_guard<std::mutex> lk(S->mu);
    ctx->last_error = e.what();
    return e.code;
  }
  S->cv.notify_one();
  return RMC_OK;
}

rmc_status rmc_poll(rmc_ctx* ctx, unsigned long long job_id, int* done, double* energies,
                    int capacity, int* job_status, double* latency_ms) {
  if (!ctx || !ctx->serving || !done) return !ctx || !done ? RMC_ERR_ARG : RMC_ERR_STATE;
  if (energies && capacity < 0) return RMC_ERR_ARG;
  ServeState* S = (ServeState*)ctx->serve;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->done.find(job_id);
  if (it == S->done.end()) {
    if (!S->pending.count(job_id)) return RMC_ERR_ARG;
    *done = 0;
    return RMC_OK;
  }
  *done = 1;
  if (energies) {
    const size_t nc = std::min(it->second.e.size(), (size_t)capacity);
    std::copy(it->second.e.begin(), it->second.e.begin() + nc, energies);
  }
  if (job_status) *job_status = it->second.status;
  if (latency_ms) *latency_ms = it->second.latency_ms;
  S->done.erase(it);
  return RMC_OK;
}

rmc_status rmc_serve_stop(rmc_ctx* ctx) {
  if (!ctx) return RMC_ERR_ARG;
  if (!ctx->serving) return RMC_ERR_STATE;
  ServeState* S = (ServeState*)ctx->serve;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv.notify_one();
  if (S->th.joinable()) S->th.join();
  ctx->serving = false;
  ctx->serve = nullptr;
  delete S;
  return RMC_OK;
}

}  // extern "C"
