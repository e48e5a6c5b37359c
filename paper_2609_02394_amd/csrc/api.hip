// librmc C ABI: context and arena, modules, leaf ED, operator projection, one
// coupling step, and the recursion over a chain (Algorithm 1 of the paper).
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "rmc_batch.h"
#include "rmc_internal.h"


using namespace rmc;

namespace {

// Largest eigenvalue of a coupling before projection, sum_i c_i P_i (x) Q_i on the
// sites its terms touch (P_i, Q_i one-site operators of the real alphabet). In the
// merged block the coupling is V^T (this) V for the isometry V of the two kept
// bases, so its largest eigenvalue is at most this value (Rayleigh quotient), a
// tighter bound than sum |c_i| when the terms do not align. Dense cyclic Jacobi on
// the 2^s states, s <= 6 sites; +inf beyond that or for an unknown operator. Cached
// by the coupling's structure.
double coupling_top(const rmc_module* A, const rmc_module* B, const rmc_bond_desc* bond) {
  static std::mutex mu;
  static std::map<std::string, double> cache;
  const int T = bond->n_terms;
  std::vector<std::pair<int, int>> qs;  // (side, site)
  for (int i = 0; i < T; ++i) {
    qs.push_back({0, A->ops[bond->opA[i]].site});
    qs.push_back({1, B->ops[bond->opB[i]].site});
  }
  std::sort(qs.begin(), qs.end());
  qs.erase(std::unique(qs.begin(), qs.end()), qs.end());
  const int ns = (int)qs.size();
  if (ns > 6) return INFINITY;
  auto qubit = [&](int side, int site) {
    return (int)(std::lower_bound(qs.begin(), qs.end(), std::make_pair(side, site)) - qs.begin());
  };
  std::string key;
  char buf[96];
  for (int i = 0; i < T; ++i) {
    const auto& a = A->ops[bond->opA[i]];
    const auto& b = B->ops[bond->opB[i]];
    if (a.op < RMC_OP_X || a.op > RMC_OP_Z || b.op < RMC_OP_X || b.op > RMC_OP_Z) return INFINITY;
    snprintf(buf, sizeof buf, "%a:%d%d:%d%d;", bond->coef[i], qubit(0, a.site), a.op, qubit(1, b.site), b.op);
    key += buf;
  }
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
  }
  const int D = 1 << ns;
  std::vector<double> M((size_t)D * D, 0.0);
  // one-site action on basis bit v: X flips (+1); T flips, +1 from 0 and -1 from 1;
  // Z keeps, +1 on 0 and -1 on 1
  auto act = [](int op, int v, int& flip, double& val) {
    flip = op == RMC_OP_Z ? 0 : 1;
    val = (op == RMC_OP_X || v == 0) ? 1.0 : -1.0;
  };
  for (int i = 0; i < T; ++i) {
    const int qa = qubit(0, A->ops[bond->opA[i]].site), qb = qubit(1, B->ops[bond->opB[i]].site);
    const int oa = A->ops[bond->opA[i]].op, ob = B->ops[bond->opB[i]].op;
    for (int r = 0; r < D; ++r) {
      int fa, fb;
      double va, vb;
      act(oa, (r >> qa) & 1, fa, va);
      act(ob, (r >> qb) & 1, fb, vb);
      const int r2 = r ^ (fa << qa) ^ (fb << qb);
      M[(size_t)r2 * D + r] += bond->coef[i] * va * vb;
    }
  }
  for (int r = 0; r < D; ++r)
    for (int c = 0; c < r; ++c) {
      const double v = 0.5 * (M[(size_t)r * D + c] + M[(size_t)c * D + r]);
      M[(size_t)r * D + c] = M[(size_t)c * D + r] = v;
    }
  double fro = 0.0;
  for (double v : M) fro += v * v;
  fro = std::sqrt(fro);
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < D; ++p)
      for (int q = p + 1; q < D; ++q) off += M[(size_t)p * D + q] * M[(size_t)p * D + q];
    if (std::sqrt(off) <= 1e-15 * (fro + 1e-300)) break;
    for (int p = 0; p < D; ++p)
      for (int q = p + 1; q < D; ++q) {
        const double apq = M[(size_t)p * D + q];
        if (apq == 0.0) continue;
        const double app = M[(size_t)p * D + p], aqq = M[(size_t)q * D + q];
        const double th = 0.5 * (aqq - app) / apq;
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < D; ++k) {
          const double mkp = M[(size_t)k * D + p], mkq = M[(size_t)k * D + q];
          M[(size_t)k * D + p] = c * mkp - sn * mkq;
          M[(size_t)k * D + q] = sn * mkp + c * mkq;
        }
        for (int k = 0; k < D; ++k) {
          const double mpk = M[(size_t)p * D + k], mqk = M[(size_t)q * D + k];
          M[(size_t)p * D + k] = c * mpk - sn * mqk;
          M[(size_t)q * D + k] = sn * mpk + c * mqk;
        }
      }
  }
  double top = -INFINITY;
  for (int r = 0; r < D; ++r) top = std::max(top, M[(size_t)r * D + r]);
  // Jacobi's rounding: a few ulps of the norm
  top += 1e-13 * (fro + 1.0);
  std::lock_guard<std::mutex> lk(mu);
  cache[key] = top;
  return top;
}

// Operators of a coupling in the streaming Kronecker kernel's layout, for every
// precision whose streaming kernel takes the size (held in the caller's scratch).
void build_packs(hipStream_t s, Scratch& sc, CoupledOp& op) {
  op.pkm = kron_pack_km(op.kA, op.kB);
  if (op.T == 0) return;  // no operators to stage
  for (int pr = 0; pr < 3; ++pr) {
    const size_t b = kron_pack_bytes(pr, op.kA, op.kB, op.T);
    op.pack[pr] = b ? static_cast<void*>(sc.get<char>(b)) : nullptr;
  }
  kron_pack(s, op.T, op.kA, op.kB, op.coef_dev, op.OAcat, op.OBcat, op.pack[0], op.pack[1],
            op.pack[2]);
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

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

void sync(rmc_ctx* ctx) { RMC_HIP(hipStreamSynchronize(ctx->stream)); }

void free_module_mem(rmc_ctx* ctx, rmc_module* m) {
  ctx->arena.release(m->E);
  m->E = nullptr;
  ctx->arena.release(m->basis);
  m->basis = nullptr;
  for (auto& o : m->ops) ctx->arena.release(o.data);
  m->ops.clear();
}

void validate_leaf(const rmc_leaf_desc* leaf) {
  RMC_CHECK(leaf != nullptr, RMC_ERR_ARG, "null leaf descriptor");
  RMC_CHECK(leaf->n_sites >= 1 && leaf->n_sites <= 12, RMC_ERR_ARG, "leaf n_sites must be 1..12");
  RMC_CHECK(leaf->n_terms >= 0 && (leaf->n_terms == 0 || leaf->terms), RMC_ERR_ARG, "bad term list");
  for (int t = 0; t < leaf->n_terms; ++t) {
    const rmc_term& tm = leaf->terms[t];
    RMC_CHECK(tm.nsite == 1 || tm.nsite == 2, RMC_ERR_ARG, "term nsite must be 1 or 2");
    for (int u = 0; u < tm.nsite; ++u) {
      RMC_CHECK(tm.site[u] >= 0 && tm.site[u] < leaf->n_sites, RMC_ERR_ARG, "term site out of range");
      RMC_CHECK(tm.op[u] >= RMC_OP_X && tm.op[u] <= RMC_OP_Z, RMC_ERR_ARG, "unknown operator");
    }
    if (tm.nsite == 2) RMC_CHECK(tm.site[0] != tm.site[1], RMC_ERR_ARG, "two-site term on one site");
  }
}

// Dense leaf H into device memory H (D x D).
void assemble_leaf(rmc_ctx* ctx, const rmc_leaf_desc* leaf, double* H) {
  std::vector<DevTerm> dt(std::max(1, leaf->n_terms));
  for (int t = 0; t < leaf->n_terms; ++t) {
    const rmc_term& tm = leaf->terms[t];
    DevTerm d{};
    d.coef = tm.coef;
    d.nsite = tm.nsite;
    for (int u = 0; u < tm.nsite; ++u) {
      d.bit[u] = leaf->n_sites - 1 - tm.site[u];
      d.op[u] = tm.op[u];
    }
    dt[t] = d;
  }
  Scratch sc(&ctx->arena);
  DevTerm* dterms = sc.get<DevTerm>(dt.size());
  RMC_HIP(hipMemcpyAsync(dterms, dt.data(), dt.size() * sizeof(DevTerm), hipMemcpyHostToDevice,
                         ctx->stream));
  leaf_assemble(ctx->stream, leaf->n_sites, leaf->n_terms, dterms, H);
  sync(ctx);  // dterms is released at scope exit
}

// ---- block-diagonal leaves ---------------------------------------------------------
// A leaf Hamiltonian whose nonzero pattern splits into several connected components
// (a conserved quantity that is diagonal in the site basis, such as total S^z for the
// Heisenberg and XXZ chains) is block diagonal after a permutation of the basis; its
// dense ED is then the union of the blocks' EDs. The components come from the term
// list with the device assembly's rule and accumulation order, so exact cancellations
// (X X - T T on |00> -> |11>) drop the same entries.
struct LeafBlocks {
  bool usable = false;  // two or more components, each within the Jacobi kernel's size
  std::vector<std::vector<int>> comps;
  int maxb = 0;
};

LeafBlocks analyse_leaf(const rmc_leaf_desc* leaf) {
  const int n = leaf->n_sites, D = 1 << n;
  std::vector<std::vector<std::pair<int, double>>> row(D);
  for (int r = 0; r < D; ++r) {
    auto& R = row[r];
    for (int t = 0; t < leaf->n_terms; ++t) {
      const rmc_term& tm = leaf->terms[t];
      int c = r;
      double sgn = 1.0;
      for (int u = 0; u < tm.nsite; ++u) {
        const int b = n - 1 - tm.site[u], br = (r >> b) & 1;
        if (tm.op[u] == RMC_OP_T) sgn *= br == 0 ? -1.0 : 1.0;
        if (tm.op[u] == RMC_OP_Z) sgn *= br == 0 ? 1.0 : -1.0;
        if (tm.op[u] != RMC_OP_Z) c ^= 1 << b;
      }
      const double val = sgn > 0.0 ? tm.coef : -tm.coef;
      auto it = std::find_if(R.begin(), R.end(), [c](const std::pair<int, double>& x) { return x.first == c; });
      if (it == R.end()) R.push_back({c, 0.0 + val});
      else it->second = it->second + val;
    }
  }
  std::vector<int> comp(D, -1);
  LeafBlocks lb;
  for (int s0 = 0; s0 < D; ++s0) {
    if (comp[s0] >= 0) continue;
    const int id = (int)lb.comps.size();
    lb.comps.push_back({s0});
    comp[s0] = id;
    for (size_t q = 0; q < lb.comps[id].size(); ++q) {
      const int r = lb.comps[id][q];
      for (auto& e : row[r])
        if (e.second != 0.0 && comp[e.first] < 0) {
          comp[e.first] = id;
          lb.comps[id].push_back(e.first);
        }
    }
  }
  for (auto& c : lb.comps) {
    std::sort(c.begin(), c.end());
    lb.maxb = std::max(lb.maxb, (int)c.size());
  }
  lb.usable = lb.comps.size() >= 2 && lb.maxb <= jacobi_max_m();
  return lb;
}

// The analysis of each distinct term list, kept for the life of the process.
const LeafBlocks& leaf_blocks(const rmc_leaf_desc* leaf) {
  static std::mutex mu;
  static std::map<std::string, LeafBlocks> cache;
  // the term list field by field (no struct padding in the key)
  std::string key(reinterpret_cast<const char*>(&leaf->n_sites), sizeof(int));
  for (int t = 0; t < leaf->n_terms; ++t) {
    const rmc_term& tm = leaf->terms[t];
    key.append(reinterpret_cast<const char*>(&tm.coef), sizeof(double));
    key.push_back((char)tm.nsite);
    for (int u = 0; u < tm.nsite; ++u) {
      key.push_back((char)tm.site[u]);
      key.push_back((char)tm.op[u]);
    }
  }
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(key);
  if (it == cache.end()) it = cache.emplace(key, analyse_leaf(leaf)).first;
  return it->second;
}

// Lowest nevs[i] eigenpairs of the block-diagonal leaves `sel` (H assembled on the
// device): every block of every leaf gathered and diagonalised by the batched Jacobi
// kernel in one launch; the leaf's eigenvalues are the sorted union (ties by block,
// then by position), its eigenvectors the block vectors scattered into full rows.
void leaf_blocks_solve(rmc_ctx* ctx, Scratch& sc, const std::vector<const rmc_leaf_desc*>& leaves,
                       const std::vector<int>& sel, const std::vector<CoupledOp>& ops,
                       const std::vector<int>& nevs, const std::vector<double*>& Xs,
                       std::vector<std::vector<double>>& evals, std::vector<SolveStats>& st) {
  hipStream_t s = ctx->stream;
  struct Blk {
    int leaf, nb;
    size_t off, offsq;
  };
  std::vector<Blk> blks;
  std::vector<int> idx;
  std::vector<std::pair<int, int>> range(leaves.size(), {0, 0});  // a leaf's blocks
  size_t sq = 0;
  int nbmax = 0;
  for (int i : sel) {
    range[i].first = (int)blks.size();
    for (const auto& c : leaf_blocks(leaves[i]).comps) {
      blks.push_back({i, (int)c.size(), idx.size(), sq});
      idx.insert(idx.end(), c.begin(), c.end());
      sq += c.size() * c.size();
      nbmax = std::max(nbmax, (int)c.size());
    }
    range[i].second = (int)blks.size();
  }
  const int NB = (int)blks.size();
  int* idx_dev = sc.get<int>(idx.size());
  double* A = sc.get<double>(sq);
  double* V = sc.get<double>(sq);
  double* Vw = sc.get<double>(sq);
  double* ev = sc.get<double>(idx.size());
  int* info = sc.get<int>(NB);
  std::vector<BlockGatherDesc> gd(NB);
  std::vector<EigDesc> ed(NB);
  for (int b = 0; b < NB; ++b) {
    const Blk& B = blks[b];
    gd[b] = BlockGatherDesc{B.nb, ops[B.leaf].n, idx_dev + B.off, ops[B.leaf].H, A + B.offsq};
    EigDesc e{};
    e.m = B.nb; e.nparts = 1; e.A = A + B.offsq; e.pstride = (long)B.nb * B.nb;
    e.evals = ev + B.off; e.V = V + B.offsq; e.Vwork = Vw + B.offsq; e.info = info + b;
    ed[b] = e;
  }
  BlockGatherDesc* gd_dev = sc.get<BlockGatherDesc>(NB);
  EigDesc* ed_dev = sc.get<EigDesc>(NB);
  RMC_HIP(hipMemcpyAsync(idx_dev, idx.data(), idx.size() * sizeof(int), hipMemcpyHostToDevice, s));
  RMC_HIP(hipMemcpyAsync(gd_dev, gd.data(), NB * sizeof(BlockGatherDesc), hipMemcpyHostToDevice, s));
  RMC_HIP(hipMemcpyAsync(ed_dev, ed.data(), NB * sizeof(EigDesc), hipMemcpyHostToDevice, s));
  gather_blocks(s, gd_dev, NB, nbmax);
  // the Jacobi launches take the blocks largest first: blocks above 56 with 1024-thread
  // workgroups, the rest with 512 threads (two workgroups a CU); the selection below
  // reads the tables in leaf order
  std::vector<EigDesc> es(NB);  // (alive until the final synchronisation)
  {
    std::vector<int> ord(NB);
    for (int b = 0; b < NB; ++b) ord[b] = b;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return blks[a].nb > blks[b].nb; });
    int nbig = 0, msmall = 0;
    for (int t = 0; t < NB; ++t) {
      es[t] = ed[ord[t]];
      if (blks[ord[t]].nb > 56) ++nbig;
      else msmall = std::max(msmall, blks[ord[t]].nb);
    }
    EigDesc* es_dev = sc.get<EigDesc>(NB);
    RMC_HIP(hipMemcpyAsync(es_dev, es.data(), NB * sizeof(EigDesc), hipMemcpyHostToDevice, s));
    jacobi_batched(s, es_dev, nbig, nbmax);
    jacobi_batched(s, es_dev + nbig, NB - nbig, msmall, 512);
  }
  // per leaf, on the device: the lowest ne of the union of its blocks' spectra (in the
  // order (eigenvalue, block, column)), their values and the scatter descriptors of the
  // rows they fill; only the kept eigenvalues and the sweep counts come back
  std::vector<LeafSelDesc> ls;
  std::vector<long> evo(leaves.size(), 0);
  long nsd = 0;
  for (int i : sel) {
    const int D = (int)(blks[range[i].second - 1].off + blks[range[i].second - 1].nb - blks[range[i].first].off);
    const int ne = std::min(nevs[i], D);
    evo[i] = nsd;
    ls.push_back(LeafSelDesc{range[i].first, range[i].second - range[i].first, ne, ops[i].n, nsd, Xs[i], nullptr});
    nsd += ne;
  }
  double* evsel = sc.get<double>(std::max(nsd, 1L));
  for (size_t t = 0; t < ls.size(); ++t) ls[t].evout = evsel + ls[t].sdbase;
  LeafSelDesc* ls_dev = sc.get<LeafSelDesc>(ls.size());
  BlockScatterDesc* sd_dev = sc.get<BlockScatterDesc>(std::max(nsd, 1L));
  RMC_HIP(hipMemcpyAsync(ls_dev, ls.data(), ls.size() * sizeof(LeafSelDesc), hipMemcpyHostToDevice, s));
  // the ranks of a leaf are a permutation of 0..D-1 unless an eigenvalue is NaN; a
  // descriptor no rank claims then stays all zero and scatters nothing
  RMC_HIP(hipMemsetAsync(sd_dev, 0, std::max(nsd, 1L) * sizeof(BlockScatterDesc), s));
  leaf_select(s, ls_dev, (int)ls.size(), ed_dev, gd_dev, sd_dev);
  scatter_block_rows(s, sd_dev, (int)nsd, nbmax);  // (each row is zeroed by the scatter kernel)
  std::vector<double> evh(nsd);
  std::vector<int> infoh(NB);
  if (nsd > 0) RMC_HIP(hipMemcpyAsync(evh.data(), evsel, nsd * sizeof(double), hipMemcpyDeviceToHost, s));
  RMC_HIP(hipMemcpyAsync(infoh.data(), info, NB * sizeof(int), hipMemcpyDeviceToHost, s));
  sync(ctx);
  for (size_t t = 0; t < ls.size(); ++t) {
    const int i = sel[t];
    int sweeps = 0;
    bool ok = true;
    for (int b = range[i].first; b < range[i].second; ++b) {
      sweeps += std::abs(infoh[b]);
      ok = ok && infoh[b] >= 0;
    }
    evals[i].assign(evh.begin() + evo[i], evh.begin() + evo[i] + ls[t].ne);
    st[i] = SolveStats();
    st[i].rr_sweeps = sweeps;
    st[i].status = ok ? RMC_OK : RMC_ERR_NOCONV;
  }
}

// Lowest eigenpairs of several dense leaves in one batched solve; builds a module
// per leaf unless q_only > 0 (then only the lowest q_only eigenvalues).
std::vector<rmc_module*> leaf_solve_batch(rmc_ctx* ctx, const std::vector<const rmc_leaf_desc*>& leaves,
                                          const std::vector<int>& ks, const std::vector<int>& q_only,
                                          const rmc_solve_opts& o,
                                          std::vector<std::vector<double>>& evals,
                                          std::vector<rmc_level_report>* reps) {
  double t0 = now_ms();
  const int P = (int)leaves.size();
  Scratch sc(&ctx->arena);
  std::vector<CoupledOp> ops(P);
  std::vector<const CoupledOp*> opp(P);
  std::vector<int> nevs(P), kreq(P);
  std::vector<double*> Xs(P);
  double* bmax = sc.get<double>(std::max(P, 1));
  // term lists of every leaf in one table, one upload, four launches
  std::vector<DevTerm> terms;
  std::vector<size_t> toff(P);
  for (int i = 0; i < P; ++i) {
    toff[i] = terms.size();
    for (int t = 0; t < leaves[i]->n_terms; ++t) {
      const rmc_term& tm = leaves[i]->terms[t];
      DevTerm d{};
      d.coef = tm.coef;
      d.nsite = tm.nsite;
      for (int u = 0; u < tm.nsite; ++u) {
        d.bit[u] = leaves[i]->n_sites - 1 - tm.site[u];
        d.op[u] = tm.op[u];
      }
      terms.push_back(d);
    }
  }
  DevTerm* terms_dev = sc.get<DevTerm>(std::max<size_t>(terms.size(), 1));
  std::vector<LeafSetDesc> ld(P);
  int ns_max = 0;
  for (int i = 0; i < P; ++i) {
    const int D = 1 << leaves[i]->n_sites;
    CoupledOp& op = ops[i];
    op.kind = 0;
    op.n = D;
    double* H = sc.get<double>((size_t)D * D);
    op.H = H;
    op.D = sc.get<double>(D);
    ld[i] = LeafSetDesc{leaves[i]->n_sites, leaves[i]->n_terms, terms_dev + toff[i], H, op.D,
                        sc.get<double>(D), bmax + i};
    ns_max = std::max(ns_max, leaves[i]->n_sites);
    kreq[i] = std::min(ks[i], D);
    nevs[i] = q_only[i] > 0 ? std::min(q_only[i], D) : std::min(D, kreq[i] + 1);
    Xs[i] = sc.get<double>((size_t)nevs[i] * D);
    opp[i] = &ops[i];
  }
  LeafSetDesc* ld_dev = sc.get<LeafSetDesc>(P);
  if (!terms.empty())
    RMC_HIP(hipMemcpyAsync(terms_dev, terms.data(), terms.size() * sizeof(DevTerm),
                           hipMemcpyHostToDevice, ctx->stream));
  RMC_HIP(hipMemcpyAsync(ld_dev, ld.data(), P * sizeof(LeafSetDesc), hipMemcpyHostToDevice, ctx->stream));
  leaf_setup_batched(ctx->stream, ld_dev, P, ns_max);
  std::vector<double> bh(P);
  RMC_HIP(hipMemcpyAsync(bh.data(), bmax, P * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  sync(ctx);
  for (int i = 0; i < P; ++i) ops[i].bup = bh[i];
  rmc_solve_opts oo = o;
  oo.precision = RMC_FP64;
  // block-diagonal leaves: blockwise Jacobi; the others: the batched block solver
  // (RMC_LEAF_BLOCKS=0 sends every leaf to the iterative solver)
  std::vector<int> blk, itr;
  {
    const char* e = getenv("RMC_LEAF_BLOCKS");
    const bool on = !(e && atoi(e) == 0);
    for (int i = 0; i < P; ++i) (on && leaf_blocks(leaves[i]).usable ? blk : itr).push_back(i);
  }
  std::vector<SolveStats> st(P);
  evals.assign(P, {});
  if (!itr.empty()) {
    std::vector<const CoupledOp*> so;
    std::vector<int> sn;
    std::vector<double*> sx;
    for (int i : itr) {
      so.push_back(opp[i]);
      sn.push_back(nevs[i]);
      sx.push_back(Xs[i]);
    }
    std::vector<std::vector<double>> se;
    std::vector<SolveStats> ss;
    eig_lowest_batch(ctx, so, sn, oo, sx, se, ss);
    for (size_t t = 0; t < itr.size(); ++t) {
      evals[itr[t]] = se[t];
      st[itr[t]] = ss[t];
    }
  }
  if (!blk.empty()) leaf_blocks_solve(ctx, sc, leaves, blk, ops, nevs, Xs, evals, st);
  const double dt = now_ms() - t0;
  if (reps) {
    reps->assign(P, rmc_level_report{});
    for (int i = 0; i < P; ++i) {
      auto& r = (*reps)[i];
      r.iters = st[i].iters;
      r.matvecs = st[i].matvecs;
      r.rr_sweeps = st[i].rr_sweeps;
      r.max_res = st[i].max_res;
      r.k_req = kreq[i];
      r.gap = INFINITY;
      r.ms = dt;
      r.width = leaves[i]->n_sites;
    }
  }
  for (int i = 0; i < P; ++i)
    if (st[i].status != RMC_OK)
      throw Error((rmc_status)st[i].status,
                  "leaf eigensolver did not converge (dim=" + std::to_string(ops[i].n) +
                      ", iters=" + std::to_string(st[i].iters) +
                      ", max_res=" + std::to_string(st[i].max_res) + ")");
  std::vector<rmc_module*> out(P, nullptr);
  try {
    std::vector<double> e_all;
    std::vector<VecDesc> copies;
    std::vector<size_t> e_off;
    long cmax = 0;
    for (int i = 0; i < P; ++i) {
      if (q_only[i] > 0) continue;
      const int D = ops[i].n;
      double gap = INFINITY;
      int k_eff = gap_cut(evals[i], kreq[i], o.gap_tol > 0 ? o.gap_tol : 1e-6, &gap);
      rmc_module* m = new rmc_module();
      m->kind = 0;
      m->n_sites = leaves[i]->n_sites;
      m->dim = D;
      m->k_eff = k_eff;
      m->gap = gap;
      m->E_host.assign(evals[i].begin(), evals[i].begin() + k_eff);
      ctx->modules.insert(m);
      out[i] = m;
      m->E = (double*)ctx->arena.alloc(k_eff * sizeof(double));
      m->basis = (double*)ctx->arena.alloc((size_t)k_eff * D * sizeof(double));
      e_off.push_back(e_all.size());
      e_all.insert(e_all.end(), m->E_host.begin(), m->E_host.end());
      VecDesc v{};
      v.nv = k_eff; v.n = D; v.out = m->basis; v.P = Xs[i];
      copies.push_back(v);
      VecDesc ve{};
      ve.nv = 1; ve.n = k_eff; ve.out = m->E;
      copies.push_back(ve);
      cmax = std::max(cmax, (long)k_eff * D);
      if (reps) {
        (*reps)[i].k_eff = k_eff;
        (*reps)[i].gap = gap;
      }
    }
    if (!copies.empty()) {
      double* e_dev = sc.get<double>(std::max<size_t>(e_all.size(), 1));
      for (size_t t = 0; t < e_off.size(); ++t) copies[2 * t + 1].P = e_dev + e_off[t];
      VecDesc* cd = sc.get<VecDesc>(copies.size());
      RMC_HIP(hipMemcpyAsync(e_dev, e_all.data(), e_all.size() * sizeof(double), hipMemcpyHostToDevice,
                             ctx->stream));
      RMC_HIP(hipMemcpyAsync(cd, copies.data(), copies.size() * sizeof(VecDesc), hipMemcpyHostToDevice,
                             ctx->stream));
      vec_batched(ctx->stream, VEC_COPY, cd, (int)copies.size(), 1, cmax);
    }
    sync(ctx);
  } catch (...) {
    for (rmc_module* m : out)
      if (m) {
        ctx->modules.erase(m);
        free_module_mem(ctx, m);
        delete m;
      }
    throw;
  }
  return out;
}

rmc_module* leaf_solve(rmc_ctx* ctx, const rmc_leaf_desc* leaf, int k, int q_only,
                       const rmc_solve_opts& o, std::vector<double>& evals, rmc_level_report* rep) {
  std::vector<std::vector<double>> ev;
  std::vector<rmc_level_report> reps;
  auto m = leaf_solve_batch(ctx, {leaf}, {k}, {q_only}, o, ev, rep ? &reps : nullptr);
  evals = ev[0];
  if (rep) *rep = reps[0];
  return m[0];
}

int find_op(const rmc_module* m, int site, int op) {
  for (size_t i = 0; i < m->ops.size(); ++i)
    if (m->ops[i].site == site && m->ops[i].op == op) return (int)i;
  return -1;
}

// Projected operator of (site, op) on module m; returns its id (index in m->ops).
int project_op(rmc_ctx* ctx, rmc_module* m, int site, int op) {
  int id = find_op(m, site, op);
  if (id >= 0) return id;
  RMC_CHECK(site >= 0 && site < m->n_sites, RMC_ERR_ARG, "operator site outside the module");
  RMC_CHECK(op >= RMC_OP_X && op <= RMC_OP_Z, RMC_ERR_ARG, "unknown operator");
  RMC_CHECK(m->basis != nullptr, RMC_ERR_STATE, "module basis already freed");
  hipStream_t s = ctx->stream;
  const int k = m->k_eff, n = m->dim;
  double* o = (double*)ctx->arena.alloc((size_t)k * k * sizeof(double));
  try {
    Scratch sc(&ctx->arena);
    double* W = sc.get<double>((size_t)k * n);
    if (m->kind == 0) {
      // W_j = O v_j, o = V W^T
      site_op_apply(s, k, m->n_sites, m->n_sites - 1 - site, op, m->basis, W);
    } else {
      const int kA = m->kA, kB = m->kB;
      if (site < m->A->n_sites) {
        int ida = project_op(ctx, m->A, site, op);
        const double* oA = m->A->ops[ida].data;
        // Z_nu = o_A C_nu (kA x kA times kA x kB), batched over nu
        gemm_f64(s, false, false, kA, kB, kA, 1.0, oA, kA, 0, m->basis, kB, n, 0.0, W, kB, n, k, 1,
                 nullptr);
      } else {
        int idb = project_op(ctx, m->B, site - m->A->n_sites, op);
        const double* oB = m->B->ops[idb].data;
        // Z_nu = C_nu o_B^T
        gemm_f64(s, false, true, kA, kB, kB, 1.0, m->basis, kB, n, oB, kB, 0, 0.0, W, kB, n, k, 1,
                 nullptr);
      }
    }
    double* kw = sc.get<double>((size_t)64 * k * k + 64);
    gemm_f64(s, false, true, k, k, n, 1.0, m->basis, n, 0, W, n, 0, 0.0, o, k, 0, 1,
             gemm_pick_ksplit(k, k, n, 1), kw);
    // no host sync: scratch released here is reused only by later work on the same
    // stream, which runs after these kernels
  } catch (...) {
    ctx->arena.release(o);
    throw;
  }
  m->ops.push_back({site, op, o});
  return (int)m->ops.size() - 1;
}

// Many projections at once (the operators every new module of a level needs): the
// same products as project_op, as one grouped GEMM for the operator applications,
// one grouped split-K GEMM for the basis contractions and one reduction. For a
// merged module, an operator of the A side acts on the rows of each k_A x k_B
// coefficient block, so the blocks are transposed first: then both sides are one
// plain (k k_X) x k_X product, Ct_v o_A^T or C_v o_B^T, and the contraction uses
// the matching (transposed or not) basis.
struct ProjReq {
  rmc_module* m;
  int site, op;
};

void project_ops_batch(rmc_ctx* ctx, const std::vector<ProjReq>& in) {
  std::vector<ProjReq> reqs;
  std::set<std::tuple<rmc_module*, int, int>> seen;
  for (const ProjReq& r : in) {
    if (find_op(r.m, r.site, r.op) >= 0 || !seen.insert({r.m, r.site, r.op}).second) continue;
    RMC_CHECK(r.site >= 0 && r.site < r.m->n_sites, RMC_ERR_ARG, "operator site outside the module");
    RMC_CHECK(r.op >= RMC_OP_X && r.op <= RMC_OP_Z, RMC_ERR_ARG, "unknown operator");
    RMC_CHECK(r.m->basis != nullptr, RMC_ERR_STATE, "module basis already freed");
    reqs.push_back(r);
  }
  if (reqs.empty()) return;
  if (reqs.size() == 1) {
    project_op(ctx, reqs[0].m, reqs[0].site, reqs[0].op);
    return;
  }
  hipStream_t s = ctx->stream;
  const int R = (int)reqs.size();
  std::vector<double*> outs(R, nullptr);
  try {
    Scratch sc(&ctx->arena);
    // child operators (present unless a caller skipped them) and transposed bases
    std::vector<const double*> child(R, nullptr);
    std::vector<char> aside(R, 0);
    std::map<rmc_module*, double*> ct;
    for (int i = 0; i < R; ++i) {
      rmc_module* m = reqs[i].m;
      if (m->kind == 0) continue;
      aside[i] = reqs[i].site < m->A->n_sites;
      if (aside[i]) {
        child[i] = m->A->ops[project_op(ctx, m->A, reqs[i].site, reqs[i].op)].data;
        if (!ct.count(m)) ct[m] = sc.get<double>((size_t)m->k_eff * m->dim);
      } else {
        child[i] = m->B->ops[project_op(ctx, m->B, reqs[i].site - m->A->n_sites, reqs[i].op)].data;
      }
    }
    std::vector<TrDesc> td;
    int tk = 0, tn = 0;
    for (auto& kv : ct) {
      rmc_module* m = kv.first;
      td.push_back(TrDesc{m->k_eff, m->kA, m->kB, 0, m->basis, kv.second});
      tk = std::max(tk, m->k_eff);
      tn = std::max(tn, m->dim);
    }
    std::vector<double*> W(R);
    std::vector<SiteOpDesc> so;
    long so_max = 0;
    std::vector<GemmDesc> g1, g2;
    std::vector<VecDesc> red;
    int M1 = 0, N1 = 0, M2 = 0;
    long kwmax = 0;
    int KS = 1;
    for (int i = 0; i < R; ++i) {
      rmc_module* m = reqs[i].m;
      const int k = m->k_eff, n = m->dim;
      W[i] = sc.get<double>((size_t)k * n);
      KS = std::max(KS, gemm_pick_ksplit(k, k, n, R));
    }
    for (int i = 0; i < R; ++i) {
      rmc_module* m = reqs[i].m;
      const int k = m->k_eff, n = m->dim;
      const double* basis = aside[i] ? ct[m] : m->basis;
      if (m->kind == 0) {
        so.push_back(SiteOpDesc{k, m->n_sites, m->n_sites - 1 - reqs[i].site, reqs[i].op, m->basis, W[i]});
        so_max = std::max(so_max, (long)k * n);
      } else {
        const int kx = aside[i] ? m->kA : m->kB, ky = aside[i] ? m->kB : m->kA;
        GemmDesc d{};
        d.M = k * ky; d.N = kx; d.K = kx;
        d.A = basis; d.lda = kx;
        d.B = child[i]; d.ldb = kx;
        d.C = W[i]; d.ldc = kx;
        d.alpha = 1.0; d.beta = 0.0; d.work = nullptr;
        g1.push_back(d);
        M1 = std::max(M1, d.M);
        N1 = std::max(N1, d.N);
      }
      outs[i] = (double*)ctx->arena.alloc((size_t)k * k * sizeof(double));
      double* kw = sc.get<double>((size_t)KS * k * k);
      GemmDesc d{};
      d.M = k; d.N = k; d.K = n;
      d.A = basis; d.lda = n;
      d.B = W[i]; d.ldb = n;
      d.alpha = 1.0; d.beta = 0.0; d.work = kw;
      g2.push_back(d);
      M2 = std::max(M2, k);
      VecDesc v{};
      v.nv = KS; v.n = k * k; v.out = outs[i]; v.P = kw;
      red.push_back(v);
      kwmax = std::max(kwmax, (long)k * k);
    }
    auto upload = [&](auto& vec) {
      typedef typename std::decay<decltype(vec)>::type::value_type T;
      T* dptr = sc.get<T>(std::max<size_t>(vec.size(), 1));
      if (!vec.empty())
        RMC_HIP(hipMemcpyAsync(dptr, vec.data(), vec.size() * sizeof(T), hipMemcpyHostToDevice, s));
      return dptr;
    };
    const TrDesc* tdd = upload(td);
    const SiteOpDesc* sod = upload(so);
    const GemmDesc* g1d = upload(g1);
    const GemmDesc* g2d = upload(g2);
    const VecDesc* rd = upload(red);
    transpose_blocks_batched(s, tdd, (int)td.size(), tk, tn);
    site_op_batched(s, sod, (int)so.size(), so_max);
    gemm_batched(s, false, true, g1d, (int)g1.size(), M1, N1, 1);
    gemm_batched(s, false, true, g2d, R, M2, M2, KS);
    vec_batched(s, VEC_REDUCE, rd, R, KS, kwmax);
    // the host descriptor tables must outlive their uploads
    sync(ctx);
  } catch (...) {
    for (double* o : outs)
      if (o) ctx->arena.release(o);
    throw;
  }
  for (int i = 0; i < R; ++i) reqs[i].m->ops.push_back({reqs[i].site, reqs[i].op, outs[i]});
}

struct CoupleReq {
  rmc_module* A;
  rmc_module* B;
  const rmc_bond_desc* bond;
  bool want_module;
  int k_keep, q;
};

// Several coupling steps (one per request) in one batched solve. k_keep: states
// kept in new modules (gap rule); q: energies returned.
std::vector<rmc_module*> couple_batch(rmc_ctx* ctx, const std::vector<CoupleReq>& reqs,
                                      const rmc_solve_opts& o,
                                      std::vector<std::vector<double>>& evals,
                                      std::vector<rmc_level_report>* reps) {
  double t0 = now_ms();
  const int P = (int)reqs.size();
  hipStream_t s = ctx->stream;
  Scratch sc(&ctx->arena);
  std::unique_ptr<HostScope> phase(new HostScope("couple.setup"));
  std::vector<CoupledOp> ops(P);
  std::vector<const CoupledOp*> opp(P);
  std::vector<int> nevs(P), kreq(P);
  std::vector<double*> Xs(P);
  // one batched set-up launch for every problem's operators (tables below)
  std::vector<OpSetDesc> setup(P);
  std::vector<double> coef_all;
  std::vector<const double*> ptr_all;
  std::vector<size_t> coef_off(P), ptr_off(P);
  long work_max = 0;
  for (int p = 0; p < P; ++p) {
    const CoupleReq& rq = reqs[p];
    rmc_module* A = rq.A;
    rmc_module* B = rq.B;
    const rmc_bond_desc* bond = rq.bond;
    const int k_keep = rq.k_keep, q = rq.q;
    RMC_CHECK(A && B && bond, RMC_ERR_ARG, "null argument");
    RMC_CHECK(A->E && B->E, RMC_ERR_STATE, "module freed");
    const int T = bond->n_terms;
    RMC_CHECK(T >= 0 && (T == 0 || (bond->coef && bond->opA && bond->opB)), RMC_ERR_ARG, "bad bond");
    const int kA = A->k_eff, kB = B->k_eff, n = kA * kB;
    RMC_CHECK(kA <= kron_max_k() && kB <= kron_max_k(), RMC_ERR_ARG, "module dimension above 192");
    if (rq.want_module) RMC_CHECK(k_keep >= 1 && q <= k_keep, RMC_ERR_ARG, "need 1 <= q <= k_keep");
    RMC_CHECK(q >= 1, RMC_ERR_ARG, "q must be >= 1");
    for (int i = 0; i < T; ++i) {
      RMC_CHECK(bond->opA[i] >= 0 && bond->opA[i] < (int)A->ops.size(), RMC_ERR_ARG, "bad opA id");
      RMC_CHECK(bond->opB[i] >= 0 && bond->opB[i] < (int)B->ops.size(), RMC_ERR_ARG, "bad opB id");
      RMC_CHECK(std::isfinite(bond->coef[i]), RMC_ERR_ARG, "non-finite coupling coefficient");
    }
    CoupledOp& op = ops[p];
    op.kind = 1;
    op.n = n;
    op.kA = kA;
    op.kB = kB;
    op.T = T;
    op.EA = A->E;
    op.EB = B->E;
    op.coef.assign(bond->coef, bond->coef + T);
    op.OAcat = sc.get<double>((size_t)std::max(T, 1) * kA * kA);
    op.OBcat = sc.get<double>((size_t)std::max(T, 1) * kB * kB);
    op.Ediag = sc.get<double>(n);
    op.D = sc.get<double>(n);
    op.pkm = kron_pack_km(kA, kB);
    for (int pr = 0; pr < 3; ++pr) {
      const size_t b = kron_pack_bytes(pr, kA, kB, T);
      op.pack[pr] = b ? static_cast<void*>(sc.get<char>(b)) : nullptr;
    }
    double csum = 0.0;
    coef_off[p] = coef_all.size();
    ptr_off[p] = ptr_all.size();
    for (int i = 0; i < T; ++i) {
      coef_all.push_back(bond->coef[i]);
      csum += std::fabs(bond->coef[i]);
    }
    for (int i = 0; i < T; ++i) ptr_all.push_back(A->ops[bond->opA[i]].data);
    for (int i = 0; i < T; ++i) ptr_all.push_back(B->ops[bond->opB[i]].data);
    OpSetDesc& sd = setup[p];
    sd.T = T; sd.kA = kA; sd.kB = kB; sd.pkm = op.pkm;
    sd.EA = A->E; sd.EB = B->E;
    sd.OAcat = op.OAcat; sd.OBcat = op.OBcat; sd.D = op.D; sd.Ediag = op.Ediag;
    sd.p64 = static_cast<double*>(op.pack[0]);
    sd.p32 = static_cast<float*>(op.pack[1]);
    sd.p16 = op.pack[2];
    const bool pk = op.pack[0] || op.pack[1] || op.pack[2];
    work_max = std::max(work_max, (long)T * (kA * kA + kB * kB) + n +
                                      (pk ? 2L * T * op.pkm * op.pkm : 0L));
    // upper end of H_eff: the largest kept energies plus the coupling's largest
    // eigenvalue, bounded by that of the unprojected coupling and by sum |c_i|
    // (projected one-site operators have spectral norm <= 1)
    const double emax = A->E_host.back() + B->E_host.back();
    const double ctop = T > 0 ? std::min(csum, coupling_top(A, B, bond)) : 0.0;
    op.bup = emax + ctop + 1e-12 * (std::fabs(emax) + csum + 1.0);
    op.precision = o.precision;
    kreq[p] = std::min(k_keep, n);
    int nev = rq.want_module ? std::min(n, kreq[p] + 1) : std::min(q, n);
    nevs[p] = std::max(nev, std::min(q, n));
    Xs[p] = sc.get<double>((size_t)nevs[p] * n);
    opp[p] = &ops[p];
  }
  {
    double* coef_dev = sc.get<double>(std::max<size_t>(coef_all.size(), 1));
    const double** ptr_dev = sc.get<const double*>(std::max<size_t>(ptr_all.size(), 1));
    OpSetDesc* sd_dev = sc.get<OpSetDesc>(P);
    for (int p = 0; p < P; ++p) {
      ops[p].coef_dev = coef_dev + coef_off[p];
      setup[p].coef = ops[p].coef_dev;
      setup[p].opa = ptr_dev + ptr_off[p];
      setup[p].opb = ptr_dev + ptr_off[p] + ops[p].T;
    }
    // pageable sources: the copies are staged before the calls return
    if (!coef_all.empty())
      RMC_HIP(hipMemcpyAsync(coef_dev, coef_all.data(), coef_all.size() * sizeof(double),
                             hipMemcpyHostToDevice, s));
    if (!ptr_all.empty())
      RMC_HIP(hipMemcpyAsync(ptr_dev, ptr_all.data(), ptr_all.size() * sizeof(double*),
                             hipMemcpyHostToDevice, s));
    RMC_HIP(hipMemcpyAsync(sd_dev, setup.data(), P * sizeof(OpSetDesc), hipMemcpyHostToDevice, s));
    op_setup_batched(s, sd_dev, P, work_max);
  }
  std::vector<SolveStats> st;
  phase.reset(new HostScope("couple.solve"));
  eig_lowest_batch(ctx, opp, nevs, o, Xs, evals, st);
  phase.reset(new HostScope("couple.modules"));
  const double dt = now_ms() - t0;
  if (reps) {
    reps->assign(P, rmc_level_report{});
    for (int p = 0; p < P; ++p) {
      auto& r = (*reps)[p];
      r.iters = st[p].iters;
      r.matvecs = st[p].matvecs;
      r.rr_sweeps = st[p].rr_sweeps;
      r.max_res = st[p].max_res;
      r.k_req = kreq[p];
      r.gap = INFINITY;
      r.ms = dt;
      r.kind = reqs[p].want_module ? 1 : 2;
      r.width = reqs[p].A->n_sites + reqs[p].B->n_sites;
    }
  }
  for (int p = 0; p < P; ++p)
    if (st[p].status != RMC_OK)
      throw Error((rmc_status)st[p].status,
                  "coupled eigensolver did not converge (n=" + std::to_string(ops[p].n) +
                      ", nev=" + std::to_string(nevs[p]) + ", iters=" + std::to_string(st[p].iters) +
                      ", max_res=" + std::to_string(st[p].max_res) + ")");
  std::vector<rmc_module*> out(P, nullptr);
  try {
    std::vector<double> e_all;
    std::vector<VecDesc> copies;
    std::vector<size_t> e_off;
    long cmax = 0;
    for (int p = 0; p < P; ++p) {
      if (!reqs[p].want_module) continue;
      const int n = ops[p].n;
      double gap = INFINITY;
      int k_eff = gap_cut(evals[p], kreq[p], o.gap_tol > 0 ? o.gap_tol : 1e-6, &gap);
      rmc_module* m = new rmc_module();
      m->kind = 1;
      m->n_sites = reqs[p].A->n_sites + reqs[p].B->n_sites;
      m->dim = n;
      m->k_eff = k_eff;
      m->kA = ops[p].kA;
      m->kB = ops[p].kB;
      m->A = reqs[p].A;
      m->B = reqs[p].B;
      m->gap = gap;
      m->E_host.assign(evals[p].begin(), evals[p].begin() + k_eff);
      ctx->modules.insert(m);
      out[p] = m;
      m->E = (double*)ctx->arena.alloc(k_eff * sizeof(double));
      m->basis = (double*)ctx->arena.alloc((size_t)k_eff * n * sizeof(double));
      e_off.push_back(e_all.size());
      e_all.insert(e_all.end(), m->E_host.begin(), m->E_host.end());
      VecDesc v{};
      v.nv = k_eff; v.n = n; v.out = m->basis; v.P = Xs[p];
      copies.push_back(v);
      VecDesc ve{};
      ve.nv = 1; ve.n = k_eff; ve.out = m->E; ve.P = nullptr;  // source set after staging
      copies.push_back(ve);
      cmax = std::max(cmax, (long)k_eff * n);
      if (reps) {
        (*reps)[p].k_eff = k_eff;
        (*reps)[p].gap = gap;
      }
    }
    if (!copies.empty()) {
      // every new module's basis and energies in one copy launch
      double* e_dev = sc.get<double>(std::max<size_t>(e_all.size(), 1));
      for (size_t i = 0; i < e_off.size(); ++i) copies[2 * i + 1].P = e_dev + e_off[i];
      VecDesc* cd = sc.get<VecDesc>(copies.size());
      RMC_HIP(hipMemcpyAsync(e_dev, e_all.data(), e_all.size() * sizeof(double), hipMemcpyHostToDevice, s));
      RMC_HIP(hipMemcpyAsync(cd, copies.data(), copies.size() * sizeof(VecDesc), hipMemcpyHostToDevice, s));
      vec_batched(s, VEC_COPY, cd, (int)copies.size(), 1, cmax);
    }
    sync(ctx);
  } catch (...) {
    for (rmc_module* m : out)
      if (m) {
        ctx->modules.erase(m);
        free_module_mem(ctx, m);
        delete m;
      }
    throw;
  }
  return out;
}

// One coupling step; out module optional.
rmc_module* couple(rmc_ctx* ctx, rmc_module* A, rmc_module* B, const rmc_bond_desc* bond,
                   int k_keep, int q, const rmc_solve_opts& o, bool want_module,
                   std::vector<double>& evals, rmc_level_report* rep) {
  std::vector<std::vector<double>> ev;
  std::vector<rmc_level_report> reps;
  auto m = couple_batch(ctx, {CoupleReq{A, B, bond, want_module, k_keep, q}}, o, ev,
                        rep ? &reps : nullptr);
  evals = ev[0];
  if (rep) *rep = reps[0];
  return m[0];
}

}  // namespace

namespace rmc {
void linalg_set_attrs();
void kron_set_attrs();

rmc_module* api_leaf_solve(rmc_ctx* ctx, const rmc_leaf_desc* leaf, int k, int q_only,
                           const rmc_solve_opts& o, std::vector<double>& evals, rmc_level_report* rep) {
  return leaf_solve(ctx, leaf, k, q_only, o, evals, rep);
}
int api_project_op(rmc_ctx* ctx, rmc_module* m, int site, int op) {
  return project_op(ctx, m, site, op);
}
void api_project_ops_batch(rmc_ctx* ctx, const std::vector<rmc_module*>& ms,
                           const std::vector<std::pair<int, int>>& so) {
  RMC_HOST_SCOPE("project.batch");
  std::vector<ProjReq> r;
  for (size_t i = 0; i < ms.size(); ++i) r.push_back(ProjReq{ms[i], so[i].first, so[i].second});
  project_ops_batch(ctx, r);
}
rmc_module* api_couple(rmc_ctx* ctx, rmc_module* A, rmc_module* B, const rmc_bond_desc* bond,
                       int k_keep, int q, const rmc_solve_opts& o, bool want_module,
                       std::vector<double>& evals, rmc_level_report* rep) {
  return couple(ctx, A, B, bond, k_keep, q, o, want_module, evals, rep);
}
std::vector<rmc_module*> api_leaf_solve_batch(rmc_ctx* ctx,
                                              const std::vector<const rmc_leaf_desc*>& leaves,
                                              const std::vector<int>& ks,
                                              const std::vector<int>& q_only,
                                              const rmc_solve_opts& o,
                                              std::vector<std::vector<double>>& evals,
                                              std::vector<rmc_level_report>* reps) {
  RMC_HOST_SCOPE("leaf.solve_batch");
  return leaf_solve_batch(ctx, leaves, ks, q_only, o, evals, reps);
}
std::vector<rmc_module*> api_couple_batch(rmc_ctx* ctx, const std::vector<rmc_module*>& As,
                                          const std::vector<rmc_module*>& Bs,
                                          const std::vector<const rmc_bond_desc*>& bonds,
                                          const std::vector<char>& want,
                                          const std::vector<int>& k_keep, const std::vector<int>& q,
                                          const rmc_solve_opts& o,
                                          std::vector<std::vector<double>>& evals,
                                          std::vector<rmc_level_report>* reps) {
  std::vector<CoupleReq> rq;
  for (size_t i = 0; i < As.size(); ++i)
    rq.push_back(CoupleReq{As[i], Bs[i], bonds[i], want[i] != 0, k_keep[i], q[i]});
  return couple_batch(ctx, rq, o, evals, reps);
}
size_t api_arena_free(rmc_ctx* ctx) { return ctx->arena.size() - ctx->arena.in_use(); }
void api_release_basis(rmc_ctx* ctx, rmc_module* m) {
  ctx->arena.release(m->basis);
  m->basis = nullptr;
}
void api_free_module(rmc_ctx* ctx, rmc_module* m) {
  RMC_HOST_SCOPE("module.free");
  ctx->modules.erase(m);
  free_module_mem(ctx, m);
  delete m;
}
}  // namespace rmc

// ---------------------------------------------------------------------------
// Scratch of the entry point that allocates nothing (rmc_kron_apply_noalloc): one
// fixed array per GPU, held until the process ends. Host code never uses its name as
// an address: rmc_create looks up each device's copy once (hipGetSymbolAddress, with
// that device current) and every launch and copy uses that address.
// ---------------------------------------------------------------------------
static constexpr size_t kNoAllocScratchBytes = (size_t)4 << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {
std::mutex scratch_mu;
std::map<int, char*> scratch_dev;  // device -> its copy of `scratch`

void scratch_setup(int device) {  // `device` must be current
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (scratch_dev.count(device)) return;
  void* p = nullptr;
  RMC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  RMC_CHECK(p != nullptr && ((uintptr_t)p & 255) == 0, RMC_ERR_HIP, "scratch array address");
  scratch_dev[device] = static_cast<char*>(p);
}

char* scratch_of(int device) {
  std::lock_guard<std::mutex> lk(scratch_mu);
  auto it = scratch_dev.find(device);
  return it == scratch_dev.end() ? nullptr : it->second;
}
}  // namespace

static void set_kernel_attrs() {
  static bool done = false;
  if (done) return;
  rmc::linalg_set_attrs();
  rmc::kron_set_attrs();
  done = true;
}

// ---------------------------------------------------------------------------
// ABI
// ---------------------------------------------------------------------------
extern "C" {

void rmc_default_opts(rmc_solve_opts* o) {
  if (!o) return;
  o->precision = RMC_FP64;
  o->tol = 1e-13;
  o->gap_tol = 1e-6;
  o->max_iter = 200;
  o->guard = 0;
  o->max_degree = 0;
  o->seed = 0x2609023940ull;
}

rmc_status rmc_create(rmc_ctx** out, int device, void* arena_dev, size_t arena_bytes,
                      void* hip_stream) {
  if (!out) return RMC_ERR_ARG;
  rmc_ctx* ctx = new rmc_ctx();
  rmc_status st = guard(ctx, [&] {
    RMC_HIP(hipSetDevice(device));
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    RMC_CHECK(arena_bytes >= (1u << 20), RMC_ERR_ARG, "arena must be at least 1 MiB");
    if (arena_dev) {
      ctx->arena_mem = arena_dev;
      ctx->own_arena = false;
    } else {
      RMC_HIP(hipMalloc(&ctx->arena_mem, arena_bytes));
      ctx->own_arena = true;
    }
    RMC_CHECK(((uintptr_t)ctx->arena_mem & 255) == 0, RMC_ERR_ARG, "arena must be 256-byte aligned");
    ctx->arena.init((char*)ctx->arena_mem, arena_bytes);
    set_kernel_attrs();
    scratch_setup(device);
  });
  if (st != RMC_OK) {
    fprintf(stderr, "rmc_create: %s\n", ctx->last_error.c_str());
    if (ctx->own_arena && ctx->arena_mem) hipFree(ctx->arena_mem);
    delete ctx;
    return st;
  }
  *out = ctx;
  return RMC_OK;
}

rmc_status rmc_serve_stop(rmc_ctx* ctx);

rmc_status rmc_destroy(rmc_ctx* ctx) {
  if (!ctx) return RMC_ERR_ARG;
  if (ctx->serving) rmc_serve_stop(ctx);
  hipStreamSynchronize(ctx->stream);
  for (rmc_module* m : ctx->modules) delete m;
  ctx->modules.clear();
  for (auto& r : ctx->prof_recs) {
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  for (hipEvent_t e : ctx->ev_pool) hipEventDestroy(e);
  for (char* h : ctx->pinned)
    if (h) hipHostFree(h);
  for (hipStream_t ls : ctx->lane_stream)
    if (ls) {
      hipStreamSynchronize(ls);
      hipStreamDestroy(ls);
    }
  for (hipEvent_t e : ctx->lane_ev)
    if (e) hipEventDestroy(e);
  if (ctx->filter_ev) hipEventDestroy(ctx->filter_ev);
  if (ctx->own_arena && ctx->arena_mem) hipFree(ctx->arena_mem);
  delete ctx;
  return RMC_OK;
}

const char* rmc_last_error(const rmc_ctx* ctx) { return ctx ? ctx->last_error.c_str() : "null ctx"; }

rmc_status rmc_arena_usage(const rmc_ctx* ctx, size_t* in_use, size_t* peak) {
  if (!ctx) return RMC_ERR_ARG;
  if (in_use) *in_use = ctx->arena.in_use();
  if (peak) *peak = ctx->arena.peak();
  return RMC_OK;
}

rmc_status rmc_module_ed(rmc_ctx* ctx, const rmc_leaf_desc* leaf, int k, const rmc_solve_opts* opts,
                         rmc_module** out) {
  if (!ctx) return RMC_ERR_ARG;
  return guard(ctx, [&] {
    validate_leaf(leaf);
    RMC_CHECK(k >= 1, RMC_ERR_ARG, "k must be >= 1");
    RMC_CHECK(out != nullptr, RMC_ERR_ARG, "null output");
    rmc_solve_opts o;
    rmc_default_opts(&o);
    if (opts) o = *opts;
    std::vector<double> ev;
    *out = leaf_solve(ctx, leaf, k, 0, o, ev, nullptr);
  });
}

rmc_status rmc_project_ops(rmc_ctx* ctx, rmc_module* m, int n_ops, const int* site, const int* op,
                           int* op_ids) {
  if (!ctx) return RMC_ERR_ARG;
  return guard(ctx, [&] {
    RMC_CHECK(m && n_ops >= 0 && (n_ops == 0 || (site && op && op_ids)), RMC_ERR_ARG, "bad arguments");
    std::vector<int> ids(n_ops);
    for (int i = 0; i < n_ops; ++i) ids[i] = project_op(ctx, m, site[i], op[i]);
    for (int i = 0; i < n_ops; ++i) op_ids[i] = ids[i];
  });
}

rmc_status rmc_couple_solve(rmc_ctx* ctx, rmc_module* A, rmc_module* B, const rmc_bond_desc* bond,
                            int k_keep, int q, const rmc_solve_opts* opts, rmc_module** out,
                            double* energies, rmc_level_report* rep) {
  if (!ctx) return RMC_ERR_ARG;
  rmc_level_report r{};
  std::vector<double> ev;
  rmc_status st = guard(ctx, [&] {
    rmc_solve_opts o;
    rmc_default_opts(&o);
    if (opts) o = *opts;
    RMC_CHECK(o.precision >= RMC_FP64 && o.precision <= RMC_BF16, RMC_ERR_ARG, "bad precision");
    rmc_module* m = couple(ctx, A, B, bond, k_keep, q, o, out != nullptr, ev, &r);
    if (out) *out = m;
  });
  if ((st == RMC_OK || st == RMC_ERR_NOCONV) && energies && !ev.empty())
    for (int i = 0; i < q && i < (int)ev.size(); ++i) energies[i] = ev[i];
  r.kind = out ? 1 : 2;
  if (rep && (st == RMC_OK || st == RMC_ERR_NOCONV)) *rep = r;
  return st;
}

rmc_status rmc_module_info(const rmc_module* m, int* k_eff, int* dim, int* n_sites, double* energies) {
  if (!m) return RMC_ERR_ARG;
  if (k_eff) *k_eff = m->k_eff;
  if (dim) *dim = m->dim;
  if (n_sites) *n_sites = m->n_sites;
  if (energies) memcpy(energies, m->E_host.data(), m->E_host.size() * sizeof(double));
  return RMC_OK;
}

rmc_status rmc_module_basis(rmc_ctx* ctx, const rmc_module* m, double* basis_host) {
  if (!ctx || !m || !basis_host) return RMC_ERR_ARG;
  return guard(ctx, [&] {
    RMC_CHECK(m->basis != nullptr, RMC_ERR_STATE, "module basis freed");
    RMC_HIP(hipMemcpyAsync(basis_host, m->basis, (size_t)m->k_eff * m->dim * sizeof(double),
                           hipMemcpyDeviceToHost, ctx->stream));
    sync(ctx);
  });
}

namespace {
// Full-space vectors of a module's retained states (k_eff x 2^n_sites, row-major):
// a leaf's basis is already in the site basis; a merged module's state mu is
// sum_{a,b} C_mu[a][b] psi_A[a] (x) psi_B[b], i.e. psi_A^T C_mu psi_B as a
// 2^{n_A} x 2^{n_B} matrix (A holds the high bits). Two GEMMs per level: one for
// all mu (C psi_B), one strided batch over mu (psi_A^T T_mu).
void lift_module(rmc_ctx* ctx, const rmc_module* m, double* out) {
  RMC_CHECK(ctx->modules.count(const_cast<rmc_module*>(m)) != 0, RMC_ERR_STATE,
            "module (or a module below it) is not owned by this context");
  RMC_CHECK(m->basis != nullptr, RMC_ERR_STATE, "module basis freed");
  hipStream_t s = ctx->stream;
  const long D = 1L << m->n_sites;
  if (m->kind == 0) {
    RMC_CHECK(m->dim == D, RMC_ERR_STATE, "module basis not in the site basis");
    copy_rows(s, m->k_eff, m->dim, m->basis, m->dim, out, m->dim);
    return;
  }
  RMC_CHECK(m->A && m->B, RMC_ERR_STATE, "merged module without children");
  const rmc_module* A = m->A;
  const rmc_module* B = m->B;
  RMC_CHECK(A->k_eff == m->kA && B->k_eff == m->kB, RMC_ERR_STATE, "children changed");
  const int DA = 1 << A->n_sites, DB = 1 << B->n_sites;
  const int k = m->k_eff, kA = m->kA, kB = m->kB;
  Scratch sc(&ctx->arena);
  double* pa = sc.get<double>((size_t)kA * DA);
  double* pb = sc.get<double>((size_t)kB * DB);
  lift_module(ctx, A, pa);
  lift_module(ctx, B, pb);
  double* T = sc.get<double>((size_t)k * kA * DB);
  // T (k kA x DB) = C (k kA x kB) psi_B (kB x DB)
  gemm_f64(s, false, false, k * kA, DB, kB, 1.0, m->basis, kB, 0, pb, DB, 0, 0.0, T, DB, 0, 1, 1,
           nullptr);
  // out_mu (DA x DB) = psi_A^T (DA x kA) T_mu (kA x DB)
  gemm_f64(s, true, false, DA, DB, kA, 1.0, pa, DA, 0, T, DB, (long)kA * DB, 0.0, out, DB,
           (long)DA * DB, k, 1, nullptr);
  // scratch released here is reused only by work enqueued later on the same stream
}
}  // namespace

rmc_status rmc_module_lift(rmc_ctx* ctx, const rmc_module* m, double* out_dev) {
  if (!ctx || !m || !out_dev) return RMC_ERR_ARG;
  return guard(ctx, [&] {
    RMC_CHECK(m->n_sites >= 1 && m->n_sites <= 24, RMC_ERR_ARG, "lifting needs 1 <= n_sites <= 24");
    lift_module(ctx, m, out_dev);
    sync(ctx);
  });
}

rmc_status rmc_module_op(rmc_ctx* ctx, const rmc_module* m, int op_id, double* op_host) {
  if (!ctx || !m || !op_host) return RMC_ERR_ARG;
  return guard(ctx, [&] {
    RMC_CHECK(op_id >= 0 && op_id < (int)m->ops.size(), RMC_ERR_ARG, "bad op id");
    RMC_HIP(hipMemcpyAsync(op_host, m->ops[op_id].data, (size_t)m->k_eff * m->k_eff * sizeof(double),
                           hipMemcpyDeviceToHost, ctx->stream));
    sync(ctx);
  });
}

rmc_status rmc_module_free(rmc_ctx* ctx, rmc_module* m) {
  if (!ctx || !m) return RMC_ERR_ARG;
  return guard(ctx, [&] {
    hipStreamSynchronize(ctx->stream);
    auto it = ctx->modules.find(m);
    RMC_CHECK(it != ctx->modules.end(), RMC_ERR_ARG, "module not owned by this context");
    for (rmc_module* o : ctx->modules)
      if (o->A == m || o->B == m) {
        if (o->A == m) o->A = nullptr;
        if (o->B == m) o->B = nullptr;
      }
    free_module_mem(ctx, m);
    ctx->modules.erase(it);
    delete m;
  });
}

rmc_status rmc_module_import(rmc_ctx* ctx, int n_sites, int k, int dim, const double* E_host,
                             const double* basis_host, int n_ops, const int* sites, const int* ops,
                             const double* op_data, rmc_module** out) {
  if (!ctx) return RMC_ERR_ARG;
  return guard(ctx, [&] {
    RMC_CHECK(out && E_host && k >= 1 && dim >= k && n_sites >= 1 && n_ops >= 0, RMC_ERR_ARG,
              "bad import arguments");
    RMC_CHECK(n_ops == 0 || (sites && ops && op_data), RMC_ERR_ARG, "null operator arrays");
    for (int i = 1; i < k; ++i) RMC_CHECK(E_host[i] >= E_host[i - 1], RMC_ERR_ARG, "E not ascending");
    rmc_module* m = new rmc_module();
    m->kind = (n_sites <= 12 && dim == (1 << n_sites)) ? 0 : 1;
    m->n_sites = n_sites;
    m->dim = dim;
    m->k_eff = k;
    m->gap = INFINITY;
    m->E_host.assign(E_host, E_host + k);
    try {
      m->E = (double*)ctx->arena.alloc(k * sizeof(double));
      RMC_HIP(hipMemcpyAsync(m->E, E_host, k * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
      if (basis_host && m->kind == 0) {
        m->basis = (double*)ctx->arena.alloc((size_t)k * dim * sizeof(double));
        RMC_HIP(hipMemcpyAsync(m->basis, basis_host, (size_t)k * dim * sizeof(double),
                               hipMemcpyHostToDevice, ctx->stream));
      }
      for (int i = 0; i < n_ops; ++i) {
        RMC_CHECK(sites[i] >= 0 && sites[i] < n_sites, RMC_ERR_ARG, "operator site out of range");
        RMC_CHECK(ops[i] >= RMC_OP_X && ops[i] <= RMC_OP_Z, RMC_ERR_ARG, "unknown operator");
        double* o = (double*)ctx->arena.alloc((size_t)k * k * sizeof(double));
        m->ops.push_back({sites[i], ops[i], o});
        RMC_HIP(hipMemcpyAsync(o, op_data + (size_t)i * k * k, (size_t)k * k * sizeof(double),
                               hipMemcpyHostToDevice, ctx->stream));
      }
      sync(ctx);
    } catch (...) {
      free_module_mem(ctx, m);
      delete m;
      throw;
    }
    ctx->modules.insert(m);
    *out = m;
  });
}

rmc_status rmc_leaf_hamiltonian(rmc_ctx* ctx, const rmc_leaf_desc* leaf, double* H_dev) {
  if (!ctx) return RMC_ERR_ARG;
  return guard(ctx, [&] {
    validate_leaf(leaf);
    RMC_CHECK(H_dev != nullptr, RMC_ERR_ARG, "null output");
    assemble_leaf(ctx, leaf, H_dev);
  });
}

rmc_status rmc_kron_apply(rmc_ctx* ctx, rmc_module* A, rmc_module* B, const rmc_bond_desc* bond,
                          int precision, int n_vec, const double* X_dev, double* Y_dev) {
  if (!ctx) return RMC_ERR_ARG;
  return guard(ctx, [&] {
    RMC_CHECK(A && B && bond && X_dev && Y_dev && n_vec >= 0, RMC_ERR_ARG, "bad arguments");
    RMC_CHECK(precision >= RMC_FP64 && precision <= RMC_BF16, RMC_ERR_ARG, "bad precision");
    const int T = bond->n_terms, kA = A->k_eff, kB = B->k_eff, n = kA * kB;
    RMC_CHECK(kA <= kron_max_k() && kB <= kron_max_k(), RMC_ERR_ARG, "module dimension above 192");
    for (int i = 0; i < T; ++i) {
      RMC_CHECK(bond->opA[i] >= 0 && bond->opA[i] < (int)A->ops.size(), RMC_ERR_ARG, "bad opA id");
      RMC_CHECK(bond->opB[i] >= 0 && bond->opB[i] < (int)B->ops.size(), RMC_ERR_ARG, "bad opB id");
    }
    hipStream_t s = ctx->stream;
    Scratch sc(&ctx->arena);
    CoupledOp op;
    op.kind = 1;
    op.n = n;
    op.kA = kA;
    op.kB = kB;
    op.T = T;
    op.coef.assign(bond->coef, bond->coef + T);
    op.coef_dev = sc.get<double>(std::max(T, 1));
    op.OAcat = sc.get<double>((size_t)std::max(T, 1) * kA * kA);
    op.OBcat = sc.get<double>((size_t)std::max(T, 1) * kB * kB);
    op.Ediag = sc.get<double>(n);
    if (T > 0)
      RMC_HIP(hipMemcpyAsync(op.coef_dev, bond->coef, T * sizeof(double), hipMemcpyHostToDevice, s));
    for (int i = 0; i < T; ++i) {
      RMC_HIP(hipMemcpyAsync(op.OAcat + (size_t)i * kA * kA, A->ops[bond->opA[i]].data,
                             (size_t)kA * kA * sizeof(double), hipMemcpyDeviceToDevice, s));
      RMC_HIP(hipMemcpyAsync(op.OBcat + (size_t)i * kB * kB, B->ops[bond->opB[i]].data,
                             (size_t)kB * kB * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    kron_diag(s, kA, kB, A->E, B->E, T, op.coef_dev, op.OAcat, op.OBcat, nullptr, op.Ediag);
    build_packs(s, sc, op);
    op_apply(ctx, op, n_vec, X_dev, Y_dev, nullptr, 1.0, 0.0, 0.0, nullptr, nullptr, precision);
    sync(ctx);
  });
}

rmc_status rmc_kron_apply_noalloc(rmc_ctx* ctx, rmc_module* A, rmc_module* B,
                                  const rmc_bond_desc* bond, int precision, int n_vec,
                                  const double* X_dev, double* Y_dev) {
  if (!ctx) return RMC_ERR_ARG;
  return guard(ctx, [&] {
    RMC_CHECK(A && B && bond && X_dev && Y_dev && n_vec >= 0, RMC_ERR_ARG, "bad arguments");
    RMC_CHECK(precision >= RMC_FP64 && precision <= RMC_BF16, RMC_ERR_ARG, "bad precision");
    RMC_CHECK(A->E && B->E, RMC_ERR_STATE, "module freed");
    const int T = bond->n_terms, kA = A->k_eff, kB = B->k_eff, n = kA * kB;
    RMC_CHECK(T >= 0 && (T == 0 || (bond->coef && bond->opA && bond->opB)), RMC_ERR_ARG, "bad bond");
    RMC_CHECK(kA <= kron_max_k() && kB <= kron_max_k(), RMC_ERR_ARG, "module dimension above 192");
    for (int i = 0; i < T; ++i) {
      RMC_CHECK(bond->opA[i] >= 0 && bond->opA[i] < (int)A->ops.size(), RMC_ERR_ARG, "bad opA id");
      RMC_CHECK(bond->opB[i] >= 0 && bond->opB[i] < (int)B->ops.size(), RMC_ERR_ARG, "bad opB id");
    }
    char* base = scratch_of(ctx->device);
    RMC_CHECK(base != nullptr, RMC_ERR_STATE, "no scratch array on this device");
    // the pieces of rmc_kron_apply's scratch, 256-byte aligned, in one fixed array
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t b_coef = al(sizeof(double) * std::max(T, 1));
    const size_t b_oa = al(sizeof(double) * std::max(T, 1) * kA * kA);
    const size_t b_ob = al(sizeof(double) * std::max(T, 1) * kB * kB);
    const size_t b_ed = al(sizeof(double) * std::max(n, 1));
    const size_t b_pk = al(kron_pack_bytes(precision, kA, kB, T));
    const size_t b_desc = al(sizeof(KronDesc));
    const size_t need = b_coef + b_oa + b_ob + b_ed + b_pk + b_desc;
    RMC_CHECK(need <= kNoAllocScratchBytes, RMC_ERR_ARG,
              "this coupling needs " + std::to_string(need) + " bytes of scratch, above the " +
                  std::to_string(kNoAllocScratchBytes) + "-byte array of rmc_kron_apply_noalloc");
    hipStream_t s = ctx->stream;
    char* q = base;
    double* coef_dev = reinterpret_cast<double*>(q); q += b_coef;
    double* OAcat = reinterpret_cast<double*>(q); q += b_oa;
    double* OBcat = reinterpret_cast<double*>(q); q += b_ob;
    double* Ediag = reinterpret_cast<double*>(q); q += b_ed;
    void* pack = b_pk ? static_cast<void*>(q) : nullptr; q += b_pk;
    KronDesc* desc = reinterpret_cast<KronDesc*>(q);
    if (T > 0)
      RMC_HIP(hipMemcpyAsync(coef_dev, bond->coef, T * sizeof(double), hipMemcpyHostToDevice, s));
    for (int i = 0; i < T; ++i) {
      RMC_HIP(hipMemcpyAsync(OAcat + (size_t)i * kA * kA, A->ops[bond->opA[i]].data,
                             (size_t)kA * kA * sizeof(double), hipMemcpyDeviceToDevice, s));
      RMC_HIP(hipMemcpyAsync(OBcat + (size_t)i * kB * kB, B->ops[bond->opB[i]].data,
                             (size_t)kB * kB * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    kron_diag(s, kA, kB, A->E, B->E, T, coef_dev, OAcat, OBcat, nullptr, Ediag);
    if (pack)
      kron_pack(s, T, kA, kB, coef_dev, OAcat, OBcat, precision == RMC_FP64 ? pack : nullptr,
                precision == RMC_FP32 ? pack : nullptr, precision == RMC_BF16 ? pack : nullptr);
    KronDesc d{};
    d.kA = kA; d.kB = kB; d.T = T; d.nv = n_vec; d.vbase = 0;
    d.pack = pack; d.pkm = kron_pack_km(kA, kB);
    d.coef = coef_dev; d.OA = OAcat; d.OB = OBcat; d.Ediag = Ediag;
    d.Y = X_dev; d.Xprev = nullptr; d.E = nullptr; d.phi = nullptr; d.out = Y_dev;
    d.s1 = 1.0; d.s2 = 0.0; d.s3 = 0.0;
    RMC_HIP(hipMemcpyAsync(desc, &d, sizeof(d), hipMemcpyHostToDevice, s));
    // never times tile candidates (no events, no synchronisation)
    kron_batched(s, desc, 1, kB, n_vec, kA, precision, T, n_vec, /*may_tune=*/false);
    RMC_HIP(hipGetLastError());
  });
}

namespace {
// A product of one-site operators on an L-site block as a FullTerm (bit L-1-s = site s).
FullTerm full_term(double coef, int L, int n, const int* site, const int* op) {
  FullTerm t{};
  t.coef = coef;
  for (int u = 0; u < n; ++u) {
    const unsigned b = 1u << (L - 1 - site[u]);
    if (op[u] == RMC_OP_X) t.flip |= b;
    if (op[u] == RMC_OP_T) t.flip |= b, t.tm |= b;
    if (op[u] == RMC_OP_Z) t.zm |= b;
  }
  return t;
}

// o = Psi (O_1 O_2 Psi^T) for a leaf basis Psi (k x 2^n rows), O_2 applied first
// (op2 = 0: a single operator).
void leaf_op_product(hipStream_t s, Scratch& sc, const rmc_module* m, int site1, int op1, int site2,
                     int op2, double* o) {
  const int k = m->k_eff, D = m->dim, n = m->n_sites;
  double* W1 = sc.get<double>((size_t)k * D);
  if (op2) {
    double* W2 = sc.get<double>((size_t)k * D);
    site_op_apply(s, k, n, n - 1 - site2, op2, m->basis, W2);
    site_op_apply(s, k, n, n - 1 - site1, op1, W2, W1);
  } else {
    site_op_apply(s, k, n, n - 1 - site1, op1, m->basis, W1);
  }
  double* kw = sc.get<double>((size_t)64 * k * k + 64);
  gemm_f64(s, false, true, k, k, D, 1.0, m->basis, D, 0, W1, D, 0, 0.0, o, k, 0, 1,
           gemm_pick_ksplit(k, k, D, 1), kw);
}

// Single-merge diagnostics of two leaf modules (the quantities of the single-merge
// bound, App. on the error bounds); out = {a, b, c, gamma, r, b^2/gamma, E0}.
void merge_bound(rmc_ctx* ctx, rmc_module* A, const rmc_leaf_desc* la, rmc_module* B,
                 const rmc_leaf_desc* lb, const rmc_bond_desc* bond, rmc_solve_opts o, double* out) {
  validate_leaf(la);
  validate_leaf(lb);
  RMC_CHECK(A && B && bond && out, RMC_ERR_ARG, "null argument");
  for (const rmc_module* m : {A, B}) {
    RMC_CHECK(ctx->modules.count(const_cast<rmc_module*>(m)) != 0, RMC_ERR_ARG,
              "module not owned by this context");
    RMC_CHECK(m->kind == 0 && m->dim == (1 << m->n_sites), RMC_ERR_ARG,
              "the diagnostics need two leaf modules");
    RMC_CHECK(m->basis != nullptr, RMC_ERR_STATE, "module basis freed");
  }
  RMC_CHECK(la->n_sites == A->n_sites && lb->n_sites == B->n_sites, RMC_ERR_ARG,
            "leaf descriptors do not match the modules");
  const int nA = A->n_sites, nB = B->n_sites, L = nA + nB;
  RMC_CHECK(L <= 24, RMC_ERR_ARG, "the full space is limited to 24 sites");
  RMC_CHECK(bond->n_terms >= 0 && (bond->n_terms == 0 || (bond->coef && bond->opA && bond->opB)),
            RMC_ERR_ARG, "bad coupling descriptor");
  const int T = bond->n_terms;
  std::vector<int> sa(T), oa(T), sb(T), ob(T);
  for (int i = 0; i < T; ++i) {
    RMC_CHECK(bond->opA[i] >= 0 && bond->opA[i] < (int)A->ops.size() && bond->opB[i] >= 0 &&
                  bond->opB[i] < (int)B->ops.size(),
              RMC_ERR_ARG, "bad operator id");
    sa[i] = A->ops[bond->opA[i]].site;
    oa[i] = A->ops[bond->opA[i]].op;
    sb[i] = B->ops[bond->opB[i]].site;
    ob[i] = B->ops[bond->opB[i]].op;
  }
  o.precision = RMC_FP64;
  hipStream_t s = ctx->stream;
  // a: lowest eigenvalue of the effective Hamiltonian, i.e. of P H P on range(P)
  std::vector<double> ev;
  couple(ctx, A, B, bond, std::max(1, A->k_eff * B->k_eff), 1, o, false, ev, nullptr);
  const double a = ev[0];
  const int kA = A->k_eff, kB = B->k_eff, DA = A->dim, DB = B->dim;
  const bool q_empty = (kA == DA && kB == DB);
  Scratch sc(&ctx->arena);
  // b^2 = lambda_max(P V Q V P) = lambda_max(P V^2 P - (P V P)^2) on the retained
  // product states (P (H_A + H_B) Q = 0): both terms from projected products of the
  // boundary operators, so -M = (P V P)^2 - P V^2 P is solved for its lowest eigenvalue
  double b = 0.0;
  if (!q_empty && T > 0) {
    const int nr = kA * kB;
    double* Ap = sc.get<double>((size_t)T * T * kA * kA);
    double* Bp = sc.get<double>((size_t)T * T * kB * kB);
    double* As = sc.get<double>((size_t)T * kA * kA);
    double* Bs = sc.get<double>((size_t)T * kB * kB);
    std::vector<double> wp(T * T), ws(T);
    for (int i = 0; i < T; ++i) {
      ws[i] = bond->coef[i];
      leaf_op_product(s, sc, A, sa[i], oa[i], 0, 0, As + (size_t)i * kA * kA);
      leaf_op_product(s, sc, B, sb[i], ob[i], 0, 0, Bs + (size_t)i * kB * kB);
      for (int j = 0; j < T; ++j) {
        wp[i * T + j] = -bond->coef[i] * bond->coef[j];
        leaf_op_product(s, sc, A, sa[i], oa[i], sa[j], oa[j], Ap + (size_t)(i * T + j) * kA * kA);
        leaf_op_product(s, sc, B, sb[i], ob[i], sb[j], ob[j], Bp + (size_t)(i * T + j) * kB * kB);
      }
    }
    double* wdev = sc.get<double>(T * T + T);
    RMC_HIP(hipMemcpyAsync(wdev, wp.data(), T * T * sizeof(double), hipMemcpyHostToDevice, s));
    RMC_HIP(hipMemcpyAsync(wdev + T * T, ws.data(), T * sizeof(double), hipMemcpyHostToDevice, s));
    double* negM = sc.get<double>((size_t)nr * nr);
    double* Vh = sc.get<double>((size_t)nr * nr);
    kron_dense(s, T * T, kA, kB, wdev, Ap, Bp, negM);
    kron_dense(s, T, kA, kB, wdev + T * T, As, Bs, Vh);
    gemm_f64(s, false, false, nr, nr, nr, 1.0, Vh, nr, 0, Vh, nr, 0, 1.0, negM, nr, 0, 1, 1, nullptr);
    double lam;
    if (nr == 1) {
      RMC_HIP(hipMemcpyAsync(&lam, negM, sizeof(double), hipMemcpyDeviceToHost, s));
      sync(ctx);
    } else {
      CoupledOp op;
      op.kind = 0;
      op.n = nr;
      op.H = negM;
      op.D = sc.get<double>(nr);
      double* rb = sc.get<double>(nr);
      double* bm = sc.get<double>(1);
      dense_diag(s, nr, negM, op.D, rb);
      vec_max(s, nr, rb, bm);
      RMC_HIP(hipMemcpyAsync(&op.bup, bm, sizeof(double), hipMemcpyDeviceToHost, s));
      sync(ctx);
      double* X = sc.get<double>(nr);
      std::vector<double> e1;
      SolveStats st;
      RMC_CHECK(eig_lowest(ctx, op, 1, o, X, e1, st) == RMC_OK, RMC_ERR_NOCONV,
                "eigensolver did not converge on P V Q V P");
      lam = e1[0];
    }
    b = std::sqrt(std::max(0.0, -lam));
  }
  // E0 = lambda_min(H) and c = lambda_min(Q H Q + sigma P) (range(P) moved to sigma >=
  // ||H||) in the full space, as one batched solve of two matrix-free operators
  std::vector<FullTerm> ft;
  std::vector<int> st2(2), op2(2);
  for (int t = 0; t < la->n_terms; ++t) {
    const rmc_term& tm = la->terms[t];
    for (int u = 0; u < tm.nsite; ++u) st2[u] = tm.site[u], op2[u] = tm.op[u];
    ft.push_back(full_term(tm.coef, L, tm.nsite, st2.data(), op2.data()));
  }
  for (int t = 0; t < lb->n_terms; ++t) {
    const rmc_term& tm = lb->terms[t];
    for (int u = 0; u < tm.nsite; ++u) st2[u] = nA + tm.site[u], op2[u] = tm.op[u];
    ft.push_back(full_term(tm.coef, L, tm.nsite, st2.data(), op2.data()));
  }
  for (int i = 0; i < T; ++i) {
    st2[0] = sa[i], op2[0] = oa[i], st2[1] = nA + sb[i], op2[1] = ob[i];
    ft.push_back(full_term(bond->coef[i], L, 2, st2.data(), op2.data()));
  }
  // grouped by flip mask, diagonal terms first: the apply kernel gathers once per group
  std::stable_sort(ft.begin(), ft.end(),
                   [](const FullTerm& x, const FullTerm& y) { return x.flip < y.flip; });
  double sigma = 0.0;
  for (auto& t : ft) sigma += std::fabs(t.coef);
  sigma = std::max(sigma, 1e-300);
  FullTerm* fdev = sc.get<FullTerm>(std::max<size_t>(ft.size(), 1));
  if (!ft.empty())
    RMC_HIP(hipMemcpyAsync(fdev, ft.data(), ft.size() * sizeof(FullTerm), hipMemcpyHostToDevice, s));
  const size_t n = (size_t)1 << L;
  std::vector<CoupledOp> ops(q_empty ? 1 : 2);
  for (size_t i = 0; i < ops.size(); ++i) {
    CoupledOp& op = ops[i];
    op.kind = 2;
    op.n = (int)n;
    op.fterms = fdev;
    op.n_fterms = (int)ft.size();
    op.nA = nA;
    op.nB = nB;
    op.bup = sigma;
    op.D = sc.get<double>(n);
    if (i == 1) {
      op.PsiA = A->basis;
      op.PsiB = B->basis;
      op.kA = kA;
      op.kB = kB;
      op.sigma = sigma;
      double* pA = sc.get<double>(DA);
      double* pB = sc.get<double>(DB);
      col_sumsq(s, kA, DA, A->basis, pA);
      col_sumsq(s, kB, DB, B->basis, pB);
      full_diag(s, L, nB, op.n_fterms, fdev, pA, pB, sigma, op.D);
    } else {
      full_diag(s, L, nB, op.n_fterms, fdev, nullptr, nullptr, 0.0, op.D);
    }
  }
  std::vector<const CoupledOp*> opp;
  std::vector<double*> Xs;
  for (auto& op : ops) {
    opp.push_back(&op);
    Xs.push_back(sc.get<double>(n));
  }
  std::vector<std::vector<double>> evs;
  std::vector<SolveStats> sts;
  eig_lowest_batch(ctx, opp, std::vector<int>(ops.size(), 1), o, Xs, evs, sts);
  for (auto& x : sts)
    RMC_CHECK(x.status == RMC_OK, RMC_ERR_NOCONV, "full-space eigensolver did not converge");
  const double E0 = evs[0][0];
  const double c = q_empty ? INFINITY : evs[1][0];
  const double g = c - a;
  out[0] = a;
  out[1] = b;
  out[2] = c;
  out[3] = g;
  out[4] = b == 0.0 ? 0.0 : 0.5 * (std::sqrt(g * g + 4.0 * b * b) - g);
  out[5] = b == 0.0 ? 0.0 : (g > 0.0 ? b * b / g : INFINITY);
  out[6] = E0;
  sync(ctx);
}
}  // namespace

rmc_status rmc_merge_bound(rmc_ctx* ctx, rmc_module* A, const rmc_leaf_desc* leaf_A, rmc_module* B,
                           const rmc_leaf_desc* leaf_B, const rmc_bond_desc* bond,
                           const rmc_solve_opts* opts, double* out_host) {
  if (!ctx) return RMC_ERR_ARG;
  return guard(ctx, [&] {
    rmc_solve_opts o;
    rmc_default_opts(&o);
    if (opts) o = *opts;
    merge_bound(ctx, A, leaf_A, B, leaf_B, bond, o, out_host);
  });
}

rmc_status rmc_profile(rmc_ctx* ctx, int enable) {
  if (!ctx) return RMC_ERR_ARG;
  return guard(ctx, [&] {
    sync(ctx);
    for (auto& r : ctx->prof_recs) {
      ctx->ev_pool.push_back(r.a);
      ctx->ev_pool.push_back(r.b);
    }
    ctx->prof_recs.clear();
    if (enable) {
      for (int k = 0; k < 3; ++k)
        for (int p = 0; p < 3; ++p) {
          ctx->prof_launches[k][p] = 0;
          ctx->prof_flops[k][p] = ctx->prof_bytes[k][p] = ctx->prof_ms[k][p] = 0.0;
        }
    }
    ctx->prof = enable != 0;
  });
}

namespace {
void profile_collect(rmc_ctx* ctx) {
  sync(ctx);
  for (auto& r : ctx->prof_recs) {
    float t = 0.f;
    RMC_HIP(hipEventElapsedTime(&t, r.a, r.b));
    ctx->prof_ms[r.kind][r.prec] += t;
    ctx->prof_flops[r.kind][r.prec] += r.flops;
    ctx->prof_bytes[r.kind][r.prec] += r.bytes;
    ctx->prof_launches[r.kind][r.prec] += 1;
    ctx->ev_pool.push_back(r.a);
    ctx->ev_pool.push_back(r.b);
  }
  ctx->prof_recs.clear();
}
}  // namespace

rmc_status rmc_profile_read(rmc_ctx* ctx, long long* launches, double* flops, double* bytes,
                            double* ms) {
  if (!ctx) return RMC_ERR_ARG;
  return guard(ctx, [&] {
    profile_collect(ctx);
    long long n = 0;
    double f = 0.0, b = 0.0, t = 0.0;
    for (int k = RMC_PROF_KRON_STEP; k <= RMC_PROF_KRON_FILTER; ++k)
      for (int p = 0; p < 3; ++p) {
        n += ctx->prof_launches[k][p];
        f += ctx->prof_flops[k][p];
        b += ctx->prof_bytes[k][p];
        t += ctx->prof_ms[k][p];
      }
    if (launches) *launches = n;
    if (flops) *flops = f;
    if (bytes) *bytes = b;
    if (ms) *ms = t;
  });
}

rmc_status rmc_profile_read_precision(rmc_ctx* ctx, int precision, long long* launches,
                                      double* flops, double* bytes, double* ms) {
  if (!ctx || precision < RMC_FP64 || precision > RMC_BF16) return RMC_ERR_ARG;
  return guard(ctx, [&] {
    profile_collect(ctx);
    const int k0 = RMC_PROF_KRON_STEP, k1 = RMC_PROF_KRON_FILTER;
    if (launches) *launches = ctx->prof_launches[k0][precision] + ctx->prof_launches[k1][precision];
    if (flops) *flops = ctx->prof_flops[k0][precision] + ctx->prof_flops[k1][precision];
    if (bytes) *bytes = ctx->prof_bytes[k0][precision] + ctx->prof_bytes[k1][precision];
    if (ms) *ms = ctx->prof_ms[k0][precision] + ctx->prof_ms[k1][precision];
  });
}

rmc_status rmc_profile_read_kernel(rmc_ctx* ctx, int kernel, int precision, long long* launches,
                                   double* flops, double* bytes, double* ms) {
  if (!ctx || precision < RMC_FP64 || precision > RMC_BF16 || kernel < RMC_PROF_KRON_STEP ||
      kernel > RMC_PROF_PAULI)
    return RMC_ERR_ARG;
  return guard(ctx, [&] {
    profile_collect(ctx);
    if (launches) *launches = ctx->prof_launches[kernel][precision];
    if (flops) *flops = ctx->prof_flops[kernel][precision];
    if (bytes) *bytes = ctx->prof_bytes[kernel][precision];
    if (ms) *ms = ctx->prof_ms[kernel][precision];
  });
}

rmc_status rmc_sym_eig(rmc_ctx* ctx, int batch, int m, const double* A_dev, double* evals_dev,
                       double* V_dev) {
  if (!ctx) return RMC_ERR_ARG;
  return guard(ctx, [&] {
    RMC_CHECK(batch >= 0 && m >= 1 && m <= jacobi_max_m(), RMC_ERR_ARG, "m must be 1..192");
    RMC_CHECK(A_dev && evals_dev && V_dev, RMC_ERR_ARG, "null pointer");
    if (batch == 0) return;
    Scratch sc(&ctx->arena);
    double* Vw = sc.get<double>((size_t)batch * m * m);
    int* info = sc.get<int>(batch);
    jacobi_eig(ctx->stream, batch, m, A_dev, (long)m * m, 1, 0, evals_dev, m, V_dev, (long)m * m, Vw,
               info);
    sync(ctx);
  });
}

}  // extern "C"
