// Leaf-module kernels: bit-index assembly of the dense leaf Hamiltonian, one-site
// operator application (for the projected boundary operators o = V^T O V),
// diagonals of the coupled operator, and the eigensolver's start block.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "rmc_batch.h"
#include "rmc_kernels.h"

namespace rmc {

// Matrix element <br|O|bc> of a one-site operator for row bit br (column bit
// bc = br ^ 1 for X and T, bc = br for Z): X -> 1; T = [[0,-1],[1,0]] -> -1 if
// br == 0 else +1; Z -> +1 if br == 0 else -1.
__device__ inline bool op_flips(int op) { return op != 3; }

__device__ inline double op_sign(int op, int br) {
  if (op == 1) return 1.0;
  if (op == 2) return br == 0 ? -1.0 : 1.0;
  return br == 0 ? 1.0 : -1.0;
}

// Entry-parallel assembly: thread (r, c) walks the term list in order and adds
// coef * (product of +-1 factors) for every term that maps row r to column c (its X / T
// sites flipped: c = r ^ flip). Each entry is accumulated in term order from +0.0,
// exactly as a dense sum of Kronecker products would be, and consecutive threads write
// consecutive entries of a row (coalesced; no separate zero pass). Each workgroup first
// turns the term list into (coef, flip, Z mask, T mask) in LDS: a term acts on row r
// with the sign (-1)^(|r & Z mask| + |~r & T mask|) (Z: -1 on a set bit; T = -i sigma^y:
// -1 on a clear bit), so an entry costs one compare per term and a sign only on a match.
struct LeafTermMask {
  double coef;
  int flip, zm, tm, pad;
};
constexpr int kLeafTermsLds = 1024;

__device__ inline LeafTermMask leaf_term_mask(const DevTerm& t) {
  LeafTermMask m{t.coef, 0, 0, 0, 0};
  for (int u = 0; u < t.nsite; ++u) {
    const int bit = 1 << t.bit[u];
    if (op_flips(t.op[u])) m.flip |= bit;
    if (t.op[u] == 3) m.zm |= bit;
    if (t.op[u] == 2) m.tm |= bit;
  }
  return m;
}

__device__ inline double leaf_entry(int r, int c, int n_terms, const LeafTermMask* tl) {
  const int x = r ^ c;
  double acc = 0.0;
  for (int t = 0; t < n_terms; ++t) {
    const LeafTermMask m = tl[t];
    if (m.flip != x) continue;
    const int odd = (__popc(r & m.zm) + __popc(~r & m.tm)) & 1;
    acc = acc + (odd ? -m.coef : m.coef);
  }
  return acc;
}

// Stages the term list of a leaf in LDS (up to kLeafTermsLds terms) and fills the D x D
// entries from e0 on, with a grid stride; longer lists read their masks from `spill`.
__device__ inline void leaf_fill(int n_sites, int n_terms, const DevTerm* __restrict__ terms,
                                 double* __restrict__ H, LeafTermMask* tl, long e0, long stride) {
  const int nl = min(n_terms, kLeafTermsLds);
  for (int t = threadIdx.x; t < nl; t += blockDim.x) tl[t] = leaf_term_mask(terms[t]);
  __syncthreads();
  const int D = 1 << n_sites;
  const long nn = (long)D * D;
  for (long e = e0; e < nn; e += stride) {
    const int r = (int)(e >> n_sites), c = (int)(e & (D - 1));
    double v = leaf_entry(r, c, nl, tl);
    for (int t = nl; t < n_terms; ++t) {  // beyond the LDS table, in the same order
      const LeafTermMask m = leaf_term_mask(terms[t]);
      if (m.flip != (r ^ c)) continue;
      const int odd = (__popc(r & m.zm) + __popc(~r & m.tm)) & 1;
      v = v + (odd ? -m.coef : m.coef);
    }
    H[e] = v;
  }
}

__global__ __launch_bounds__(256) void leaf_assemble_kernel(int n_sites, int n_terms,
                                                            const DevTerm* __restrict__ terms,
                                                            double* __restrict__ H) {
  __shared__ LeafTermMask tl[kLeafTermsLds];
  leaf_fill(n_sites, n_terms, terms, H, tl, blockIdx.x * 256L + threadIdx.x, (long)gridDim.x * 256);
}

void leaf_assemble(hipStream_t s, int n_sites, int n_terms, const DevTerm* terms, double* H) {
  const long D = 1L << n_sites, nn = D * D;
  const int blocks = (int)std::min<long>((nn + 255) / 256, 4096);
  hipLaunchKernelGGL(leaf_assemble_kernel, dim3(blocks), dim3(256), 0, s, n_sites, n_terms, terms, H);
}

// ---- batched leaf set-up (every leaf of a level in three launches) -----------------
// The entry-parallel assembly of leaf_assemble_kernel for every leaf of a batch.
__global__ __launch_bounds__(256) void leaf_assemble_batched_kernel(const LeafSetDesc* __restrict__ descs) {
  __shared__ LeafTermMask tl[kLeafTermsLds];
  const LeafSetDesc d = descs[blockIdx.y];
  leaf_fill(d.n_sites, d.n_terms, d.terms, d.H, tl, blockIdx.x * 256L + threadIdx.x, (long)gridDim.x * 256);
}

// Diagonal and Gershgorin row bounds (as dense_diag_kernel), one workgroup per row.
__global__ __launch_bounds__(256) void leaf_diag_batched_kernel(const LeafSetDesc* __restrict__ descs) {
  __shared__ double red[4];
  const LeafSetDesc d = descs[blockIdx.y];
  const int n = 1 << d.n_sites;
  const int i = blockIdx.x;
  if (i >= n) return;
  const double* row = d.H + (long)i * n;
  double acc = 0.0;
  for (int j = threadIdx.x; j < n; j += 256)
    if (j != i) acc += fabs(row[j]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = (red[0] + red[1]) + (red[2] + red[3]);
    d.D[i] = row[i];
    d.rb[i] = row[i] + s;
  }
}

// bmax = max over rows of the Gershgorin bound (as vec_max_kernel).
__global__ __launch_bounds__(256) void leaf_bound_batched_kernel(const LeafSetDesc* __restrict__ descs) {
  __shared__ double red[256];
  const LeafSetDesc d = descs[blockIdx.x];
  const int n = 1 << d.n_sites;
  double m = -INFINITY;
  for (int i = threadIdx.x; i < n; i += 256) m = fmax(m, d.rb[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) d.bmax[0] = red[0];
}

void leaf_setup_batched(hipStream_t s, const LeafSetDesc* d, int P, int n_sites_max) {
  if (P <= 0) return;
  const long D = 1L << n_sites_max, nn = D * D;
  const int ab = (int)std::min<long>((nn + 255) / 256, 1024);
  hipLaunchKernelGGL(leaf_assemble_batched_kernel, dim3(ab, P), dim3(256), 0, s, d);
  hipLaunchKernelGGL(leaf_diag_batched_kernel, dim3((unsigned)D, P), dim3(256), 0, s, d);
  hipLaunchKernelGGL(leaf_bound_batched_kernel, dim3(P), dim3(256), 0, s, d);
}

// (O v)[r] = sum_c O[r][c] v[c] = sign(op, bit of r) * v[r ^ flip].
__global__ void site_op_apply_kernel(int nv, int D, int bit, int op, const double* __restrict__ V,
                                     double* __restrict__ W) {
  long total = (long)nv * D;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total;
       t += (long)gridDim.x * blockDim.x) {
    int j = (int)(t / D), r = (int)(t % D);
    int br = (r >> bit) & 1;
    int c = op_flips(op) ? (r ^ (1 << bit)) : r;
    W[t] = op_sign(op, br) * V[(long)j * D + c];
  }
}

__global__ void site_op_batched_kernel(const SiteOpDesc* __restrict__ descs) {
  const SiteOpDesc d = descs[blockIdx.y];
  const int D = 1 << d.n_sites;
  const long total = (long)d.nv * D;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total;
       t += (long)gridDim.x * blockDim.x) {
    int j = (int)(t / D), r = (int)(t % D);
    int br = (r >> d.bit) & 1;
    int c = op_flips(d.op) ? (r ^ (1 << d.bit)) : r;
    d.W[t] = op_sign(d.op, br) * d.V[(long)j * D + c];
  }
}

void site_op_batched(hipStream_t s, const SiteOpDesc* d, int P, long total_max) {
  if (P <= 0 || total_max <= 0) return;
  const int blocks = (int)std::min<long>((total_max + 255) / 256, 1024);
  hipLaunchKernelGGL(site_op_batched_kernel, dim3(blocks, P), dim3(256), 0, s, d);
}

void site_op_apply(hipStream_t s, int nv, int n_sites, int bit, int op, const double* V, double* W) {
  int D = 1 << n_sites;
  long total = (long)nv * D;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(site_op_apply_kernel, dim3(blocks), dim3(256), 0, s, nv, D, bit, op, V, W);
}

__global__ void kron_diag_kernel(int kA, int kB, const double* __restrict__ EA, const double* __restrict__ EB,
                                 int T, const double* __restrict__ coef, const double* __restrict__ OA,
                                 const double* __restrict__ OB, double* __restrict__ D,
                                 double* __restrict__ Ediag) {
  int n = kA * kB;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
    int a = t / kB, b = t % kB;
    double e = EA[a] + EB[b];
    double d = e;
    for (int i = 0; i < T; ++i)
      d += coef[i] * OA[(long)i * kA * kA + (long)a * kA + a] * OB[(long)i * kB * kB + (long)b * kB + b];
    if (D) D[t] = d;
    if (Ediag) Ediag[t] = e;
  }
}

void kron_diag(hipStream_t s, int kA, int kB, const double* EA, const double* EB, int T,
               const double* coef_dev, const double* OAcat, const double* OBcat, double* D,
               double* Ediag) {
  int n = kA * kB;
  hipLaunchKernelGGL(kron_diag_kernel, dim3((n + 255) / 256), dim3(256), 0, s, kA, kB, EA, EB, T,
                     coef_dev, OAcat, OBcat, D, Ediag);
}

__global__ __launch_bounds__(256) void dense_diag_kernel(int n, const double* __restrict__ H,
                                                         double* __restrict__ D, double* __restrict__ bound) {
  __shared__ double red[4];
  int i = blockIdx.x;
  const double* row = H + (long)i * n;
  double acc = 0.0;
  for (int j = threadIdx.x; j < n; j += 256)
    if (j != i) acc += fabs(row[j]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = (red[0] + red[1]) + (red[2] + red[3]);
    D[i] = row[i];
    bound[i] = row[i] + s;
  }
}

void dense_diag(hipStream_t s, int n, const double* H, double* D, double* rowbound) {
  hipLaunchKernelGGL(dense_diag_kernel, dim3(n), dim3(256), 0, s, n, H, D, rowbound);
}

// SplitMix64 (Steele, Lea, Flood 2014) as a counter-based generator.
__device__ inline uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

__global__ void rank_select_kernel(int n, int m, const double* __restrict__ D, int* __restrict__ sel) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    double di = D[i];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      double dj = D[j];
      rank += (dj < di) || (dj == di && j < i);
    }
    if (rank < m) sel[rank] = i;
  }
}

__global__ void start_block_kernel(int n, int m, const int* __restrict__ sel, double eps, uint64_t seed,
                                   double* __restrict__ X) {
  long total = (long)m * n;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total;
       t += (long)gridDim.x * blockDim.x) {
    int j = (int)(t / n), i = (int)(t % n);
    uint64_t h = splitmix64(seed ^ splitmix64((uint64_t)t));
    double u = (double)(h >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
    double v = eps * u;
    if (sel[j] == i) v += 1.0;
    X[t] = v;
  }
}

void start_block(hipStream_t s, int n, int m, const double* D, double eps, unsigned long long seed,
                 int* sel, double* X) {
  hipLaunchKernelGGL(rank_select_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, m, D, sel);
  long total = (long)m * n;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(start_block_kernel, dim3(blocks), dim3(256), 0, s, n, m, sel, eps,
                     (uint64_t)seed, X);
}

// sel[r] = index of the entry of rank r among the m smallest of D (ties by index), one
// workgroup per problem. An MSD radix select over order-preserving 64-bit keys
// (8 passes of 8 bits, LDS histograms) finds the key K of rank m-1 and how many
// entries equal to K are needed; the entries below K plus the lowest-index entries
// equal to K are then gathered and ranked among themselves (m <= 192).
// inclusive prefix sum over a 256-thread workgroup (wave shuffles, then the wave
// totals); wsum: 4 entries of LDS. Contains the barriers it needs.
__device__ inline unsigned scan256(unsigned v, unsigned* wsum) {
  const int tid = threadIdx.x, lane = tid & 63;
  unsigned x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const unsigned y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) wsum[tid >> 6] = x;
  __syncthreads();
  for (int w = 0; w < (tid >> 6); ++w) x += wsum[w];
  __syncthreads();
  return x;
}

__device__ inline unsigned long long order_key(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x + 0.0);  // -0 -> +0
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__global__ __launch_bounds__(256) void rank_select_batched_kernel(const StartDesc* __restrict__ descs) {
  __shared__ unsigned int hist[256];
  __shared__ unsigned long long s_prefix, s_mask;
  __shared__ int s_need;
  __shared__ int cnt_eq[256];
  __shared__ int n_less;
  __shared__ unsigned long long ck[192];
  __shared__ int ci[192];
  __shared__ unsigned wsum[4];
  const StartDesc d = descs[blockIdx.x];
  const int n = d.n, m = d.m, tid = threadIdx.x;
  if (m <= 0 || m > 192) return;
  if (tid == 0) { s_prefix = 0; s_mask = 0; s_need = m; n_less = 0; }
  __syncthreads();
  for (int pass = 0; pass < 8; ++pass) {
    const int shift = 56 - 8 * pass;
    hist[tid] = 0;
    __syncthreads();
    const unsigned long long pre = s_prefix, msk = s_mask;
    for (int i = tid; i < n; i += 256) {
      const unsigned long long k = order_key(d.D[i]);
      if ((k & msk) == pre) atomicAdd(&hist[(k >> shift) & 255u], 1u);
    }
    __syncthreads();
    // the first bin whose running count reaches the rank still needed: bin b with
    // excl(b) < need <= incl(b) (the counts under the prefix cover need)
    const int need = s_need;
    const unsigned hv = hist[tid];
    const unsigned incl = scan256(hv, wsum), excl = incl - hv;
    if ((int)excl < need && (int)incl >= need) {
      s_need = need - (int)excl;
      s_prefix = pre | ((unsigned long long)tid << shift);
      s_mask = msk | (255ull << shift);
    }
    __syncthreads();
  }
  const unsigned long long K = s_prefix;
  const int need = s_need;  // entries equal to K to take (>= 1)
  // contiguous index chunk per thread: counts of entries equal to K, exclusive scan
  const int chunk = (n + 255) / 256;
  const int lo = min(n, tid * chunk), hi = min(n, lo + chunk);
  int ce = 0;
  for (int i = lo; i < hi; ++i) {
    const unsigned long long k = order_key(d.D[i]);
    if (k < K) {
      const int slot = atomicAdd(&n_less, 1);
      ck[slot] = k;
      ci[slot] = i;
    } else if (k == K) {
      ++ce;
    }
  }
  cnt_eq[tid] = (int)scan256((unsigned)ce, wsum) - ce;  // exclusive
  __syncthreads();
  const int base_less = m - need;  // == n_less
  int before = cnt_eq[tid];
  for (int i = lo; i < hi && before < need; ++i) {
    const unsigned long long k = order_key(d.D[i]);
    if (k == K) {
      ck[base_less + before] = k;
      ci[base_less + before] = i;
      ++before;
    }
  }
  __syncthreads();
  // rank the m candidates by (key, index)
  for (int c = tid; c < m; c += 256) {
    const unsigned long long kc = ck[c];
    const int ic = ci[c];
    int r = 0;
    for (int e = 0; e < m; ++e) r += (ck[e] < kc) || (ck[e] == kc && ci[e] < ic);
    d.sel[r] = ic;
  }
}

__global__ void start_block_batched_kernel(const StartDesc* __restrict__ descs) {
  const StartDesc d = descs[blockIdx.z];
  const long total = (long)d.m * d.n;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total;
       t += (long)gridDim.x * blockDim.x) {
    int j = (int)(t / d.n), i = (int)(t % d.n);
    uint64_t h = splitmix64((uint64_t)d.seed ^ splitmix64((uint64_t)t));
    double u = (double)(h >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
    double v = d.eps * u;
    if (d.sel[j] == i) v += 1.0;
    d.X[t] = v;
  }
}

// ---- block-diagonal leaves -----------------------------------------------------------
__global__ __launch_bounds__(256) void gather_blocks_kernel(const BlockGatherDesc* __restrict__ descs) {
  const BlockGatherDesc& d = descs[blockIdx.y];
  const long total = (long)d.nb * d.nb;
  for (long t = blockIdx.x * 256L + threadIdx.x; t < total; t += (long)gridDim.x * 256) {
    const int i = (int)(t / d.nb), j = (int)(t - (long)i * d.nb);
    d.A[t] = d.H[(long)d.idx[i] * d.D + d.idx[j]];
  }
}

void gather_blocks(hipStream_t s, const BlockGatherDesc* d, int P, int nbmax) {
  if (P <= 0 || nbmax <= 0) return;
  const long tot = (long)nbmax * nbmax;
  const int bx = (int)std::min<long>((tot + 255) / 256, 64);
  hipLaunchKernelGGL(gather_blocks_kernel, dim3(bx, P), dim3(256), 0, s, d);
}

// One workgroup per output row: the row is zeroed, then (after the barrier) the block's
// entries are written, so no separate fill per leaf is needed.
__global__ __launch_bounds__(256) void scatter_block_rows_kernel(const BlockScatterDesc* __restrict__ descs) {
  const BlockScatterDesc& d = descs[blockIdx.x];
  for (int t = threadIdx.x; t < d.n; t += 256) d.out[t] = 0.0;
  __syncthreads();
  for (int r = threadIdx.x; r < d.nb; r += 256) d.out[d.idx[r]] = d.V[(long)r * d.nb + d.col];
}

void scatter_block_rows(hipStream_t s, const BlockScatterDesc* d, int P, int nbmax) {
  if (P <= 0 || nbmax <= 0) return;
  hipLaunchKernelGGL(scatter_block_rows_kernel, dim3(P), dim3(256), 0, s, d);
}

// One workgroup per leaf, a thread per eigenvalue of the leaf. Within its own block an
// eigenvalue's column is its count of smaller keys (the block is ascending, equal values
// in column order); every other block adds the count of its values below (blocks after
// it) or not above (blocks before it: equal values there come first), by bisection.
__global__ __launch_bounds__(256) void leaf_select_kernel(const LeafSelDesc* __restrict__ descs,
                                                          const EigDesc* __restrict__ ed,
                                                          const BlockGatherDesc* __restrict__ gd,
                                                          BlockScatterDesc* __restrict__ sd) {
  const LeafSelDesc L = descs[blockIdx.x];
  const EigDesc* eb = ed + L.b0;
  const double* ev0 = eb[0].evals;  // the leaf's eigenvalues, block after block
  const int D = (int)(eb[L.nblk - 1].evals - ev0) + eb[L.nblk - 1].m;
  for (int e = threadIdx.x; e < D; e += 256) {
    const double v = ev0[e];
    int rank = 0, b = 0, j = 0;
    for (int q = 0; q < L.nblk; ++q) {
      const double* x = eb[q].evals;
      const int nb = eb[q].m, o = (int)(x - ev0);
      if (e >= o && e < o + nb) {
        b = q;
        j = e - o;
        rank += j;
        continue;
      }
      const bool before = o + nb <= e;
      int lo = 0, hi = nb;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const double xm = x[mid];
        if (before ? xm <= v : xm < v) lo = mid + 1;
        else hi = mid;
      }
      rank += lo;
    }
    if (rank < L.ne) {
      L.evout[rank] = v;
      sd[L.sdbase + rank] = BlockScatterDesc{eb[b].m, j, L.n, 0, gd[L.b0 + b].idx, eb[b].V, L.X + (long)rank * L.n};
    }
  }
}

void leaf_select(hipStream_t s, const LeafSelDesc* d, int P, const EigDesc* ed, const BlockGatherDesc* gd,
                 BlockScatterDesc* sd) {
  if (P <= 0) return;
  hipLaunchKernelGGL(leaf_select_kernel, dim3(P), dim3(256), 0, s, d, ed, gd, sd);
}

void start_batched(hipStream_t s, const StartDesc* d, int P, int nmax, int mmax) {
  if (P <= 0) return;
  hipLaunchKernelGGL(rank_select_batched_kernel, dim3(P), dim3(256), 0, s, d);
  long tot = (long)nmax * mmax;
  int bx2 = (int)((tot + 255) / 256);
  if (bx2 > 2048) bx2 = 2048;
  hipLaunchKernelGGL(start_block_batched_kernel, dim3(bx2, 1, P), dim3(256), 0, s, d);
}

}  // namespace rmc
