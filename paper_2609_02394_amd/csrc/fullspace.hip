// Full-space kernels of the single-merge truncation diagnostics (Sec. IV, single-merge
// bound; App. on the error bounds): the Hamiltonian of the merged block applied
// matrix-free as a sum of Pauli strings on 2^L amplitudes (the bit-index rule of the
// leaf assembly, without storing the matrix), the projector P onto the retained
// product sector built from GEMMs, and the small dense pieces of ||P H Q||_2.
//
// These run at L <= 24 for one merge; every kernel is a coalesced grid-stride loop
// bound by HBM / L2 traffic (a gather y[r ^ flip] keeps a wavefront inside one or two
// 512-byte segments for any flip).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "rmc_batch.h"

namespace rmc {

namespace {

__device__ inline double term_sign(unsigned r, unsigned zm, unsigned tm) {
  const unsigned odd = (__popc(r & zm) + __popc(~r & tm)) & 1u;
  return odd ? -1.0 : 1.0;
}

__global__ __launch_bounds__(256) void pauli_batched_kernel(const PauliDesc* __restrict__ descs) {
  const PauliDesc& d = descs[blockIdx.y];
  const long n = 1L << d.n_sites;
  const long total = n * d.nv;
  const unsigned mask = (unsigned)(n - 1);
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long base = e & ~(long)mask;  // first amplitude of this vector
    const unsigned r = (unsigned)(e & mask);
    const double* y = d.Y + base;
    const double* u = d.sub ? d.sub + base : nullptr;
    // terms arrive grouped by flip mask (all diagonal terms first): one gather serves
    // every term of a group
    double acc = 0.0, v = 0.0;
    unsigned last = ~0u;
    for (int t = 0; t < d.n_terms; ++t) {
      const FullTerm tm = d.terms[t];
      if (tm.flip != last) {
        const unsigned c = r ^ tm.flip;
        v = y[c];
        if (u) v -= u[c];
        last = tm.flip;
      }
      acc += tm.coef * term_sign(r, tm.zm, tm.tm) * v;
    }
    double o = d.s1 * acc;
    if (d.Y0) o += d.s2 * d.Y0[e];
    if (d.Xprev) o += d.s3 * d.Xprev[e];
    d.out[e] = o;
  }
}

__global__ __launch_bounds__(256) void lincomb_batched_kernel(const LinDesc* __restrict__ descs) {
  const LinDesc& d = descs[blockIdx.y];
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < d.n; e += (long)gridDim.x * blockDim.x) {
    double o = 0.0;
#pragma unroll
    for (int i = 0; i < 5; ++i)
      if (d.U[i]) o += d.w[i] * d.U[i][e];
    d.out[e] = o;
  }
}

__global__ __launch_bounds__(256) void full_diag_kernel(int n_sites, int nB, int n_terms,
                                                        const FullTerm* __restrict__ terms,
                                                        const double* __restrict__ pA,
                                                        const double* __restrict__ pB, double sigma,
                                                        double* __restrict__ D) {
  const long n = 1L << n_sites;
  const unsigned bmask = (1u << nB) - 1u;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const unsigned r = (unsigned)e;
    double acc = 0.0;
    for (int t = 0; t < n_terms; ++t) {
      const FullTerm tm = terms[t];
      if (tm.flip == 0) acc += tm.coef * term_sign(r, tm.zm, tm.tm);
    }
    if (pA) acc += sigma * pA[r >> nB] * pB[r & bmask];
    D[e] = acc;
  }
}

__global__ __launch_bounds__(256) void col_sumsq_kernel(int k, int D, const double* __restrict__ Psi,
                                                        double* __restrict__ p) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= D) return;
  double acc = 0.0;
  for (int i = 0; i < k; ++i) {
    const double v = Psi[(long)i * D + j];
    acc += v * v;
  }
  p[j] = acc;
}

__global__ __launch_bounds__(256) void kron_dense_kernel(int T, int kA, int kB, const double* __restrict__ w,
                                                         const double* __restrict__ Acat,
                                                         const double* __restrict__ Bcat,
                                                         double* __restrict__ M) {
  const long nr = (long)kA * kB;
  const long total = nr * nr;
  const long sa = (long)kA * kA, sb = (long)kB * kB;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long row = e / nr, col = e - row * nr;
    const int a = (int)(row / kB), b = (int)(row - (long)a * kB);
    const int a2 = (int)(col / kB), b2 = (int)(col - (long)a2 * kB);
    double acc = 0.0;
    for (int t = 0; t < T; ++t)
      acc += w[t] * Acat[t * sa + (long)a * kA + a2] * Bcat[t * sb + (long)b * kB + b2];
    M[e] = acc;
  }
}

unsigned grid_for(long elems) {
  return (unsigned)std::max<long>(1, std::min<long>((elems + 255) / 256, 8192));
}

}  // namespace

void pauli_batched(hipStream_t s, const PauliDesc* d, int P, long elems_max) {
  if (P <= 0 || elems_max <= 0) return;
  hipLaunchKernelGGL(pauli_batched_kernel, dim3(grid_for(elems_max), P), dim3(256), 0, s, d);
}

void lincomb_batched(hipStream_t s, const LinDesc* d, int P, long nmax) {
  if (P <= 0 || nmax <= 0) return;
  hipLaunchKernelGGL(lincomb_batched_kernel, dim3(grid_for(nmax), P), dim3(256), 0, s, d);
}

void full_diag(hipStream_t s, int n_sites, int nB, int n_terms, const FullTerm* terms,
               const double* pA, const double* pB, double sigma, double* D) {
  hipLaunchKernelGGL(full_diag_kernel, dim3(grid_for(1L << n_sites)), dim3(256), 0, s, n_sites, nB,
                     n_terms, terms, pA, pB, sigma, D);
}

void col_sumsq(hipStream_t s, int k, int D, const double* Psi, double* p) {
  hipLaunchKernelGGL(col_sumsq_kernel, dim3((D + 255) / 256), dim3(256), 0, s, k, D, Psi, p);
}

void kron_dense(hipStream_t s, int T, int kA, int kB, const double* w, const double* Acat,
                const double* Bcat, double* M) {
  const long nr = (long)kA * kB;
  hipLaunchKernelGGL(kron_dense_kernel, dim3(grid_for(nr * nr)), dim3(256), 0, s, T, kA, kB, w, Acat,
                     Bcat, M);
}

}  // namespace rmc
