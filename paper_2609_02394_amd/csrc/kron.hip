// Kronecker-sum matvec of one coupling step (the effective Hamiltonian of the
// assembled effective-Hamiltonian equation applied without forming it):
//
//   out_j = s1 * ( sum_i c_i O_A^i Y_j (O_B^i)^T + (E_A[a] + E_B[b]) .* Y_j )
//         + s2 * Y_j + s3 * Xprev_j
//
//         [ + s1 * phi_j * Ecorr_j ]
// for a block of vectors Y_j, each a k_A x k_B row-major coefficient matrix. The
// optional Ecorr term is the FP64 residual that drives the defect form of the
// Chebyshev filter in the FP32/BF16 forms (see solver.hip).
// (A (x) B) vec(X) = vec(A X B^T) for row-major vec, so this is exactly H_eff Y_j.
//
// Batched over problems (descriptor per problem, blockIdx.z). One workgroup
// (4 waves) owns one vector j and one 16-wide column tile
// [b0, b0+16) of the output:
//   stage 1: Z_i[:, tile] = Y_j (O_B^i[tile, :])^T   (k_A x 16, K = k_B) -> LDS
//   stage 2: acc[:, tile] = sum_i c_i O_A^i Z_i[:, tile]     (K = k_A)
//   epilogue: scale, diagonal, Chebyshev three-term recurrence, store FP64.
// Each wave owns the 16-row tiles w, w+4, ... in both stages. Operands come from
// global memory (L2-resident at these sizes); the MFMA K index is permuted so that
// every lane reads contiguous elements: within a K step, lane group g = lane/16
// takes a contiguous run of K instead of every fourth element (the sum over K is
// order-free up to rounding).
//
// Precisions: FP64 (v_mfma_f64_16x16x4_f64), FP32 (v_mfma_f32_16x16x4_f32) and
// BF16 inputs with FP32 accumulation (v_mfma_f32_16x16x32_bf16). Storage stays
// FP64; low precision applies to the products and their accumulation.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "rmc_batch.h"
#include "rmc_internal.h"

namespace rmc {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int KR_TCH = 4;  // terms per LDS chunk

template <int P>
struct KTraits;
template <>
struct KTraits<0> {  // FP64
  static constexpr int KS = 4;  // K per MFMA
  typedef double zt;
  typedef d4 acc;
};
template <>
struct KTraits<1> {  // FP32
  static constexpr int KS = 4;
  typedef float zt;
  typedef f4 acc;
};
template <>
struct KTraits<2> {  // BF16 in, FP32 accumulate
  static constexpr int KS = 32;
  typedef float zt;
  typedef f4 acc;
};

// Row of accumulator register r in lane group g: the FP64 16x16x4 instruction
// places D[4r+g][lane%16] in register r, the FP32 and BF16 ones D[4g+r][lane%16].
template <int P>
__device__ inline int acc_row(int g, int r) {
  return P == 0 ? 4 * r + g : 4 * g + r;
}

__device__ inline double ld_or0(const double* __restrict__ p, bool ok) { return ok ? *p : 0.0; }

// One MFMA step. a_run/b_run: the lane's contiguous K run (length L = KS/4 for
// FP64/FP32 -> 1 element per MFMA, 8 for BF16).
template <int P>
struct Mfma;
template <>
struct Mfma<0> {
  __device__ static inline d4 step(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<1> {
  __device__ static inline f4 step(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<2> {
  __device__ static inline f4 step(bf8 a, bf8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

// acc += A(rows r0.., K) * B(K, cols) with A(i,k) = Arow(i)[k] (row-major, ld lda,
// rows < M, k < K) scaled by `scale`, and B(k,j) supplied by a functor.
template <int P, class BFn>
__device__ inline typename KTraits<P>::acc mma_tile(typename KTraits<P>::acc acc,
                                                    const double* __restrict__ A, int lda, int row,
                                                    bool row_ok, int K, double scale, BFn bfn) {
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4;
  if constexpr (P == 0 || P == 1) {
    // K in chunks of 64: all operands of a chunk are loaded before its 16 MFMAs so
    // the loads overlap; two accumulators alternate so consecutive MFMAs do not
    // wait on each other. Within a step of 16, lane group g takes k = kb + 4g + s.
    typename KTraits<P>::acc acc2 = {0, 0, 0, 0};
    for (int kc = 0; kc < K; kc += 64) {
      double av[16], bv[16];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int k = kc + 16 * u + 4 * g + s;
          const bool ok = k < K;
          av[4 * u + s] = ld_or0(A + (long)row * lda + k, ok && row_ok);
          bv[4 * u + s] = ok ? bfn(k) : 0.0;
        }
#pragma unroll
      for (int u = 0; u < 16; u += 2) {
        if constexpr (P == 0) {
          acc = Mfma<0>::step(av[u] * scale, bv[u], acc);
          acc2 = Mfma<0>::step(av[u + 1] * scale, bv[u + 1], acc2);
        } else {
          acc = Mfma<1>::step((float)(av[u] * scale), (float)bv[u], acc);
          acc2 = Mfma<1>::step((float)(av[u + 1] * scale), (float)bv[u + 1], acc2);
        }
      }
    }
    acc += acc2;
  } else {
    // K step of 32: lane group g takes k = kb + 8g + s, s = 0..7
    for (int kb = 0; kb < K; kb += 32) {
      const int k0 = kb + 8 * g;
      bf8 a8, b8;
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int k = k0 + s;
        const bool ok = k < K;
        float av = (float)(ld_or0(A + (long)row * lda + k, ok && row_ok) * scale);
        float bv = ok ? (float)bfn(k) : 0.0f;
        a8[s] = (__bf16)av;
        b8[s] = (__bf16)bv;
      }
      acc = Mfma<2>::step(a8, b8, acc);
    }
  }
  return acc;
}

// Stage-1 product of one 16-row tile for up to KR_TCH terms: z[t] += Yrow . OBrow_t
// (K = kB), the Y operand loaded once per K chunk and shared by the terms.
template <int P>
__device__ inline void stage1_tile(typename KTraits<P>::acc* z, int tn, const double* __restrict__ yrow,
                                   bool rok, int K, const double* __restrict__ obrow, bool bok,
                                   long tstride) {
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4;
  if constexpr (P == 0 || P == 1) {
    for (int kc = 0; kc < K; kc += 64) {
      double av[16];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int k = kc + 16 * u + 4 * g + s;
          av[4 * u + s] = (rok && k < K) ? yrow[k] : 0.0;
        }
#pragma unroll
      for (int t = 0; t < KR_TCH; ++t) {
        if (t >= tn) break;
        const double* ob = obrow + t * tstride;
        double bv[16];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const int k = kc + 16 * u + 4 * g + s;
            bv[4 * u + s] = (bok && k < K) ? ob[k] : 0.0;
          }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          if constexpr (P == 0)
            z[t] = Mfma<0>::step(av[u], bv[u], z[t]);
          else
            z[t] = Mfma<1>::step((float)av[u], (float)bv[u], z[t]);
        }
      }
    }
  } else {
    for (int kc = 0; kc < K; kc += 32) {
      bf8 a8;
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int k = kc + 8 * g + s;
        a8[s] = (__bf16)(float)((rok && k < K) ? yrow[k] : 0.0);
      }
#pragma unroll
      for (int t = 0; t < KR_TCH; ++t) {
        if (t >= tn) break;
        const double* ob = obrow + t * tstride;
        bf8 b8;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const int k = kc + 8 * g + s;
          b8[s] = (__bf16)(float)((bok && k < K) ? ob[k] : 0.0);
        }
        z[t] = Mfma<2>::step(a8, b8, z[t]);
      }
    }
  }
}

// One workgroup: vector j of descriptor d, output columns [b0, b0+16).
template <int P>
__device__ void kron_body(const KronDesc& d, int j, int b0, char* smem_raw) {
  typedef typename KTraits<P>::zt zt;
  typedef typename KTraits<P>::acc accT;
  zt* Zs = reinterpret_cast<zt*>(smem_raw);  // [KR_TCH][kApad][16]
  const int kA = d.kA, kB = d.kB, T = d.T;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, l16 = lane & 15;
  const int n = kA * kB;
  const int RT = (kA + 15) >> 4;
  const int kApad = RT * 16;
  const double* Yj = d.Y + (long)j * n;

  constexpr int MAXRT = 4;  // row tiles per wave (kA <= 256)
  accT acc[MAXRT];
#pragma unroll
  for (int t = 0; t < MAXRT; ++t) acc[t] = accT{0, 0, 0, 0};

  for (int t0 = 0; t0 < T; t0 += KR_TCH) {
    const int tn = min(KR_TCH, T - t0);
    // stage 1: Z_i = Y_j (O_B^i[tile,:])^T, rows = a, cols = tile, K = kB; the rows
    // of Y_j are loaded once per K chunk for all terms of the chunk
    {
      const int bcol = b0 + l16;
      const bool bok = bcol < kB;
#pragma unroll
      for (int q = 0; q < MAXRT; ++q) {
        const int rt = wave + 4 * q;
        if (rt >= RT) break;
        const int row = rt * 16 + l16;
        const bool rok = row < kA;
        accT z[KR_TCH];
#pragma unroll
        for (int ti = 0; ti < KR_TCH; ++ti) z[ti] = accT{0, 0, 0, 0};
        stage1_tile<P>(z, tn, Yj + (long)row * kB, rok, kB,
                       d.OB + (long)t0 * kB * kB + (long)bcol * kB, bok, (long)kB * kB);
#pragma unroll
        for (int ti = 0; ti < KR_TCH; ++ti) {
          if (ti >= tn) break;
          zt* Zt = Zs + ((long)ti * kApad) * 16;
#pragma unroll
          for (int r = 0; r < 4; ++r) Zt[(rt * 16 + acc_row<P>(g, r)) * 16 + l16] = (zt)z[ti][r];
        }
      }
    }
    __syncthreads();
    // stage 2: acc += c_i O_A^i Z_i
    for (int ti = 0; ti < tn; ++ti) {
      const double* OAi = d.OA + (long)(t0 + ti) * kA * kA;
      const double ci = d.coef[t0 + ti];
      const zt* Zt = Zs + ((long)ti * kApad) * 16;
#pragma unroll
      for (int q = 0; q < MAXRT; ++q) {
        const int rt = wave + 4 * q;
        if (rt >= RT) break;
        const int row = rt * 16 + l16;
        acc[q] = mma_tile<P>(acc[q], OAi, kA, row, row < kA, kA, ci,
                             [&](int k) -> double { return (double)Zt[k * 16 + l16]; });
      }
    }
    __syncthreads();
  }
  // epilogue: register r of each row tile holds row acc_row<P>(g, r), column l16
  const int col = b0 + l16;
  if (col >= kB) return;
  const double* Xp = d.Xprev ? d.Xprev + (long)j * n : nullptr;
  const double* Ej = d.E ? d.E + (long)j * n : nullptr;
  const double ph = d.E ? d.s1 * d.phi[j] : 0.0;
  double* oj = d.out + (long)j * n;
#pragma unroll
  for (int q = 0; q < MAXRT; ++q) {
    const int rt = wave + 4 * q;
    if (rt >= RT) break;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = rt * 16 + acc_row<P>(g, r);
      if (row >= kA) continue;
      const long idx = (long)row * kB + col;
      const double y = Yj[idx];
      double v = d.s1 * ((double)acc[q][r] + d.Ediag[idx] * y) + d.s2 * y;
      if (Xp) v += d.s3 * Xp[idx];
      if (Ej) v += ph * Ej[idx];
      oj[idx] = v;
    }
  }
}

template <int P>
__global__ __launch_bounds__(256) void kron_batched_kernel(const KronDesc* __restrict__ descs) {
  extern __shared__ char smem_raw[];
  const KronDesc d = descs[blockIdx.z];
  const int j = blockIdx.y, b0 = blockIdx.x * 16;
  if (j >= d.nv || b0 >= d.kB) return;
  kron_body<P>(d, j, b0, smem_raw);
}

static size_t kron_lds_bytes(int kA, int prec) {
  int kApad = ((kA + 15) / 16) * 16;
  size_t el = prec == 0 ? sizeof(double) : sizeof(float);
  return (size_t)KR_TCH * kApad * 16 * el;
}

int kron_max_k() { return 256; }

void kron_set_attrs() {
  const int lds = 160 * 1024 - 1024;
  hipFuncSetAttribute(reinterpret_cast<const void*>(&kron_batched_kernel<0>),
                      hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  hipFuncSetAttribute(reinterpret_cast<const void*>(&kron_batched_kernel<1>),
                      hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  hipFuncSetAttribute(reinterpret_cast<const void*>(&kron_batched_kernel<2>),
                      hipFuncAttributeMaxDynamicSharedMemorySize, lds);
}

void kron_batched(hipStream_t s, const KronDesc* d, int P, int kBmax, int nvmax, int kAmax,
                  int precision) {
  if (P <= 0 || nvmax <= 0 || kBmax <= 0) return;
  dim3 grid((kBmax + 15) / 16, nvmax, P);
  size_t lds = kron_lds_bytes(kAmax, precision);
  switch (precision) {
    case RMC_FP64:
      hipLaunchKernelGGL(kron_batched_kernel<0>, grid, dim3(256), lds, s, d);
      break;
    case RMC_FP32:
      hipLaunchKernelGGL(kron_batched_kernel<1>, grid, dim3(256), lds, s, d);
      break;
    default:
      hipLaunchKernelGGL(kron_batched_kernel<2>, grid, dim3(256), lds, s, d);
      break;
  }
}

}  // namespace rmc
