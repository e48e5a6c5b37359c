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
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>

#include "rmc_batch.h"
#include "rmc_internal.h"

namespace rmc {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

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

// Lane-run operand loads. Within a K chunk (64 for FP64/FP32, 32 for BF16) lane
// group g = lane/16 takes a contiguous run of K: for FP64/FP32 step u (0..3) of the
// chunk covers k = kc + 16u + 4g + s (s = 0..3, one MFMA per (u, s)); for BF16 the
// chunk is one MFMA with k = kc + 8g + s (s = 0..7).
template <int P>
struct Run;
// The loads sit in branches whose result is only used after the last of them (the
// scaling and conversion come afterwards), so a run's loads issue together instead of
// waiting one by one.
template <>
struct Run<0> {
  double v[16];
  __device__ void load(const double* __restrict__ row, bool ok, int kc, int K, double scale, int g) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = kc + 16 * u + 4 * g + s;
        double x = 0.0;
        if (ok && k < K) x = row[k];
        v[4 * u + s] = x;
      }
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] *= scale;
  }
  template <class F>
  __device__ void load_fn(F f, int kc, int K, int g) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = kc + 16 * u + 4 * g + s;
        double x = 0.0;
        if (k < K) x = f(k);
        v[4 * u + s] = x;
      }
  }
};
template <>
struct Run<1> {
  float v[16];
  __device__ void load(const double* __restrict__ row, bool ok, int kc, int K, double scale, int g) {
    double x[16];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = kc + 16 * u + 4 * g + s;
        x[4 * u + s] = 0.0;
        if (ok && k < K) x[4 * u + s] = row[k];
      }
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = (float)(x[i] * scale);
  }
  template <class F>
  __device__ void load_fn(F f, int kc, int K, int g) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = kc + 16 * u + 4 * g + s;
        double x = 0.0;
        if (k < K) x = f(k);
        v[4 * u + s] = (float)x;
      }
  }
};
template <>
struct Run<2> {
  bf8 v;
  __device__ void load(const double* __restrict__ row, bool ok, int kc, int K, double scale, int g) {
    double x[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int k = kc + 8 * g + s;
      x[s] = 0.0;
      if (ok && k < K) x[s] = row[k];
    }
#pragma unroll
    for (int s = 0; s < 8; ++s) v[s] = (__bf16)(float)(x[s] * scale);
  }
  template <class F>
  __device__ void load_fn(F f, int kc, int K, int g) {
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int k = kc + 8 * g + s;
      double x = 0.0;
      if (k < K) x = f(k);
      v[s] = (__bf16)(float)x;
    }
  }
};

template <int P>
__device__ inline void mma_run(typename KTraits<P>::acc& c, const Run<P>& a, const Run<P>& b) {
  if constexpr (P == 2) {
    c = Mfma<2>::step(a.v, b.v, c);
  } else {
#pragma unroll
    for (int u = 0; u < 16; ++u) c = Mfma<P>::step(a.v[u], b.v[u], c);
  }
}

template <int P>
constexpr int kchunk() {
  return P == 2 ? 32 : 64;
}

// One workgroup: vector j of descriptor d, output columns [b0, b0 + 16 CT). Each
// wave owns the 16-row tiles w, w+4, ... (at most MRT) and all CT column sub-tiles
// of them, so a row operand loaded once feeds CT products. Terms go through LDS
// in chunks of TCH = 4/CT.
template <int P, int CT, int MRT>
__device__ void kron_body(const KronDesc& d, int j, int b0, char* smem_raw) {
  typedef typename KTraits<P>::zt zt;
  typedef typename KTraits<P>::acc accT;
  constexpr int TCH = 4 / CT;
  constexpr int W = 16 * CT;  // LDS row width of Z
  constexpr int KC = kchunk<P>();
  zt* Zs = reinterpret_cast<zt*>(smem_raw);  // [TCH][kApad][W]
  const int kA = d.kA, kB = d.kB, T = d.T;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, l16 = lane & 15;
  const int n = kA * kB;
  const int RT = (kA + 15) >> 4;
  const int kApad = RT * 16;
  const double* Yj = d.Y + (long)j * n;

  accT acc[MRT][CT];
#pragma unroll
  for (int q = 0; q < MRT; ++q)
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[q][c] = accT{0, 0, 0, 0};

  for (int t0 = 0; t0 < T; t0 += TCH) {
    const int tn = min(TCH, T - t0);
    // stage 1: Z_t[:, tile] = Y_j (O_B^t[tile, :])^T, K = kB
#pragma unroll
    for (int q = 0; q < MRT; ++q) {
      const int rt = wave + 4 * q;
      if (rt >= RT) break;
      const int row = rt * 16 + l16;
      const bool rok = row < kA;
      accT z[CT][TCH];
#pragma unroll
      for (int c = 0; c < CT; ++c)
#pragma unroll
        for (int t = 0; t < TCH; ++t) z[c][t] = accT{0, 0, 0, 0};
      for (int kc = 0; kc < kB; kc += KC) {
        Run<P> a;
        a.load(Yj + (long)row * kB, rok, kc, kB, 1.0, g);
#pragma unroll
        for (int c = 0; c < CT; ++c) {
          const int bcol = b0 + 16 * c + l16;
          const bool bok = bcol < kB;
#pragma unroll
          for (int t = 0; t < TCH; ++t) {
            if (t >= tn) break;
            Run<P> b;
            b.load(d.OB + (long)(t0 + t) * kB * kB + (long)bcol * kB, bok, kc, kB, 1.0, g);
            mma_run<P>(z[c][t], a, b);
          }
        }
      }
#pragma unroll
      for (int t = 0; t < TCH; ++t) {
        if (t >= tn) break;
        zt* Zt = Zs + (long)t * kApad * W;
#pragma unroll
        for (int c = 0; c < CT; ++c)
#pragma unroll
          for (int r = 0; r < 4; ++r) Zt[(rt * 16 + acc_row<P>(g, r)) * W + 16 * c + l16] = (zt)z[c][t][r];
      }
    }
    __syncthreads();
    // stage 2: acc += c_t O_A^t Z_t, K = kA
    for (int t = 0; t < tn; ++t) {
      const double* OAt = d.OA + (long)(t0 + t) * kA * kA;
      const double ct = d.coef[t0 + t];
      const zt* Zt = Zs + (long)t * kApad * W;
#pragma unroll
      for (int q = 0; q < MRT; ++q) {
        const int rt = wave + 4 * q;
        if (rt >= RT) break;
        const int row = rt * 16 + l16;
        for (int kc = 0; kc < kA; kc += KC) {
          Run<P> a;
          a.load(OAt + (long)row * kA, row < kA, kc, kA, ct, g);
#pragma unroll
          for (int c = 0; c < CT; ++c) {
            Run<P> b;
            b.load_fn([&](int k) -> double { return (double)Zt[k * W + 16 * c + l16]; }, kc, kA, g);
            mma_run<P>(acc[q][c], a, b);
          }
        }
      }
    }
    __syncthreads();
  }
  // epilogue: register r of a tile holds row acc_row<P>(g, r), column l16 of its sub-tile
  const double* Xp = d.Xprev ? d.Xprev + (long)j * n : nullptr;
  const double* Ej = d.E ? d.E + (long)j * n : nullptr;
  const double ph = d.E ? d.s1 * d.phi[j] : 0.0;
  double* oj = d.out + (long)j * n;
#pragma unroll
  for (int q = 0; q < MRT; ++q) {
    const int rt = wave + 4 * q;
    if (rt >= RT) break;
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      const int col = b0 + 16 * c + l16;
      // the sub-tile's operands first (loaded together), then the outputs
      double yv[4], dv[4], xv[4], ev[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rt * 16 + acc_row<P>(g, r);
        const long idx = (long)row * kB + col;
        yv[r] = dv[r] = xv[r] = ev[r] = 0.0;
        if (row < kA && col < kB) {
          yv[r] = Yj[idx];
          dv[r] = d.Ediag[idx];
          if (Xp) xv[r] = Xp[idx];
          if (Ej) ev[r] = Ej[idx];
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rt * 16 + acc_row<P>(g, r);
        if (row >= kA || col >= kB) continue;
        const long idx = (long)row * kB + col;
        const double y = yv[r];
        double v = d.s1 * ((double)acc[q][c][r] + dv[r] * y) + d.s2 * y;
        if (Xp) v += d.s3 * xv[r];
        if (Ej) v += ph * ev[r];
        oj[idx] = v;
      }
    }
  }
}

template <int P, int CT, int MRT>
__global__ __launch_bounds__(256) void kron_batched_kernel(const KronDesc* __restrict__ descs) {
  extern __shared__ char smem_raw[];
  const KronDesc d = descs[blockIdx.z];
  const int j = blockIdx.y, b0 = blockIdx.x * 16 * CT;
  if (j >= d.nv || b0 >= d.kB) return;
  kron_body<P, CT, MRT>(d, j, b0, smem_raw);
}

// ---- streaming variant (k_A, k_B <= KM) ----------------------------------------------
// A persistent grid: workgroup L owns the launch-wide vectors [L V / G, (L+1) V / G)
// (V vectors over all descriptors, G workgroups) and walks them one (vector, term)
// step at a time. The padded KM x KM tiles of one step live in LDS in the MFMA
// input type: Bs = O_B^t, As = c_t O_A^t and Zt = Z^T, so every MFMA operand is one
// contiguous K run of an LDS row (vector LDS reads):
//   stage 1: Z = Y_j (O_B^t)^T   A operand: rows of Y_j (registers), B: rows of Bs
//   stage 2: acc += As Z         A operand: rows of As, B: rows of Zt
// Wave (rt, cw) owns row tile rt and column tiles [cw CPW, (cw+1) CPW) of Z and of
// the output. The operators of the next step are loaded from global memory into
// registers while the current step computes and are written to LDS behind the two
// barriers of the step (O_B in flight during stage 1 and stored after it, c O_A in
// flight during stage 2 and stored after it); the rows of the next vector are
// prefetched the same way. Logical workgroups are spread so that each
// XCD (hardware workgroup id mod 8) owns a contiguous run of vectors, which keeps
// one problem's operators in one L2. Tiles are zero-padded to KM, so the K loops
// unroll fully and padded rows and columns contribute exact zeros.
template <int P>
struct SK;
template <>
struct SK<0> {
  typedef double lt;  // LDS / operand element
  typedef d4 acc;
  static constexpr int KR = 4;   // contiguous K per lane per chunk
  static constexpr int CH = 16;  // K per chunk
};
template <>
struct SK<1> {
  typedef float lt;
  typedef f4 acc;
  static constexpr int KR = 4;
  static constexpr int CH = 16;
};
template <>
struct SK<2> {
  typedef __bf16 lt;
  typedef f4 acc;
  static constexpr int KR = 8;
  static constexpr int CH = 32;
};

template <int P>
constexpr int sk_pitch(int KM) {
  return KM + 16 / (int)sizeof(typename SK<P>::lt);  // 16-byte row padding
}

// Rounds to the element type through FP32 (for BF16: RNE to FP32, then RNE to BF16;
// the empty asm keeps the compiler from fusing the two into one slower rounding).
template <int P>
__device__ inline typename SK<P>::lt to_lt(double x) {
  if constexpr (P == 0) {
    return x;
  } else if constexpr (P == 1) {
    return (float)x;
  } else {
    float f = (float)x;
    asm volatile("" : "+v"(f));
    return (__bf16)f;
  }
}

// Global-address-space views: loads through them compile to global (not flat)
// memory instructions, which LDS waits do not have to drain.
template <class T>
using gptr = const __attribute__((address_space(1))) T*;
template <class T>
using gptr_w = __attribute__((address_space(1))) T*;
template <class T>
__device__ inline gptr<T> gview(const T* p) {
  return (gptr<T>)p;
}
template <class T>
__device__ inline gptr_w<T> gview_w(T* p) {
  return (gptr_w<T>)p;
}

// Four consecutive tile elements (the unit of the staging copies) as one vector.
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
template <int P>
struct Grp;
template <>
struct Grp<0> {
  typedef d4 t;
};
template <>
struct Grp<1> {
  typedef f4 t;
};
template <>
struct Grp<2> {
  typedef bf4 t;
};

// The KR-element K run of chunk u of an LDS row for lane group g.
template <int P>
struct Frag {
  typename SK<P>::lt v[SK<P>::KR];
  __device__ void load(const typename SK<P>::lt* row, int u, int g) {
    const typename SK<P>::lt* q = row + SK<P>::CH * u + SK<P>::KR * g;
    if constexpr (P == 0) {
      const double2 a = *reinterpret_cast<const double2*>(q);
      const double2 b = *reinterpret_cast<const double2*>(q + 2);
      v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    } else if constexpr (P == 1) {
      const float4 a = *reinterpret_cast<const float4*>(q);
      v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    } else {
      const uint4 a = *reinterpret_cast<const uint4*>(q);
      *reinterpret_cast<uint4*>(v) = a;
    }
  }
};

template <int P>
__device__ inline void mma_frag(typename SK<P>::acc& c, const typename SK<P>::lt* a, const Frag<P>& b) {
  if constexpr (P == 2) {
    bf8 av, bv;
#pragma unroll
    for (int e = 0; e < 8; ++e) { av[e] = a[e]; bv[e] = b.v[e]; }
    c = Mfma<2>::step(av, bv, c);
  } else {
#pragma unroll
    for (int s = 0; s < 4; ++s) c = Mfma<P>::step(a[s], b.v[s], c);
  }
}

// Two workgroups share a CU where their LDS fits (the SH forms up to KM = 96), else one.
template <int P, int KM, bool SH>
constexpr int sk_blocks_per_cu() {
  return SH && 2 * 2 * KM * sk_pitch<P>(KM) * (int)sizeof(typename SK<P>::lt) <= 160 * 1024 ? 2 : 1;
}

template <int P, int KM, int NWC, bool SH>
__global__ __launch_bounds__(64 * (KM / 16) * NWC, (sk_blocks_per_cu<P, KM, SH>())) void kron_stream_kernel(
    const KronDesc* __restrict__ descs, int P_, long V, int G) {
  typedef typename SK<P>::lt lt;
  typedef typename SK<P>::acc accT;
  constexpr int RTM = KM / 16;            // row (and column) tiles
  constexpr int CPW = RTM / NWC;          // column tiles per wave
  constexpr int NT = 64 * RTM * NWC;      // threads
  constexpr int PW = sk_pitch<P>(KM);
  constexpr int KR = SK<P>::KR, CH = SK<P>::CH;
  constexpr int NCH = KM / CH;            // K chunks
  constexpr int NYE = KM / 4;             // Y elements per lane (NCH * KR)
  constexpr int NG = KM * KM / (4 * NT);  // 4-element staging groups per thread per matrix
  // epilogue prefetch where the registers allow it (the FP64 single-buffer forms and
  // the widest tiles are at the register limit already); the next vector's rows are
  // prefetched up to KM = 96 and loaded at the vector boundary beyond
  constexpr bool EPF = KM <= 64 && !(P == 0 && NWC == 1);
  // FP64 at KM = 96: the vector's rows (stage 1's A operand) are read from L2 chunk by
  // chunk instead of being held in registers (24 doubles a lane would spill)
  constexpr bool YG = P == 0 && KM > 64;
  constexpr bool YPF = KM <= 96 && !YG;
  // the epilogue's loads of a column tile issued together (where the registers allow;
  // elsewhere each element's loads go out alone)
  constexpr bool EPB = YG || EPF || KM == 128;
  static_assert(RTM % NWC == 0 && NG * 4 * NT == KM * KM, "tile split");
  extern __shared__ char smem_raw[];
  lt* Bs = reinterpret_cast<lt*>(smem_raw);
  lt* As = SH ? Bs : Bs + KM * PW;  // SH: one buffer holds O_B, then c O_A, of a step
  lt* Zt = As + KM * PW;

  // XCD x (blockIdx % 8) owns the launch's vectors [x V/8, (x+1) V/8); its GX
  // workgroups take them in turn, so that at any time they work on neighbouring
  // vectors, mostly of one problem, whose operator tiles its L2 serves to all of them
  const int w = blockIdx.x;
  const int GX = G >> 3;
  const long v0 = (long)(w & 7) * V / 8 + (w >> 3), v1 = (long)((w & 7) + 1) * V / 8;
  if (v0 >= v1) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, l16 = lane & 15;
  const int rt = wave / NWC, c0 = (wave % NWC) * CPW;

  // descriptor of vector v0: the last one whose vbase <= v0 (empty ones share vbase)
  int p = 0;
  {
    int lo = 0, hi = P_ - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (descs[mid].vbase <= v0) lo = mid;
      else hi = mid - 1;
    }
    p = lo;
  }
  int j = (int)(v0 - descs[p].vbase), t = 0;
  long v = v0;

  typedef typename Grp<P>::t gv;
  gv pf[NG];  // next operator tile in flight (O_B, then c O_A)
  auto load_tile = [&](const KronDesc* e, int tt, bool isA) {
    const int pk = e->pkm;
    const bool on = tt < e->T;
    // a term-less descriptor has no pack: read nothing and stage zeros
    gptr<lt> base = on ? gview(static_cast<const lt*>(e->pack)) + ((long)tt * 2 + (isA ? 1 : 0)) * pk * pk
                       : nullptr;
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      const int q = tid + i * NT, r = q / (KM / 4), cc = (q % (KM / 4)) * 4;
      const bool in = on && r < pk && cc < pk;
      gv x = gv{0, 0, 0, 0};
      if (in) x = *reinterpret_cast<gptr<gv>>(base + r * pk + cc);
      pf[i] = x;
    }
  };
  auto store_tile = [&](lt* dst) {
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      const int q = tid + i * NT, r = q / (KM / 4), cc = (q % (KM / 4)) * 4;
      lt* o = dst + r * PW + cc;
      if constexpr (P == 0) {  // rows are 16-byte aligned
        *reinterpret_cast<double2*>(o) = double2{pf[i][0], pf[i][1]};
        *reinterpret_cast<double2*>(o + 2) = double2{pf[i][2], pf[i][3]};
      } else {
        *reinterpret_cast<gv*>(o) = pf[i];
      }
    }
  };
  lt yf[YG ? 1 : NYE], yn[YPF ? NYE : 1];
  auto load_y = [&](const KronDesc* e, int jj, lt* dst) {
    const int kA = e->kA, kB = e->kB;
    gptr<double> Y = gview(e->Y) + (long)jj * kA * kB;
    const int a = rt * 16 + l16;
#pragma unroll
    for (int u = 0; u < NCH; ++u)
#pragma unroll
      for (int x = 0; x < KR; ++x) {
        const int k = CH * u + KR * g + x;
        const bool in = a < kA && k < kB;
        const double y = Y[in ? (long)a * kB + k : 0];
        dst[u * KR + x] = to_lt<P>(in ? y : 0.0);
      }
  };

  load_tile(descs + p, 0, false);
  store_tile(Bs);
  if constexpr (!SH) {
    load_tile(descs + p, 0, true);
    store_tile(As);
  }
  if constexpr (!YG) load_y(descs + p, j, yf);
  __syncthreads();
  accT acc[CPW];
  while (true) {
    const KronDesc* d = descs + p;
    const int Td = d->T > 0 ? d->T : 1;
    // coordinates of the next step
    bool has_next = true;
    int nj = j, nt = t + 1, np = p;
    if (nt >= Td) {
      nt = 0;
      if (v + GX >= v1) {
        has_next = false;
      } else {
        nj = j + GX;
        while (nj >= descs[np].nv) {
          nj -= descs[np].nv;
          ++np;
        }
      }
    }
    const KronDesc* nd = descs + np;
    if constexpr (SH) load_tile(d, t, true);  // this step's c O_A, stored after stage 1
    else if (has_next) load_tile(nd, nt, false);
    if constexpr (YPF)
      if (has_next && nt == 0) load_y(nd, nj, yn);
    if (t == 0) {
#pragma unroll
      for (int c = 0; c < CPW; ++c) acc[c] = accT{0, 0, 0, 0};
    }
    // stage 1: Z tile = Y rows x (O_B rows)^T -> Zt
    {
      accT z[CPW];
#pragma unroll
      for (int c = 0; c < CPW; ++c) z[c] = accT{0, 0, 0, 0};
      if constexpr (YG) {
        // the row's next chunk is in flight while the current one computes (two buffers
        // taken in turn, so no register copy waits for a load); the loads are
        // unconditional: a padded entry, or the chunk after the last (k >= KM >= kB),
        // reads the row's first element, which is dropped
        static_assert(NCH % 2 == 0, "chunk pairs");
        const int kA = d->kA, kB = d->kB;
        const int a = rt * 16 + l16;
        const bool ain = a < kA;
        gptr<double> Yr = gview(d->Y) + (long)j * kA * kB + (long)(ain ? a : 0) * kB;
        double y0[KR], y1[KR];
        auto ld = [&](double* yb, int u) {
#pragma unroll
          for (int x = 0; x < KR; ++x) {
            const int k = CH * u + KR * g + x;
            yb[x] = Yr[k < kB ? k : 0];
          }
        };
        auto mm = [&](const double* yb, int u) {
          lt ya[KR];
#pragma unroll
          for (int x = 0; x < KR; ++x) {
            const int k = CH * u + KR * g + x;
            ya[x] = (ain && k < kB) ? yb[x] : 0.0;
          }
#pragma unroll
          for (int c = 0; c < CPW; ++c) {
            Frag<P> b;
            b.load(Bs + ((c0 + c) * 16 + l16) * PW, u, g);
            mma_frag<P>(z[c], ya, b);
          }
        };
        ld(y0, 0);
#pragma unroll 1
        for (int u = 0; u < NCH; u += 2) {
          ld(y1, u + 1);
          __builtin_amdgcn_sched_barrier(0);  // the scheduler keeps the loads ahead
          mm(y0, u);
          ld(y0, u + 2);
          __builtin_amdgcn_sched_barrier(0);
          mm(y1, u + 1);
        }
      } else {
#pragma unroll
        for (int u = 0; u < NCH; ++u)
#pragma unroll
          for (int c = 0; c < CPW; ++c) {
            Frag<P> b;
            b.load(Bs + ((c0 + c) * 16 + l16) * PW, u, g);
            mma_frag<P>(z[c], yf + u * KR, b);
          }
      }
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        lt* zr = Zt + ((c0 + c) * 16 + l16) * PW + rt * 16;
        if constexpr (P == 0) {
#pragma unroll
          for (int r = 0; r < 4; ++r) zr[acc_row<0>(g, r)] = z[c][r];
        } else if constexpr (P == 1) {
          *reinterpret_cast<float4*>(zr + 4 * g) = float4{z[c][0], z[c][1], z[c][2], z[c][3]};
        } else {
          lt h[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) h[r] = (__bf16)z[c][r];
          *reinterpret_cast<uint2*>(zr + 4 * g) = *reinterpret_cast<const uint2*>(h);
        }
      }
    }
    __syncthreads();
    if constexpr (SH) {
      store_tile(As);
      __syncthreads();
      if (has_next) load_tile(nd, nt, false);
    } else if (has_next) {
      store_tile(Bs);
      load_tile(nd, nt, true);
    }
    // On a vector's last step, the epilogue's HBM operands (previous iterate and
    // defect term) are loaded before stage 2 so that stage 2 hides their latency.
    const bool last = t == Td - 1;
    double exq[EPF ? CPW : 1][4], eeq[EPF ? CPW : 1][4];
    if constexpr (EPF) {
      if (last) {
        const int kA = d->kA, kB = d->kB;
        const long n = (long)kA * kB;
        gptr<double> Xp = d->Xprev ? gview(d->Xprev) + (long)j * n : nullptr;
        gptr<double> Ej = d->E ? gview(d->E) + (long)j * n : nullptr;
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
          const int col = (c0 + c) * 16 + l16;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = rt * 16 + acc_row<P>(g, r);
            const long idx = (row < kA && col < kB) ? (long)row * kB + col : 0;
            exq[c][r] = Xp ? Xp[idx] : 0.0;
            eeq[c][r] = Ej ? Ej[idx] : 0.0;
          }
        }
      }
    }
    // stage 2: acc += As rows x Z
#pragma unroll
    for (int u = 0; u < NCH; ++u) {
      Frag<P> a;
      a.load(As + (rt * 16 + l16) * PW, u, g);
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        Frag<P> b;
        b.load(Zt + ((c0 + c) * 16 + l16) * PW, u, g);
        mma_frag<P>(acc[c], a.v, b);
      }
    }
    if (last) {
      const int kA = d->kA, kB = d->kB, n = kA * kB;
      const double s1 = d->s1, s2 = d->s2, s3 = d->s3;
      gptr<double> Yj = gview(d->Y) + (long)j * n;
      gptr<double> Ed = gview(d->Ediag);
      gptr<double> Xp = d->Xprev ? gview(d->Xprev) + (long)j * n : nullptr;
      gptr<double> Ej = d->E ? gview(d->E) + (long)j * n : nullptr;
      const double ph = d->E ? s1 * d->phi[j] : 0.0;
      gptr_w<double> oj = gview_w(d->out) + (long)j * n;
      // one column tile at a time: its operands are loaded unconditionally (a padded
      // element reads element 0 and drops it), so they issue together
#pragma unroll
      for (int c = 0; c < (EPB ? CPW : 0); ++c) {
        const int col = (c0 + c) * 16 + l16;
        double yv[4], dv[4], xv[4], ev[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = rt * 16 + acc_row<P>(g, r);
          const long idx = (row < kA && col < kB) ? (long)row * kB + col : 0;
          yv[r] = Yj[idx];
          dv[r] = Ed[idx];
          if constexpr (EPF) {
            xv[r] = exq[c][r];
            ev[r] = eeq[c][r];
          } else {
            xv[r] = Xp ? Xp[idx] : 0.0;
            ev[r] = Ej ? Ej[idx] : 0.0;
          }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = rt * 16 + acc_row<P>(g, r);
          if (row < kA && col < kB) {
            const long idx = (long)row * kB + col;
            const double y = yv[r];
            // explicit fused multiply-adds: the fused filter kernel rounds the same way
            double o = fma(s1, fma(dv[r], y, (double)acc[c][r]), s2 * y);
            if (Xp) o = fma(s3, xv[r], o);
            if (Ej) o = fma(ph, ev[r], o);
            oj[idx] = o;
          }
        }
      }
#pragma unroll
      for (int c = 0; c < (EPB ? 0 : CPW); ++c) {
        const int col = (c0 + c) * 16 + l16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = rt * 16 + acc_row<P>(g, r);
          if (row < kA && col < kB) {
            const long idx = (long)row * kB + col;
            const double y = Yj[idx];
            double o = fma(s1, fma(Ed[idx], y, (double)acc[c][r]), s2 * y);
            if (Xp) o = fma(s3, Xp[idx], o);
            if (Ej) o = fma(ph, Ej[idx], o);
            oj[idx] = o;
          }
        }
      }
    }
    __syncthreads();
    if (!has_next) break;
    if constexpr (SH) {
      store_tile(Bs);
      __syncthreads();
    } else {
      store_tile(As);
    }
    if (nt == 0) {
      if constexpr (YPF) {
#pragma unroll
        for (int e = 0; e < NYE; ++e) yf[e] = yn[e];
      } else if constexpr (!YG) {
        load_y(nd, nj, yf);  // every wave is past its last read of yf (barrier above)
      }
      v += GX;
    }
    p = np;
    j = nj;
    t = nt;
  }
}

// ---- fused Chebyshev filter ---------------------------------------------------------
__device__ inline int tid_of() { return threadIdx.x; }

// Every step of the filter's recurrence acts on each vector alone, so one workgroup
// carries a vector through all of its steps: the FP64 iterates D_k, D_{k-1}, the
// defect E_j and the diagonal stay in registers (one 16 x 16 tile per wave, in the
// accumulator layout), the low-precision copy of D_k that feeds the MFMAs sits in
// LDS, and the problem's 2T operator tiles are resident in LDS for as long as the
// workgroup stays on that problem. HBM sees E_j and X_j once and out_j once per
// vector instead of four vectors per step. Per step and term: stage 1 (Z = D O_B^T,
// stored transposed, double-buffered across terms) and stage 2 (acc += c O_A Z),
// one barrier after each stage 1 and one after the new iterate is written.
// The arithmetic is that of the per-step kernel in the same order.
//
// RES = false is the form for operators too large to stay resident: LDS holds the
// iterate, one Z^T buffer and the current term's two operator tiles; the next term's
// tiles are loaded into registers while the current term computes and are stored
// behind its two barriers (O_B after stage 1, c O_A after stage 2).
template <int P, int KM, int CPW, bool RES>
__global__ __launch_bounds__(64 * (KM / 16) * (KM / 16) / CPW) void kron_filter_kernel(
    const FilterDesc* __restrict__ descs, int P_, long V, int G) {
  typedef typename SK<P>::lt lt;
  typedef typename SK<P>::acc accT;
  typedef typename Grp<P>::t gv;
  constexpr int RTM = KM / 16;
  constexpr int NWR = RTM / CPW;  // waves per row tile; wave (rt, cw) owns CPW column tiles
  constexpr int NT = 64 * RTM * NWR;
  constexpr int PW = sk_pitch<P>(KM);
  constexpr int NCH = KM / SK<P>::CH;
  constexpr int TILE = KM * PW;
  constexpr int NG = RES ? 1 : KM * KM / (4 * NT);  // streamed form: staging groups per thread
  // one tile per wave holds the defect and the diagonal in registers; with more tiles
  // per wave they are re-read each step (L2-resident) to stay within the registers
  constexpr bool HOLD = CPW == 1;
  static_assert(RTM % CPW == 0, "column tiles per wave");
  static_assert(RES || NG * 4 * NT == KM * KM, "tile staging");
  extern __shared__ char smem_raw[];
  lt* Ys = reinterpret_cast<lt*>(smem_raw);
  lt* Zt0 = Ys + TILE;
  // resident: tile 2t O_B^t, tile 2t+1 c_t O_A^t; streamed: the current term's pair
  lt* Ops = Zt0 + (RES ? 2 : 1) * TILE;
  gv pfB[NG], pfA[NG];
  // streamed form: term tt of problem e into the staging registers (zeros past pkm)
  auto fetch = [&](const FilterDesc* e, int tt) {
    gptr<lt> base = gview(static_cast<const lt*>(e->pack)) + (long)tt * 2 * e->pkm * e->pkm;
    const int pkm = e->pkm;
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      const int q = tid_of() + i * NT, r = q / (KM / 4), cc = (q % (KM / 4)) * 4;
      gv xb = gv{0, 0, 0, 0}, xa = gv{0, 0, 0, 0};
      if (r < pkm && cc < pkm) {
        xb = *reinterpret_cast<gptr<gv>>(base + r * pkm + cc);
        xa = *reinterpret_cast<gptr<gv>>(base + (long)pkm * pkm + r * pkm + cc);
      }
      pfB[i] = xb;
      pfA[i] = xa;
    }
  };
  auto put = [&](lt* dst, const gv* pf) {
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      const int q = tid_of() + i * NT, r = q / (KM / 4), cc = (q % (KM / 4)) * 4;
      lt* o = dst + r * PW + cc;
      if constexpr (P == 0) {
        *reinterpret_cast<double2*>(o) = double2{pf[i][0], pf[i][1]};
        *reinterpret_cast<double2*>(o + 2) = double2{pf[i][2], pf[i][3]};
      } else {
        *reinterpret_cast<gv*>(o) = pf[i];
      }
    }
  };
  int staged = -1;  // streamed form: problem whose term-0 tiles sit in LDS

  // XCD x (blockIdx % 8) owns the launch's vectors [x V/8, (x+1) V/8). Resident form:
  // each of its GX workgroups takes a contiguous run (fewer operator loads into LDS);
  // streamed form: they take the vectors in turn, so that at any time they work on
  // neighbouring vectors of mostly one problem and share its tiles in L2
  const int w = blockIdx.x;
  const int GX = G >> 3;
  const int vs = RES ? 1 : GX;
  long v0, v1;
  if constexpr (RES) {
    const int L = (w & 7) * GX + (w >> 3);
    v0 = (long)L * V / G;
    v1 = (long)(L + 1) * V / G;
  } else {
    v0 = (long)(w & 7) * V / 8 + (w >> 3);
    v1 = (long)((w & 7) + 1) * V / 8;
  }
  if (v0 >= v1) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, l16 = lane & 15;
  const int rt = wave / NWR, c0 = (wave % NWR) * CPW;

  int p = 0;
  {
    int lo = 0, hi = P_ - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (descs[mid].vbase <= v0) lo = mid;
      else hi = mid - 1;
    }
    p = lo;
  }
  int j = (int)(v0 - descs[p].vbase);
  int loaded = -1;
  for (long v = v0; v < v1; v += vs) {
    while (j >= descs[p].nv) {
      j -= descs[p].nv;
      ++p;
    }
    const FilterDesc* d = descs + p;
    const int kA = d->kA, kB = d->kB, T = d->T, steps = d->steps, nv = d->nv;
    const long n = (long)kA * kB;
    if (RES && loaded != p) {
      __syncthreads();  // every wave is done with the previous operators
      // the pack's tiles are pkm x pkm (the problem's own padded size, <= KM): rows and
      // columns past pkm are staged as zeros
      gptr<lt> pk = gview(static_cast<const lt*>(d->pack));
      const int pkm = d->pkm;
      for (int q = tid; q < 2 * T * (KM * KM / 4); q += NT) {
        const int tile = q / (KM * KM / 4), rem = q - tile * (KM * KM / 4);
        const int r = rem / (KM / 4), cc = (rem % (KM / 4)) * 4;
        gv x = gv{0, 0, 0, 0};
        if (r < pkm && cc < pkm) x = *reinterpret_cast<gptr<gv>>(pk + (long)tile * pkm * pkm + r * pkm + cc);
        lt* o = Ops + tile * TILE + r * PW + cc;
        if constexpr (P == 0) {
          *reinterpret_cast<double2*>(o) = double2{x[0], x[1]};
          *reinterpret_cast<double2*>(o + 2) = double2{x[2], x[3]};
        } else {
          *reinterpret_cast<gv*>(o) = x;
        }
      }
      loaded = p;
    }
    gptr<double> Ej = gview(d->E) + (long)j * n;
    gptr<double> Edg = gview(d->Ediag);
    double Dc[CPW][4], Dp[CPW][4], Ev[HOLD ? CPW : 1][4], Ed[HOLD ? CPW : 1][4];
    int idx[CPW][4];
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const int col = (c0 + c) * 16 + l16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rt * 16 + acc_row<P>(g, r);
        const bool in = row < kA && col < kB;
        idx[c][r] = in ? row * kB + col : -1;
        // unconditional loads (a padded element reads element 0 and discards it), so the
        // group issues together and costs one round trip
        Dc[c][r] = Ej[in ? idx[c][r] : 0];
        if constexpr (HOLD) Ed[c][r] = Edg[in ? idx[c][r] : 0];
      }
    }
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const int col = (c0 + c) * 16 + l16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rt * 16 + acc_row<P>(g, r);
        const bool in = idx[c][r] >= 0;
        const double e0 = in ? Dc[c][r] : 0.0;
        if constexpr (HOLD) {
          Ev[c][r] = e0;
          Ed[c][r] = in ? Ed[c][r] : 0.0;
        }
        Dc[c][r] = d->r0 * e0;
        Dp[c][r] = 0.0;
        Ys[row * PW + col] = to_lt<P>(Dc[c][r]);
      }
    }
    if constexpr (!RES) {
      // every wave is past its last read of the operator tiles (the previous vector's
      // last barrier) when the first problem, or one after a term-less problem, starts
      if (T > 0 && staged != p) {
        fetch(d, 0);
        put(Ops, pfB);
        put(Ops + TILE, pfA);
        staged = p;
      }
    }
    __syncthreads();
    for (int k = 1; k <= steps; ++k) {
      const double s1 = d->sc[3 * (k - 1)], s2 = d->sc[3 * (k - 1) + 1], s3 = d->sc[3 * (k - 1) + 2];
      const double ph = s1 * d->phi[(long)(k - 1) * nv + j];
      accT acc[CPW];
#pragma unroll
      for (int c = 0; c < CPW; ++c) acc[c] = accT{0, 0, 0, 0};
      for (int t = 0; t < T; ++t) {
        lt* Zt = Zt0 + (RES ? (t & 1) * TILE : 0);
        lt* Bs = Ops + (RES ? 2 * t * TILE : 0);
        lt* As = Bs + TILE;
        // streamed form: the next term's tiles (this problem's next term, its term 0 for
        // the next step, or the next vector's problem), loaded during this term
        const FilterDesc* nd = nullptr;
        if constexpr (!RES) {
          if (t + 1 < T) {
            nd = d;
          } else if (k < steps) {
            nd = d;
          } else if (v + vs < v1) {
            int pn = p, jn = j + vs;
            while (jn >= descs[pn].nv) {
              jn -= descs[pn].nv;
              ++pn;
            }
            nd = descs + pn;
            staged = descs[pn].T > 0 ? pn : -1;
          }
          if (nd && nd->T > 0) fetch(nd, t + 1 < T ? t + 1 : 0);
          else nd = nullptr;
        }
        accT z[CPW];
#pragma unroll
        for (int c = 0; c < CPW; ++c) z[c] = accT{0, 0, 0, 0};
#pragma unroll
        for (int u = 0; u < NCH; ++u) {
          Frag<P> a;
          a.load(Ys + (rt * 16 + l16) * PW, u, g);
#pragma unroll
          for (int c = 0; c < CPW; ++c) {
            Frag<P> b;
            b.load(Bs + ((c0 + c) * 16 + l16) * PW, u, g);
            mma_frag<P>(z[c], a.v, b);
          }
        }
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
          lt* zr = Zt + ((c0 + c) * 16 + l16) * PW + rt * 16;
          if constexpr (P == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) zr[acc_row<0>(g, r)] = z[c][r];
          } else if constexpr (P == 1) {
            *reinterpret_cast<float4*>(zr + 4 * g) = float4{z[c][0], z[c][1], z[c][2], z[c][3]};
          } else {
            lt h[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) h[r] = (__bf16)z[c][r];
            *reinterpret_cast<uint2*>(zr + 4 * g) = *reinterpret_cast<const uint2*>(h);
          }
        }
        __syncthreads();
        if constexpr (!RES)
          if (nd) put(Bs, pfB);  // every wave is past stage 1's reads of O_B
#pragma unroll
        for (int u = 0; u < NCH; ++u) {
          Frag<P> a;
          a.load(As + (rt * 16 + l16) * PW, u, g);
#pragma unroll
          for (int c = 0; c < CPW; ++c) {
            Frag<P> b;
            b.load(Zt + ((c0 + c) * 16 + l16) * PW, u, g);
            mma_frag<P>(acc[c], a.v, b);
          }
        }
        if constexpr (!RES) {
          __syncthreads();          // every wave is past stage 2's reads of c O_A and Z^T
          if (nd) put(As, pfA);     // visible to the next stage 2 after the next barrier
        }
      }
      // the per-step kernel's epilogue, on the register-resident iterates
#pragma unroll
      for (int c = 0; c < CPW; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const bool in = idx[c][r] >= 0;
          double ed, ev;
          if constexpr (HOLD) {
            ed = Ed[c][r];
            ev = Ev[c][r];
          } else {
            ed = Edg[in ? idx[c][r] : 0];
            ev = Ej[in ? idx[c][r] : 0];
            ed = in ? ed : 0.0;
            ev = in ? ev : 0.0;
          }
          double o = fma(s1, fma(ed, Dc[c][r], (double)acc[c][r]), s2 * Dc[c][r]);
          if (k > 1) o = fma(s3, Dp[c][r], o);  // the first step has no previous iterate
          o = fma(ph, ev, o);
          Dp[c][r] = Dc[c][r];
          Dc[c][r] = in ? o : 0.0;
        }
      if (k < steps) {
#pragma unroll
        for (int c = 0; c < CPW; ++c)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            Ys[(rt * 16 + acc_row<P>(g, r)) * PW + (c0 + c) * 16 + l16] = to_lt<P>(Dc[c][r]);
        __syncthreads();
      }
    }
    const double phP = d->phi[(long)steps * nv + j];
    gptr<double> Xj = gview(d->X) + (long)j * n;
    gptr_w<double> oj = gview_w(d->out) + (long)j * n;
    double xv[CPW][4];
#pragma unroll
    for (int c = 0; c < CPW; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) xv[c][r] = Xj[idx[c][r] >= 0 ? idx[c][r] : 0];
#pragma unroll
    for (int c = 0; c < CPW; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (idx[c][r] >= 0)
          oj[idx[c][r]] = __dadd_rn(__dmul_rn(phP, xv[c][r]), Dc[c][r]);  // as the scale-add kernel
    j += vs;
  }
}

// A wave-uniform value passed through an empty asm statement: the compiler can neither
// hoist what is computed from it out of a loop nor fold it (the value is unchanged).
__device__ inline unsigned opaque_uniform(unsigned x) {
  unsigned v = __builtin_amdgcn_readfirstlane(x);
  asm volatile("" : "+s"(v));
  return v;
}
template <class T>
__device__ inline T* opaque_uniform_ptr(T* p) {
  const unsigned long long v = (unsigned long long)p;
  const unsigned lo = opaque_uniform((unsigned)v), hi = opaque_uniform((unsigned)(v >> 32));
  return reinterpret_cast<T*>(((unsigned long long)hi << 32) | lo);
}
// A raw buffer resource over `bytes` bytes at a wave-uniform address (word 3: the CDNA
// raw-buffer format). Loads through it take a 32-bit byte offset in a VGPR and the base
// in SGPRs, so a group of them needs no 64-bit address per element.
__device__ inline __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ inline double buf_f64(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}

// Wide tiles (KM = 96): the whole filter as above, operators streamed through LDS, but
// within the register budget of 12 waves that own three column tiles each: one staging
// buffer for the next term's tiles (O_B fetched at the start of a term and stored after
// stage 1, then c O_A fetched and stored after stage 2), the defect and the diagonal
// E_A[a] + E_B[b] (the sum the set-up stores, so the same value) re-read from L2 every
// step, element indices recomputed, and the K loops not unrolled so that few operand
// fragments are in flight. LDS holds the low-precision iterate, Z^T and the current
// term's two tiles. The epilogue's loads go out unconditionally (a padded element reads
// a valid in-range address and discards it), so they issue together and cost one round
// trip, not one each. Same arithmetic, in the same
// order, as the per-step kernel's epilogue. (The staging loads stay conditional: a select
// on their value would wait for them before the stage they are meant to overlap.)
template <int P, int KM, int CPW>
__global__ __launch_bounds__(64 * (KM / 16) * (KM / 16) / CPW) void kron_filter_wide_kernel(
    const FilterDesc* __restrict__ descs, int P_, long V, int G) {
  typedef typename SK<P>::lt lt;
  typedef typename SK<P>::acc accT;
  typedef typename Grp<P>::t gv;
  constexpr int RTM = KM / 16;
  constexpr int NWR = RTM / CPW;  // waves per row tile
  constexpr int NT = 64 * RTM * NWR;
  constexpr int PW = sk_pitch<P>(KM);
  constexpr int NCH = KM / SK<P>::CH;
  constexpr int TILE = KM * PW;
  constexpr int NG = KM * KM / (4 * NT);  // staging groups per thread per tile
  static_assert(RTM % CPW == 0 && NG * 4 * NT == KM * KM, "tile split");
  extern __shared__ char smem_raw[];
  lt* Ys = reinterpret_cast<lt*>(smem_raw);
  lt* Zt = Ys + TILE;
  lt* Bs = Zt + TILE;
  lt* As = Bs + TILE;
  gv pf[NG];
  // tile `which` (0: O_B, 1: c O_A) of term tt of a pack with tile size pkm into pf
  // (zeros past pkm)
  auto fetch = [&](const lt* pack, int pkm, int tt, int which) {
    gptr<lt> base = gview(pack) + ((long)tt * 2 + which) * pkm * pkm;
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      const int q = (int)threadIdx.x + i * NT, r = q / (KM / 4), cc = (q % (KM / 4)) * 4;
      gv x = gv{0, 0, 0, 0};  // (a branch, not a select: no wait before the stage)
      if (r < pkm && cc < pkm) x = *reinterpret_cast<gptr<gv>>(base + r * pkm + cc);
      pf[i] = x;
    }
  };
  auto put = [&](lt* dst) {
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      const int q = (int)threadIdx.x + i * NT, r = q / (KM / 4), cc = (q % (KM / 4)) * 4;
      *reinterpret_cast<gv*>(dst + r * PW + cc) = pf[i];
    }
  };

  // XCD x (blockIdx % 8) owns the launch's vectors [x V/8, (x+1) V/8); its GX
  // workgroups take them in turn (stride GX), so that at any time they work on
  // neighbouring vectors, mostly of one problem, whose operator tiles its L2 then
  // serves to all of them
  const int w = blockIdx.x;
  const int GX = G >> 3;
  const long r0 = (long)(w & 7) * V / 8, r1 = (long)((w & 7) + 1) * V / 8;
  const long v0 = r0 + (w >> 3);
  if (v0 >= r1) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, l16 = lane & 15;
  const int rt = wave / NWR, c0 = (wave % NWR) * CPW;
  const int arow = rt * 16 + l16;  // this lane's operand row

  int p = 0;
  {
    int lo = 0, hi = P_ - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (descs[mid].vbase <= v0) lo = mid;
      else hi = mid - 1;
    }
    p = lo;
  }
  int j = (int)(v0 - descs[p].vbase);
  int staged = -1;  // problem whose term-0 tiles sit in LDS
  for (long v = v0; v < r1; v += GX) {
    while (j >= descs[p].nv) {
      j -= descs[p].nv;
      ++p;
    }
    const FilterDesc* d = descs + p;
    const int kA = d->kA, kB = d->kB, T = d->T, steps = d->steps, nv = d->nv;
    // a filter has degree >= 2, so at least one step (the host never builds fewer); said
    // here so that the compiler keeps no copy of the starting iterate for an empty loop
    __builtin_assume(steps >= 1);
    const lt* packd = opaque_uniform_ptr(static_cast<const lt*>(d->pack));
    const int pkmd = (int)opaque_uniform((unsigned)d->pkm);
    // the problem of the next vector of this workgroup, whose term-0 tiles the last
    // term of this vector stages
    int pn = p, Tn = 0, pkmn = 0;
    const lt* packn = nullptr;
    if (v + GX < r1) {
      int jn = j + GX;
      while (jn >= descs[pn].nv) {
        jn -= descs[pn].nv;
        ++pn;
      }
      Tn = descs[pn].T;
      packn = opaque_uniform_ptr(static_cast<const lt*>(descs[pn].pack));
      pkmn = (int)opaque_uniform((unsigned)descs[pn].pkm);
    }
    const long n = (long)kA * kB;
    gptr<double> Ej = gview(d->E) + (long)j * n;
    double Dc[CPW][4], Dp[CPW][4];
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const int col = (c0 + c) * 16 + l16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rt * 16 + acc_row<P>(g, r);
        const bool in = row < kA && col < kB;
        Dc[c][r] = Ej[in ? row * kB + col : 0];
      }
    }
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const int col = (c0 + c) * 16 + l16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rt * 16 + acc_row<P>(g, r);
        const bool in = row < kA && col < kB;
        Dc[c][r] = d->r0 * (in ? Dc[c][r] : 0.0);
        Dp[c][r] = 0.0;
        Ys[row * PW + col] = to_lt<P>(Dc[c][r]);
      }
    }
    if (T > 0 && staged != p) {  // every wave is past the previous vector's last reads
      fetch(packd, pkmd, 0, 0);
      put(Bs);
      fetch(packd, pkmd, 0, 1);
      put(As);
      staged = p;
    }
    __syncthreads();
    for (int k = 1; k <= steps; ++k) {
      const double s1 = d->sc[3 * (k - 1)], s2 = d->sc[3 * (k - 1) + 1], s3 = d->sc[3 * (k - 1) + 2];
      const double ph = s1 * d->phi[(long)(k - 1) * nv + j];
      accT acc[CPW];
#pragma unroll
      for (int c = 0; c < CPW; ++c) acc[c] = accT{0, 0, 0, 0};
      for (int t = 0; t < T; ++t) {
        // the tiles the next term uses: this problem's next term, its term 0 for the
        // next step, or the next vector's problem; nothing to stage when they are the
        // ones already in LDS (a single-term problem)
        const lt* npack = nullptr;
        int npkm = 0, ntt = 0;
        if (t + 1 < T) {
          npack = packd;
          npkm = pkmd;
          ntt = t + 1;
        } else if (k < steps) {
          if (T > 1) {
            npack = packd;
            npkm = pkmd;
          }
        } else if (v + GX < r1) {
          if (Tn > 0 && !(pn == p && T == 1)) {
            npack = packn;
            npkm = pkmn;
          }
          staged = Tn > 0 ? pn : -1;
        }
        if (npack) fetch(npack, npkm, ntt, 0);
        // stage 1: Z = D O_B^T, stored transposed
        accT z[CPW];
#pragma unroll
        for (int c = 0; c < CPW; ++c) z[c] = accT{0, 0, 0, 0};
#pragma unroll 1
        for (int u = 0; u < NCH; ++u) {
          Frag<P> a;
          a.load(Ys + arow * PW, u, g);
#pragma unroll
          for (int c = 0; c < CPW; ++c) {
            Frag<P> b;
            b.load(Bs + ((c0 + c) * 16 + l16) * PW, u, g);
            mma_frag<P>(z[c], a.v, b);
          }
        }
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
          lt* zr = Zt + ((c0 + c) * 16 + l16) * PW + rt * 16;
          if constexpr (P == 1) {
            *reinterpret_cast<float4*>(zr + 4 * g) = float4{z[c][0], z[c][1], z[c][2], z[c][3]};
          } else {
            lt h[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) h[r] = (__bf16)z[c][r];
            *reinterpret_cast<uint2*>(zr + 4 * g) = *reinterpret_cast<const uint2*>(h);
          }
        }
        __syncthreads();
        if (npack) {  // every wave is past stage 1's reads of O_B
          put(Bs);
          fetch(npack, npkm, ntt, 1);
        }
        // stage 2: acc += c O_A Z
#pragma unroll 1
        for (int u = 0; u < NCH; ++u) {
          Frag<P> a;
          a.load(As + arow * PW, u, g);
#pragma unroll
          for (int c = 0; c < CPW; ++c) {
            Frag<P> b;
            b.load(Zt + ((c0 + c) * 16 + l16) * PW, u, g);
            mma_frag<P>(acc[c], a.v, b);
          }
        }
        __syncthreads();  // every wave is past stage 2's reads of c O_A and Z^T
        if (npack) put(As);  // visible to the next stage 2 after the next barrier
      }
      // the per-step kernel's epilogue on the register-resident iterates; the defect and
      // the module energies come from L2 through buffer loads (uniform bases, 32-bit
      // offsets), all issued before the first use
      const __amdgpu_buffer_rsrc_t rE = buf_rsrc(opaque_uniform_ptr(d->E + (size_t)j * n), (unsigned)n * 8u);
      const __amdgpu_buffer_rsrc_t rA = buf_rsrc(opaque_uniform_ptr(d->EA), (unsigned)kA * 8u);
      const __amdgpu_buffer_rsrc_t rB = buf_rsrc(opaque_uniform_ptr(d->EB), (unsigned)kB * 8u);
      // (laundered: offsets recomputed every step rather than kept live across the loop)
      const int kBs = (int)opaque_uniform((unsigned)kB);
      double ev[CPW][4], ea[4], ebv[CPW];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rt * 16 + acc_row<P>(g, r);
        ea[r] = buf_f64(rA, (unsigned)(row < kA ? row : 0) * 8u);
      }
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        const int col = (c0 + c) * 16 + l16;
        ebv[c] = buf_f64(rB, (unsigned)(col < kB ? col : 0) * 8u);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = rt * 16 + acc_row<P>(g, r);
          const bool in = row < kA && col < kB;
          ev[c][r] = buf_f64(rE, in ? (unsigned)(row * kBs + col) * 8u : 0u);
        }
      }
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        const int col = (c0 + c) * 16 + l16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = rt * 16 + acc_row<P>(g, r);
          const bool in = row < kA && col < kB;
          const double ed = in ? ea[r] + ebv[c] : 0.0;
          const double e1 = in ? ev[c][r] : 0.0;
          double o = fma(s1, fma(ed, Dc[c][r], (double)acc[c][r]), s2 * Dc[c][r]);
          if (k > 1) o = fma(s3, Dp[c][r], o);  // the first step has no previous iterate
          o = fma(ph, e1, o);
          Dp[c][r] = Dc[c][r];
          Dc[c][r] = in ? o : 0.0;
        }
      }
      if (k < steps) {
#pragma unroll
        for (int c = 0; c < CPW; ++c)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            Ys[(rt * 16 + acc_row<P>(g, r)) * PW + (c0 + c) * 16 + l16] = to_lt<P>(Dc[c][r]);
        __syncthreads();
      }
    }
    // out_j = phi_P X_j + D_P (as the scale-add kernel rounds)
    const double phP = d->phi[(long)steps * nv + j];
    const __amdgpu_buffer_rsrc_t rX = buf_rsrc(opaque_uniform_ptr(d->X + (size_t)j * n), (unsigned)n * 8u);
    char* ob = opaque_uniform_ptr(reinterpret_cast<char*>(d->out) + (size_t)j * n * sizeof(double));
    double xv[CPW][4];
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const int col = (c0 + c) * 16 + l16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rt * 16 + acc_row<P>(g, r);
        xv[c][r] = buf_f64(rX, row < kA && col < kB ? (unsigned)(row * kB + col) * 8u : 0u);
      }
    }
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const int col = (c0 + c) * 16 + l16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rt * 16 + acc_row<P>(g, r);
        if (row < kA && col < kB) {
          const unsigned off = (unsigned)(row * kB + col) * 8u;
          *reinterpret_cast<gptr_w<double>>(gview_w(ob) + off) = __dadd_rn(__dmul_rn(phP, xv[c][r]), Dc[c][r]);
        }
      }
    }
    j += GX;
  }
}

typedef void (*FilterKernel)(const FilterDesc*, int, long, int);

// Column tiles per wave of the fused filter (RMC_FILTER_CPW = 1, 2 or 4): more tiles per
// wave reuse each row fragment across them (fewer LDS reads per MFMA) with fewer waves.
static int filter_cpw() {
  static const int c = [] {
    const char* e = getenv("RMC_FILTER_CPW");
    const int v = e ? atoi(e) : 1;
    return (v == 2 || v == 4) ? v : 1;
  }();
  return c;
}

// Streamed form: column tiles per wave of the one instance per precision and tile size
// (0: none). FP64 at KM = 64 takes two tiles per wave for the registers. Wider tiles
// need three or more tiles per wave (the 16-wave limit), and those forms spill
// registers, so they are left out.
static int filter_streamed_cpw(int prec, int km) {
  if (prec == RMC_FP64) return km <= 32 ? 1 : (km <= 64 ? 2 : 0);
  if (km <= 32) return 0;  // resident at this size in every precision
  if (km <= 64) return 1;
  // 96: 6 x 6 tiles, 12 waves of three column tiles. 128 stays on the per-step path:
  // four FP32 tiles of 128 do not fit in LDS, and in BF16 the FP64 iterates of 64 tiles
  // spill registers with 16 waves of four tiles or 8 waves of eight
  return km <= 96 ? 3 : 0;
}

template <int P, int KM>
static FilterKernel filter_kernel_cpw(int cpw) {
  if constexpr (KM / 16 >= 4)
    if (cpw == 4) return kron_filter_kernel<P, KM, 4, true>;
  if (cpw >= 2) return kron_filter_kernel<P, KM, 2, true>;
  return kron_filter_kernel<P, KM, 1, true>;
}

// res: operators resident in LDS; else the streamed form (one per precision and size,
// column tiles per wave fixed by the 16-wave limit: 1 at KM <= 64, 3 at 96, 4 at 128)
static FilterKernel filter_kernel(int prec, int km, int cpw, bool res = true) {
  if (!res) {
    switch (filter_streamed_cpw(prec, km)) {
      case 0: return nullptr;
      case 1: return prec == RMC_FP64 ? kron_filter_kernel<0, 32, 1, false>
                                      : (prec == RMC_FP32 ? kron_filter_kernel<1, 64, 1, false> : kron_filter_kernel<2, 64, 1, false>);
      case 3: return prec == RMC_FP32 ? kron_filter_wide_kernel<1, 96, 3> : kron_filter_wide_kernel<2, 96, 3>;
      default: return kron_filter_kernel<0, 64, 2, false>;
    }
  }
  if (prec == RMC_FP64) return km <= 32 ? filter_kernel_cpw<0, 32>(cpw) : nullptr;
  if (prec == RMC_FP32)
    return km <= 32 ? filter_kernel_cpw<1, 32>(cpw) : (km <= 64 ? filter_kernel_cpw<1, 64>(cpw) : nullptr);
  return km <= 32 ? filter_kernel_cpw<2, 32>(cpw) : (km <= 64 ? filter_kernel_cpw<2, 64>(cpw) : nullptr);
}

static int filter_threads(int prec, int km, int cpw, bool res = true) {
  const int rtm = km / 16;
  int c = cpw;
  if (!res) c = filter_streamed_cpw(prec, km);
  else if (cpw == 4 && rtm < 4) c = 2;
  return 64 * rtm * rtm / c;
}

static size_t filter_lds_bytes(int prec, int KM, int T, bool res = true) {
  const int esz = prec == RMC_FP64 ? 8 : (prec == RMC_FP32 ? 4 : 2);
  return (size_t)(res ? 3 + 2 * std::max(T, 0) : 4) * KM * (KM + 16 / esz) * esz;
}

static constexpr size_t kFilterLdsMax = 159 * 1024;

static size_t kron_lds_bytes(int kA, int prec) {
  // TCH * kApad * 16 * CT elements = 64 * kApad for every CT
  const int kApad = ((kA + 15) / 16) * 16;
  return (size_t)64 * kApad * (prec == 0 ? sizeof(double) : sizeof(float));
}

int kron_max_k() { return 192; }

typedef void (*KronKernel)(const KronDesc*);

template <int P, int CT>
static KronKernel pick_mrt(int mrt) {
  switch (mrt) {
    case 1: return kron_batched_kernel<P, CT, 1>;
    case 2: return kron_batched_kernel<P, CT, 2>;
    default: return kron_batched_kernel<P, CT, 3>;
  }
}

template <int P>
static KronKernel pick_ct(int ct, int mrt) {
  switch (ct) {
    case 1: return pick_mrt<P, 1>(mrt);
    case 2: return pick_mrt<P, 2>(mrt);
    default: return mrt == 3 ? pick_mrt<P, 2>(mrt) : pick_mrt<P, 4>(mrt);
  }
}

static KronKernel kron_kernel(int prec, int ct, int mrt) {
  switch (prec) {
    case RMC_FP64: return pick_ct<0>(ct, mrt);
    case RMC_FP32: return pick_ct<1>(ct, mrt);
    default: return pick_ct<2>(ct, mrt);
  }
}

typedef void (*StreamKernel)(const KronDesc*, int, long, int);

// Streaming kernels by precision, padded size KM and column split NWC; null where
// the three KM x KM tiles do not fit in LDS.
static StreamKernel stream_kernel(int prec, int km, int nwc, bool sh = false) {
#define RMC_SK(P_, KM_)                                                                \
  if (km <= KM_)                                                                       \
    return nwc == 1 ? (sh ? kron_stream_kernel<P_, KM_, 1, true> : kron_stream_kernel<P_, KM_, 1, false>) \
                    : (sh ? kron_stream_kernel<P_, KM_, 2, true> : kron_stream_kernel<P_, KM_, 2, false>);
  // the widest tiles fit in LDS only with one buffer for both operators (SH)
  if (prec == RMC_FP64) {
    RMC_SK(0, 32) RMC_SK(0, 64)
    // 96: one LDS buffer for both operators (two 96-wide FP64 tiles), two waves a row tile
    if (km <= 96) return (sh && nwc == 2) ? kron_stream_kernel<0, 96, 2, true> : nullptr;
  } else if (prec == RMC_FP32) {
    RMC_SK(1, 32) RMC_SK(1, 64) RMC_SK(1, 96)
    if (km <= 128) return (sh && nwc == 1) ? kron_stream_kernel<1, 128, 1, true> : nullptr;
  } else {
    RMC_SK(2, 32) RMC_SK(2, 64) RMC_SK(2, 96)
    if (km <= 128 && nwc == 1) return sh ? kron_stream_kernel<2, 128, 1, true> : kron_stream_kernel<2, 128, 1, false>;
  }
#undef RMC_SK
  return nullptr;
}

// Some streaming kernel (either LDS form, one or two waves a row tile) takes tiles of
// this size and precision: the operators are then packed for it. Every streaming
// launch reads the packs, so a variant is a candidate only where this holds.
static bool has_stream(int prec, int km) {
  for (int nwc : {1, 2})
    for (bool sh : {false, true})
      if (stream_kernel(prec, km, nwc, sh) != nullptr) return true;
  return false;
}

static int stream_km(int km) { return km <= 32 ? 32 : (km <= 64 ? 64 : (km <= 96 ? 96 : 128)); }

static size_t stream_lds_bytes(int prec, int KM, bool sh = false) {
  const int esz = prec == RMC_FP64 ? 8 : (prec == RMC_FP32 ? 4 : 2);
  return (size_t)(sh ? 2 : 3) * KM * (KM + 16 / esz) * esz;
}

// Workgroups of a streaming launch: resident workgroups per CU times the CU count
// (a multiple of 8 for the XCD mapping), at most one per vector.
static int stream_grid(const void* k, int threads, size_t lds, long V) {
  static std::mutex mu;
  static std::map<std::pair<const void*, size_t>, int> per_cu;
  static int cus = 0;
  int n;
  {
    std::lock_guard<std::mutex> lk(mu);
    if (cus == 0) {
      int dev = 0;
      (void)hipGetDevice(&dev);
      if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
          cus <= 0)
        cus = 256;
    }
    auto it = per_cu.find({k, lds});
    if (it == per_cu.end()) {
      int b = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k, threads, lds) != hipSuccess || b <= 0)
        b = 1;
      it = per_cu.emplace(std::make_pair(k, lds), b).first;
    }
    n = it->second * cus;
  }
  // RMC_KRON_MAX_GRID caps the grid, so that each workgroup walks many vectors (tests)
  if (const char* f = getenv("RMC_KRON_MAX_GRID")) {
    const int cap = atoi(f);
    if (cap >= 8) n = std::min(n, cap);
  }
  // as few workgroups as give the same makespan: every workgroup walks
  // ceil(V / n) vectors at most, so ceil(V / that) workgroups suffice and the CUs
  // left over take other streams' work (the solver's other lanes)
  const long per = (V + n - 1) / n;
  const long g = std::min<long>(n, (V + per - 1) / per);
  return (int)(((g + 7) / 8) * 8);
}

void kron_set_attrs() {
  const int lds = 160 * 1024 - 1024;
  for (int p = 0; p < 3; ++p)
    for (int km : {32, 64, 96, 128})
      for (int nwc : {1, 2})
        for (bool sh : {false, true})
          if (StreamKernel k = stream_kernel(p, km, nwc, sh))
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  for (int p = 0; p < 3; ++p)
    for (int ct : {1, 2, 4})
      for (int mrt = 1; mrt <= 3; ++mrt)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kron_kernel(p, ct, mrt)),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  for (int p = 0; p < 3; ++p)
    for (int km : {32, 64, 96, 128})
      for (int cpw : {1, 2, 4})
        for (bool res : {true, false})
          if (FilterKernel k = filter_kernel(p, km, cpw, res))
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFilterLdsMax);
}

// Resident form where its LDS fits, else the streamed form (RMC_FILTER_STREAMED=1
// takes the streamed form wherever it exists, to test it).
static bool filter_resident(int precision, int km, int T) {
  const char* fe = getenv("RMC_FILTER_STREAMED");
  const bool force_streamed = fe && atoi(fe) != 0;
  const bool res_ok = filter_kernel(precision, km, 1, true) != nullptr &&
                      filter_lds_bytes(precision, km, T, true) <= kFilterLdsMax;
  const bool str_ok = filter_kernel(precision, km, 1, false) != nullptr &&
                      filter_lds_bytes(precision, km, T, false) <= kFilterLdsMax;
  return res_ok && !(force_streamed && str_ok);
}

bool kron_filter_fits(int precision, int kA, int kB, int T) {
  const int km = stream_km(std::max(kA, kB));
  if (!has_stream(precision, km)) return false;  // no operator pack for this size
  return (filter_kernel(precision, km, 1, true) && filter_lds_bytes(precision, km, T, true) <= kFilterLdsMax) ||
         (filter_kernel(precision, km, 1, false) && filter_lds_bytes(precision, km, T, false) <= kFilterLdsMax);
}

void kron_filter_batched(hipStream_t s, const FilterDesc* d, int P, long total_vecs, int precision,
                         int kmax, int Tmax) {
  if (P <= 0 || total_vecs <= 0) return;
  const int KM = stream_km(kmax);
  const bool res = filter_resident(precision, KM, Tmax);
  const int cpw = filter_cpw();
  FilterKernel k = filter_kernel(precision, KM, cpw, res);
  const int threads = filter_threads(precision, KM, cpw, res);
  const size_t lds = filter_lds_bytes(precision, KM, Tmax, res);
  const int G = stream_grid(reinterpret_cast<const void*>(k), threads, lds, total_vecs);
  hipLaunchKernelGGL(k, dim3(G), dim3(threads), lds, s, d, P, total_vecs, G);
}

// ---- operator packs for the streaming kernel ----------------------------------------
// pack[t][0] = O_B^t, pack[t][1] = c_t O_A^t, each pkm x pkm zero-padded, in the
// element type of the precision (rounded through FP32 for BF16, as the kernel
// rounds its vectors).
__global__ void kron_pack_kernel(int T, int kA, int kB, int pkm, const double* __restrict__ coef,
                                 const double* __restrict__ OA, const double* __restrict__ OB,
                                 double* p64, float* p32, __bf16* p16) {
  const int t = blockIdx.y >> 1, isA = blockIdx.y & 1;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T || i >= (long)pkm * pkm) return;
  const int r = (int)(i / pkm), c = (int)(i % pkm);
  const int k = isA ? kA : kB;
  double v = 0.0;
  if (r < k && c < k)
    v = isA ? coef[t] * OA[(long)t * kA * kA + (long)r * kA + c] : OB[(long)t * kB * kB + (long)r * kB + c];
  const long o = ((long)t * 2 + isA) * pkm * pkm + i;
  if (p64) p64[o] = v;
  if (p32) p32[o] = (float)v;
  if (p16) p16[o] = to_lt<2>(v);
}

// One workgroup row per problem; a grid-stride loop over the concatenated work of
// the problem: T k_A^2 copies, T k_B^2 copies, n diagonal entries, the pack entries.
// The values are those of the per-operator path (same sums in the same order).
__global__ __launch_bounds__(256) void op_setup_kernel(const OpSetDesc* __restrict__ descs) {
  const OpSetDesc d = descs[blockIdx.y];
  const int T = d.T, kA = d.kA, kB = d.kB, pk = d.pkm;
  const long a2 = (long)kA * kA, b2 = (long)kB * kB, n = (long)kA * kB;
  const long nA = T * a2, nB = T * b2;
  const bool packs = d.p64 || d.p32 || d.p16;
  const long nP = packs ? 2L * T * pk * pk : 0;
  const long total = nA + nB + n + nP;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < total; i += (long)gridDim.x * 256) {
    if (i < nA) {
      d.OAcat[i] = d.opa[i / a2][i % a2];
    } else if (i < nA + nB) {
      const long j = i - nA;
      d.OBcat[j] = d.opb[j / b2][j % b2];
    } else if (i < nA + nB + n) {
      const long t = i - nA - nB;
      const int a = (int)(t / kB), b = (int)(t % kB);
      const double e = d.EA[a] + d.EB[b];
      double v = e;
      for (int q = 0; q < T; ++q) v += d.coef[q] * d.opa[q][(long)a * kA + a] * d.opb[q][(long)b * kB + b];
      if (d.D) d.D[t] = v;
      d.Ediag[t] = e;
    } else {
      const long o = i - nA - nB - n;
      const long pp = (long)pk * pk;
      const int t = (int)(o / (2 * pp)), isA = (int)((o / pp) & 1);
      const int r = (int)((o % pp) / pk), c = (int)(o % pk);
      const int k = isA ? kA : kB;
      double v = 0.0;
      if (r < k && c < k) v = isA ? d.coef[t] * d.opa[t][(long)r * kA + c] : d.opb[t][(long)r * kB + c];
      if (d.p64) d.p64[o] = v;
      if (d.p32) d.p32[o] = (float)v;
      if (d.p16) static_cast<__bf16*>(d.p16)[o] = to_lt<2>(v);
    }
  }
}

void op_setup_batched(hipStream_t s, const OpSetDesc* d, int P, long work_max) {
  if (P <= 0 || work_max <= 0) return;
  const long b = (work_max + 255) / 256;
  const int gx = (int)(b > 512 ? 512 : b);
  hipLaunchKernelGGL(op_setup_kernel, dim3(gx, P), dim3(256), 0, s, d);
}

int kron_pack_km(int kA, int kB) { return stream_km(std::max(kA, kB)); }

size_t kron_pack_bytes(int precision, int kA, int kB, int T) {
  if (T <= 0) return 0;
  const int km = kron_pack_km(kA, kB);
  if (!has_stream(precision, km)) return 0;
  const size_t esz = precision == RMC_FP64 ? 8 : (precision == RMC_FP32 ? 4 : 2);
  return (size_t)T * 2 * km * km * esz;
}

void kron_pack(hipStream_t s, int T, int kA, int kB, const double* coef, const double* OA,
               const double* OB, void* p64, void* p32, void* p16) {
  if (T <= 0 || (!p64 && !p32 && !p16)) return;
  const int pkm = kron_pack_km(kA, kB);
  dim3 grid((unsigned)(((long)pkm * pkm + 255) / 256), 2 * T);
  hipLaunchKernelGGL(kron_pack_kernel, grid, dim3(256), 0, s, T, kA, kB, pkm, coef, OA, OB,
                     static_cast<double*>(p64), static_cast<float*>(p32), static_cast<__bf16*>(p16));
}

// ---- tile-shape autotuner ---------------------------------------------------------
// The column sub-tiles per workgroup (CT = 1, 2 or 4) are chosen per launch shape
// (precision, k_A, k_B, T, vectors in the launch rounded to a power of two) by timing
// every candidate on the first launch of that shape; candidates 8 to 11 are the
// streaming kernel (k <= 64 in FP64, 96 in FP32, 128 in BF16). The timed launches are
// ordinary launches (the output does not alias the inputs). The CT candidates give
// bit-identical results; the streaming one sums K in another order, so it agrees
// with them to rounding. The
// choice is cached for the process and, if RMC_TUNE_CACHE names a file, read from
// and appended to that file, which makes a run reproducible bit for bit.
namespace {
std::mutex tune_mu;
std::map<std::string, int> tune_cache;
bool tune_loaded = false;

void tune_load() {
  if (tune_loaded) return;
  tune_loaded = true;
  const char* f = getenv("RMC_TUNE_CACHE");
  if (!f) return;
  FILE* fp = fopen(f, "r");
  if (!fp) return;
  char key[128];
  int v;
  while (fscanf(fp, "%127s %d", key, &v) == 2) tune_cache[key] = v;
  fclose(fp);
}

void tune_store(const std::string& key, int v) {
  const char* f = getenv("RMC_TUNE_CACHE");
  if (!f) return;
  FILE* fp = fopen(f, "a");
  if (!fp) return;
  fprintf(fp, "%s %d\n", key.c_str(), v);
  fclose(fp);
}
}  // namespace

static bool tuning_enabled = true;
static thread_local bool thread_tuning = true;
void kron_set_tuning(bool on) { tuning_enabled = on; }
void kron_thread_tuning(bool on) { thread_tuning = on; }

int kron_batched(hipStream_t s, const KronDesc* d, int P, int kBmax, int nvmax, int kAmax,
                 int precision, int T, long total_vecs, bool may_tune, bool strict) {
  if (P <= 0 || nvmax <= 0 || kBmax <= 0 || total_vecs <= 0) return 0;
  const int RT = (kAmax + 15) / 16;
  const int mrt = RT <= 4 ? 1 : (RT <= 8 ? 2 : 3);
  const size_t lds = kron_lds_bytes(kAmax, precision);
  const int KM = stream_km(std::max(kAmax, kBmax));
  // candidates: 1, 2, 4 = column sub-tiles of the tiled kernel; 8, 9 = streaming
  // kernel with one or two waves per row tile; 10, 11 = the same with one LDS buffer
  // for both operators of a step (two more barriers, one tile less of LDS)
  auto valid = [&](int c) {
    if (c >= 8 && c <= 11)
      return has_stream(precision, KM) && stream_kernel(precision, KM, (c - 8) % 2 + 1, c >= 10) != nullptr;
    if (c == 1) return true;
    if (c != 2 && c != 4) return false;
    if (16 * c > ((kBmax + 15) / 16) * 16 * 2) return false;  // at most two half-empty tiles
    return !(c == 4 && mrt == 3);                             // that variant spills registers
  };
  auto launch = [&](int c) {
    if (c >= 8) {
      const int nwc = (c - 8) % 2 + 1;
      const bool sh = c >= 10;
      StreamKernel k = stream_kernel(precision, KM, nwc, sh);
      const int threads = 4 * KM * nwc;
      const size_t slds = stream_lds_bytes(precision, KM, sh);
      const int G = stream_grid(reinterpret_cast<const void*>(k), threads, slds, total_vecs);
      hipLaunchKernelGGL(k, dim3(G), dim3(threads), slds, s, d, P, total_vecs, G);
      return;
    }
    dim3 grid((kBmax + 16 * c - 1) / (16 * c), nvmax, P);
    hipLaunchKernelGGL(kron_kernel(precision, c, mrt), grid, dim3(256), lds, s, d);
  };
  // RMC_KRON_VARIANT forces a candidate, e.g. to test it: where it does not take the
  // shape, a strict launch fails and any other takes the autotuner's choice
  if (const char* f = getenv("RMC_KRON_VARIANT")) {
    const int c = atoi(f);
    if (valid(c)) {
      launch(c);
      return c;
    }
    RMC_CHECK(!strict, RMC_ERR_ARG,
              "Kronecker variant " + std::to_string(c) + " does not take this shape (precision " +
                  std::to_string(precision) + ", k_A " + std::to_string(kAmax) + ", k_B " +
                  std::to_string(kBmax) + ")");
  }
  int lg = 0;
  while ((1L << (lg + 1)) <= total_vecs) ++lg;
  char kb[128];
  snprintf(kb, sizeof(kb), "p%d_a%d_b%d_t%d_v%d", precision, kAmax, kBmax, T, lg);
  const std::string key(kb);
  int ct = -1;
  {
    std::lock_guard<std::mutex> lk(tune_mu);
    tune_load();
    auto it = tune_cache.find(key);
    if (it != tune_cache.end() && valid(it->second)) ct = it->second;
  }
  if (ct < 0 && (!tuning_enabled || !may_tune || !thread_tuning)) ct = valid(8) ? 8 : (valid(2) ? 2 : 1);
  if (ct < 0) {
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    float best = 1e30f;
    int best_ct = 1;
    for (int c : {1, 2, 4, 8, 9, 10, 11}) {
      if (!valid(c)) continue;
      launch(c);  // warm
      float tmin = 1e30f;
      for (int rep = 0; rep < 2; ++rep) {
        hipEventRecord(e0, s);
        launch(c);
        hipEventRecord(e1, s);
        hipEventSynchronize(e1);
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        tmin = std::min(tmin, ms);
      }
      if (tmin < best) {
        best = tmin;
        best_ct = c;
      }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    ct = best_ct;
    std::lock_guard<std::mutex> lk(tune_mu);
    tune_cache[key] = ct;
    tune_store(key, ct);
  }
  launch(ct);
  return ct;
}

}  // namespace rmc
