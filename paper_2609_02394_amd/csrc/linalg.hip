// Dense FP64 building blocks of the eigensolver on gfx950: an MFMA GEMM with
// split-K, vector norms, Cholesky + triangular inverse (CholeskyQR2), and a
// parallel cyclic Jacobi eigensolver for the Rayleigh-Ritz matrices.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "rmc_batch.h"
#include "rmc_kernels.h"

namespace rmc {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------------------
// GEMM: 64x64 output tile per 256-thread workgroup, K staged 16 at a time in LDS.
// Each wave owns a 32x32 quadrant = 2x2 tiles of v_mfma_f64_16x16x4_f64.
// Operand lanes: A[i][k] with i = lane%16, k = lane/16; B[k][j] with j = lane%16,
// k = lane/16; for this FP64 instruction accumulator register r holds
// D[4*r + lane/16][lane%16] (measured on gfx950).
// ---------------------------------------------------------------------------
constexpr int GB_M = 64, GB_N = 64, GB_K = 16;

// One 64x64 output tile over K range [kbeg, kend): LDS double-buffered, the next
// 16-deep K slice is loaded into registers while the MFMAs consume the current one.
__device__ inline void gemm_tile(int tA, int tB, int M, int N, const double* __restrict__ Ab, long lda,
                                 const double* __restrict__ Bb, long ldb, int row0, int col0,
                                 int kbeg, int kend, d4 (&acc)[2][2]) {
  __shared__ double As[2][GB_K][GB_M + 1];
  __shared__ double Bs[2][GB_K][GB_N + 1];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  double ra[4], rb[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = tid + e * 256;
      int i, k;
      if (!tA) { i = idx / GB_K; k = idx % GB_K; } else { k = idx / GB_M; i = idx % GB_M; }
      const int gi = row0 + i, gk = k0 + k;
      ra[e] = (gi < M && gk < kend) ? (tA ? Ab[(long)gk * lda + gi] : Ab[(long)gi * lda + gk]) : 0.0;
      int j, kb;
      if (!tB) { kb = idx / GB_N; j = idx % GB_N; } else { j = idx / GB_K; kb = idx % GB_K; }
      const int gj = col0 + j, gkb = k0 + kb;
      rb[e] = (gj < N && gkb < kend) ? (tB ? Bb[(long)gj * ldb + gkb] : Bb[(long)gkb * ldb + gj]) : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = tid + e * 256;
      int i, k;
      if (!tA) { i = idx / GB_K; k = idx % GB_K; } else { k = idx / GB_M; i = idx % GB_M; }
      As[buf][k][i] = ra[e];
      int j, kb;
      if (!tB) { kb = idx / GB_N; j = idx % GB_N; } else { j = idx / GB_K; kb = idx % GB_K; }
      Bs[buf][kb][j] = rb[e];
    }
  };
  if (kbeg >= kend) return;
  load(kbeg);
  store(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = kbeg; k0 < kend; k0 += GB_K) {
    const bool more = k0 + GB_K < kend;
    if (more) load(k0 + GB_K);
#pragma unroll
    for (int kk = 0; kk < GB_K; kk += 4) {
      const int kr = kk + (lane >> 4);
      const double a0 = As[buf][kr][wm + (lane & 15)];
      const double a1 = As[buf][kr][wm + 16 + (lane & 15)];
      const double b0 = Bs[buf][kr][wn + (lane & 15)];
      const double b1 = Bs[buf][kr][wn + 16 + (lane & 15)];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
}

__global__ __launch_bounds__(256) void gemm_f64_kernel(
    int tA, int tB, int M, int N, int K, int kchunk, double alpha, const double* __restrict__ A,
    long lda, long sA, const double* __restrict__ B, long ldb, long sB, double beta,
    double* __restrict__ C, long ldc, long sC, int batch, int ksplit, double* __restrict__ work,
    int to_parts) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int bz = blockIdx.z;
  const int b = bz / ksplit, ks = bz % ksplit;
  const int row0 = blockIdx.y * GB_M, col0 = blockIdx.x * GB_N;
  const int kbeg = ks * kchunk;
  const int kend = min(K, kbeg + kchunk);
  d4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  gemm_tile(tA, tB, M, N, A + (long)b * sA, lda, B + (long)b * sB, ldb, row0, col0, kbeg, kend, acc);

  if (ksplit > 1 || to_parts) {
    double* P = work + ((long)ks * batch + b) * (long)M * N;
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int gi = row0 + wm + ti * 16 + 4 * r + (lane >> 4);
          int gj = col0 + wn + tj * 16 + (lane & 15);
          if (gi < M && gj < N) P[(long)gi * N + gj] = alpha * acc[ti][tj][r];
        }
    return;
  }
  double* Cb = C + (long)b * sC;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int gi = row0 + wm + ti * 16 + 4 * r + (lane >> 4);
        int gj = col0 + wn + tj * 16 + (lane & 15);
        if (gi < M && gj < N) {
          double v = alpha * acc[ti][tj][r];
          if (beta != 0.0) v += beta * Cb[(long)gi * ldc + gj];
          Cb[(long)gi * ldc + gj] = v;
        }
      }
}

__global__ void splitk_reduce_kernel(int M, int N, int batch, int ksplit, const double* __restrict__ work,
                                     double beta, double* __restrict__ C, long ldc, long sC) {
  long total = (long)batch * M * N;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total;
       t += (long)gridDim.x * blockDim.x) {
    int b = (int)(t / ((long)M * N));
    long r = t % ((long)M * N);
    int i = (int)(r / N), j = (int)(r % N);
    double v = 0.0;
    for (int ks = 0; ks < ksplit; ++ks) v += work[((long)ks * batch + b) * (long)M * N + r];
    double* c = C + (long)b * sC + (long)i * ldc + j;
    if (beta != 0.0) v += beta * *c;
    *c = v;
  }
}

// Grouped GEMM: problem = blockIdx.z / ksplit, split = blockIdx.z % ksplit, each
// problem with its own sizes, pointers and scalars.
__global__ __launch_bounds__(256) void gemm_grouped_kernel(int tA, int tB, int ksplit,
                                                           const GemmDesc* __restrict__ descs) {
  const GemmDesc d = descs[blockIdx.z / ksplit];
  const int ks = blockIdx.z % ksplit;
  const int M = d.M, N = d.N, K = d.K;
  const int row0 = blockIdx.y * GB_M, col0 = blockIdx.x * GB_N;
  if (row0 >= M || col0 >= N) return;
  int kchunk = (K + ksplit - 1) / ksplit;
  kchunk = ((kchunk + GB_K - 1) / GB_K) * GB_K;
  if (kchunk < GB_K) kchunk = GB_K;
  const int kbeg = ks * kchunk;
  const int kend = min(K, kbeg + kchunk);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  d4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  gemm_tile(tA, tB, M, N, d.A, d.lda, d.B, d.ldb, row0, col0, kbeg, kend, acc);
  const bool parts = d.work != nullptr;
  double* P = parts ? d.work + (long)ks * M * N : nullptr;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int gi = row0 + wm + ti * 16 + 4 * r + (lane >> 4);
        int gj = col0 + wn + tj * 16 + (lane & 15);
        if (gi < M && gj < N) {
          double v = d.alpha * acc[ti][tj][r];
          if (parts) {
            P[(long)gi * N + gj] = v;
          } else {
            if (d.beta != 0.0) v += d.beta * d.C[(long)gi * d.ldc + gj];
            d.C[(long)gi * d.ldc + gj] = v;
          }
        }
      }
}

// The same product for 64 < M <= 16 MT (a Rayleigh-Ritz block with its guard vectors,
// MT = 5: 80 rows; MT = 8: 128 rows): one 16 MT x 16 NW output tile per workgroup of NW
// waves, so M is not padded to two 64-row tiles and the wide operand B is read once, not
// once per row tile. Wave w owns columns 16w..16w+15 as MT 16 x 16 MFMA tiles down the
// rows.
template <int MT, int NW>
__global__ __launch_bounds__(64 * NW) void gemm_grouped_tall_kernel(int tA, int tB, int ksplit,
                                                                    const GemmDesc* __restrict__ descs) {
  constexpr int GM = 16 * MT, GN = 16 * NW, NT = 64 * NW;
  constexpr int NA = (GM * GB_K + NT - 1) / NT;  // A elements each thread stages per K slice
  constexpr int NB = GB_K * GN / NT;             // B elements
  static_assert(NB * NT == GB_K * GN, "B slice split");
  __shared__ double As[2][GB_K][GM + 1];
  __shared__ double Bs[2][GB_K][GN + 1];
  const GemmDesc d = descs[blockIdx.z / ksplit];
  const int ks = blockIdx.z % ksplit;
  const int M = d.M, N = d.N, K = d.K;
  const int col0 = blockIdx.x * GN;
  if (col0 >= N || M <= 0) return;
  int kchunk = (K + ksplit - 1) / ksplit;
  kchunk = ((kchunk + GB_K - 1) / GB_K) * GB_K;
  if (kchunk < GB_K) kchunk = GB_K;
  const int kbeg = ks * kchunk;
  const int kend = min(K, kbeg + kchunk);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  d4 acc[MT];
#pragma unroll
  for (int i = 0; i < MT; ++i) acc[i] = d4{0.0, 0.0, 0.0, 0.0};
  double ra[NA], rb[NB];
  auto load = [&](int k0) {
#pragma unroll
    for (int e = 0; e < NA; ++e) {
      const int idx = tid + e * NT;  // the last round may run past GM * 16: nothing to load
      int i, k;
      if (!tA) { i = idx / GB_K; k = idx % GB_K; } else { k = idx / GM; i = idx % GM; }
      const int gk = k0 + k;
      ra[e] = (idx < GM * GB_K && i < M && gk < kend)
                  ? (tA ? d.A[(long)gk * d.lda + i] : d.A[(long)i * d.lda + gk]) : 0.0;
    }
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      const int idx = tid + e * NT;
      int j, kb;
      if (!tB) { kb = idx / GN; j = idx % GN; } else { j = idx / GB_K; kb = idx % GB_K; }
      const int gj = col0 + j, gkb = k0 + kb;
      rb[e] = (gj < N && gkb < kend) ? (tB ? d.B[(long)gj * d.ldb + gkb] : d.B[(long)gkb * d.ldb + gj]) : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int e = 0; e < NA; ++e) {
      const int idx = tid + e * NT;
      if (idx >= GM * GB_K) break;
      int i, k;
      if (!tA) { i = idx / GB_K; k = idx % GB_K; } else { k = idx / GM; i = idx % GM; }
      As[buf][k][i] = ra[e];
    }
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      const int idx = tid + e * NT;
      int j, kb;
      if (!tB) { kb = idx / GN; j = idx % GN; } else { j = idx / GB_K; kb = idx % GB_K; }
      Bs[buf][kb][j] = rb[e];
    }
  };
  if (kbeg < kend) {
    load(kbeg);
    store(0);
    __syncthreads();
    int buf = 0;
    for (int k0 = kbeg; k0 < kend; k0 += GB_K) {
      const bool more = k0 + GB_K < kend;
      if (more) load(k0 + GB_K);
#pragma unroll
      for (int kk = 0; kk < GB_K; kk += 4) {
        const int kr = kk + (lane >> 4);
        const double b = Bs[buf][kr][wave * 16 + (lane & 15)];
#pragma unroll
        for (int t = 0; t < MT; ++t)
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(As[buf][kr][t * 16 + (lane & 15)], b, acc[t], 0, 0, 0);
      }
      if (more) store(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }
  const bool parts = d.work != nullptr;
  double* P = parts ? d.work + (long)ks * M * N : nullptr;
  const int gj = col0 + wave * 16 + (lane & 15);
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gi = t * 16 + 4 * r + (lane >> 4);
      if (gi < M && gj < N) {
        double v = d.alpha * acc[t][r];
        if (parts) {
          P[(long)gi * N + gj] = v;
        } else {
          if (d.beta != 0.0) v += d.beta * d.C[(long)gi * d.ldc + gj];
          d.C[(long)gi * d.ldc + gj] = v;
        }
      }
    }
}

void gemm_batched(hipStream_t s, bool tA, bool tB, const GemmDesc* d, int P, int Mmax, int Nmax,
                  int ksplit) {
  if (P <= 0 || Mmax <= 0 || Nmax <= 0) return;
  if (ksplit < 1) ksplit = 1;
  if (Mmax > GB_M && Mmax <= 128) {
    // up to 80 rows (a block with its guard vectors): 80 x 64 tiles (4 waves); up to 128:
    // 128 x 128 tiles (8 waves), so the small operand (a rotation, a triangular factor)
    // is re-read half as often per output (41% -> 57% MFMA busy on 128-row products;
    // 128-wide tiles at 64 and 80 rows measured no faster)
    if (Mmax <= 80) {
      dim3 grid((Nmax + 63) / 64, 1, P * ksplit);
      hipLaunchKernelGGL((gemm_grouped_tall_kernel<5, 4>), grid, dim3(256), 0, s, (int)tA, (int)tB, ksplit, d);
    } else {
      dim3 grid((Nmax + 127) / 128, 1, P * ksplit);
      hipLaunchKernelGGL((gemm_grouped_tall_kernel<8, 8>), grid, dim3(512), 0, s, (int)tA, (int)tB, ksplit, d);
    }
    return;
  }
  dim3 grid((Nmax + GB_N - 1) / GB_N, (Mmax + GB_M - 1) / GB_M, P * ksplit);
  hipLaunchKernelGGL(gemm_grouped_kernel, grid, dim3(256), 0, s, (int)tA, (int)tB, ksplit, d);
}

// ---- Gram partials of tall-skinny blocks -------------------------------------------
// One workgroup (8 waves) per (problem, K-slice): the slice of every row of A (and of
// B unless B == A) is staged in LDS 32 columns at a time, and each wave accumulates
// its 16x16 output tiles with FP64 MFMA. Lane group g takes the K run 8g..8g+7 of a
// chunk (the order of K inside an MFMA step is free), so operands are contiguous
// LDS reads. Rows past ca / cb are staged as zeros. A slice past n writes zeros.
// For A A^T, and for a product the caller declares symmetric (Q^T H Q), only the tiles
// on and above the diagonal are formed and each is written to both triangles. ROWS bounds ca, cb (LDS is sized for it). A chunk is loaded in
// K pairs (16-byte loads when n is even) from clamped addresses, all of a thread's
// loads at once, and the out-of-block elements are zeroed when stored; for up to 80
// rows the next chunk is in flight while the current one computes.
constexpr int GR_KC = 32, GR_PW = GR_KC + 2;

template <int TPW, int ROWS>
__global__ __launch_bounds__(512) void gram_kernel(const GramDesc* __restrict__ descs) {
  constexpr int HK = GR_KC / 2;                  // K pairs per row and chunk
  constexpr int NPF = (ROWS * HK + 511) / 512;   // pairs staged per thread and operand
  // the next chunk in flight during the current one (one workgroup a CU from 81 rows
  // on); for the widest blocks the registers do not allow it and a chunk is loaded and
  // stored in one go
  constexpr bool PF = ROWS <= 128;
  __shared__ double As[ROWS * GR_PW];
  __shared__ double Bs[ROWS * GR_PW];
  const GramDesc d = descs[blockIdx.y];
  const int ca = d.ca, cb = d.cb, n = d.n;
  const int s = blockIdx.x, ks = d.ks;  // (the grid's x is the call's largest ks)
  if (ca <= 0 || cb <= 0 || s >= ks) return;
  int lk = (n + ks - 1) / ks;
  lk = ((lk + GR_KC - 1) / GR_KC) * GR_KC;
  const int k0 = s * lk, k1 = min(n, k0 + lk);
  const bool same = d.A == d.B && ca == cb;
  const bool tri = same || (d.sym && ca == cb);  // upper tiles only, mirrored
  const int TA = (ca + 15) / 16, TB = (cb + 15) / 16;
  const int ra = TA * 16, rb = TB * 16;
  const int nt = tri ? TA * (TA + 1) / 2 : TA * TB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, l16 = lane & 15;
  // rows start 16-byte aligned when n is even (the arena aligns blocks to 256 bytes),
  // and then a chunk's pairs never straddle the slice end (k0, k1 even)
  const bool pairs = (n & 1) == 0;
  // output tile of slot i: row-major over TA x TB, or the upper triangle row by row
  auto tile_of = [&](int t, int& tr, int& tc) {
    if (!tri) { tr = t / TB; tc = t % TB; return; }
    int r = 0, left = t;
    while (left >= TA - r) { left -= TA - r; ++r; }
    tr = r; tc = r + left;
  };
  typedef const __attribute__((address_space(1))) double gdbl;  // global, not flat, loads
  typedef const __attribute__((address_space(1))) d2 gd2;
  d2 pa[NPF], pb[NPF];
  auto fetch = [&](const double* M, int c, int kc, d2* st) {
#pragma unroll
    for (int i = 0; i < NPF; ++i) {
      const int e = tid + i * 512, row = e / HK, k = kc + 2 * (e % HK);
      gdbl* rp = (gdbl*)M + (long)(row < c ? row : 0) * n;
      if (pairs) {
        st[i] = *reinterpret_cast<gd2*>(rp + (k < k1 ? k : 0));
      } else {
        st[i].x = rp[k < k1 ? k : 0];
        st[i].y = rp[k + 1 < k1 ? k + 1 : 0];
      }
    }
  };
  auto put = [&](int c, int r, int kc, const d2* st, double* dst) {
#pragma unroll
    for (int i = 0; i < NPF; ++i) {
      const int e = tid + i * 512, row = e / HK, cp = e % HK, k = kc + 2 * cp;
      if (row < r) {
        const bool rin = row < c;
        d2 v;
        v.x = rin && k < k1 ? st[i].x : 0.0;
        v.y = rin && k + 1 < k1 ? st[i].y : 0.0;
        *reinterpret_cast<d2*>(dst + row * GR_PW + 2 * cp) = v;
      }
    }
  };
  d4 acc[TPW];
  int tco[TPW];  // tile coordinates tr << 8 | tc of slot i
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    acc[i] = d4{0.0, 0.0, 0.0, 0.0};
    int tr = 0, tc = 0;
    if (wave + 8 * i < nt) tile_of(wave + 8 * i, tr, tc);
    tco[i] = tr << 8 | tc;
  }
  const double* Bsrc = same ? As : Bs;
  if (PF && k0 < k1) {
    fetch(d.A, ca, k0, pa);
    if (!same) fetch(d.B, cb, k0, pb);
    put(ca, ra, k0, pa, As);
    if (!same) put(cb, rb, k0, pb, Bs);
    __syncthreads();
  }
  for (int kc = k0; kc < k1; kc += GR_KC) {
    const bool more = kc + GR_KC < k1;
    if constexpr (PF) {
      if (more) {
        fetch(d.A, ca, kc + GR_KC, pa);
        if (!same) fetch(d.B, cb, kc + GR_KC, pb);
      }
    } else {  // A, then B through the same registers
      fetch(d.A, ca, kc, pa);
      put(ca, ra, kc, pa, As);
      if (!same) {
        fetch(d.B, cb, kc, pa);
        put(cb, rb, kc, pa, Bs);
      }
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int t = wave + 8 * i;
      if (t >= nt) break;
      const int tr = tco[i] >> 8, tc = tco[i] & 255;
      const double* ar = As + (tr * 16 + l16) * GR_PW + 8 * g;
      const double* br = Bsrc + (tc * 16 + l16) * GR_PW + 8 * g;
      double av[8], bv[8];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double2 x = *reinterpret_cast<const double2*>(ar + 2 * q);
        const double2 y = *reinterpret_cast<const double2*>(br + 2 * q);
        av[2 * q] = x.x; av[2 * q + 1] = x.y;
        bv[2 * q] = y.x; bv[2 * q + 1] = y.y;
      }
#pragma unroll
      for (int st = 0; st < 8; ++st) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[st], bv[st], acc[i], 0, 0, 0);
    }
    __syncthreads();
    if (PF && more) {
      put(ca, ra, kc + GR_KC, pa, As);
      if (!same) put(cb, rb, kc + GR_KC, pb, Bs);
      __syncthreads();
    }
  }
  double* out = d.work + (long)s * ca * cb;
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const int t = wave + 8 * i;
    if (t >= nt) break;
    int tr, tc;
    tile_of(t, tr, tc);
    const int col = tc * 16 + l16;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = tr * 16 + 4 * r + g;  // FP64 accumulator layout
      if (row < ca && col < cb) {
        out[(long)row * cb + col] = acc[i][r];
        if (tri && tr != tc) out[(long)col * cb + row] = acc[i][r];
      }
    }
  }
}

void gram_batched(hipStream_t s, const GramDesc* d, int P, int ks, int cmax) {
  if (P <= 0 || cmax <= 0) return;
  if (ks < 1) ks = 1;  // the largest ks of the descriptors
  const int t = (cmax + 15) / 16;
  if (t <= 5)
    hipLaunchKernelGGL((gram_kernel<4, 80>), dim3(ks, P), dim3(512), 0, s, d);
  else if (t <= 8)  // up to 128 rows: 70 KB of LDS, two workgroups a CU
    hipLaunchKernelGGL((gram_kernel<8, 128>), dim3(ks, P), dim3(512), 0, s, d);
  else
    hipLaunchKernelGGL((gram_kernel<18, 192>), dim3(ks, P), dim3(512), 0, s, d);
}

int gemm_pick_ksplit(int M, int N, int K, int batch) {
  long tiles = (long)((M + GB_M - 1) / GB_M) * ((N + GB_N - 1) / GB_N) * batch;
  if (tiles >= 256) return 1;
  long want = 512 / tiles;
  long maxk = (K + 63) / 64;  // keep at least 64 of K per split
  long ks = want < maxk ? want : maxk;
  if (ks > 64) ks = 64;
  return ks < 1 ? 1 : (int)ks;
}

void gemm_f64(hipStream_t s, bool tA, bool tB, int M, int N, int K, double alpha,
              const double* A, long lda, long sA, const double* B, long ldb, long sB,
              double beta, double* C, long ldc, long sC, int batch, int ksplit, double* work) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  if (K <= 0) K = 0;  // the kernel then writes C = beta * C
  if (ksplit < 1 || work == nullptr || K == 0) ksplit = 1;
  int kchunk = (K + ksplit - 1) / ksplit;
  kchunk = ((kchunk + GB_K - 1) / GB_K) * GB_K;
  if (kchunk < GB_K) kchunk = GB_K;
  ksplit = K > 0 ? (K + kchunk - 1) / kchunk : 1;
  dim3 grid((N + GB_N - 1) / GB_N, (M + GB_M - 1) / GB_M, batch * ksplit);
  hipLaunchKernelGGL(gemm_f64_kernel, grid, dim3(256), 0, s, (int)tA, (int)tB, M, N, K, kchunk,
                     alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, ksplit, work, 0);
  if (ksplit > 1) {
    long total = (long)batch * M * N;
    int blocks = (int)((total + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3(blocks), dim3(256), 0, s, M, N, batch, ksplit,
                       work, beta, C, ldc, sC);
  }
}

int gemm_f64_partials(hipStream_t s, bool tA, bool tB, int M, int N, int K, const double* A,
                      long lda, const double* B, long ldb, int ksplit, double* work) {
  if (M <= 0 || N <= 0) return 1;
  if (K < 0) K = 0;
  if (ksplit < 1 || K == 0) ksplit = 1;
  int kchunk = (K + ksplit - 1) / ksplit;
  kchunk = ((kchunk + GB_K - 1) / GB_K) * GB_K;
  if (kchunk < GB_K) kchunk = GB_K;
  ksplit = K > 0 ? (K + kchunk - 1) / kchunk : 1;
  dim3 grid((N + GB_N - 1) / GB_N, (M + GB_M - 1) / GB_M, ksplit);
  hipLaunchKernelGGL(gemm_f64_kernel, grid, dim3(256), 0, s, (int)tA, (int)tB, M, N, K, kchunk, 1.0,
                     A, lda, 0L, B, ldb, 0L, 0.0, (double*)nullptr, 0L, 0L, 1, ksplit, work, 1);
  return ksplit;
}

// ---------------------------------------------------------------------------
// Elementwise and reductions.
// ---------------------------------------------------------------------------
__global__ void axpy_epilogue_kernel(int nv, int n, double* __restrict__ out, const double* __restrict__ Y,
                                     const double* __restrict__ Xp, const double* __restrict__ diag,
                                     double s1, double s2, double s3, int out_zero) {
  long total = (long)nv * n;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total;
       t += (long)gridDim.x * blockDim.x) {
    int i = (int)(t % n);
    double y = Y[t];
    double v = out_zero ? 0.0 : out[t];
    if (diag) v += s1 * diag[i] * y;
    v += s2 * y;
    if (Xp) v += s3 * Xp[t];
    out[t] = v;
  }
}

void axpy_epilogue(hipStream_t s, int nv, int n, double* out, const double* Y, const double* Xprev,
                   const double* diag, double s1, double s2, double s3, bool out_is_zero) {
  long total = (long)nv * n;
  if (total <= 0) return;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(axpy_epilogue_kernel, dim3(blocks), dim3(256), 0, s, nv, n, out, Y,
                     s3 != 0.0 ? Xprev : nullptr, diag, s1, s2, s3, (int)out_is_zero);
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block (256 threads) sum in a fixed order: per-wave shuffle tree, then 4 partials.
__device__ inline double block_sum256(double v, double* red) {
  v = wave_sum(v);
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = v;
  __syncthreads();
  double t = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return t;
}

__global__ __launch_bounds__(256) void row_norms_kernel(int n, double* __restrict__ Y, double* __restrict__ norms,
                                                        int normalize) {
  __shared__ double red[4];
  double* y = Y + (long)blockIdx.x * n;
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += y[i] * y[i];
  double s = sqrt(block_sum256(acc, red));
  if (threadIdx.x == 0) norms[blockIdx.x] = s;
  if (normalize && s > 0.0) {
    double inv = 1.0 / s;
    for (int i = threadIdx.x; i < n; i += 256) y[i] *= inv;
  }
}

void row_norms(hipStream_t s, int nv, int n, double* Y, double* norms, bool normalize) {
  if (nv <= 0) return;
  hipLaunchKernelGGL(row_norms_kernel, dim3(nv), dim3(256), 0, s, n, Y, norms, (int)normalize);
}

__global__ __launch_bounds__(256) void residual_norms_kernel(int n, const double* __restrict__ HX,
                                                             const double* __restrict__ X,
                                                             const double* __restrict__ theta,
                                                             double* __restrict__ res) {
  __shared__ double red[4];
  const double* hx = HX + (long)blockIdx.x * n;
  const double* x = X + (long)blockIdx.x * n;
  double th = theta[blockIdx.x];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    double r = hx[i] - th * x[i];
    acc += r * r;
  }
  double s = sqrt(block_sum256(acc, red));
  if (threadIdx.x == 0) res[blockIdx.x] = s;
}

void residual_norms(hipStream_t s, int nv, int n, const double* HX, const double* X,
                    const double* theta, double* res) {
  if (nv <= 0) return;
  hipLaunchKernelGGL(residual_norms_kernel, dim3(nv), dim3(256), 0, s, n, HX, X, theta, res);
}

// out_j = a[j] * P_j + b * Q_j (Q may be null), rows of length n.
__global__ void rows_scale_add_kernel(int nv, int n, double* __restrict__ out, const double* __restrict__ Pm,
                                      const double* __restrict__ a, double asgn, double b,
                                      const double* __restrict__ Qm) {
  long total = (long)nv * n;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total;
       t += (long)gridDim.x * blockDim.x) {
    int j = (int)(t / n);
    double v = asgn * a[j] * Pm[t];
    if (Qm) v += b * Qm[t];
    out[t] = v;
  }
}

void rows_scale_add(hipStream_t s, int nv, int n, double* out, const double* P, const double* a,
                    double asgn, double b, const double* Q) {
  long total = (long)nv * n;
  if (total <= 0) return;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(rows_scale_add_kernel, dim3(blocks), dim3(256), 0, s, nv, n, out, P, a, asgn, b, Q);
}

__global__ void copy_rows_kernel(int nv, int n, const double* __restrict__ src, long lds,
                                 double* __restrict__ dst, long ldd) {
  long total = (long)nv * n;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total;
       t += (long)gridDim.x * blockDim.x) {
    int j = (int)(t / n), i = (int)(t % n);
    dst[(long)j * ldd + i] = src[(long)j * lds + i];
  }
}

void copy_rows(hipStream_t s, int nv, int n, const double* src, long ld_src, double* dst,
               long ld_dst) {
  long total = (long)nv * n;
  if (total <= 0) return;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(copy_rows_kernel, dim3(blocks), dim3(256), 0, s, nv, n, src, ld_src, dst,
                     ld_dst);
}

__global__ __launch_bounds__(256) void vec_max_kernel(int n, const double* __restrict__ v,
                                                      double* __restrict__ out) {
  __shared__ double red[256];
  double m = -INFINITY;
  for (int i = threadIdx.x; i < n; i += 256) m = fmax(m, v[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

void vec_max(hipStream_t s, int n, const double* v, double* out) {
  hipLaunchKernelGGL(vec_max_kernel, dim3(1), dim3(256), 0, s, n, v, out);
}

// 1/sqrt(x) and 1/x for x > 0 (normal range): the hardware estimates refined by two
// Newton steps (each one squares the relative error). Only the rotation's c stays
// tied to working precision through these (c^2 (1 + t^2) = 1); an inexact t leaves
// a slightly larger off-diagonal entry for the next sweep.
__device__ inline double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * (1.5 - 0.5 * x * y * y);
  y = y * (1.5 - 0.5 * x * y * y);
  return y;
}
__device__ inline double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = y * (2.0 - x * y);
  y = y * (2.0 - x * y);
  return y;
}

// ---------------------------------------------------------------------------
// Cholesky + in-place inverse of the lower factor, one 1024-thread workgroup
// (a 32 x 32 thread grid), packed lower triangle in LDS (m <= 192 -> at most
// 151 KB). The input Gram matrix may be given as nparts split-K partial
// sums (stride pstride), added in a fixed order while loading. The factor is
// taken of the equilibrated D^-1 G D^-1 (d_i = sqrt(G_ii)) and the output is
// L^-1 D^-1 = (D L)^-1, so rows of any scale need no normalisation beforehand
// (CholeskyQR is invariant to it) and the pivots stay on the unit scale.
// ---------------------------------------------------------------------------
constexpr int JMAX = 192;
constexpr int CHOL_THREADS = 1024;
__device__ inline int lidx(int i, int j) { return i * (i + 1) / 2 + j; }  // j <= i

__device__ inline int tri_row(int t) {  // row i of packed lower index t
  int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while (i * (i + 1) / 2 > t) --i;
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  return i;
}

__device__ void chol_inv_body(int m, const double* __restrict__ G, int nparts, long pstride,
                              double shift, double* __restrict__ Linv, int* __restrict__ info,
                              double* L, double* col, double* dinv) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int ty = tid >> 5, tx = tid & 31;  // 32 x 32 thread grid
  const int np = m * (m + 1) / 2;
  // equilibration: factor D^-1 G D^-1 (d_i = sqrt(G_ii), 1 for an empty row) and
  // return L^-1 D^-1, the inverse of G's own lower factor D L
  for (int i = tid; i < m; i += nt) {
    double v = 0.0;
    for (int ks = 0; ks < nparts; ++ks) v += G[(long)ks * pstride + (long)i * m + i];
    dinv[i] = v > 0.0 ? 1.0 / sqrt(v) : 1.0;
  }
  __syncthreads();
  for (int t = tid; t < np; t += nt) {
    int i = tri_row(t);
    int j = t - i * (i + 1) / 2;
    double v = 0.0;
    for (int ks = 0; ks < nparts; ++ks) {
      const double* g = G + (long)ks * pstride;
      v += 0.5 * (g[(long)i * m + j] + g[(long)j * m + i]);
    }
    v *= dinv[i] * dinv[j];
    if (i == j) v += shift;
    L[t] = v;
  }
  __syncthreads();
  int fail = 0;
  // right-looking factorisation; col[] keeps the sqrt of the pivots
  for (int j = 0; j < m; ++j) {
    const double d = L[lidx(j, j)];
    if (!(d > 0.0)) { fail = 1; break; }
    const double sd = sqrt(d);
    if (tid == 0) col[j] = sd;
    const double inv = 1.0 / sd;
    for (int i = j + 1 + tid; i < m; i += nt) L[lidx(i, j)] *= inv;
    __syncthreads();
    for (int r = j + 1 + ty; r < m; r += 32) {
      const int base = r * (r + 1) / 2;
      const double lrj = L[base + j];
      for (int c = j + 1 + tx; c <= r; c += 32) L[base + c] -= lrj * L[c * (c + 1) / 2 + j];
    }
    __syncthreads();
  }
  if (tid == 0) info[0] = fail;
  if (fail) return;
  for (int j = tid; j < m; j += nt) L[lidx(j, j)] = col[j];
  __syncthreads();
  // in-place inverse, columns right to left: X[i][j] = -(sum_{k=j+1..i} X[i][k] L[k][j]) / L[j][j]
  for (int j = m - 1; j >= 0; --j) {
    for (int i = j + 1 + tid; i < m; i += nt) col[i] = L[lidx(i, j)];
    const double d = L[lidx(j, j)];
    __syncthreads();
    for (int i0 = j + 1; i0 < m; i0 += 32) {
      const int i = i0 + ty;
      double acc = 0.0;
      const int base = i * (i + 1) / 2;
      if (i < m)
        for (int k = j + 1 + tx; k <= i; k += 32) acc += L[base + k] * col[k];
#pragma unroll
      for (int off = 16; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 32);
      if (i < m && tx == 0) L[base + j] = -acc / d;
    }
    if (tid == 0) L[lidx(j, j)] = 1.0 / d;
    __syncthreads();
  }
  for (long t = tid; t < (long)m * m; t += nt) {
    int i = (int)(t / m), j = (int)(t % m);
    Linv[t] = j <= i ? L[lidx(i, j)] * dinv[j] : 0.0;
  }
}

// The same factorisation (equilibrated the same way) and inverse for m <= 80 by
// 8-wide blocks, so that a panel
// costs three barriers instead of eight steps of two. Matrix in LDS with an odd row
// stride, padded to a multiple of 8 with the identity. Per panel: wave 0 factors the
// 8 x 8 diagonal block in registers (lane (r, c), shuffles), the rows below are solved
// against it, then the trailing matrix takes the rank-8 update. The inverse X = L^{-1}
// goes to the unused upper triangle (X[i][j] at (j, i)) and its diagonal to xd: the
// diagonal blocks first (one wave each), then the blocks below them one block
// diagonal at a time, X_IJ = -X_II (sum_{J <= K < I} L_IK X_KJ).
constexpr int CB_MAX = 80;
size_t chol_blocked_lds_bytes(int m) {
  const int mp = (m + 7) & ~7;
  return ((size_t)mp * (mp + 1) + 3 * (size_t)mp + 2) * sizeof(double);
}

__device__ __forceinline__ void chol_blocked_body(int m, const double* __restrict__ G, int nparts, long pstride,
                                                  double shift, double* __restrict__ Linv,
                                                  int* __restrict__ info, double* sm) {
  const int mp = (m + 7) & ~7, nb = mp / 8, LD = mp + 1;
  double* A = sm;            // [mp][LD]
  double* xd = A + mp * LD;  // diagonal of X
  double* rd = xd + mp;      // 1 / L[i][i]
  double* dv = rd + mp;      // 1 / d_i of the equilibration
  int* flag = (int*)(dv + mp);
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = tid >> 6;
  const int r8 = lane >> 3, c8 = lane & 7;
  for (int i = tid; i < mp; i += nt) {
    double v = 0.0;
    if (i < m)
      for (int ks = 0; ks < nparts; ++ks) v += G[(long)ks * pstride + (long)i * m + i];
    dv[i] = v > 0.0 ? 1.0 / sqrt(v) : 1.0;
  }
  __syncthreads();
  for (int t = tid; t < mp * mp; t += nt) {
    const int i = t / mp, j = t % mp;
    if (j > i) continue;
    double v = (i == j) ? 1.0 : 0.0;
    if (i < m) {
      v = 0.0;
      for (int ks = 0; ks < nparts; ++ks) {
        const double* g = G + (long)ks * pstride;
        v += 0.5 * (g[(long)i * m + j] + g[(long)j * m + i]);
      }
      v *= dv[i] * dv[j];
      if (i == j) v += shift;
    }
    A[i * LD + j] = v;
  }
  if (tid == 0) *flag = 0;
  __syncthreads();
  for (int J = 0; J < nb; ++J) {
    const int j0 = 8 * J;
    if (wave == 0) {
      double D = (c8 <= r8) ? A[(j0 + r8) * LD + j0 + c8] : 0.0;
      bool bad = false;
      for (int k = 0; k < 8; ++k) {
        const double dkk = __shfl(D, k * 9, 64);
        if (!(dkk > 0.0)) { bad = true; break; }
        const double inv = rsqrt_nr(dkk);
        if (c8 == k) D = (r8 == k) ? dkk * inv : (r8 > k ? D * inv : D);
        const double lrk = __shfl(D, r8 * 8 + k, 64);
        const double lck = __shfl(D, c8 * 8 + k, 64);
        if (r8 > k && c8 > k && c8 <= r8) D -= lrk * lck;
        if (lane == 0) rd[j0 + k] = inv;
      }
      if (bad) {
        if (lane == 0) *flag = 1;
      } else if (c8 <= r8) {
        A[(j0 + r8) * LD + j0 + c8] = D;
      }
    }
    __syncthreads();
    if (*flag) break;
    // rows below the block: x L_JJ^T = a
    for (int i = j0 + 8 + tid; i < mp; i += nt) {
      double x[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) x[c] = A[i * LD + j0 + c];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        double a = x[c];
#pragma unroll
        for (int k = 0; k < c; ++k) a -= x[k] * A[(j0 + c) * LD + j0 + k];
        x[c] = a * rd[j0 + c];
      }
#pragma unroll
      for (int c = 0; c < 8; ++c) A[i * LD + j0 + c] = x[c];
    }
    __syncthreads();
    // trailing rank-8 update
    const int t0 = j0 + 8, nr = mp - t0;
    for (int e = tid; e < nr * nr; e += nt) {
      const int i = t0 + e / nr, k = t0 + e % nr;
      if (k > i) continue;
      double acc = A[i * LD + k];
#pragma unroll
      for (int c = 0; c < 8; ++c) acc -= A[i * LD + j0 + c] * A[k * LD + j0 + c];
      A[i * LD + k] = acc;
    }
    __syncthreads();
  }
  if (*flag) {
    if (tid == 0) info[0] = 1;
    return;
  }
  // diagonal blocks of X, wave J
  if (wave < nb) {
    const int j0 = 8 * wave;
    double X = (r8 == c8) ? rd[j0 + r8] : 0.0;
    for (int rr = 1; rr < 8; ++rr) {
      double acc = 0.0;
      for (int k = 0; k < rr; ++k) {
        const double xkc = __shfl(X, k * 8 + c8, 64);
        if (k >= c8) acc += A[(j0 + rr) * LD + j0 + k] * xkc;
      }
      if (r8 == rr && c8 < rr) X = -acc * rd[j0 + rr];
    }
    if (c8 < r8) A[(j0 + c8) * LD + j0 + r8] = X;
    else if (c8 == r8) xd[j0 + r8] = X;
  }
  __syncthreads();
  // blocks (J + d, J), one wave each
  for (int d = 1; d < nb; ++d) {
    const int J = wave;
    if (J < nb - d) {
      const int I = J + d, i0 = 8 * I, j0 = 8 * J;
      double T = 0.0;
      for (int a = j0; a < i0; ++a) {
        const int b = j0 + c8;
        const double xab = a > b ? A[b * LD + a] : (a == b ? xd[a] : 0.0);
        T += A[(i0 + r8) * LD + a] * xab;
      }
      double X = 0.0;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const double tkc = __shfl(T, k * 8 + c8, 64);
        const double xrk = k < r8 ? A[(i0 + k) * LD + i0 + r8] : (k == r8 ? xd[i0 + r8] : 0.0);
        X -= xrk * tkc;
      }
      A[(j0 + c8) * LD + i0 + r8] = X;
    }
    __syncthreads();
  }
  for (int t = tid; t < m * m; t += nt) {
    const int i = t / m, j = t % m;
    Linv[t] = (j < i ? A[j * LD + i] : (j == i ? xd[i] : 0.0)) * dv[j];
  }
  if (tid == 0) info[0] = 0;
}

__global__ __launch_bounds__(CHOL_THREADS) void chol_inv_kernel(int m, const double* __restrict__ G, int nparts,
                                                                long pstride, double shift,
                                                                double* __restrict__ Linv, int* __restrict__ info) {
  extern __shared__ double sm[];
  chol_inv_body(m, G, nparts, pstride, shift, Linv, info, sm, sm + m * (m + 1) / 2, sm + m * (m + 1) / 2 + m);
}

size_t chol_lds_bytes(int m) { return ((size_t)m * (m + 1) / 2 + 2 * (size_t)m) * sizeof(double); }

void chol_inv(hipStream_t s, int m, const double* G, int nparts, long pstride, double shift,
              double* Linv, int* info) {
  hipLaunchKernelGGL(chol_inv_kernel, dim3(1), dim3(CHOL_THREADS), chol_lds_bytes(m), s, m, G,
                     nparts < 1 ? 1 : nparts, pstride, shift, Linv, info);
}

__global__ __launch_bounds__(CHOL_THREADS) void chol_batched_kernel(const CholDesc* __restrict__ descs) {
  extern __shared__ double sm[];
  const CholDesc d = descs[blockIdx.x];
  double* L = sm;
  double* col = sm + d.m * (d.m + 1) / 2;
  double* dinv = col + d.m;
  const bool blk = d.m <= CB_MAX;
  if (blk) chol_blocked_body(d.m, d.G, d.nparts, d.pstride, 0.0, d.Linv, d.info, sm);
  else chol_inv_body(d.m, d.G, d.nparts, d.pstride, 0.0, d.Linv, d.info, L, col, dinv);
  __syncthreads();
  const int failed = d.info[0];
  __syncthreads();
  if (failed) {  // shifted CholeskyQR: retry with the shift, flag it in info[1]
    if (blk) chol_blocked_body(d.m, d.G, d.nparts, d.pstride, d.shift, d.Linv, d.info, sm);
    else chol_inv_body(d.m, d.G, d.nparts, d.pstride, d.shift, d.Linv, d.info, L, col, dinv);
    if (threadIdx.x == 0) d.info[1] = 1;
  } else if (threadIdx.x == 0) {
    d.info[1] = 0;
  }
}

void chol_batched(hipStream_t s, const CholDesc* d, int P, int mmax) {
  if (P <= 0) return;
  const size_t lds = std::max(chol_lds_bytes(mmax), chol_blocked_lds_bytes(std::min(mmax, CB_MAX)));
  hipLaunchKernelGGL(chol_batched_kernel, dim3(P), dim3(CHOL_THREADS), lds, s, d);
}

// ---------------------------------------------------------------------------
// Parallel cyclic Jacobi (round-robin ordering) for symmetric m x m, m <= 192.
// Packed upper triangle of A in LDS; eigenvectors accumulated in LDS when they
// fit beside it, else in global memory (Vwork). Rotation of pair (p,q) skipped
// when |a_pq| <= max(eps sqrt|a_pp a_qq|, eps ||A||_F); before each sweep all
// off-diagonal entries are tested and the loop ends when none exceeds that.
// ---------------------------------------------------------------------------
constexpr int JAC_THREADS = 1024;
__device__ inline int uidx(int i, int j) { return j * (j + 1) / 2 + i; }  // i <= j
__device__ inline int sidx(int i, int j) { return i <= j ? uidx(i, j) : uidx(j, i); }
__device__ inline int rr_player(int pos, int step, int M) {
  if (pos == 0) return 0;
  int x = pos - 1 + step;  // < 2 (M - 1)
  if (x >= M - 1) x -= M - 1;
  return 1 + x;
}

size_t jacobi_lds_doubles(int m, bool vlds) {
  const int M = m + (m & 1), H = M / 2;
  // A (packed upper), two rotation buffers (c, s, t doubles; p, q, active ints),
  // reduction scratch and flag
  size_t d = (size_t)M * (M + 1) / 2 + 6 * (size_t)H + 3 * (size_t)H + 2 + 64;
  if (vlds) d += (size_t)m * m;
  return d;
}
static bool jacobi_v_in_lds(int m) { return jacobi_lds_doubles(m, true) * 8 <= 156 * 1024; }


// Parallel cyclic Jacobi (round-robin ordering: M-1 rounds of M/2 disjoint pairs per
// sweep), one 1024-thread workgroup, A packed in LDS. Each round has two phases
// separated by barriers: (R) the round's rotations are computed from A while every
// thread applies the previous round's rotations to V (double-buffered rotation
// tables), (U) the 2x2 blocks of A touched by each pair of rotations are updated,
// one flat work item per block. Rotation (Rutishauser's form of the symmetric 2x2
// Schur decomposition): d = a_qq - a_pp, h = 2 a_pq, t = sign(d) h / (|d| + hypot(d, h)),
// c = 1/sqrt(1 + t^2), s = t c (reciprocals and roots by refined estimates). A pair is rotated when a_pq^2 > eps^2 |a_pp a_qq| and
// |a_pq| > eps ||A||_F; the sweep loop stops when no pair qualifies.
__device__ __forceinline__ void jacobi_body(int m, const double* __restrict__ Ab, int nparts, long pstride,
                            double* __restrict__ evals, double* __restrict__ Vout,
                            double* __restrict__ Vg, int vlds, int max_sweeps, int* __restrict__ info,
                            double* sm) {
  const int M = m + (m & 1);
  const int H = M / 2;
  double* A = sm;                        // M*(M+1)/2
  double* cs = A + M * (M + 1) / 2;      // [2][H]
  double* sn = cs + 2 * H;               // [2][H]
  double* tn = sn + 2 * H;               // [2][H]
  int* pp = (int*)(tn + 2 * H);          // [2][H]
  int* qq = pp + 2 * H;                  // [2][H]
  int* act = qq + 2 * H;                 // [2][H]
  double* red = (double*)(((uintptr_t)(act + 2 * H) + 15) & ~(uintptr_t)15);  // 64
  int* flag = (int*)(red + 32);
  double* V = vlds ? (red + 64) : Vg;
  const int tid = threadIdx.x, nt = blockDim.x;

  double nrm = 0.0;
  const int np = M * (M + 1) / 2;
  for (int t = tid; t < np; t += nt) {
    int j = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while (j * (j + 1) / 2 > t) --j;
    while ((j + 1) * (j + 2) / 2 <= t) ++j;
    int i = t - j * (j + 1) / 2;
    double v = 0.0;
    if (j < m)
      for (int ks = 0; ks < nparts; ++ks) {
        const double* g = Ab + (long)ks * pstride;
        v += 0.5 * (g[(long)i * m + j] + g[(long)j * m + i]);
      }
    A[t] = v;
    nrm += (i == j ? 1.0 : 2.0) * v * v;
  }
  for (long t = tid; t < (long)m * m; t += nt) V[t] = ((t / m) == (t % m)) ? 1.0 : 0.0;
  nrm = wave_sum(nrm);
  if ((tid & 63) == 0) red[tid >> 6] = nrm;
  __syncthreads();
  double fro = 0.0;
  for (int w = 0; w < (nt >> 6); ++w) fro += red[w];
  fro = sqrt(fro);
  const double eps = 2.220446049250313e-16, eps2 = eps * eps;
  const double floor_abs = eps * fro;
  const int npair = H * (H + 1) / 2;  // blocks (k, l), k <= l

  // V update: thread (k, g) applies rotation k to the rows g, g + VG, g + 2 VG, ...
  // (VG row groups), so each thread reads its rotation's table entries once per round
  const int VG = nt / H;
  const int vk = tid % H, vg = tid / H;
  auto apply_v = [&](int b) {
    if (vg >= VG || !act[b * H + vk]) return;
    const int p = pp[b * H + vk], q = qq[b * H + vk];
    const double c = cs[b * H + vk], s = sn[b * H + vk];
    for (int r = vg; r < m; r += VG) {
      double* row = V + (long)r * m;
      const double vp = row[p], vq = row[q];
      row[p] = c * vp - s * vq;
      row[q] = s * vp + c * vq;
    }
  };
  // this thread's first 2x2 block (k, l), k <= l, of the A update (the same in every
  // round); further blocks (m > 88) are decoded on the fly
  int uk0 = 0, ul0 = 0;
  if (tid < npair) {
    int l = (int)((sqrtf(8.0f * tid + 1.0f) - 1.0f) * 0.5f);
    while (l * (l + 1) / 2 > tid) --l;
    while ((l + 1) * (l + 2) / 2 <= tid) ++l;
    ul0 = l;
    uk0 = tid - l * (l + 1) / 2;
  }

  int sweeps = 0;
  bool converged = false;
  for (;;) {
    // any off-diagonal entry above its threshold?
    if (tid == 0) *flag = 0;
    __syncthreads();
    for (int t = tid; t < np; t += nt) {
      int j = (int)((sqrtf(8.0f * t + 1.0f) - 1.0f) * 0.5f);
      while (j * (j + 1) / 2 > t) --j;
      while ((j + 1) * (j + 2) / 2 <= t) ++j;
      const int i = t - j * (j + 1) / 2;
      if (i == j || j >= m) continue;
      const double apq = A[t];
      if (apq * apq > eps2 * fabs(A[uidx(i, i)] * A[uidx(j, j)]) && fabs(apq) > floor_abs) *flag = 1;
    }
    __syncthreads();
    if (*flag == 0) { converged = true; break; }
    if (sweeps >= max_sweeps) break;
    ++sweeps;
    __syncthreads();
    for (int step = 0; step < M - 1; ++step) {
      const int b = step & 1;
      int any_rot = 0;
      // (R) rotations of this round; V update with the previous round's
      for (int k = tid; k < H; k += nt) {
        int p = rr_player(k, step, M), q = rr_player(M - 1 - k, step, M);
        if (p > q) { int t = p; p = q; q = t; }
        double c = 1.0, s = 0.0, t = 0.0;
        int a = 0;
        if (q < m) {
          const double apq = A[uidx(p, q)];
          const double app = A[uidx(p, p)], aqq = A[uidx(q, q)];
          if (apq * apq > eps2 * fabs(app * aqq) && fabs(apq) > floor_abs) {
            const double d = aqq - app, h = 2.0 * apq;
            const double x = d * d + h * h;
            const double r = x * rsqrt_nr(x);
            t = (d >= 0.0 ? h : -h) * rcp_nr(fabs(d) + r);
            c = rsqrt_nr(1.0 + t * t);
            s = t * c;
            a = 1;
          }
        }
        pp[b * H + k] = p; qq[b * H + k] = q; cs[b * H + k] = c; sn[b * H + k] = s;
        tn[b * H + k] = t; act[b * H + k] = a;
        any_rot |= a;
      }
      if (step > 0) apply_v(b ^ 1);
      // barrier and vote: a round with no rotation leaves A as it is
      if (!__syncthreads_or(any_rot)) continue;
      // (U) 2x2 blocks of A, one flat work item per block (k, l), k <= l
      const int* p_ = pp + b * H;
      const int* q_ = qq + b * H;
      const int* a_ = act + b * H;
      for (int w = tid; w < npair; w += nt) {
        int l = ul0, k = uk0;
        if (w != tid) {
          l = (int)((sqrtf(8.0f * w + 1.0f) - 1.0f) * 0.5f);
          while (l * (l + 1) / 2 > w) --l;
          while ((l + 1) * (l + 2) / 2 <= w) ++l;
          k = w - l * (l + 1) / 2;
        }
        if (!a_[k] && !a_[l]) continue;
        const int pk = p_[k], qk = q_[k];
        if (k == l) {
          const double apq = A[uidx(pk, qk)];
          const double tk = tn[b * H + k];
          A[uidx(pk, pk)] -= tk * apq;
          A[uidx(qk, qk)] += tk * apq;
          A[uidx(pk, qk)] = 0.0;
          continue;
        }
        const int pl = p_[l], ql = q_[l];
        const double ck = cs[b * H + k], sk = sn[b * H + k], cl = cs[b * H + l], sl = sn[b * H + l];
        const int i00 = sidx(pk, pl), i01 = sidx(pk, ql), i10 = sidx(qk, pl), i11 = sidx(qk, ql);
        const double m00 = A[i00], m01 = A[i01], m10 = A[i10], m11 = A[i11];
        const double r00 = ck * m00 - sk * m10, r01 = ck * m01 - sk * m11;
        const double r10 = sk * m00 + ck * m10, r11 = sk * m01 + ck * m11;
        A[i00] = r00 * cl - r01 * sl;
        A[i01] = r00 * sl + r01 * cl;
        A[i10] = r10 * cl - r11 * sl;
        A[i11] = r10 * sl + r11 * cl;
      }
      __syncthreads();
    }
    apply_v((M - 2) & 1);  // the sweep's last round
    __syncthreads();
  }
  for (int i = tid; i < m; i += nt) {
    double di = A[uidx(i, i)];
    int rank = 0;
    for (int j = 0; j < m; ++j) {
      double dj = A[uidx(j, j)];
      rank += (dj < di) || (dj == di && j < i);
    }
    evals[rank] = di;
    for (int r = 0; r < m; ++r) Vout[(long)r * m + rank] = V[(long)r * m + i];
  }
  if (tid == 0) info[0] = converged ? sweeps : -(sweeps + 1);
}

// ---------------------------------------------------------------------------
// The same cyclic Jacobi for 8 <= m <= 80 with A and V kept in the frame of the
// round-robin schedule. Positions 0..M-1 are paired (k, M-1-k) into H = M/2 slots;
// after every round each index moves from position j to j-1 (position 1 to M-1,
// position 0 fixed), which is what makes the schedule visit every pair once per
// sweep. Storing A and V by position instead of by index makes every address a
// thread touches fixed for the whole run: a round reads one buffer and writes the
// rotated values to the positions they move to in the other.
//   A: for each slot pair (k <= l) the 2x2 block of entries between positions
//      {k, M-1-k} x {l, M-1-l}, as four planes (LL, LR, RL, RR) of H(H+1)/2 blocks.
//   V: column of position j (the eigenvector estimate of the index there), rows in
//      pairs so that a lane moves 16 bytes.
// Roles (1024 threads): wave 0 lane k updates the block holding the two indices
// that meet in slot k next round and computes that rotation from the updated entry
// and the new diagonals (a rotation table carries c, s and the pair's diagonals
// after its rotation), so a round needs one barrier; waves 1..15 update the other
// blocks and the eigenvectors. Same rotation and thresholds as jacobi_body; m odd
// is padded with a zero index whose rotations never qualify.
// ---------------------------------------------------------------------------
constexpr int JS_MIN = 8, JS_MAX = 80;
constexpr int JS_HALF_MAX = 56;  // largest m the body takes with 512 threads

__device__ inline int js_next(int j, int M) { return j == 0 ? 0 : (j == M - 1 ? 1 : j + 1); }  // pos -> its index's previous pos
__device__ inline int js_prev(int x, int M) { return x == 0 ? 0 : (x == 1 ? M - 1 : x - 1); }  // where pos x moves
__device__ inline int js_blk(int k, int l) { return l * (l + 1) / 2 + k; }
// plane * npair + block of the entry at positions (i, j) after the move
__device__ inline int js_dest(int i, int j, int M, int H, int npair) {
  const int i2 = js_prev(i, M), j2 = js_prev(j, M);
  const int si = i2 < H ? i2 : M - 1 - i2, ri = i2 < H ? 0 : 1;
  const int sj = j2 < H ? j2 : M - 1 - j2, rj = j2 < H ? 0 : 1;
  if (si < sj) return (ri * 2 + rj) * npair + js_blk(si, sj);
  if (si > sj) return (rj * 2 + ri) * npair + js_blk(sj, si);
  return ((i2 == j2) ? (ri ? 3 : 0) : 1) * npair + js_blk(si, si);
}
size_t jacobi_shift_lds_doubles(int m) {
  const int M = m + (m & 1), H = M / 2, np = H * (H + 1) / 2;
  return 8 * (size_t)np + 2 * (size_t)M * M + 8 * (size_t)H + (size_t)M + 64 + 8;
}
__device__ inline void js_rot(double apq, double app, double aqq, double eps2, double floor_abs,
                              double& c, double& s, double& t) {
  c = 1.0; s = 0.0; t = 0.0;
  if (apq * apq > eps2 * fabs(app * aqq) && fabs(apq) > floor_abs) {
    const double d = aqq - app, h = 2.0 * apq;
    const double x = d * d + h * h;
    const double r = x * rsqrt_nr(x);
    t = (d >= 0.0 ? h : -h) * rcp_nr(fabs(d) + r);
    c = rsqrt_nr(1.0 + t * t);
    s = t * c;
  }
}

__device__ __forceinline__ void jacobi_shift_body(int m, const double* __restrict__ Ab, int nparts, long pstride,
                                  double* __restrict__ evals, double* __restrict__ Vout, int max_sweeps,
                                  int* __restrict__ info, double* sm) {
  constexpr int VJ = 2;  // eigenvector items per thread: ceil(H / ((1024 - 64) / (M / 2))) <= 2
  const int M = m + (m & 1), H = M / 2, hp = M / 2;
  const int npair = H * (H + 1) / 2;
  double* PL = sm;                                // [2][4][npair]
  double* VP = PL + 8 * npair;                    // [2][M][M]
  double2* CS = (double2*)(VP + 2 * M * M);       // [2][H] (c, s)
  double2* DD = CS + 2 * H;                       // [2][H] pair diagonals after the rotation
  double* dpos = (double*)(DD + 2 * H);           // [M]
  double* red = dpos + M;
  int* flag = (int*)(red + 32);
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63;
  const bool w0 = tid < 64;

  auto a_at = [&](int i, int j) -> double {
    if (i >= m || j >= m) return 0.0;
    double v = 0.0;
    for (int ks = 0; ks < nparts; ++ks) {
      const double* g = Ab + (long)ks * pstride;
      v += 0.5 * (g[(long)i * m + j] + g[(long)j * m + i]);
    }
    return v;
  };
  double nrm = 0.0;
  for (int w = tid; w < npair; w += nt) {
    int l = (int)((sqrtf(8.0f * w + 1.0f) - 1.0f) * 0.5f);
    while (l * (l + 1) / 2 > w) --l;
    while ((l + 1) * (l + 2) / 2 <= w) ++l;
    const int k = w - l * (l + 1) / 2;
    const double e0 = a_at(k, l), e1 = a_at(k, M - 1 - l), e2 = a_at(M - 1 - k, l), e3 = a_at(M - 1 - k, M - 1 - l);
    PL[w] = e0; PL[npair + w] = e1; PL[2 * npair + w] = e2; PL[3 * npair + w] = e3;
    nrm += (k == l) ? e0 * e0 + 2.0 * e1 * e1 + e3 * e3 : 2.0 * (e0 * e0 + e1 * e1 + e2 * e2 + e3 * e3);
  }
  for (int t = tid; t < M * M; t += nt) VP[t] = ((t / M) == (t % M)) ? 1.0 : 0.0;
  nrm = wave_sum(nrm);
  if ((tid & 63) == 0) red[tid >> 6] = nrm;
  __syncthreads();
  double fro = 0.0;
  for (int w = 0; w < (nt >> 6); ++w) fro += red[w];
  fro = sqrt(fro);
  const double eps = 2.220446049250313e-16, eps2 = eps * eps;
  const double floor_abs = eps * fro;

  // This thread's block. The block holding the indices that meet in slot kp next
  // round joins slots a = slot(js_next(kp)) and b = slot(js_next(M-1-kp)); these are
  // (k, k+2) for k <= H-3, (0, 1) and (H-2, H-1). Wave 0 lane kp takes it; waves
  // 1.. take the other blocks in column order (column l >= 1 starts at index
  // 1 + (l-1) l / 2 of that order).
  int bk = -1, bl = -1, sel = 0, pa = 0, psa = 0, pb = 0, psb = 0;
  if (w0) {
    if (lane < H) {
      const int x = js_next(lane, M), y = js_next(M - 1 - lane, M);
      pa = x < H ? x : M - 1 - x; psa = x < H ? 0 : 1;
      pb = y < H ? y : M - 1 - y; psb = y < H ? 0 : 1;
      bk = min(pa, pb); bl = max(pa, pb);
      sel = pa < pb ? psa * 2 + psb : psb * 2 + psa;
    }
  } else {
    const int j = tid - 64;
    if (j == 0) {
      bk = 0; bl = 0;
    } else if (j < npair - H) {
      int l = 1;
      while (l + 1 < H && 1 + l * (l + 1) / 2 <= j) ++l;
      const int r = j - (1 + (l - 1) * l / 2);
      bl = l;
      if (l == 1) bk = 1;
      else if (l == H - 1) bk = r < H - 3 ? r : r + 2;
      else bk = r < l - 2 ? r : r + 1;
    }
  }
  const bool has_blk = bk >= 0;
  int myb = 0, d0 = 0, d1 = 0, d2 = 0, d3 = 0;
  if (has_blk) {
    myb = js_blk(bk, bl);
    d0 = js_dest(bk, bl, M, H, npair);
    d1 = js_dest(bk, M - 1 - bl, M, H, npair);
    d2 = js_dest(M - 1 - bk, bl, M, H, npair);
    d3 = js_dest(M - 1 - bk, M - 1 - bl, M, H, npair);
  }
  // eigenvector items (waves 1..): row pair vr, slots vrg, vrg + RG
  const int RG = (nt - 64) / hp;
  const int vr = (tid - 64) % hp, vrg = (tid - 64) / hp;
  int vs0[VJ], vs1[VJ], vd0[VJ], vd1[VJ], vk[VJ];
#pragma unroll
  for (int j = 0; j < VJ; ++j) {
    const int k = vrg + j * RG;
    vk[j] = (!w0 && vrg < RG && k < H) ? k : -1;
    const int kk = vk[j] < 0 ? 0 : k;
    vs0[j] = kk * hp + vr; vs1[j] = (M - 1 - kk) * hp + vr;
    vd0[j] = js_prev(kk, M) * hp + vr; vd1[j] = js_prev(M - 1 - kk, M) * hp + vr;
  }
  for (int k = tid; k < H; k += nt) {
    const int w = js_blk(k, k);
    const double app = PL[w], apq = PL[npair + w], aqq = PL[3 * npair + w];
    double c, s, t;
    js_rot(apq, app, aqq, eps2, floor_abs, c, s, t);
    CS[k] = make_double2(c, s);
    DD[k] = make_double2(app - t * apq, aqq + t * apq);
  }

  int sweeps = 0, rc = 0;
  bool converged = false;
  for (;;) {
    // any off-diagonal entry above its threshold?
    const double* src = PL + (rc & 1) * 4 * npair;
    if (tid == 0) *flag = 0;
    for (int k = tid; k < H; k += nt) {
      const int w = js_blk(k, k);
      dpos[k] = src[w];
      dpos[M - 1 - k] = src[3 * npair + w];
    }
    __syncthreads();
    if (has_blk) {
      bool big = false;
      auto test = [&](double apq, int i, int j) {
        big |= apq * apq > eps2 * fabs(dpos[i] * dpos[j]) && fabs(apq) > floor_abs;
      };
      const int kL = bk, kR = M - 1 - bk, lL = bl, lR = M - 1 - bl;
      if (bk == bl) {
        test(src[npair + myb], kL, kR);
      } else {
        test(src[myb], kL, lL); test(src[npair + myb], kL, lR);
        test(src[2 * npair + myb], kR, lL); test(src[3 * npair + myb], kR, lR);
      }
      if (big) *flag = 1;
    }
    __syncthreads();
    if (*flag == 0) { converged = true; break; }
    if (sweeps >= max_sweeps) break;
    ++sweeps;
    for (int step = 0; step < M - 1; ++step, ++rc) {
      const int bb = rc & 1;
      const double* S = PL + bb * 4 * npair;
      double* D = PL + (bb ^ 1) * 4 * npair;
      const double2* Vs = (const double2*)(VP + bb * M * M);
      double2* Vd = (double2*)(VP + (bb ^ 1) * M * M);
      const double2* cs_ = CS + bb * H;
      const double2* dd_ = DD + bb * H;
      if (!w0) {
        double2 c_[VJ], x0[VJ], x1[VJ];
#pragma unroll
        for (int j = 0; j < VJ; ++j)
          if (vk[j] >= 0) { c_[j] = cs_[vk[j]]; x0[j] = Vs[vs0[j]]; x1[j] = Vs[vs1[j]]; }
        if (has_blk) {
          if (bk == bl) {
            const double2 dk = dd_[bk];
            const bool act = cs_[bk].y != 0.0;
            D[d0] = dk.x;
            D[d1] = act ? 0.0 : S[npair + myb];
            D[d3] = dk.y;
          } else {
            const double2 k2 = cs_[bk], l2 = cs_[bl];
            const double m00 = S[myb], m01 = S[npair + myb], m10 = S[2 * npair + myb], m11 = S[3 * npair + myb];
            const double r00 = k2.x * m00 - k2.y * m10, r01 = k2.x * m01 - k2.y * m11;
            const double r10 = k2.y * m00 + k2.x * m10, r11 = k2.y * m01 + k2.x * m11;
            D[d0] = r00 * l2.x - r01 * l2.y;
            D[d1] = r00 * l2.y + r01 * l2.x;
            D[d2] = r10 * l2.x - r11 * l2.y;
            D[d3] = r10 * l2.y + r11 * l2.x;
          }
        }
#pragma unroll
        for (int j = 0; j < VJ; ++j)
          if (vk[j] >= 0) {
            const double c = c_[j].x, s = c_[j].y;
            Vd[vd0[j]] = make_double2(c * x0[j].x - s * x1[j].x, c * x0[j].y - s * x1[j].y);
            Vd[vd1[j]] = make_double2(s * x0[j].x + c * x1[j].x, s * x0[j].y + c * x1[j].y);
          }
      } else if (has_blk) {
        const double2 k2 = cs_[bk], l2 = cs_[bl];
        const double2 da = dd_[pa], db = dd_[pb];
        const double m00 = S[myb], m01 = S[npair + myb], m10 = S[2 * npair + myb], m11 = S[3 * npair + myb];
        const double r00 = k2.x * m00 - k2.y * m10, r01 = k2.x * m01 - k2.y * m11;
        const double r10 = k2.y * m00 + k2.x * m10, r11 = k2.y * m01 + k2.x * m11;
        const double n00 = r00 * l2.x - r01 * l2.y, n01 = r00 * l2.y + r01 * l2.x;
        const double n10 = r10 * l2.x - r11 * l2.y, n11 = r10 * l2.y + r11 * l2.x;
        D[d0] = n00; D[d1] = n01; D[d2] = n10; D[d3] = n11;
        const double apq = sel == 0 ? n00 : sel == 1 ? n01 : sel == 2 ? n10 : n11;
        const double app = psa ? da.y : da.x, aqq = psb ? db.y : db.x;
        double c, s, t;
        js_rot(apq, app, aqq, eps2, floor_abs, c, s, t);
        CS[(bb ^ 1) * H + lane] = make_double2(c, s);
        DD[(bb ^ 1) * H + lane] = make_double2(app - t * apq, aqq + t * apq);
      }
      __syncthreads();
    }
  }
  // eigenpairs by position, ascending; with m odd the padding index sits at the
  // position that holds index M-1 after rc moves
  const int ph = (m & 1) ? (M - 2 - rc % (M - 1) + (M - 1)) % (M - 1) + 1 : -1;
  const double* src = PL + (rc & 1) * 4 * npair;
  const double* Vf = VP + (rc & 1) * M * M;
  for (int k = tid; k < H; k += nt) {
    const int w = js_blk(k, k);
    dpos[k] = src[w];
    dpos[M - 1 - k] = src[3 * npair + w];
  }
  __syncthreads();
  for (int i = tid; i < M; i += nt) {
    if (i == ph) continue;
    const double di = dpos[i];
    int rank = 0;
    for (int j = 0; j < M; ++j)
      if (j != ph) rank += (dpos[j] < di) || (dpos[j] == di && j < i);
    evals[rank] = di;
    for (int r = 0; r < m; ++r) Vout[(long)r * m + rank] = Vf[(long)i * M + r];
  }
  if (tid == 0) info[0] = converged ? sweeps : -(sweeps + 1);
}

// ---------------------------------------------------------------------------
// The same cyclic Jacobi, one barrier a round, with A and V kept by index and updated
// in place: 81 <= m <= 112 with V in LDS, and even m from 114 to 146 with V in global
// memory (the workgroup's own Vwork). The position-frame storage above needs A and V
// twice and from m = 81 on no longer fits in LDS; in place needs them once: the
// rotations of a round act on disjoint index pairs, so every entry of A (in the 2x2
// block of two slots) and of V (a row pair of one column) that a round touches is
// read and written by one thread, and only the rotation tables are double-buffered.
// Slots, the fixed owner of each block and the next round's rotation, computed by the
// thread of the slot (threads 0..H-1) from the entry its block has just produced, are
// those of the position-frame form; the indices in slot k's positions k, M-1-k at
// round r come from the round-robin schedule (rr_player). A is packed upper, V by
// column (the eigenvector estimate of each index) with rows in pairs. Same rotation
// and thresholds as jacobi_body; m odd is padded with a zero index M-1 whose rotations
// never qualify (V in LDS only: in global memory V takes exactly m x m).
// ---------------------------------------------------------------------------
constexpr int JI_MIN = 81, JI_MAX = 112;   // V in LDS
constexpr int JG_MIN = 114, JG_MAX = 146;  // V in global memory, m even (H <= 73)

size_t jacobi_inplace_lds_doubles(int m, bool vg) {
  const int M = m + (m & 1), H = M / 2;
  const size_t na = ((size_t)M * (M + 1) / 2 + 1) & ~(size_t)1;
  return na + (vg ? 0 : (size_t)M * M) + 8 * (size_t)H + 40;
}

// VG: V in global memory (Vg); BJ blocks and VJ eigenvector items (in groups of VH,
// loaded together) at most per thread past the next-rotation threads:
//   V in LDS (H <= 56): 64 next-rotation threads, 960 others: BJ = 2, VJ = 4;
//   V in global (H <= 73): 128 next-rotation threads from H = 65 on, 896 others:
//   H (H - 1) / 2 <= 3 * 896 blocks, ceil(H / floor(896 / H)) <= 7 items.
template <bool VG, int BJ, int VJ, int VH>
__device__ __forceinline__ void jacobi_inplace_body(int m, const double* __restrict__ Ab, int nparts, long pstride,
                                    double* __restrict__ evals, double* __restrict__ Vout,
                                    double* __restrict__ Vg, int max_sweeps, int* __restrict__ info,
                                    double* sm) {
  static_assert(VJ % VH == 0, "item groups");
  const int M = m + (m & 1), H = M / 2;
  const int na = (M * (M + 1) / 2 + 1) & ~1;
  double* A = sm;                                           // packed upper, by index
  double2* V2 = VG ? (double2*)Vg : (double2*)(A + na);     // [M][H]: column i, rows 2 rp, 2 rp + 1
  double2* CS = (double2*)(A + na) + (VG ? 0 : M * H);      // [2][H] (c, s)
  double2* DD = CS + 2 * H;                                 // [2][H] the pair's diagonals after its rotation
  double* red = (double*)(DD + 2 * H);                      // 32
  int* flag = (int*)(red + 32);
  const int tid = threadIdx.x, nt = blockDim.x;
  const int NRT = ((H + 63) / 64) * 64;  // next-rotation threads (whole waves)
  const bool w0 = tid < NRT;

  double nrm = 0.0;
  const int np = M * (M + 1) / 2;
  for (int t = tid; t < np; t += nt) {
    int j = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while (j * (j + 1) / 2 > t) --j;
    while ((j + 1) * (j + 2) / 2 <= t) ++j;
    const int i = t - j * (j + 1) / 2;
    double v = 0.0;
    if (j < m)
      for (int ks = 0; ks < nparts; ++ks) {
        const double* g = Ab + (long)ks * pstride;
        v += 0.5 * (g[(long)i * m + j] + g[(long)j * m + i]);
      }
    A[t] = v;
    nrm += (i == j ? 1.0 : 2.0) * v * v;
  }
  for (int t = tid; t < M * H; t += nt) {
    const int i = t / H, rp = t % H;
    V2[t] = make_double2(2 * rp == i ? 1.0 : 0.0, 2 * rp + 1 == i ? 1.0 : 0.0);
  }
  nrm = wave_sum(nrm);
  if ((tid & 63) == 0) red[tid >> 6] = nrm;
  __syncthreads();
  double fro = 0.0;
  for (int w = 0; w < (nt >> 6); ++w) fro += red[w];
  fro = sqrt(fro);
  const double eps = 2.220446049250313e-16, eps2 = eps * eps;
  const double floor_abs = eps * fro;

  // This thread's blocks (slots k <= l). Thread kp < H owns the block holding the two
  // indices that meet in slot kp next round: they sit this round at positions
  // js_next(kp) (slot pa, side psa) and js_next(M-1-kp) (slot pb, side psb). The
  // threads past NRT own the other blocks in column order, as in the position-frame
  // form.
  int bkl[BJ];  // block q as k << 8 | l, or -1
  int pa = 0, psa = 0, pb = 0, psb = 0, sel = 0;
#pragma unroll
  for (int q = 0; q < BJ; ++q) bkl[q] = -1;
  if (w0) {
    if (tid < H) {
      const int x = js_next(tid, M), y = js_next(M - 1 - tid, M);
      pa = x < H ? x : M - 1 - x; psa = x < H ? 0 : 1;
      pb = y < H ? y : M - 1 - y; psb = y < H ? 0 : 1;
      bkl[0] = min(pa, pb) << 8 | max(pa, pb);
      sel = pa < pb ? psa * 2 + psb : psb * 2 + psa;
    }
  } else {
#pragma unroll
    for (int q = 0; q < BJ; ++q) {
      const int j = tid - NRT + q * (nt - NRT);
      if (j == 0) {
        bkl[q] = 0;
      } else if (j < H * (H - 1) / 2) {
        int l = 1;
        while (l + 1 < H && 1 + l * (l + 1) / 2 <= j) ++l;
        const int r = j - (1 + (l - 1) * l / 2);
        int k;
        if (l == 1) k = 1;
        else if (l == H - 1) k = r < H - 3 ? r : r + 2;
        else k = r < l - 2 ? r : r + 1;
        bkl[q] = k << 8 | l;
      }
    }
  }
  // eigenvector items (threads past NRT): row pair vr of the columns in slots vrg + j RG
  const int RG = (nt - NRT) / H;
  const int vr = (tid - NRT) % H, vrg = (tid - NRT) / H;
  const bool vown = !w0 && vrg < RG;
  auto vk = [&](int j) { const int k = vrg + j * RG; return vown && k < H ? k : -1; };
  // rotations of round 0 (every index at its own position)
  for (int k = tid; k < H; k += nt) {
    const int p = k, q = M - 1 - k;
    const double app = A[uidx(p, p)], apq = A[uidx(p, q)], aqq = A[uidx(q, q)];
    double c, s, t;
    js_rot(apq, app, aqq, eps2, floor_abs, c, s, t);
    CS[k] = make_double2(c, s);
    DD[k] = make_double2(app - t * apq, aqq + t * apq);
  }

  int sweeps = 0, rc = 0;
  bool converged = false;
  for (;;) {
    // any off-diagonal entry above its threshold? (a sweep starts at round 0, where
    // slot k holds the indices k and M-1-k)
    if (tid == 0) *flag = 0;
    __syncthreads();
    bool big = false;
    auto test = [&](int i, int j) {
      const double apq = A[sidx(i, j)];
      big |= apq * apq > eps2 * fabs(A[uidx(i, i)] * A[uidx(j, j)]) && fabs(apq) > floor_abs;
    };
#pragma unroll
    for (int q = 0; q < BJ; ++q) {
      if (bkl[q] < 0) continue;
      const int k = bkl[q] >> 8, l = bkl[q] & 255;
      if (k == l) {
        test(k, M - 1 - k);
      } else {
        test(k, l); test(k, M - 1 - l); test(M - 1 - k, l); test(M - 1 - k, M - 1 - l);
      }
    }
    if (big) *flag = 1;
    __syncthreads();
    if (*flag == 0) { converged = true; break; }
    if (sweeps >= max_sweeps) break;
    ++sweeps;
    for (int step = 0; step < M - 1; ++step, ++rc) {
      const int bb = rc & 1;
      const double2* cs_ = CS + bb * H;
      const double2* dd_ = DD + bb * H;
      if (!w0) {
        // the entries a round touches are this thread's alone: the eigenvector items go
        // in groups of VH (loads together, then the rotated stores), the first group's
        // loads ahead of the block updates
        double2 c_[VH], x0[VH], x1[VH];
        int i0[VH], i1[VH];
        auto vload = [&](int j0) {
#pragma unroll
          for (int j = 0; j < VH; ++j)
            if (vk(j0 + j) >= 0) {
              const int k = vk(j0 + j);
              i0[j] = rr_player(k, step, M) * H + vr;
              i1[j] = rr_player(M - 1 - k, step, M) * H + vr;
              c_[j] = cs_[k];
              x0[j] = V2[i0[j]];
              x1[j] = V2[i1[j]];
            }
        };
        auto vstore = [&](int j0) {
#pragma unroll
          for (int j = 0; j < VH; ++j)
            if (vk(j0 + j) >= 0 && c_[j].y != 0.0) {
              const double c = c_[j].x, s = c_[j].y;
              V2[i0[j]] = make_double2(c * x0[j].x - s * x1[j].x, c * x0[j].y - s * x1[j].y);
              V2[i1[j]] = make_double2(s * x0[j].x + c * x1[j].x, s * x0[j].y + c * x1[j].y);
            }
        };
        // (V in global memory: every group before the blocks, so that no group's
        // registers are live across the block updates)
        if constexpr (VG) {
#pragma unroll
          for (int j0 = 0; j0 < VJ; j0 += VH) {
            vload(j0);
            vstore(j0);
          }
        } else {
          vload(0);
        }
#pragma unroll
        for (int q = 0; q < BJ; ++q) {
          if (bkl[q] < 0) continue;
          const int k = bkl[q] >> 8, l = bkl[q] & 255;
          const int Pk = rr_player(k, step, M), Qk = rr_player(M - 1 - k, step, M);
          const double2 k2 = cs_[k];
          if (k == l) {
            const double2 dk = dd_[k];
            A[uidx(Pk, Pk)] = dk.x;
            A[uidx(Qk, Qk)] = dk.y;
            if (k2.y != 0.0) A[sidx(Pk, Qk)] = 0.0;
          } else {
            const int Pl = rr_player(l, step, M), Ql = rr_player(M - 1 - l, step, M);
            const int i00 = sidx(Pk, Pl), i01 = sidx(Pk, Ql), i10 = sidx(Qk, Pl), i11 = sidx(Qk, Ql);
            const double2 l2 = cs_[l];
            const double m00 = A[i00], m01 = A[i01], m10 = A[i10], m11 = A[i11];
            const double r00 = k2.x * m00 - k2.y * m10, r01 = k2.x * m01 - k2.y * m11;
            const double r10 = k2.y * m00 + k2.x * m10, r11 = k2.y * m01 + k2.x * m11;
            A[i00] = r00 * l2.x - r01 * l2.y;
            A[i01] = r00 * l2.y + r01 * l2.x;
            A[i10] = r10 * l2.x - r11 * l2.y;
            A[i11] = r10 * l2.y + r11 * l2.x;
          }
        }
        if constexpr (!VG) {
          vstore(0);
#pragma unroll
          for (int j0 = VH; j0 < VJ; j0 += VH) {
            vload(j0);
            vstore(j0);
          }
        }
      } else if (bkl[0] >= 0) {
        const int k = bkl[0] >> 8, l = bkl[0] & 255;
        const int Pk = rr_player(k, step, M), Qk = rr_player(M - 1 - k, step, M);
        const int Pl = rr_player(l, step, M), Ql = rr_player(M - 1 - l, step, M);
        const int i00 = sidx(Pk, Pl), i01 = sidx(Pk, Ql), i10 = sidx(Qk, Pl), i11 = sidx(Qk, Ql);
        const double2 ka = cs_[k], la = cs_[l];
        const double2 da = dd_[pa], db = dd_[pb];
        const double m00 = A[i00], m01 = A[i01], m10 = A[i10], m11 = A[i11];
        const double r00 = ka.x * m00 - ka.y * m10, r01 = ka.x * m01 - ka.y * m11;
        const double r10 = ka.y * m00 + ka.x * m10, r11 = ka.y * m01 + ka.x * m11;
        const double n00 = r00 * la.x - r01 * la.y, n01 = r00 * la.y + r01 * la.x;
        const double n10 = r10 * la.x - r11 * la.y, n11 = r10 * la.y + r11 * la.x;
        A[i00] = n00; A[i01] = n01; A[i10] = n10; A[i11] = n11;
        const double apq = sel == 0 ? n00 : sel == 1 ? n01 : sel == 2 ? n10 : n11;
        const double app = psa ? da.y : da.x, aqq = psb ? db.y : db.x;
        double c, s, t;
        js_rot(apq, app, aqq, eps2, floor_abs, c, s, t);
        CS[(bb ^ 1) * H + tid] = make_double2(c, s);
        DD[(bb ^ 1) * H + tid] = make_double2(app - t * apq, aqq + t * apq);
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < m; i += nt) {
    const double di = A[uidx(i, i)];
    int rank = 0;
    for (int j = 0; j < m; ++j) {
      const double dj = A[uidx(j, j)];
      rank += (dj < di) || (dj == di && j < i);
    }
    evals[rank] = di;
    const double* col = reinterpret_cast<const double*>(V2 + (long)i * H);
    for (int r = 0; r < m; ++r) Vout[(long)r * m + rank] = col[r];
  }
  if (tid == 0) info[0] = converged ? sweeps : -(sweeps + 1);
}

// V in global memory: a function of its own, so that its register pressure stays out
// of the kernel's other bodies
__device__ __noinline__ void jacobi_inplace_global(int m, const double* Ab, int nparts, long pstride,
                                                  double* evals, double* Vout, double* Vg, int max_sweeps,
                                                  int* info, double* sm) {
  jacobi_inplace_body<true, 3, 8, 4>(m, Ab, nparts, pstride, evals, Vout, Vg, max_sweeps, info, sm);
}

// Largest launch that takes the in-place body with V in global memory: alone on a CU
// it is faster than the two-barrier body (m = 128, random: 5.1 against 7.2 ms), but
// every round moves the eigenvector matrix through L2, and with many workgroups a CU
// the L2 traffic makes it slower (512 problems: 19.8 against 15.1 ms)
constexpr int JG_BATCH = 128;

// the in-place body for m, if it takes m: V in LDS (BJ 2, VJ 4), or in global memory
// where the launch allows it (glob)
__device__ __forceinline__ bool jacobi_inplace(int m, const double* Ab, int nparts, long pstride,
                                               double* evals, double* Vout, double* Vg, int max_sweeps,
                                               int* info, double* sm, bool glob) {
  if (m >= JI_MIN && m <= JI_MAX) {
    jacobi_inplace_body<false, 2, 4, 2>(m, Ab, nparts, pstride, evals, Vout, nullptr, max_sweeps, info, sm);
    return true;
  }
  if (glob && m >= JG_MIN && m <= JG_MAX && (m & 1) == 0) {
    jacobi_inplace_global(m, Ab, nparts, pstride, evals, Vout, Vg, max_sweeps, info, sm);
    return true;
  }
  return false;
}

__global__ __launch_bounds__(JAC_THREADS) void jacobi_kernel(int m, const double* __restrict__ Ain, long sA,
                                                             int nparts, long pstride,
                                                             double* __restrict__ evals, long sE,
                                                             double* __restrict__ Vout, long sV,
                                                             double* __restrict__ Vwork, int vlds,
                                                             int max_sweeps, int* __restrict__ info) {
  // vlds: bit 0 V in LDS for the two-barrier body, bit 1 the global-V in-place body allowed
  extern __shared__ double sm[];
  const int b = blockIdx.x;
  if (m >= JS_MIN && m <= JS_MAX)
    jacobi_shift_body(m, Ain + (long)b * sA, nparts, pstride, evals + (long)b * sE, Vout + (long)b * sV,
                      max_sweeps, info + b, sm);
  else if (jacobi_inplace(m, Ain + (long)b * sA, nparts, pstride, evals + (long)b * sE, Vout + (long)b * sV,
                          Vwork + (long)b * m * m, max_sweeps, info + b, sm, (vlds & 2) != 0))
    ;
  else
    jacobi_body(m, Ain + (long)b * sA, nparts, pstride, evals + (long)b * sE, Vout + (long)b * sV,
                Vwork + (long)b * m * m, vlds & 1, max_sweeps, info + b, sm);
}

__global__ __launch_bounds__(JAC_THREADS) void jacobi_batched_kernel(const EigDesc* __restrict__ descs,
                                                                     int vlds, int max_sweeps) {
  // vlds: as for jacobi_kernel
  extern __shared__ double sm[];
  const EigDesc d = descs[blockIdx.x];
  if (d.m >= JS_MIN && d.m <= JS_MAX)
    jacobi_shift_body(d.m, d.A, d.nparts, d.pstride, d.evals, d.V, max_sweeps, d.info, sm);
  else if (jacobi_inplace(d.m, d.A, d.nparts, d.pstride, d.evals, d.V, d.Vwork, max_sweeps, d.info, sm,
                          (vlds & 2) != 0))
    ;
  else
    jacobi_body(d.m, d.A, d.nparts, d.pstride, d.evals, d.V, d.Vwork, vlds & 1, max_sweeps, d.info, sm);
}

// LDS for a launch whose largest matrix is mmax: either body may run
static size_t jacobi_launch_lds(int mmax, int vl) {
  // the generic body runs below JS_MIN and above JI_MAX only
  size_t d = jacobi_lds_doubles(mmax > JI_MAX ? mmax : std::min(mmax, JS_MIN - 1), vl);
  if (mmax >= JS_MIN) d = std::max(d, jacobi_shift_lds_doubles(std::min(mmax, JS_MAX)));
  if (mmax >= JI_MIN) d = std::max(d, jacobi_inplace_lds_doubles(std::min(mmax, JI_MAX), false));
  if (mmax >= JG_MIN) d = std::max(d, jacobi_inplace_lds_doubles(std::min(mmax, JG_MAX), true));
  return d * sizeof(double);
}

void jacobi_batched(hipStream_t s, const EigDesc* d, int P, int mmax, int threads) {
  if (P <= 0) return;
  const int vl = jacobi_v_in_lds(mmax) ? 1 : 0;
  size_t lds = jacobi_launch_lds(mmax, vl);
  // half-size workgroups only where the m <= 80 body's work split holds with 448
  // threads besides wave 0 (two eigenvector items and one block per thread)
  const int nt = (threads == JAC_THREADS / 2 && mmax <= JS_HALF_MAX) ? JAC_THREADS / 2 : JAC_THREADS;
  hipLaunchKernelGGL(jacobi_batched_kernel, dim3(P), dim3(nt), lds, s, d, vl | (P <= JG_BATCH ? 2 : 0), 40);
}

// Row-block vector operations (one workgroup per row for the reductions).
__global__ __launch_bounds__(256) void vec_batched_kernel(int op, const VecDesc* __restrict__ descs) {
  __shared__ double red[4];
  const VecDesc d = descs[blockIdx.z];
  const int n = d.n;
  if (op == VEC_NORMALIZE || op == VEC_RESIDUAL) {
    const int j = blockIdx.x;
    if (j >= d.nv) return;
    double acc = 0.0;
    // rows of even length start 16-byte aligned (the arena is 256-byte aligned): pairs
    // of elements move as one 16-byte access; each thread's partial sum keeps the order
    // i, i + 1 within a pair and ascending pairs
    const bool pairs = (n & 1) == 0;
    if (op == VEC_NORMALIZE) {
      double* y = d.out + (long)j * n;
      if (pairs) {
        double2* y2 = reinterpret_cast<double2*>(y);
        for (int i = threadIdx.x; i < n / 2; i += 256) {
          const double2 v = y2[i];
          acc += v.x * v.x;
          acc += v.y * v.y;
        }
      } else {
        for (int i = threadIdx.x; i < n; i += 256) acc += y[i] * y[i];
      }
      double nr = sqrt(block_sum256(acc, red));
      if (threadIdx.x == 0 && d.norms) d.norms[j] = nr;
      if (nr > 0.0) {
        double inv = 1.0 / nr;
        if (pairs) {
          double2* y2 = reinterpret_cast<double2*>(y);
          for (int i = threadIdx.x; i < n / 2; i += 256) {
            const double2 v = y2[i];
            y2[i] = double2{v.x * inv, v.y * inv};
          }
        } else {
          for (int i = threadIdx.x; i < n; i += 256) y[i] *= inv;
        }
      }
    } else {
      const double* hx = d.P + (long)j * n;
      const double* x = d.Q + (long)j * n;
      const double th = d.a[j];
      double* rout = d.out ? d.out + (long)j * n : nullptr;
      if (pairs) {
        const double2* h2 = reinterpret_cast<const double2*>(hx);
        const double2* x2 = reinterpret_cast<const double2*>(x);
        double2* r2 = reinterpret_cast<double2*>(rout);
        for (int i = threadIdx.x; i < n / 2; i += 256) {
          const double2 h = h2[i], v = x2[i];
          const double ra = h.x - th * v.x, rb = h.y - th * v.y;
          acc += ra * ra;
          acc += rb * rb;
          if (rout) r2[i] = double2{ra, rb};
        }
      } else {
        for (int i = threadIdx.x; i < n; i += 256) {
          double r = hx[i] - th * x[i];
          acc += r * r;
          if (rout) rout[i] = r;
        }
      }
      double nr = sqrt(block_sum256(acc, red));
      if (threadIdx.x == 0) d.norms[j] = nr;
    }
    return;
  }
  if (op == VEC_REDUCE) {
    for (long t = blockIdx.x * 256L + threadIdx.x; t < n; t += (long)gridDim.x * 256) {
      double v = 0.0;
      for (int j = 0; j < d.nv; ++j) v += d.P[(long)j * n + t];
      d.out[t] = v;
    }
    return;
  }
  const long total = (long)d.nv * n;
  for (long t = blockIdx.x * 256L + threadIdx.x; t < total; t += (long)gridDim.x * 256) {
    const int j = (int)(t / n);
    double v;
    if (op == VEC_SCALE_ADD) {
      v = d.asgn * d.a[j] * d.P[t];
      if (d.Q) v += d.b * d.Q[t];
    } else if (op == VEC_COPY) {
      v = d.P[t];
    } else {  // VEC_AXPY3
      v = d.out[t] + d.b * d.P[t];
      if (d.Q) v += d.c * d.Q[t];
    }
    d.out[t] = v;
  }
}

void vec_batched(hipStream_t s, VecOp op, const VecDesc* d, int P, int nvmax, long elems_max) {
  if (P <= 0) return;
  int gx;
  if (op == VEC_NORMALIZE || op == VEC_RESIDUAL) {
    gx = nvmax;
  } else {
    long b = (elems_max + 255) / 256;
    gx = (int)(b > 1024 ? 1024 : b);
  }
  if (gx <= 0) return;
  hipLaunchKernelGGL(vec_batched_kernel, dim3(gx, 1, P), dim3(256), 0, s, (int)op, d);
}

// One workgroup per filter, a thread per vector: its phi_k by the recurrence, every
// product and the difference rounded on their own (no contraction), as on the host.
__global__ __launch_bounds__(128) void filter_phi_kernel(const PhiDesc* __restrict__ descs) {
  const PhiDesc d = descs[blockIdx.x];
  for (int j = threadIdx.x; j < d.cn; j += 128) {
    const double t = d.t[j];
    double pk = __dmul_rn(d.r0, t), pm1 = 1.0;
    d.phi[j] = pk;
    for (int k = 1; k <= d.steps; ++k) {
      const double a = d.sc[3 * (k - 1)];
      const double b = k == 1 ? d.b1 : -d.sc[3 * (k - 1) + 2];
      const double nx = __dsub_rn(__dmul_rn(__dmul_rn(a, t), pk), __dmul_rn(b, pm1));
      pm1 = pk;
      pk = nx;
      d.phi[(long)k * d.cn + j] = pk;
    }
  }
}

void filter_phi_batched(hipStream_t s, const PhiDesc* d, int P) {
  if (P <= 0) return;
  hipLaunchKernelGGL(filter_phi_kernel, dim3(P), dim3(128), 0, s, d);
}

int jacobi_max_m() { return JMAX; }

// Ct_v = (C_v)^T for the k_A x k_B coefficient blocks C_v of a merged basis:
// Ct[v][b k_A + a] = C[v][a k_B + b], one descriptor per module (blockIdx.z).
__global__ __launch_bounds__(256) void transpose_blocks_kernel(const TrDesc* __restrict__ descs) {
  const TrDesc d = descs[blockIdx.z];
  const int v = blockIdx.y;
  if (v >= d.k) return;
  const int n = d.kA * d.kB;
  const double* src = d.C + (long)v * n;
  double* dst = d.Ct + (long)v * n;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < n; e += gridDim.x * 256) {
    const int a = e / d.kB, b = e % d.kB;
    dst[(long)b * d.kA + a] = src[e];
  }
}

void transpose_blocks_batched(hipStream_t s, const TrDesc* d, int P, int kmax, int nmax) {
  if (P <= 0 || kmax <= 0 || nmax <= 0) return;
  const int gx = std::min((nmax + 255) / 256, 16);
  hipLaunchKernelGGL(transpose_blocks_kernel, dim3(gx, kmax, P), dim3(256), 0, s, d);
}

void linalg_set_attrs() {
  const int lds = 160 * 1024 - 1024;
  hipFuncSetAttribute(reinterpret_cast<const void*>(&jacobi_kernel),
                      hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  hipFuncSetAttribute(reinterpret_cast<const void*>(&chol_inv_kernel),
                      hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  hipFuncSetAttribute(reinterpret_cast<const void*>(&chol_batched_kernel),
                      hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  hipFuncSetAttribute(reinterpret_cast<const void*>(&jacobi_batched_kernel),
                      hipFuncAttributeMaxDynamicSharedMemorySize, lds);
}

void jacobi_eig(hipStream_t s, int batch, int m, const double* A, long sA, int nparts,
                long pstride, double* evals, long sE, double* V, long sV, double* Vwork, int* info) {
  const int vl = jacobi_v_in_lds(m) ? 1 : 0;
  size_t lds = jacobi_launch_lds(m, vl);
  hipLaunchKernelGGL(jacobi_kernel, dim3(batch), dim3(JAC_THREADS), lds, s, m, A, sA,
                     nparts < 1 ? 1 : nparts, pstride, evals, sE, V, sV, Vwork,
                     vl | (batch <= JG_BATCH ? 2 : 0), 40, info);
}

}  // namespace rmc
