// Dense FP64 building blocks of the eigensolver on gfx950: an MFMA GEMM with
// split-K, vector norms, Cholesky + triangular inverse (CholeskyQR2), and a
// parallel cyclic Jacobi eigensolver for the Rayleigh-Ritz matrices.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "rmc_kernels.h"

namespace rmc {

typedef double d4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// GEMM: 64x64 output tile per 256-thread workgroup, K staged 16 at a time in LDS.
// Each wave owns a 32x32 quadrant = 2x2 tiles of v_mfma_f64_16x16x4_f64.
// Operand lanes: A[i][k] with i = lane%16, k = lane/16; B[k][j] with j = lane%16,
// k = lane/16; for this FP64 instruction accumulator register r holds
// D[4*r + lane/16][lane%16] (measured on gfx950).
// ---------------------------------------------------------------------------
constexpr int GB_M = 64, GB_N = 64, GB_K = 16;

__global__ __launch_bounds__(256) void gemm_f64_kernel(
    int tA, int tB, int M, int N, int K, int kchunk, double alpha, const double* __restrict__ A,
    long lda, long sA, const double* __restrict__ B, long ldb, long sB, double beta,
    double* __restrict__ C, long ldc, long sC, int batch, int ksplit, double* __restrict__ work) {
  __shared__ double As[GB_K][GB_M + 1];
  __shared__ double Bs[GB_K][GB_N + 1];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int bz = blockIdx.z;
  const int b = bz / ksplit, ks = bz % ksplit;
  const int row0 = blockIdx.y * GB_M, col0 = blockIdx.x * GB_N;
  const double* Ab = A + (long)b * sA;
  const double* Bb = B + (long)b * sB;
  const int kbeg = ks * kchunk;
  const int kend = min(K, kbeg + kchunk);

  d4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  for (int k0 = kbeg; k0 < kend; k0 += GB_K) {
    // A tile: GB_M x GB_K elements, 4 per thread.
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      int idx = tid + e * 256;
      int i, k;
      if (!tA) { i = idx / GB_K; k = idx % GB_K; } else { k = idx / GB_M; i = idx % GB_M; }
      int gi = row0 + i, gk = k0 + k;
      double v = 0.0;
      if (gi < M && gk < kend) v = tA ? Ab[(long)gk * lda + gi] : Ab[(long)gi * lda + gk];
      As[k][i] = v;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      int idx = tid + e * 256;
      int j, k;
      if (!tB) { k = idx / GB_N; j = idx % GB_N; } else { j = idx / GB_K; k = idx % GB_K; }
      int gj = col0 + j, gk = k0 + k;
      double v = 0.0;
      if (gj < N && gk < kend) v = tB ? Bb[(long)gj * ldb + gk] : Bb[(long)gk * ldb + gj];
      Bs[k][j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GB_K; kk += 4) {
      const int kr = kk + (lane >> 4);
      double a0 = As[kr][wm + (lane & 15)];
      double a1 = As[kr][wm + 16 + (lane & 15)];
      double b0 = Bs[kr][wn + (lane & 15)];
      double b1 = Bs[kr][wn + 16 + (lane & 15)];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }

  if (ksplit > 1) {
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
                     alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, ksplit, work);
  if (ksplit > 1) {
    long total = (long)batch * M * N;
    int blocks = (int)((total + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3(blocks), dim3(256), 0, s, M, N, batch, ksplit,
                       work, beta, C, ldc, sC);
  }
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

// ---------------------------------------------------------------------------
// Cholesky + inverse of the lower factor, one 1024-thread workgroup, packed
// lower triangle in LDS (m <= 192 -> at most 148 KB).
// ---------------------------------------------------------------------------
constexpr int JMAX = 192;
__device__ inline int lidx(int i, int j) { return i * (i + 1) / 2 + j; }  // j <= i

__global__ __launch_bounds__(1024) void chol_inv_kernel(int m, const double* __restrict__ G, double shift,
                                                        double* __restrict__ Linv, int* __restrict__ info) {
  extern __shared__ double L[];
  __shared__ int fail;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int np = m * (m + 1) / 2;
  for (int t = tid; t < np; t += nt) {
    int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while (i * (i + 1) / 2 > t) --i;
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    int j = t - i * (i + 1) / 2;
    double v = 0.5 * (G[(long)i * m + j] + G[(long)j * m + i]);
    if (i == j) v += shift;
    L[t] = v;
  }
  if (tid == 0) fail = 0;
  __syncthreads();
  for (int j = 0; j < m; ++j) {
    if (tid == 0) {
      double d = L[lidx(j, j)];
      if (!(d > 0.0)) fail = 1;
      else L[lidx(j, j)] = sqrt(d);
    }
    __syncthreads();
    if (fail) break;
    double djj = L[lidx(j, j)];
    for (int i = j + 1 + tid; i < m; i += nt) L[lidx(i, j)] /= djj;
    __syncthreads();
    int r0 = j + 1, w = m - r0;
    int ntri = w * (w + 1) / 2;
    for (int t = tid; t < ntri; t += nt) {
      int a = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
      while (a * (a + 1) / 2 > t) --a;
      while ((a + 1) * (a + 2) / 2 <= t) ++a;
      int c = t - a * (a + 1) / 2;
      int r = r0 + a, cc = r0 + c;
      L[lidx(r, cc)] -= L[lidx(r, j)] * L[lidx(cc, j)];
    }
    __syncthreads();
  }
  if (tid == 0) info[0] = fail;
  if (fail) return;
  // Column c of L^{-1} by forward substitution (one thread per column).
  for (int c = tid; c < m; c += nt) {
    double* X = Linv;
    for (int i = 0; i < c; ++i) X[(long)i * m + c] = 0.0;
    X[(long)c * m + c] = 1.0 / L[lidx(c, c)];
    for (int i = c + 1; i < m; ++i) {
      double acc = 0.0;
      const int base = i * (i + 1) / 2;
      for (int k = c; k < i; ++k) acc += L[base + k] * X[(long)k * m + c];
      X[(long)i * m + c] = -acc / L[base + i];
    }
  }
}

void chol_inv(hipStream_t s, int m, const double* G, double shift, double* Linv, int* info) {
  size_t lds = (size_t)m * (m + 1) / 2 * sizeof(double);
  hipLaunchKernelGGL(chol_inv_kernel, dim3(1), dim3(1024), lds, s, m, G, shift, Linv, info);
}

// ---------------------------------------------------------------------------
// Parallel cyclic Jacobi (round-robin ordering). Packed upper triangle of A in
// LDS; eigenvector accumulation in global memory (Vwork), one workgroup per
// matrix. A rotation of pair (p,q) is skipped when |a_pq| is below
// max(eps*sqrt(|a_pp a_qq|), eps*||A||_F); the sweep loop ends after a sweep
// with no rotation.
// ---------------------------------------------------------------------------
__device__ inline int uidx(int i, int j) {  // i <= j, packed upper by columns
  return j * (j + 1) / 2 + i;
}
__device__ inline int sidx(int i, int j) { return i <= j ? uidx(i, j) : uidx(j, i); }

__device__ inline int rr_player(int pos, int step, int M) {
  if (pos == 0) return 0;
  return 1 + (pos - 1 + step) % (M - 1);
}

__global__ __launch_bounds__(1024) void jacobi_kernel(int m, const double* __restrict__ Ain, long sA,
                                                      double* __restrict__ evals, long sE,
                                                      double* __restrict__ Vout, long sV,
                                                      double* __restrict__ Vwork, int max_sweeps,
                                                      int* __restrict__ info) {
  extern __shared__ double sm[];
  const int M = m + (m & 1);
  const int H = M / 2;
  double* A = sm;                         // M*(M+1)/2
  double* cs = A + M * (M + 1) / 2;       // H
  double* sn = cs + H;                    // H
  double* tn = sn + H;                    // H
  int* pp = (int*)(tn + H);               // H
  int* qq = pp + H;                       // H
  int* act = qq + H;                      // H
  __shared__ int s_rot;
  __shared__ double red[16];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int b = blockIdx.x;
  const double* Ab = Ain + (long)b * sA;
  double* V = Vwork + (long)b * m * m;

  // load (symmetrised), dummy row/col for odd m
  double nrm = 0.0;
  const int np = M * (M + 1) / 2;
  for (int t = tid; t < np; t += nt) {
    int j = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while (j * (j + 1) / 2 > t) --j;
    while ((j + 1) * (j + 2) / 2 <= t) ++j;
    int i = t - j * (j + 1) / 2;
    double v = 0.0;
    if (j < m) v = 0.5 * (Ab[(long)i * m + j] + Ab[(long)j * m + i]);
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
  const double eps = 2.220446049250313e-16;
  const double floor_abs = eps * fro;

  int sweeps = 0;
  bool converged = (M <= 1);
  for (; sweeps < max_sweeps && !converged; ++sweeps) {
    if (tid == 0) s_rot = 0;
    __syncthreads();
    for (int step = 0; step < M - 1; ++step) {
      if (tid < H) {
        int p = rr_player(tid, step, M), q = rr_player(M - 1 - tid, step, M);
        if (p > q) { int t = p; p = q; q = t; }
        double c = 1.0, s = 0.0, t = 0.0;
        int a = 0;
        if (q < m) {
          double apq = A[uidx(p, q)];
          double app = A[uidx(p, p)], aqq = A[uidx(q, q)];
          double thr = fmax(eps * sqrt(fabs(app * aqq)), floor_abs);
          if (fabs(apq) > thr) {
            double tau = (aqq - app) / (2.0 * apq);
            t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            a = 1;
            s_rot = 1;
          }
        }
        pp[tid] = p; qq[tid] = q; cs[tid] = c; sn[tid] = s; tn[tid] = t; act[tid] = a;
      }
      __syncthreads();
      // two-sided update of all 2x2 blocks (k <= l)
      const int nb = H * (H + 1) / 2;
      for (int t = tid; t < nb; t += nt) {
        int l = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
        while (l * (l + 1) / 2 > t) --l;
        while ((l + 1) * (l + 2) / 2 <= t) ++l;
        int k = t - l * (l + 1) / 2;
        if (!act[k] && !act[l]) continue;
        int pk = pp[k], qk = qq[k];
        if (k == l) {
          double apq = A[uidx(pk, qk)];
          double tk = tn[k];
          A[uidx(pk, pk)] -= tk * apq;
          A[uidx(qk, qk)] += tk * apq;
          A[uidx(pk, qk)] = 0.0;
          continue;
        }
        int pl = pp[l], ql = qq[l];
        double ck = cs[k], sk = sn[k], cl = cs[l], sl = sn[l];
        int i00 = sidx(pk, pl), i01 = sidx(pk, ql), i10 = sidx(qk, pl), i11 = sidx(qk, ql);
        double m00 = A[i00], m01 = A[i01], m10 = A[i10], m11 = A[i11];
        // rows: J_k^T M
        double r00 = ck * m00 - sk * m10, r01 = ck * m01 - sk * m11;
        double r10 = sk * m00 + ck * m10, r11 = sk * m01 + ck * m11;
        // cols: (.) J_l
        A[i00] = r00 * cl - r01 * sl;
        A[i01] = r00 * sl + r01 * cl;
        A[i10] = r10 * cl - r11 * sl;
        A[i11] = r10 * sl + r11 * cl;
      }
      // eigenvector columns
      const long nv = (long)m * H;
      for (long t = tid; t < nv; t += nt) {
        int k = (int)(t % H);
        int r = (int)(t / H);
        if (!act[k]) continue;
        int p = pp[k], q = qq[k];
        double c = cs[k], s = sn[k];
        double vp = V[(long)r * m + p], vq = V[(long)r * m + q];
        V[(long)r * m + p] = c * vp - s * vq;
        V[(long)r * m + q] = s * vp + c * vq;
      }
      __syncthreads();
    }
    converged = (s_rot == 0);
    __syncthreads();
  }
  // sort eigenvalues ascending (ties by index) and permute eigenvector columns
  for (int i = tid; i < m; i += nt) {
    double di = A[uidx(i, i)];
    int rank = 0;
    for (int j = 0; j < m; ++j) {
      double dj = A[uidx(j, j)];
      rank += (dj < di) || (dj == di && j < i);
    }
    evals[(long)b * sE + rank] = di;
    for (int r = 0; r < m; ++r) Vout[(long)b * sV + (long)r * m + rank] = V[(long)r * m + i];
  }
  if (tid == 0) info[b] = converged ? sweeps : -sweeps;
}

int jacobi_max_m() { return JMAX; }

void linalg_set_attrs() {
  const int lds = 160 * 1024 - 1024;
  hipFuncSetAttribute(reinterpret_cast<const void*>(&jacobi_kernel),
                      hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  hipFuncSetAttribute(reinterpret_cast<const void*>(&chol_inv_kernel),
                      hipFuncAttributeMaxDynamicSharedMemorySize, lds);
}

void jacobi_eig(hipStream_t s, int batch, int m, const double* A, long sA, double* evals, long sE,
                double* V, long sV, double* Vwork, int* info) {
  int M = m + (m & 1);
  size_t lds = (size_t)M * (M + 1) / 2 * sizeof(double) + (size_t)(M / 2) * (3 * sizeof(double) + 3 * sizeof(int));
  hipLaunchKernelGGL(jacobi_kernel, dim3(batch), dim3(1024), lds, s, m, A, sA, evals, sE, V, sV,
                     Vwork, 40, info);
}

}  // namespace rmc
