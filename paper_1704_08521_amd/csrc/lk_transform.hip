// Tensor-product transforms of the pressure-correction solve: every grid line
// along one axis is multiplied by the same n x n mode matrix (S^T M forward, S
// backward).  Both kernels are register-tiled dense contractions on the vector
// FMA units with LDS staging; one block owns the whole transformed dimension
// (up to 16*TM rows), so each data tile is read from HBM once.
#include <hip/hip_runtime.h>

#include "lk_device.h"

namespace lk {
namespace {

constexpr int TPR = 16;  // thread rows
constexpr int TPC = 16;  // thread columns

// Left transform: C[m][n] = sum_k A[m][k] B[k][n]; A is the n_axis x n_axis mode
// matrix, B the data with "segmented" columns: column n starts at
// (n / nseg) * seg_stride + n % nseg and consecutive k are kstride apart.  C has
// B's layout.  With scale set, C[m][n] is divided by lam_m + ly[j] + lx[i]
// (n = j*nx + i), and the constant mode (m, j, i) = (zm, zj, zi) is zeroed.
template <typename T, int TM, int TN, int TBK>
__global__ void __launch_bounds__(TPR* TPC) k_tp_left(int M, int N, int K, const T* __restrict__ A,
                                                      const T* __restrict__ B, T* __restrict__ C, int nseg,
                                                      long seg_stride, long kstride, const double* __restrict__ lm,
                                                      const double* __restrict__ ly, const double* __restrict__ lx,
                                                      int nxs, int zm, int zj, int zi) {
  constexpr int BM = TPR * TM, BN = TPC * TN;
  __shared__ T As[TBK][BM + 1];
  __shared__ T Bs[TBK][BN];
  const int tid = threadIdx.x;
  const int tx = tid % TPC, ty = tid / TPC;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  // B-tile loads: thread loads column (tid % BN) for rows (tid / BN) + q*(256/BN)
  const int lcol = tid % BN, lrow = tid / BN;
  constexpr int LROWS = (TPR * TPC) / BN;
  const int gnl = n0 + lcol;
  const long boff = (gnl < N) ? (long)(gnl / nseg) * seg_stride + (gnl % nseg) : 0;
  T acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int c = 0; c < TN; ++c) acc[a][c] = T(0);
  // global -> registers (all loads issued back to back from in-range addresses),
  // registers -> LDS one chunk later so the next chunk is in flight during compute
  constexpr int NTH = TPR * TPC;
  constexpr int NA = (BM * TBK + NTH - 1) / NTH;
  constexpr int NB = (TBK * BN) / NTH;
  T ra[NA], rb[NB];
  auto gload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + q * NTH;
      const int mm = e / TBK, kk = e % TBK;
      const int gm = m0 + mm, gk = k0 + kk;
      const bool ok = e < BM * TBK && gm < M && gk < K;
      const T x = A[ok ? (long)gm * K + gk : 0];
      ra[q] = ok ? x : T(0);
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int gk = k0 + lrow + q * LROWS;
      const bool ok = gnl < N && gk < K;
      const T x = B[ok ? boff + (long)gk * kstride : 0];
      rb[q] = ok ? x : T(0);
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + q * NTH;
      if (e < BM * TBK) As[e % TBK][e / TBK] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) Bs[lrow + q * LROWS][lcol] = rb[q];
  };
  gload(0);
  for (int k0 = 0; k0 < K; k0 += TBK) {
    sstore();
    __syncthreads();
    if (k0 + TBK < K) gload(k0 + TBK);
#pragma unroll 4
    for (int kk = 0; kk < TBK; ++kk) {
      T av[TM], bv[TN];
#pragma unroll
      for (int a = 0; a < TM; ++a) av[a] = As[kk][ty + TPR * a];
#pragma unroll
      for (int c = 0; c < TN; ++c) bv[c] = Bs[kk][tx + TPC * c];
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int c = 0; c < TN; ++c) acc[a][c] = fma(av[a], bv[c], acc[a][c]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int c = 0; c < TN; ++c) {
    const int gn = n0 + tx + TPC * c;
    if (gn >= N) continue;
    const long off = (long)(gn / nseg) * seg_stride + (gn % nseg);
    const int jj = lm ? gn / nxs : 0, ii = lm ? gn % nxs : 0;
    const double sxy = lm ? ly[jj] + lx[ii] : 0.0;
#pragma unroll
    for (int a = 0; a < TM; ++a) {
      const int gm = m0 + ty + TPR * a;
      if (gm >= M) continue;
      T val = acc[a][c];
      if (lm) val = (gm == zm && jj == zj && ii == zi) ? T(0) : (T)((double)val / (lm[gm] + sxy));
      C[off + (long)gm * kstride] = val;
    }
  }
}

// Right transform: C[m][n] = sum_k A[m][k] B[k][n]; A is the data (lines of
// length K, contiguous), B the K x N mode matrix (transposed), C lines of N.
template <typename T, int TM, int TN, int TBK>
__global__ void __launch_bounds__(TPR* TPC) k_tp_right(int M, int N, int K, const T* __restrict__ A,
                                                       const T* __restrict__ B, T* __restrict__ C) {
  constexpr int BM = TPR * TM, BN = TPC * TN;
  __shared__ T As[TBK][BM + 1];
  __shared__ T Bs[TBK][BN];
  const int tid = threadIdx.x;
  const int tx = tid % TPC, ty = tid / TPC;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  T acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int c = 0; c < TN; ++c) acc[a][c] = T(0);
  constexpr int NTH = TPR * TPC;
  constexpr int NA = (BM * TBK) / NTH;
  constexpr int NB = (TBK * BN + NTH - 1) / NTH;
  T ra[NA], rb[NB];
  auto gload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + q * NTH;
      const int mm = e / TBK, kk = e % TBK;
      const int gm = m0 + mm, gk = k0 + kk;
      const bool ok = gm < M && gk < K;
      const T x = A[ok ? (long)gm * K + gk : 0];
      ra[q] = ok ? x : T(0);
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = tid + q * NTH;
      const int kk = e / BN, nn = e % BN;
      const int gk = k0 + kk, gn = n0 + nn;
      const bool ok = e < TBK * BN && gk < K && gn < N;
      const T x = B[ok ? (long)gk * N + gn : 0];
      rb[q] = ok ? x : T(0);
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + q * NTH;
      As[e % TBK][e / TBK] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = tid + q * NTH;
      if (e < TBK * BN) Bs[e / BN][e % BN] = rb[q];
    }
  };
  gload(0);
  for (int k0 = 0; k0 < K; k0 += TBK) {
    sstore();
    __syncthreads();
    if (k0 + TBK < K) gload(k0 + TBK);
#pragma unroll 4
    for (int kk = 0; kk < TBK; ++kk) {
      T av[TM], bv[TN];
#pragma unroll
      for (int a = 0; a < TM; ++a) av[a] = As[kk][ty + TPR * a];
#pragma unroll
      for (int c = 0; c < TN; ++c) bv[c] = Bs[kk][tx + TPC * c];
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int c = 0; c < TN; ++c) acc[a][c] = fma(av[a], bv[c], acc[a][c]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < TM; ++a) {
    const int gm = m0 + ty + TPR * a;
    if (gm >= M) continue;
#pragma unroll
    for (int c = 0; c < TN; ++c) {
      const int gn = n0 + tx + TPC * c;
      if (gn < N) C[(long)gm * N + gn] = acc[a][c];
    }
  }
}

// ------------------------------------------------ mirror-symmetric axes
// On a grid symmetric under i -> n-1-i every mode of an axis is even or odd, so a
// transform splits into two half-size ones.  Modes are stored parity-sorted (he even
// modes, then ho odd ones; he = ceil(n/2), ho = floor(n/2)).  Forward: line values are
// folded on load, f_i + f_{n-1-i} (even; the middle value alone when n is odd) and
// f_i - f_{n-1-i} (odd), and contracted with the even (he x he) or odd (ho x ho) half
// matrix; blocks with blockIdx.y (left) / blockIdx.x (right) below nbe do the even
// half.  Backward: a_i = sum_e Se[i][e] c_e and b_i = sum_o So[i][o] c_o for i < he,
// written as phi_i = a_i + b_i and phi_{n-1-i} = a_i - b_i.

// Left, forward: C[r][col] (r parity-sorted mode) = sum_k Ah[r'][k] fold(B)[k][col];
// B and C have the segmented-column layout of k_tp_left; optional eigenvalue scaling.
template <typename T, int TM, int TN, int TBK>
__global__ void __launch_bounds__(TPR* TPC) k_tpf_left(int n, int he, int ho, int nbe, int N, const T* __restrict__ Ae,
                                                       const T* __restrict__ Ao, const T* __restrict__ B,
                                                       T* __restrict__ C, int nseg, long seg_stride, long kstride,
                                                       const double* __restrict__ lm, const double* __restrict__ ly,
                                                       const double* __restrict__ lx, int nxs, int zm, int zj, int zi) {
  constexpr int BM = TPR * TM, BN = TPC * TN;
  __shared__ T As[TBK][BM + 1];
  __shared__ T Bs[TBK][BN];
  const bool odd = (int)blockIdx.y >= nbe;
  const int M = odd ? ho : he, K = M;
  const T* A = odd ? Ao : Ae;
  const T sgn = odd ? T(-1) : T(1);
  const int rowoff = odd ? he : 0;
  const int tid = threadIdx.x;
  const int tx = tid % TPC, ty = tid / TPC;
  const int m0 = (odd ? (int)blockIdx.y - nbe : (int)blockIdx.y) * BM, n0 = blockIdx.x * BN;
  const int lcol = tid % BN, lrow = tid / BN;
  constexpr int LROWS = (TPR * TPC) / BN;
  const int gnl = n0 + lcol;
  const long boff = (gnl < N) ? (long)(gnl / nseg) * seg_stride + (gnl % nseg) : 0;
  T acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int c = 0; c < TN; ++c) acc[a][c] = T(0);
  constexpr int NTH = TPR * TPC;
  constexpr int NA = (BM * TBK + NTH - 1) / NTH;
  constexpr int NB = (TBK * BN) / NTH;
  T ra[NA], rb[NB];
  auto gload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + q * NTH;
      const int mm = e / TBK, kk = e % TBK;
      const int gm = m0 + mm, gk = k0 + kk;
      const bool ok = e < BM * TBK && gm < M && gk < K;
      const T x = A[ok ? (long)gm * K + gk : 0];
      ra[q] = ok ? x : T(0);
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int gk = k0 + lrow + q * LROWS;
      const bool ok = gnl < N && gk < K;
      const int gm = n - 1 - gk;
      const T x1 = B[ok ? boff + (long)gk * kstride : 0];
      const T x2 = B[ok ? boff + (long)gm * kstride : 0];
      rb[q] = ok ? (gm == gk ? x1 : x1 + sgn * x2) : T(0);
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + q * NTH;
      if (e < BM * TBK) As[e % TBK][e / TBK] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) Bs[lrow + q * LROWS][lcol] = rb[q];
  };
  gload(0);
  for (int k0 = 0; k0 < K; k0 += TBK) {
    sstore();
    __syncthreads();
    if (k0 + TBK < K) gload(k0 + TBK);
#pragma unroll 4
    for (int kk = 0; kk < TBK; ++kk) {
      T av[TM], bv[TN];
#pragma unroll
      for (int a = 0; a < TM; ++a) av[a] = As[kk][ty + TPR * a];
#pragma unroll
      for (int c = 0; c < TN; ++c) bv[c] = Bs[kk][tx + TPC * c];
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int c = 0; c < TN; ++c) acc[a][c] = fma(av[a], bv[c], acc[a][c]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int c = 0; c < TN; ++c) {
    const int gn = n0 + tx + TPC * c;
    if (gn >= N) continue;
    const long off = (long)(gn / nseg) * seg_stride + (gn % nseg);
    const int jj = lm ? gn / nxs : 0, ii = lm ? gn % nxs : 0;
    const double sxy = lm ? ly[jj] + lx[ii] : 0.0;
#pragma unroll
    for (int a = 0; a < TM; ++a) {
      const int lr = m0 + ty + TPR * a;
      if (lr >= M) continue;
      const int gm = rowoff + lr;
      T val = acc[a][c];
      if (lm) val = (gm == zm && jj == zj && ii == zi) ? T(0) : (T)((double)val / (lm[gm] + sxy));
      C[off + (long)gm * kstride] = val;
    }
  }
}

// Left, backward: rows i < he of a = Se c_e (Se: he x he) and b = So c_o (So: he x ho),
// C[i] = a + b and C[n-1-i] = a - b; B (parity-sorted modes) and C have the
// segmented-column layout.
template <typename T, int TM, int TN, int TBK>
__global__ void __launch_bounds__(TPR* TPC) k_tpu_left(int n, int he, int ho, int N, const T* __restrict__ Se,
                                                       const T* __restrict__ So, const T* __restrict__ B,
                                                       T* __restrict__ C, int nseg, long seg_stride, long kstride) {
  constexpr int BM = TPR * TM, BN = TPC * TN;
  __shared__ T As[TBK][BM + 1];
  __shared__ T Bs[TBK][BN];
  const int tid = threadIdx.x;
  const int tx = tid % TPC, ty = tid / TPC;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int lcol = tid % BN, lrow = tid / BN;
  constexpr int LROWS = (TPR * TPC) / BN;
  const int gnl = n0 + lcol;
  const long boff = (gnl < N) ? (long)(gnl / nseg) * seg_stride + (gnl % nseg) : 0;
  T acc[2][TM][TN];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int c = 0; c < TN; ++c) acc[h][a][c] = T(0);
  constexpr int NTH = TPR * TPC;
  constexpr int NA = (BM * TBK + NTH - 1) / NTH;
  constexpr int NB = (TBK * BN) / NTH;
  T ra[NA], rb[NB];
  // phase 0: even modes (K = he, rows 0..he-1 of B); phase 1: odd modes (K = ho, rows he..)
  auto gload = [&](int ph, int k0) {
    const T* A = ph ? So : Se;
    const int K = ph ? ho : he;
    const int kb = ph ? he : 0;
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + q * NTH;
      const int mm = e / TBK, kk = e % TBK;
      const int gm = m0 + mm, gk = k0 + kk;
      const bool ok = e < BM * TBK && gm < he && gk < K;
      const T x = A[ok ? (long)gm * K + gk : 0];
      ra[q] = ok ? x : T(0);
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int gk = k0 + lrow + q * LROWS;
      const bool ok = gnl < N && gk < K;
      const T x = B[ok ? boff + (long)(kb + gk) * kstride : 0];
      rb[q] = ok ? x : T(0);
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + q * NTH;
      if (e < BM * TBK) As[e % TBK][e / TBK] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) Bs[lrow + q * LROWS][lcol] = rb[q];
  };
#pragma unroll
  for (int ph = 0; ph < 2; ++ph) {
    const int K = ph ? ho : he;
    gload(ph, 0);
    for (int k0 = 0; k0 < K; k0 += TBK) {
      sstore();
      __syncthreads();
      if (k0 + TBK < K) gload(ph, k0 + TBK);
#pragma unroll 4
      for (int kk = 0; kk < TBK; ++kk) {
        T av[TM], bv[TN];
#pragma unroll
        for (int a = 0; a < TM; ++a) av[a] = As[kk][ty + TPR * a];
#pragma unroll
        for (int c = 0; c < TN; ++c) bv[c] = Bs[kk][tx + TPC * c];
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
          for (int c = 0; c < TN; ++c) acc[ph][a][c] = fma(av[a], bv[c], acc[ph][a][c]);
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int c = 0; c < TN; ++c) {
    const int gn = n0 + tx + TPC * c;
    if (gn >= N) continue;
    const long off = (long)(gn / nseg) * seg_stride + (gn % nseg);
#pragma unroll
    for (int a = 0; a < TM; ++a) {
      const int i = m0 + ty + TPR * a;
      if (i >= he) continue;
      const T va = acc[0][a][c], vb = acc[1][a][c];
      C[off + (long)i * kstride] = va + vb;
      if (i < ho) C[off + (long)(n - 1 - i) * kstride] = va - vb;
    }
  }
}

// Right, forward: C[line][r] (parity-sorted mode) = sum_k fold(A)[line][k] Bh[k][r'];
// A: lines of n contiguous values; Bh: FTe (he x he) or FTo (ho x ho); C: lines of n.
template <typename T, int TM, int TN, int TBK>
__global__ void __launch_bounds__(TPR* TPC) k_tpf_right(int n, int he, int ho, int nbe, int Mlines,
                                                        const T* __restrict__ A, const T* __restrict__ Be,
                                                        const T* __restrict__ Bo, T* __restrict__ C) {
  constexpr int BM = TPR * TM, BN = TPC * TN;
  __shared__ T As[TBK][BM + 1];
  __shared__ T Bs[TBK][BN];
  const bool odd = (int)blockIdx.x >= nbe;
  const int N = odd ? ho : he, K = N;
  const T* B = odd ? Bo : Be;
  const T sgn = odd ? T(-1) : T(1);
  const int coloff = odd ? he : 0;
  const int tid = threadIdx.x;
  const int tx = tid % TPC, ty = tid / TPC;
  const int m0 = blockIdx.y * BM, n0 = (odd ? (int)blockIdx.x - nbe : (int)blockIdx.x) * BN;
  T acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int c = 0; c < TN; ++c) acc[a][c] = T(0);
  constexpr int NTH = TPR * TPC;
  constexpr int NA = (BM * TBK) / NTH;
  constexpr int NB = (TBK * BN + NTH - 1) / NTH;
  T ra[NA], rb[NB];
  auto gload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + q * NTH;
      const int mm = e / TBK, kk = e % TBK;
      const int gm = m0 + mm, gk = k0 + kk;
      const bool ok = gm < Mlines && gk < K;
      const int gr = n - 1 - gk;
      const T x1 = A[ok ? (long)gm * n + gk : 0];
      const T x2 = A[ok ? (long)gm * n + gr : 0];
      ra[q] = ok ? (gr == gk ? x1 : x1 + sgn * x2) : T(0);
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = tid + q * NTH;
      const int kk = e / BN, nn = e % BN;
      const int gk = k0 + kk, gn = n0 + nn;
      const bool ok = e < TBK * BN && gk < K && gn < N;
      const T x = B[ok ? (long)gk * N + gn : 0];
      rb[q] = ok ? x : T(0);
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + q * NTH;
      As[e % TBK][e / TBK] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = tid + q * NTH;
      if (e < TBK * BN) Bs[e / BN][e % BN] = rb[q];
    }
  };
  gload(0);
  for (int k0 = 0; k0 < K; k0 += TBK) {
    sstore();
    __syncthreads();
    if (k0 + TBK < K) gload(k0 + TBK);
#pragma unroll 4
    for (int kk = 0; kk < TBK; ++kk) {
      T av[TM], bv[TN];
#pragma unroll
      for (int a = 0; a < TM; ++a) av[a] = As[kk][ty + TPR * a];
#pragma unroll
      for (int c = 0; c < TN; ++c) bv[c] = Bs[kk][tx + TPC * c];
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int c = 0; c < TN; ++c) acc[a][c] = fma(av[a], bv[c], acc[a][c]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < TM; ++a) {
    const int gm = m0 + ty + TPR * a;
    if (gm >= Mlines) continue;
#pragma unroll
    for (int c = 0; c < TN; ++c) {
      const int gn = n0 + tx + TPC * c;
      if (gn < N) C[(long)gm * n + coloff + gn] = acc[a][c];
    }
  }
}

// Right, backward: for each line, a_i = sum_e c_e SeT[e][i], b_i = sum_o c_o SoT[o][i]
// (i < he; SeT: he x he, SoT: ho x he), C[line][i] = a + b, C[line][n-1-i] = a - b.
template <typename T, int TM, int TN, int TBK>
__global__ void __launch_bounds__(TPR* TPC) k_tpu_right(int n, int he, int ho, int Mlines, const T* __restrict__ A,
                                                        const T* __restrict__ SeT, const T* __restrict__ SoT,
                                                        T* __restrict__ C) {
  constexpr int BM = TPR * TM, BN = TPC * TN;
  __shared__ T As[TBK][BM + 1];
  __shared__ T Bs[TBK][BN];
  const int tid = threadIdx.x;
  const int tx = tid % TPC, ty = tid / TPC;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  T acc[2][TM][TN];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int c = 0; c < TN; ++c) acc[h][a][c] = T(0);
  constexpr int NTH = TPR * TPC;
  constexpr int NA = (BM * TBK) / NTH;
  constexpr int NB = (TBK * BN + NTH - 1) / NTH;
  T ra[NA], rb[NB];
  auto gload = [&](int ph, int k0) {
    const T* B = ph ? SoT : SeT;
    const int K = ph ? ho : he;
    const int kb = ph ? he : 0;
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + q * NTH;
      const int mm = e / TBK, kk = e % TBK;
      const int gm = m0 + mm, gk = k0 + kk;
      const bool ok = gm < Mlines && gk < K;
      const T x = A[ok ? (long)gm * n + kb + gk : 0];
      ra[q] = ok ? x : T(0);
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = tid + q * NTH;
      const int kk = e / BN, nn = e % BN;
      const int gk = k0 + kk, gn = n0 + nn;
      const bool ok = e < TBK * BN && gk < K && gn < he;
      const T x = B[ok ? (long)gk * he + gn : 0];
      rb[q] = ok ? x : T(0);
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + q * NTH;
      As[e % TBK][e / TBK] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = tid + q * NTH;
      if (e < TBK * BN) Bs[e / BN][e % BN] = rb[q];
    }
  };
#pragma unroll
  for (int ph = 0; ph < 2; ++ph) {
    const int K = ph ? ho : he;
    gload(ph, 0);
    for (int k0 = 0; k0 < K; k0 += TBK) {
      sstore();
      __syncthreads();
      if (k0 + TBK < K) gload(ph, k0 + TBK);
#pragma unroll 4
      for (int kk = 0; kk < TBK; ++kk) {
        T av[TM], bv[TN];
#pragma unroll
        for (int a = 0; a < TM; ++a) av[a] = As[kk][ty + TPR * a];
#pragma unroll
        for (int c = 0; c < TN; ++c) bv[c] = Bs[kk][tx + TPC * c];
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
          for (int c = 0; c < TN; ++c) acc[ph][a][c] = fma(av[a], bv[c], acc[ph][a][c]);
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int a = 0; a < TM; ++a) {
    const int gm = m0 + ty + TPR * a;
    if (gm >= Mlines) continue;
#pragma unroll
    for (int c = 0; c < TN; ++c) {
      const int i = n0 + tx + TPC * c;
      if (i >= he) continue;
      const T va = acc[0][a][c], vb = acc[1][a][c];
      C[(long)gm * n + i] = va + vb;
      if (i < ho) C[(long)gm * n + (n - 1 - i)] = va - vb;
    }
  }
}

// Register tile along the transformed dimension: the smallest that covers n with 16
// threads, except that 161..224 uses 7 (two blocks of 112), which measured faster at
// n = 200 than one block of 13 (n > 256 uses several blocks).
inline int pick_tile(int n) {
  if (n > 160 && n <= 224) return 7;
  const int need = (n + 15) / 16;
  const int opts[] = {1, 2, 4, 8, 10, 13, 16};
  for (int t : opts)
    if (t >= need) return t;
  return 16;
}

template <typename T, int TM>
hipError_t left_launch(int M, int N, int K, const T* A, const T* B, T* C, int nseg, long seg_stride, long kstride,
                       const double* lm, const double* ly, const double* lx, int nxs, int zm, int zj, int zi,
                       hipStream_t st) {
  dim3 grid(blocks_for(N, TPC * 4), blocks_for(M, TPR * TM), 1);
  hipLaunchKernelGGL((k_tp_left<T, TM, 4, 16>), grid, dim3(TPR * TPC), 0, st, M, N, K, A, B, C, nseg, seg_stride, kstride,
                     lm, ly, lx, nxs, zm, zj, zi);
  return hipGetLastError();
}

template <typename T, int TN>
hipError_t right_launch(int M, int N, int K, const T* A, const T* B, T* C, hipStream_t st) {
  dim3 grid(blocks_for(N, TPC * TN), blocks_for(M, TPR * 4), 1);
  hipLaunchKernelGGL((k_tp_right<T, 4, TN, 16>), grid, dim3(TPR * TPC), 0, st, M, N, K, A, B, C);
  return hipGetLastError();
}


// ------------------------------------------------ matrix-core (MFMA) transforms
// The folded transforms of a mirror-symmetric axis as 16x16x4 MFMA contractions
// (FP64 or FP32 matrix cores).  One wave owns W tiles of 16 columns (left) or 16
// lines (right) and every output mode of both parities, so each input value is read
// from HBM once and folded in registers; no LDS.  The half matrices come packed in
// fragment order: P[(kq * RT + t) * 64 + l] = Mat(o = 16 t + l % 16, k = 4 kq + l / 16),
// zero outside the matrix, where o is the output index (mode forward, point backward)
// and k the contracted one.  One 64-value load per fragment, and the same pack serves
// as the A operand (left: Mat x data) and as the B operand (right: data x Mat^T).
// (Fragments are grouped 16 bytes per lane: see mf_pack_index.)
// Lane l of a 16x16x4 step holds A[l % 16][l / 16] and B[l / 16][l % 16]; it receives
// D[row(l / 16, r)][l % 16], r = 0..3, with row = 4 g + r (FP32) or g + 4 r (FP64), as
// measured on gfx950.
template <typename T>
struct Mf;
template <>
struct Mf<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int g, int r) { return g + 4 * r; }
};
template <>
struct Mf<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int g, int r) { return 4 * g + r; }
};

// v / a for the eigenvalue scaling, a > 0: hardware reciprocal refined by two Newton
// steps and one residual correction of the quotient (within an ulp of v / a, a third of
// the instructions of the IEEE division sequence).  The FP32 solve divides in FP32
// (reciprocal and one Newton step).
__device__ __forceinline__ float mf_div(float v, double a) {
  const float af = (float)a;
  float y = __builtin_amdgcn_rcpf(af);
  y = fmaf(fmaf(-af, y, 1.0f), y, y);
  return v * y;
}
__device__ __forceinline__ double mf_div(double v, double a) {
  double y = __builtin_amdgcn_rcp(a);
  double e = fma(-a, y, 1.0);
  y = fma(e, y, y);
  e = fma(-a, y, 1.0);
  y = fma(e, y, y);
  const double q = v * y;
  return fma(fma(-a, q, v), y, q);
}

// Data fragments of contraction index k (= 4 kq + l / 16) for the W tiles: element
// (tile c, k) lives at src[base[c] + k * kstr].  mf_load issues the two raw loads (k and
// its mirror n-1-k forward, the even mode k and the odd mode he+k backward) from
// in-range addresses; mf_fold combines them only when the step is computed, so the loads
// stay in flight meanwhile.  Forward: s = f_k + f_{n-1-k} (f_k alone on the middle row),
// d = f_k - f_{n-1-k}.  Backward: s = c_k, d = c_{he+k}.
template <typename T, int W, bool FOLD>
__device__ __forceinline__ void mf_load(const T* __restrict__ src, const long (&base)[W], const bool (&ok)[W],
                                        long kstr, int n, int he, int ho, int k, T (&x1)[W], T (&x2)[W]) {
  const bool ke = k < he, ko = k < ho;
  const long k1 = k, k2 = FOLD ? (long)(n - 1 - k) : (long)(he + k);
#pragma unroll
  for (int c = 0; c < W; ++c) {
    const bool oe = ok[c] & ke, oo = ok[c] & (FOLD ? ke : ko);
    x1[c] = src[oe ? base[c] + k1 * kstr : 0];
    x2[c] = src[oo ? base[c] + k2 * kstr : 0];
  }
}
// Optional scaling of the backward operands (SCALE: the pressure solve's division by the
// sum of the axis eigenvalues, done where the z backward transform loads its modes):
// column c's mode k is divided by lm[k] + sxy[c], and the constant mode (zm in a
// zero-mode column, zc[c]) is set to zero.
template <typename T, int W, bool FOLD, bool SCALE>
__device__ __forceinline__ void mf_fold(const bool (&ok)[W], int n, int he, int ho, int k, const T (&x1)[W],
                                        const T (&x2)[W], int zm, double le, double lo, const double (&sxy)[W],
                                        const bool (&zc)[W], T (&s)[W], T (&d)[W]) {
  const bool ke = k < he, ko = k < ho;
#pragma unroll
  for (int c = 0; c < W; ++c) {
    const bool oe = ok[c] & ke;
    if (FOLD) {
      s[c] = oe ? (n - 1 - k == k ? x1[c] : x1[c] + x2[c]) : T(0);
      d[c] = (oe & ko) ? x1[c] - x2[c] : T(0);
    } else if (SCALE) {  // padding and the constant mode stay exactly zero (no 0/0)
      s[c] = (!oe || (zc[c] && k == zm)) ? T(0) : mf_div(x1[c], le + sxy[c]);
      d[c] = (!(ok[c] & ko) || (zc[c] && he + k == zm)) ? T(0) : mf_div(x2[c], lo + sxy[c]);
    } else {
      s[c] = oe ? x1[c] : T(0);
      d[c] = (ok[c] & ko) ? x2[c] : T(0);
    }
  }
}

// Accumulates the even and odd contractions of one wave: acc_e += Pe x s, acc_o += Po x d
// over the KQP steps of the (padded) packs.  Vector-memory loads complete in issue order,
// so every load of a step - raw data (HBM), pack fragments (L1/L2) and eigenvalues alike -
// is issued PD steps ahead into a register ring (PD = 1 in use: the registers a deeper
// ring costs buy more as a third wave per SIMD); the step loop has no conditional exits
// (KQP is a multiple of PD, the padding steps hold zero fragments and masked data), which
// lets the compiler wait for exactly the oldest step's loads instead of draining all of
// them at the loop head.  LEFT: the pack is the A operand; otherwise the data is.
template <typename T, int RT, int W, bool FOLD, bool LEFT, bool SCALE, int PD>
__device__ __forceinline__ void mf_contract(const T* __restrict__ Pe, const T* __restrict__ Po,
                                            const T* __restrict__ src, const long (&base)[W], const bool (&ok)[W],
                                            long kstr, int n, int he, int ho, const double* __restrict__ lm, int zm,
                                            const double (&sxy)[W], const bool (&zc)[W],
                                            typename Mf<T>::v4 (&ae)[RT][W], typename Mf<T>::v4 (&ao)[RT][W]) {
  const int lane = threadIdx.x & 63, g = lane >> 4;
  const int KQP = mf_steps(he, PD);
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int c = 0; c < W; ++c) {
      ae[t][c] = typename Mf<T>::v4{0, 0, 0, 0};
      ao[t][c] = typename Mf<T>::v4{0, 0, 0, 0};
    }
  constexpr int FG = 16 / sizeof(T), RTG = mf_tile_groups(RT, FG);
  typedef T VG __attribute__((ext_vector_type(FG)));
  VG pe[PD][RTG], po[PD][RTG];
  T r1[PD][W], r2[PD][W];
  double le[PD], lo[PD];
#define LK_MF_ISSUE(u, kq)                                                              \
  {                                                                                     \
    const int kc = min(kq, KQP - 1); /* the last steps re-read in-range fragments */    \
    _Pragma("unroll") for (int tg = 0; tg < RTG; ++tg) {                                \
      pe[u][tg] = *(const VG*)(Pe + mf_pack_index(kc, tg * FG, lane, RT, FG));          \
      po[u][tg] = *(const VG*)(Po + mf_pack_index(kc, tg * FG, lane, RT, FG));          \
    }                                                                                   \
    mf_load<T, W, FOLD>(src, base, ok, kstr, n, he, ho, 4 * kc + g, r1[u], r2[u]);      \
    if (SCALE) {                                                                        \
      le[u] = lm[min(4 * kc + g, he - 1)];                                              \
      lo[u] = lm[he + min(4 * kc + g, max(ho - 1, 0))];                                 \
    } else {                                                                            \
      le[u] = lo[u] = 1.0;                                                              \
    }                                                                                   \
  }
#pragma unroll
  for (int u = 0; u < PD; ++u) LK_MF_ISSUE(u, u)
  for (int kq0 = 0; kq0 < KQP; kq0 += PD) {
#pragma unroll
    for (int u = 0; u < PD; ++u) {
      const int kq = kq0 + u;
      T s[W], d[W];
      mf_fold<T, W, FOLD, SCALE>(ok, n, he, ho, 4 * kq + g, r1[u], r2[u], zm, le[u], lo[u], sxy, zc, s, d);
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int c = 0; c < W; ++c) {
          const T fe = pe[u][t / FG][t % FG], fo = po[u][t / FG][t % FG];
          if (LEFT) {
            ae[t][c] = Mf<T>::mma(fe, s[c], ae[t][c]);
            ao[t][c] = Mf<T>::mma(fo, d[c], ao[t][c]);
          } else {
            ae[t][c] = Mf<T>::mma(s[c], fe, ae[t][c]);
            ao[t][c] = Mf<T>::mma(d[c], fo, ao[t][c]);
          }
        }
      LK_MF_ISSUE(u, kq + PD)
    }
  }
#undef LK_MF_ISSUE
}

// Left, forward (folded); layout as k_tpf_left (the eigenvalue scaling is left to the
// backward transform).
template <typename T, int RT, int W, int PD, int LB>
__global__ void __launch_bounds__(256, LB) k_mff_left(int n, int he, int ho, int N, const T* __restrict__ Pe,
                                                  const T* __restrict__ Po, const T* __restrict__ B, T* __restrict__ C,
                                                  int nseg, long seg_stride, long kstride) {
  const int lane = threadIdx.x & 63, g = lane >> 4, cl = lane & 15;
  const int col0 = (blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 16 * W;
  if (col0 >= N) return;
  long base[W];
  bool ok[W], zc[W];
  double sxy[W];
#pragma unroll
  for (int c = 0; c < W; ++c) {
    const int col = col0 + 16 * c + cl;
    ok[c] = col < N;
    base[c] = ok[c] ? (long)(col / nseg) * seg_stride + col % nseg : 0;
    zc[c] = false;
    sxy[c] = 0.0;
  }
  typename Mf<T>::v4 ae[RT][W], ao[RT][W];
  mf_contract<T, RT, W, true, true, false, PD>(Pe, Po, B, base, ok, kstride, n, he, ho, nullptr, -1, sxy, zc, ae, ao);
#pragma unroll
  for (int c = 0; c < W; ++c) {
    if (!ok[c]) continue;
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = 16 * t + Mf<T>::row(g, r);
        if (o < he) C[base[c] + (long)o * kstride] = ae[t][c][r];
        if (o < ho) C[base[c] + (long)(he + o) * kstride] = ao[t][c][r];
      }
  }
}

// Left, backward (unfolded); layout as k_tpu_left.
// With lm set, the input modes are first divided by lm[mode] + ly[j] + lx[i] (column
// (j, i) = (col / nxs, col % nxs)) and the constant mode (zm, zj, zi) is zeroed.
template <typename T, int RT, int W, bool SCALE, int PD, int LB>
__global__ void __launch_bounds__(256, LB) k_mfu_left(int n, int he, int ho, int N, const T* __restrict__ Pse,
                                                  const T* __restrict__ Pso, const T* __restrict__ B, T* __restrict__ C,
                                                  int nseg, long seg_stride, long kstride, const double* __restrict__ lm,
                                                  const double* __restrict__ ly, const double* __restrict__ lx, int nxs,
                                                  int zm, int zj, int zi) {
  const int lane = threadIdx.x & 63, g = lane >> 4, cl = lane & 15;
  const int col0 = (blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 16 * W;
  if (col0 >= N) return;
  long base[W];
  bool ok[W], zc[W];
  double sxy[W];
#pragma unroll
  for (int c = 0; c < W; ++c) {
    const int col = col0 + 16 * c + cl;
    ok[c] = col < N;
    base[c] = ok[c] ? (long)(col / nseg) * seg_stride + col % nseg : 0;
    const int jj = ok[c] && SCALE ? col / nxs : 0, ii = ok[c] && SCALE ? col % nxs : 0;
    zc[c] = SCALE && jj == zj && ii == zi;
    sxy[c] = SCALE ? ly[jj] + lx[ii] : 0.0;
  }
  typename Mf<T>::v4 aa[RT][W], ab[RT][W];
  mf_contract<T, RT, W, false, true, SCALE, PD>(Pse, Pso, B, base, ok, kstride, n, he, ho, lm, zm, sxy, zc, aa, ab);
#pragma unroll
  for (int c = 0; c < W; ++c) {
    if (!ok[c]) continue;
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * t + Mf<T>::row(g, r);
        const T va = aa[t][c][r], vb = ab[t][c][r];
        if (i < he) C[base[c] + (long)i * kstride] = va + vb;
        if (i < ho) C[base[c] + (long)(n - 1 - i) * kstride] = va - vb;
      }
  }
}

// Right, forward (folded): lines of n contiguous values in A, C.
template <typename T, int RT, int W, int PD, int LB>
__global__ void __launch_bounds__(256, LB) k_mff_right(int n, int he, int ho, int Mlines, const T* __restrict__ A,
                                                   const T* __restrict__ Pe, const T* __restrict__ Po,
                                                   T* __restrict__ C) {
  const int lane = threadIdx.x & 63, g = lane >> 4, cl = lane & 15;
  const int line0 = (blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 16 * W;
  if (line0 >= Mlines) return;
  long base[W];
  bool ok[W];
#pragma unroll
  for (int c = 0; c < W; ++c) {
    const int line = line0 + 16 * c + cl;
    ok[c] = line < Mlines;
    base[c] = ok[c] ? (long)line * n : 0;
  }
  typename Mf<T>::v4 ae[RT][W], ao[RT][W];
  bool zc[W];
  double sxy[W];
#pragma unroll
  for (int c = 0; c < W; ++c) {
    zc[c] = false;
    sxy[c] = 0.0;
  }
  mf_contract<T, RT, W, true, false, false, PD>(Pe, Po, A, base, ok, 1, n, he, ho, nullptr, -1, sxy, zc, ae, ao);
#pragma unroll
  for (int c = 0; c < W; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int line = line0 + 16 * c + Mf<T>::row(g, r);
      if (line >= Mlines) continue;
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        const int o = 16 * t + cl;
        if (o < he) C[(long)line * n + o] = ae[t][c][r];
        if (o < ho) C[(long)line * n + he + o] = ao[t][c][r];
      }
    }
}

// Right, backward (unfolded): lines of parity-sorted modes in A, of points in C.
template <typename T, int RT, int W, int PD, int LB>
__global__ void __launch_bounds__(256, LB) k_mfu_right(int n, int he, int ho, int Mlines, const T* __restrict__ A,
                                                   const T* __restrict__ Pse, const T* __restrict__ Pso,
                                                   T* __restrict__ C) {
  const int lane = threadIdx.x & 63, g = lane >> 4, cl = lane & 15;
  const int line0 = (blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 16 * W;
  if (line0 >= Mlines) return;
  long base[W];
  bool ok[W];
#pragma unroll
  for (int c = 0; c < W; ++c) {
    const int line = line0 + 16 * c + cl;
    ok[c] = line < Mlines;
    base[c] = ok[c] ? (long)line * n : 0;
  }
  typename Mf<T>::v4 aa[RT][W], ab[RT][W];
  bool zc[W];
  double sxy[W];
#pragma unroll
  for (int c = 0; c < W; ++c) {
    zc[c] = false;
    sxy[c] = 0.0;
  }
  mf_contract<T, RT, W, false, false, false, PD>(Pse, Pso, A, base, ok, 1, n, he, ho, nullptr, -1, sxy, zc, aa, ab);
#pragma unroll
  for (int c = 0; c < W; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int line = line0 + 16 * c + Mf<T>::row(g, r);
      if (line >= Mlines) continue;
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        const int i = 16 * t + cl;
        const T va = aa[t][c][r], vb = ab[t][c][r];
        if (i < he) C[(long)line * n + i] = va + vb;
        if (i < ho) C[(long)line * n + (n - 1 - i)] = va - vb;
      }
    }
}

}  // namespace

template <typename T>
hipError_t launch_tp_left(int M, int N, int K, const T* A, const T* B, T* C, int nseg, long seg_stride,
                          long kstride, const double* lm, const double* ly, const double* lx, int nxs, int zm, int zj,
                          int zi, hipStream_t st) {
  switch (pick_tile(M)) {
    case 1: return left_launch<T, 1>(M, N, K, A, B, C, nseg, seg_stride, kstride, lm, ly, lx, nxs, zm, zj, zi, st);
    case 2: return left_launch<T, 2>(M, N, K, A, B, C, nseg, seg_stride, kstride, lm, ly, lx, nxs, zm, zj, zi, st);
    case 4: return left_launch<T, 4>(M, N, K, A, B, C, nseg, seg_stride, kstride, lm, ly, lx, nxs, zm, zj, zi, st);
    case 8: return left_launch<T, 8>(M, N, K, A, B, C, nseg, seg_stride, kstride, lm, ly, lx, nxs, zm, zj, zi, st);
    case 7: return left_launch<T, 7>(M, N, K, A, B, C, nseg, seg_stride, kstride, lm, ly, lx, nxs, zm, zj, zi, st);
    case 10: return left_launch<T, 10>(M, N, K, A, B, C, nseg, seg_stride, kstride, lm, ly, lx, nxs, zm, zj, zi, st);
    case 13: return left_launch<T, 13>(M, N, K, A, B, C, nseg, seg_stride, kstride, lm, ly, lx, nxs, zm, zj, zi, st);
    default: return left_launch<T, 16>(M, N, K, A, B, C, nseg, seg_stride, kstride, lm, ly, lx, nxs, zm, zj, zi, st);
  }
}

template <typename T>
hipError_t launch_tp_right(int M, int N, int K, const T* A, const T* B, T* C, hipStream_t st) {
  switch (pick_tile(N)) {
    case 1: return right_launch<T, 1>(M, N, K, A, B, C, st);
    case 2: return right_launch<T, 2>(M, N, K, A, B, C, st);
    case 4: return right_launch<T, 4>(M, N, K, A, B, C, st);
    case 8: return right_launch<T, 8>(M, N, K, A, B, C, st);
    case 7: return right_launch<T, 7>(M, N, K, A, B, C, st);
    case 10: return right_launch<T, 10>(M, N, K, A, B, C, st);
    case 13: return right_launch<T, 13>(M, N, K, A, B, C, st);
    default: return right_launch<T, 16>(M, N, K, A, B, C, st);
  }
}

// Contraction chunk for a half of length k: 20 when it pads less than 16 (k = 100 at
// n = 200 measured 5-10% faster), else 16.
inline bool chunk20(int k) { return (k + 19) / 20 * 20 - k < (k + 15) / 16 * 16 - k; }

// Tile along a half (he <= 112 in one block, larger halves in several).
inline int pick_half_tile(int h) {
  const int need = (h + 15) / 16;
  const int opts[] = {1, 2, 4, 7, 8, 10, 13, 16};
  for (int t : opts)
    if (t >= need) return t;
  return 16;
}

template <typename T>
hipError_t launch_tpf_left(int n, int N, const T* Ae, const T* Ao, const T* B, T* C, int nseg, long seg_stride,
                           long kstride, const double* lm, const double* ly, const double* lx, int nxs, int zm, int zj,
                           int zi, hipStream_t st) {
  const int he = (n + 1) / 2, ho = n / 2;
#define TPF(TM)                                                                                                  \
  {                                                                                                              \
    const int nbe = (int)blocks_for(he, TPR * TM), nbo = (int)blocks_for(ho > 0 ? ho : 1, TPR * TM);           \
    const dim3 grid(blocks_for(N, TPC * 4), nbe + nbo);                                                          \
    if (chunk20(he))                                                                                             \
      hipLaunchKernelGGL((k_tpf_left<T, TM, 4, 20>), grid, dim3(TPR * TPC), 0, st, n, he, ho, nbe, N, Ae, Ao, B, C, \
                         nseg, seg_stride, kstride, lm, ly, lx, nxs, zm, zj, zi);                                \
    else                                                                                                         \
      hipLaunchKernelGGL((k_tpf_left<T, TM, 4, 16>), grid, dim3(TPR * TPC), 0, st, n, he, ho, nbe, N, Ae, Ao, B, C, \
                         nseg, seg_stride, kstride, lm, ly, lx, nxs, zm, zj, zi);                                \
    break;                                                                                                       \
  }
  switch (pick_half_tile(he)) {
    case 1: TPF(1)
    case 2: TPF(2)
    case 4: TPF(4)
    case 7: TPF(7)
    case 8: TPF(8)
    case 10: TPF(10)
    case 13: TPF(13)
    default: TPF(16)
  }
#undef TPF
  return hipGetLastError();
}

template <typename T>
hipError_t launch_tpu_left(int n, int N, const T* Se, const T* So, const T* B, T* C, int nseg, long seg_stride,
                           long kstride, hipStream_t st) {
  const int he = (n + 1) / 2, ho = n / 2;
  // two row blocks per half at n = 200 (the grid would otherwise hold only one block per column tile)
#define TPU(TM)                                                                                                  \
  {                                                                                                              \
    const dim3 grid(blocks_for(N, TPC * 4), blocks_for(he, TPR * TM));                                           \
    if (chunk20(he))                                                                                             \
      hipLaunchKernelGGL((k_tpu_left<T, TM, 4, 20>), grid, dim3(TPR * TPC), 0, st, n, he, ho, N, Se, So, B, C, nseg, \
                         seg_stride, kstride);                                                                   \
    else                                                                                                         \
      hipLaunchKernelGGL((k_tpu_left<T, TM, 4, 16>), grid, dim3(TPR * TPC), 0, st, n, he, ho, N, Se, So, B, C, nseg, \
                         seg_stride, kstride);                                                                   \
    break;                                                                                                       \
  }
  switch (pick_half_tile((he + 1) / 2)) {
    case 1: TPU(1)
    case 2: TPU(2)
    case 4: TPU(4)
    case 7: TPU(7)
    default: TPU(8)
  }
#undef TPU
  return hipGetLastError();
}

template <typename T>
hipError_t launch_tpf_right(int n, int Mlines, const T* A, const T* Be, const T* Bo, T* C, hipStream_t st) {
  const int he = (n + 1) / 2, ho = n / 2;
#define TPFR(TN)                                                                                               \
  {                                                                                                            \
    const int nbe = (int)blocks_for(he, TPC * TN), nbo = (int)blocks_for(ho > 0 ? ho : 1, TPC * TN);         \
    hipLaunchKernelGGL((k_tpf_right<T, 4, TN, 16>), dim3(nbe + nbo, blocks_for(Mlines, TPR * 4)),             \
                       dim3(TPR * TPC), 0, st, n, he, ho, nbe, Mlines, A, Be, Bo, C);                          \
    break;                                                                                                     \
  }
  switch (pick_half_tile(he)) {
    case 1: TPFR(1)
    case 2: TPFR(2)
    case 4: TPFR(4)
    case 7: TPFR(7)
    case 8: TPFR(8)
    case 10: TPFR(10)
    case 13: TPFR(13)
    default: TPFR(16)
  }
#undef TPFR
  return hipGetLastError();
}

template <typename T>
hipError_t launch_tpu_right(int n, int Mlines, const T* A, const T* SeT, const T* SoT, T* C, hipStream_t st) {
  const int he = (n + 1) / 2, ho = n / 2;
#define TPUR(TN)                                                                                               \
  {                                                                                                            \
    const dim3 grid(blocks_for(he, TPC * TN), blocks_for(Mlines, TPR * 4));                                    \
    if (chunk20(he))                                                                                           \
      hipLaunchKernelGGL((k_tpu_right<T, 4, TN, 20>), grid, dim3(TPR * TPC), 0, st, n, he, ho, Mlines, A, SeT, SoT, C); \
    else                                                                                                       \
      hipLaunchKernelGGL((k_tpu_right<T, 4, TN, 16>), grid, dim3(TPR * TPC), 0, st, n, he, ho, Mlines, A, SeT, SoT, C); \
    break;                                                                                                     \
  }
  switch (pick_half_tile((he + 1) / 2)) {
    case 1: TPUR(1)
    case 2: TPUR(2)
    case 4: TPUR(4)
    case 7: TPUR(7)
    default: TPUR(8)
  }
#undef TPUR
  return hipGetLastError();
}

template hipError_t launch_tp_left<double>(int, int, int, const double*, const double*, double*, int, long, long,
                                           const double*, const double*, const double*, int, int, int, int,
                                           hipStream_t);
template hipError_t launch_tp_left<float>(int, int, int, const float*, const float*, float*, int, long, long,
                                          const double*, const double*, const double*, int, int, int, int,
                                          hipStream_t);
template hipError_t launch_tp_right<double>(int, int, int, const double*, const double*, double*, hipStream_t);
template hipError_t launch_tp_right<float>(int, int, int, const float*, const float*, float*, hipStream_t);

#define LK_TPF_INST(T)                                                                                           \
  template hipError_t launch_tpf_left<T>(int, int, const T*, const T*, const T*, T*, int, long, long, const double*, \
                                         const double*, const double*, int, int, int, int, hipStream_t);          \
  template hipError_t launch_tpu_left<T>(int, int, const T*, const T*, const T*, T*, int, long, long, hipStream_t); \
  template hipError_t launch_tpf_right<T>(int, int, const T*, const T*, const T*, T*, hipStream_t);                \
  template hipError_t launch_tpu_right<T>(int, int, const T*, const T*, const T*, T*, hipStream_t);
LK_TPF_INST(double)
LK_TPF_INST(float)
#undef LK_TPF_INST


// ------------------------------------------------ matrix-core launchers
// RT = ceil(he / 16) row tiles per wave (he <= 128); 4 waves per block.
#define LK_MF_SWITCH(RT_, BODY) \
  switch (RT_) {                \
    case 1: BODY(1) break;      \
    case 2: BODY(2) break;      \
    case 3: BODY(3) break;      \
    case 4: BODY(4) break;      \
    case 5: BODY(5) break;      \
    case 6: BODY(6) break;      \
    case 7: BODY(7) break;      \
    case 8: BODY(8) break;      \
    default: return hipErrorInvalidValue; \
  }
// Waves per SIMD: a 200^3 transform is 2500 waves, and at 2 per SIMD (2048 slots) the
// last 452 form a second round that costs half the kernel time (measured: 40 us for 2048
// waves, 60 us for 2304..2500).  With a one-step prefetch ring the FP64 kernels fit 3 per
// SIMD (168 registers) and all 2500 waves run in one round (51-57 us); the FP32 ones do
// best at 2, and so do FP64 kernels with 8 row tiles (n > 224), which spill at 3.
constexpr int kMfW = 1;
template <typename T, int RT>
constexpr int mf_lb() { return sizeof(T) == sizeof(double) && RT < 8 ? 3 : 2; }

template <typename T>
hipError_t launch_mff_left(int n, int N, const T* Pe, const T* Po, const T* B, T* C, int nseg, long seg_stride,
                           long kstride, hipStream_t st) {
  const int he = (n + 1) / 2, ho = n / 2;
  const dim3 grid(blocks_for(blocks_for(N, 16 * kMfW), 4));
#define BODY(RT) hipLaunchKernelGGL((k_mff_left<T, RT, kMfW, kMfPD, mf_lb<T, RT>()>), grid, dim3(256), 0, st, n, he, ho, N, Pe, Po, B, C, nseg, \
                                    seg_stride, kstride);
  LK_MF_SWITCH((he + 15) / 16, BODY)
#undef BODY
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mfu_left(int n, int N, const T* Pse, const T* Pso, const T* B, T* C, int nseg, long seg_stride,
                           long kstride, const double* lm, const double* ly, const double* lx, int nxs, int zm, int zj,
                           int zi, hipStream_t st) {
  const int he = (n + 1) / 2, ho = n / 2;
  const dim3 grid(blocks_for(blocks_for(N, 16 * kMfW), 4));
#define BODY(RT)                                                                                                   \
  if (lm)                                                                                                          \
    hipLaunchKernelGGL((k_mfu_left<T, RT, kMfW, true, kMfPD, mf_lb<T, RT>()>), grid, dim3(256), 0, st, n, he, ho, N, Pse, Pso, B, C, nseg,  \
                       seg_stride, kstride, lm, ly, lx, nxs, zm, zj, zi);                                          \
  else                                                                                                             \
    hipLaunchKernelGGL((k_mfu_left<T, RT, kMfW, false, kMfPD, mf_lb<T, RT>()>), grid, dim3(256), 0, st, n, he, ho, N, Pse, Pso, B, C, nseg, \
                       seg_stride, kstride, lm, ly, lx, nxs, zm, zj, zi);
  LK_MF_SWITCH((he + 15) / 16, BODY)
#undef BODY
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mff_right(int n, int Mlines, const T* A, const T* Pe, const T* Po, T* C, hipStream_t st) {
  const int he = (n + 1) / 2, ho = n / 2;
  const dim3 grid(blocks_for(blocks_for(Mlines, 16 * kMfW), 4));
#define BODY(RT) hipLaunchKernelGGL((k_mff_right<T, RT, kMfW, kMfPD, mf_lb<T, RT>()>), grid, dim3(256), 0, st, n, he, ho, Mlines, A, Pe, Po, C);
  LK_MF_SWITCH((he + 15) / 16, BODY)
#undef BODY
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mfu_right(int n, int Mlines, const T* A, const T* Pse, const T* Pso, T* C, hipStream_t st) {
  const int he = (n + 1) / 2, ho = n / 2;
  const dim3 grid(blocks_for(blocks_for(Mlines, 16 * kMfW), 4));
#define BODY(RT) hipLaunchKernelGGL((k_mfu_right<T, RT, kMfW, kMfPD, mf_lb<T, RT>()>), grid, dim3(256), 0, st, n, he, ho, Mlines, A, Pse, Pso, C);
  LK_MF_SWITCH((he + 15) / 16, BODY)
#undef BODY
  return hipGetLastError();
}
#undef LK_MF_SWITCH

#define LK_MF_INST(T)                                                                                            \
  template hipError_t launch_mff_left<T>(int, int, const T*, const T*, const T*, T*, int, long, long, hipStream_t); \
  template hipError_t launch_mfu_left<T>(int, int, const T*, const T*, const T*, T*, int, long, long, const double*, \
                                         const double*, const double*, int, int, int, int, hipStream_t);          \
  template hipError_t launch_mff_right<T>(int, int, const T*, const T*, const T*, T*, hipStream_t);                \
  template hipError_t launch_mfu_right<T>(int, int, const T*, const T*, const T*, T*, hipStream_t);
LK_MF_INST(double)
LK_MF_INST(float)
#undef LK_MF_INST

}  // namespace lk
