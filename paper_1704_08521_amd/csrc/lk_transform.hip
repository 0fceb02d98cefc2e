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

template hipError_t launch_tp_left<double>(int, int, int, const double*, const double*, double*, int, long, long,
                                           const double*, const double*, const double*, int, int, int, int,
                                           hipStream_t);
template hipError_t launch_tp_left<float>(int, int, int, const float*, const float*, float*, int, long, long,
                                          const double*, const double*, const double*, int, int, int, int,
                                          hipStream_t);
template hipError_t launch_tp_right<double>(int, int, int, const double*, const double*, double*, hipStream_t);
template hipError_t launch_tp_right<float>(int, int, int, const float*, const float*, float*, hipStream_t);

}  // namespace lk
