// Device kernels of the SIMPLE-evaluated Krylov vector (gfx950, wave64).
//
// Staggered layout, x fastest: u[k][j][i] (i = 0..nx), v[k][j][i] (j = 0..ny),
// w[k][j][i] (k = 0..nz), cells p[k][j][i].  Wall-normal faces are read as zero.
#include <hip/hip_runtime.h>

#include "lk_internal.h"

namespace lk {
namespace {

__device__ __forceinline__ double lerp(double a0, double a1, double t) {
  return (1.0 - t) * a0 + t * a1;
}

struct Idx {
  int nx, ny, nz;
  __device__ __forceinline__ size_t u(int k, int j, int i) const {
    return ((size_t)k * ny + j) * (nx + 1) + i;
  }
  __device__ __forceinline__ size_t v(int k, int j, int i) const {
    return ((size_t)k * (ny + 1) + j) * nx + i;
  }
  __device__ __forceinline__ size_t w(int k, int j, int i) const {
    return ((size_t)k * ny + j) * nx + i;
  }
  __device__ __forceinline__ size_t c(int k, int j, int i) const {
    return ((size_t)k * ny + j) * nx + i;
  }
};

// Loads that read wall-normal faces as zero.
struct Vel {
  const double* u;
  const double* v;
  const double* w;
  Idx I;
  __device__ __forceinline__ double U(int k, int j, int i) const {
    return (i == 0 || i == I.nx) ? 0.0 : u[I.u(k, j, i)];
  }
  __device__ __forceinline__ double V(int k, int j, int i) const {
    return (j == 0 || j == I.ny) ? 0.0 : v[I.v(k, j, i)];
  }
  __device__ __forceinline__ double W(int k, int j, int i) const {
    return (k == 0 || k == I.nz) ? 0.0 : w[I.w(k, j, i)];
  }
};

// ------------------------------------------------------------------ momentum
// x-momentum at the interior x-face (i, j, k), 1 <= i <= nx-1.
template <bool LID>
__device__ double mom_u(const GridDev& g, const Vel& A, const Vel& B, int i, int j, int k,
                        double rre, double s, double lid_u) {
  const int nx = g.x.n, ny = g.y.n, nz = g.z.n;
  const double bc = B.U(k, j, i);
  const double bxm = B.U(k, j, i - 1), bxp = B.U(k, j, i + 1);
  // Laplacian: normal (x) part, tangential y and z parts with wall fluxes
  double lap = ((bxp - bc) * g.x.rd[i] - (bc - bxm) * g.x.rd[i - 1]) * g.x.rdd[i];
  {
    const double fm = (j > 0) ? (bc - B.U(k, j - 1, i)) * g.y.rdd[j] : bc * g.y.rdd[0];
    const double fp = (j < ny - 1) ? (B.U(k, j + 1, i) - bc) * g.y.rdd[j + 1] : -bc * g.y.rdd[ny];
    lap += (fp - fm) * g.y.rd[j];
  }
  {
    const double top = LID ? lid_u : 0.0;
    const double fm = (k > 0) ? (bc - B.U(k - 1, j, i)) * g.z.rdd[k] : bc * g.z.rdd[0];
    const double fp = (k < nz - 1) ? (B.U(k + 1, j, i) - bc) * g.z.rdd[k + 1] : (top - bc) * g.z.rdd[nz];
    lap += (fp - fm) * g.z.rd[k];
  }
  // convection: normal flux at the centres i-1, i
  const double ac = A.U(k, j, i);
  const double am = 0.5 * (A.U(k, j, i - 1) + ac), ap = 0.5 * (ac + A.U(k, j, i + 1));
  const double bm = 0.5 * (bxm + bc), bp = 0.5 * (bc + bxp);
  double conv = 2.0 * (ap * bp - am * bm) * g.x.rdd[i];
  // y-flux on edges (xf[i], yf[jj]), jj = j, j+1
  const double tx = g.x.th[i];
  double e[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int jj = j + q;
    if (jj == 0 || jj == ny) {
      e[q] = 0.0;
    } else {
      const double ty = g.y.th[jj];
      const double av = lerp(A.V(k, jj, i - 1), A.V(k, jj, i), tx);
      const double bv = lerp(B.V(k, jj, i - 1), B.V(k, jj, i), tx);
      const double au = lerp(A.U(k, jj - 1, i), A.U(k, jj, i), ty);
      const double bu = lerp(B.U(k, jj - 1, i), B.U(k, jj, i), ty);
      e[q] = av * bu + bv * au;
    }
  }
  conv += (e[1] - e[0]) * g.y.rd[j];
  // z-flux on edges (xf[i], zf[kk]), kk = k, k+1
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int kk = k + q;
    if (kk == 0 || kk == nz) {
      e[q] = 0.0;
    } else {
      const double tz = g.z.th[kk];
      const double aw = lerp(A.W(kk, j, i - 1), A.W(kk, j, i), tx);
      const double bw = lerp(B.W(kk, j, i - 1), B.W(kk, j, i), tx);
      const double au = lerp(A.U(kk - 1, j, i), A.U(kk, j, i), tz);
      const double bu = lerp(B.U(kk - 1, j, i), B.U(kk, j, i), tz);
      e[q] = aw * bu + bw * au;
    }
  }
  conv += (e[1] - e[0]) * g.z.rd[k];
  (void)nx;
  return rre * lap - s * conv;
}

// y-momentum at the interior y-face (i, j, k), 1 <= j <= ny-1.
template <bool LID>
__device__ double mom_v(const GridDev& g, const Vel& A, const Vel& B, int i, int j, int k,
                        double rre, double s, double lid_v) {
  const int nx = g.x.n, ny = g.y.n, nz = g.z.n;
  const double bc = B.V(k, j, i);
  const double bym = B.V(k, j - 1, i), byp = B.V(k, j + 1, i);
  double lap = ((byp - bc) * g.y.rd[j] - (bc - bym) * g.y.rd[j - 1]) * g.y.rdd[j];
  {
    const double fm = (i > 0) ? (bc - B.V(k, j, i - 1)) * g.x.rdd[i] : bc * g.x.rdd[0];
    const double fp = (i < nx - 1) ? (B.V(k, j, i + 1) - bc) * g.x.rdd[i + 1] : -bc * g.x.rdd[nx];
    lap += (fp - fm) * g.x.rd[i];
  }
  {
    const double top = LID ? lid_v : 0.0;
    const double fm = (k > 0) ? (bc - B.V(k - 1, j, i)) * g.z.rdd[k] : bc * g.z.rdd[0];
    const double fp = (k < nz - 1) ? (B.V(k + 1, j, i) - bc) * g.z.rdd[k + 1] : (top - bc) * g.z.rdd[nz];
    lap += (fp - fm) * g.z.rd[k];
  }
  const double ty = g.y.th[j];
  double e[2];
  // x-flux on edges (xf[ii], yf[j]), ii = i, i+1
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int ii = i + q;
    if (ii == 0 || ii == nx) {
      e[q] = 0.0;
    } else {
      const double tx = g.x.th[ii];
      const double au = lerp(A.U(k, j - 1, ii), A.U(k, j, ii), ty);
      const double bu = lerp(B.U(k, j - 1, ii), B.U(k, j, ii), ty);
      const double av = lerp(A.V(k, j, ii - 1), A.V(k, j, ii), tx);
      const double bv = lerp(B.V(k, j, ii - 1), B.V(k, j, ii), tx);
      e[q] = au * bv + bu * av;
    }
  }
  double conv = (e[1] - e[0]) * g.x.rd[i];
  // normal flux at the centres j-1, j
  const double ac = A.V(k, j, i);
  const double am = 0.5 * (A.V(k, j - 1, i) + ac), ap = 0.5 * (ac + A.V(k, j + 1, i));
  const double bm = 0.5 * (bym + bc), bp = 0.5 * (bc + byp);
  conv += 2.0 * (ap * bp - am * bm) * g.y.rdd[j];
  // z-flux on edges (yf[j], zf[kk])
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int kk = k + q;
    if (kk == 0 || kk == nz) {
      e[q] = 0.0;
    } else {
      const double tz = g.z.th[kk];
      const double aw = lerp(A.W(kk, j - 1, i), A.W(kk, j, i), ty);
      const double bw = lerp(B.W(kk, j - 1, i), B.W(kk, j, i), ty);
      const double av = lerp(A.V(kk - 1, j, i), A.V(kk, j, i), tz);
      const double bv = lerp(B.V(kk - 1, j, i), B.V(kk, j, i), tz);
      e[q] = aw * bv + bw * av;
    }
  }
  conv += (e[1] - e[0]) * g.z.rd[k];
  return rre * lap - s * conv;
}

// z-momentum at the interior z-face (i, j, k), 1 <= k <= nz-1.
__device__ double mom_w(const GridDev& g, const Vel& A, const Vel& B, int i, int j, int k,
                        double rre, double s) {
  const int nx = g.x.n, ny = g.y.n, nz = g.z.n;
  const double bc = B.W(k, j, i);
  const double bzm = B.W(k - 1, j, i), bzp = B.W(k + 1, j, i);
  double lap = ((bzp - bc) * g.z.rd[k] - (bc - bzm) * g.z.rd[k - 1]) * g.z.rdd[k];
  {
    const double fm = (i > 0) ? (bc - B.W(k, j, i - 1)) * g.x.rdd[i] : bc * g.x.rdd[0];
    const double fp = (i < nx - 1) ? (B.W(k, j, i + 1) - bc) * g.x.rdd[i + 1] : -bc * g.x.rdd[nx];
    lap += (fp - fm) * g.x.rd[i];
  }
  {
    const double fm = (j > 0) ? (bc - B.W(k, j - 1, i)) * g.y.rdd[j] : bc * g.y.rdd[0];
    const double fp = (j < ny - 1) ? (B.W(k, j + 1, i) - bc) * g.y.rdd[j + 1] : -bc * g.y.rdd[ny];
    lap += (fp - fm) * g.y.rd[j];
  }
  const double tz = g.z.th[k];
  double e[2];
  // x-flux on edges (xf[ii], zf[k])
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int ii = i + q;
    if (ii == 0 || ii == nx) {
      e[q] = 0.0;
    } else {
      const double tx = g.x.th[ii];
      const double au = lerp(A.U(k - 1, j, ii), A.U(k, j, ii), tz);
      const double bu = lerp(B.U(k - 1, j, ii), B.U(k, j, ii), tz);
      const double aw = lerp(A.W(k, j, ii - 1), A.W(k, j, ii), tx);
      const double bw = lerp(B.W(k, j, ii - 1), B.W(k, j, ii), tx);
      e[q] = au * bw + bu * aw;
    }
  }
  double conv = (e[1] - e[0]) * g.x.rd[i];
  // y-flux on edges (yf[jj], zf[k])
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int jj = j + q;
    if (jj == 0 || jj == ny) {
      e[q] = 0.0;
    } else {
      const double ty = g.y.th[jj];
      const double av = lerp(A.V(k - 1, jj, i), A.V(k, jj, i), tz);
      const double bv = lerp(B.V(k - 1, jj, i), B.V(k, jj, i), tz);
      const double aw = lerp(A.W(k, jj - 1, i), A.W(k, jj, i), ty);
      const double bw = lerp(B.W(k, jj - 1, i), B.W(k, jj, i), ty);
      e[q] = av * bw + bv * aw;
    }
  }
  conv += (e[1] - e[0]) * g.y.rd[j];
  // normal flux at the centres k-1, k
  const double ac = A.W(k, j, i);
  const double am = 0.5 * (A.W(k - 1, j, i) + ac), ap = 0.5 * (ac + A.W(k + 1, j, i));
  const double bm = 0.5 * (bzm + bc), bp = 0.5 * (bc + bzp);
  conv += 2.0 * (ap * bp - am * bm) * g.z.rdd[k];
  return rre * lap - s * conv;
}

template <bool LID>
__global__ void __launch_bounds__(256) k_momentum(GridDev g, Vel A, Vel B, double* __restrict__ out_u,
                                                  double* __restrict__ out_v, double* __restrict__ out_w,
                                                  double rre, double s, double lid_u, double lid_v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = blockIdx.z;
  const int nx = g.x.n, ny = g.y.n, nz = g.z.n;
  if (i > nx || j > ny || k > nz) return;
  const Idx& I = A.I;
  if (j < ny && k < nz) {
    out_u[I.u(k, j, i)] = (i == 0 || i == nx) ? 0.0 : mom_u<LID>(g, A, B, i, j, k, rre, s, lid_u);
  }
  if (i < nx && k < nz) {
    out_v[I.v(k, j, i)] = (j == 0 || j == ny) ? 0.0 : mom_v<LID>(g, A, B, i, j, k, rre, s, lid_v);
  }
  if (i < nx && j < ny) {
    out_w[I.w(k, j, i)] = (k == 0 || k == nz) ? 0.0 : mom_w(g, A, B, i, j, k, rre, s);
  }
}

// ---------------------------------------------------------- block reductions
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
  return x;
}

// Sum of one value per thread over a block of kReduceBlock threads; result in thread 0.
__device__ double block_sum(double x) {
  __shared__ double red[kReduceBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  x = wave_sum(x);
  if (lane == 0) red[wid] = x;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
    for (int q = 0; q < kReduceBlock / 64; ++q) t += red[q];
  }
  return t;
}

// ---------------------------------------------------------------- divergence
__global__ void __launch_bounds__(kReduceBlock) k_divergence(GridDev g, Vel V, double* __restrict__ r,
                                                             double* __restrict__ partials) {
  const int nx = g.x.n, ny = g.y.n, nz = g.z.n;
  const size_t ncell = (size_t)nx * ny * nz;
  const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double contrib = 0.0;
  if (c < ncell) {
    const int i = (int)(c % nx);
    const int j = (int)((c / nx) % ny);
    const int k = (int)(c / ((size_t)nx * ny));
    const double dv = (V.U(k, j, i + 1) - V.U(k, j, i)) * g.x.rd[i] +
                      (V.V(k, j + 1, i) - V.V(k, j, i)) * g.y.rd[j] +
                      (V.W(k + 1, j, i) - V.W(k, j, i)) * g.z.rd[k];
    r[c] = dv;
    contrib = g.x.d[i] * g.y.d[j] * g.z.d[k] * dv * dv;
  }
  if (partials) {
    const double t = block_sum(contrib);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
  }
}

// ---------------------------------------------------------------- correction
__global__ void __launch_bounds__(256) k_correct(GridDev g, const double* __restrict__ w,
                                                 const double* __restrict__ phi, double* __restrict__ v,
                                                 double* __restrict__ p, int accumulate) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = blockIdx.z;
  const int nx = g.x.n, ny = g.y.n, nz = g.z.n;
  if (i > nx || j > ny || k > nz) return;
  const Idx I{nx, ny, nz};
  const size_t nu = (size_t)(nx + 1) * ny * nz, nv = (size_t)nx * (ny + 1) * nz;
  const double* src = accumulate ? v : w;
  if (j < ny && k < nz) {
    const size_t q = I.u(k, j, i);
    double val = 0.0;
    if (i > 0 && i < nx) val = src[q] - (phi[I.c(k, j, i)] - phi[I.c(k, j, i - 1)]) * g.x.rdd[i];
    v[q] = val;
  }
  if (i < nx && k < nz) {
    const size_t q = nu + I.v(k, j, i);
    double val = 0.0;
    if (j > 0 && j < ny) val = src[q] - (phi[I.c(k, j, i)] - phi[I.c(k, j - 1, i)]) * g.y.rdd[j];
    v[q] = val;
  }
  if (i < nx && j < ny) {
    const size_t q = nu + nv + I.w(k, j, i);
    double val = 0.0;
    if (k > 0 && k < nz) val = src[q] - (phi[I.c(k, j, i)] - phi[I.c(k - 1, j, i)]) * g.z.rdd[k];
    v[q] = val;
    if (p && k < nz) {
      const size_t c = I.c(k, j, i);
      p[c] = accumulate ? p[c] + phi[c] : phi[c];
    }
  }
}

// ------------------------------------------------------------- misc vectors
__global__ void __launch_bounds__(1024) k_sum(const double* __restrict__ partials, int n,
                                              double* __restrict__ out) {
  // fixed order: thread t sums t, t+1024, ...; then a fixed tree
  __shared__ double sh[1024];
  double t = 0.0;
  for (int q = threadIdx.x; q < n; q += 1024) t += partials[q];
  sh[threadIdx.x] = t;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

__global__ void __launch_bounds__(kReduceBlock) k_dot(const double* __restrict__ a,
                                                      const double* __restrict__ b, size_t n,
                                                      double* __restrict__ partials) {
  double t = 0.0;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) t += a[q] * b[q];
  t = block_sum(t);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ void k_axpy(size_t n, double a, const double* __restrict__ x, double* __restrict__ y) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) y[q] += a * x[q];
}

__global__ void k_scale(size_t n, double a, double* __restrict__ x) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) x[q] *= a;
}

__global__ void k_d2f(size_t n, const double* __restrict__ in, float* __restrict__ out) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) out[q] = (float)in[q];
}

__global__ void k_f2d(size_t n, const float* __restrict__ in, double* __restrict__ out, int acc) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) out[q] = acc ? out[q] + (double)in[q] : (double)in[q];
}

// SplitMix64 in counter mode (Steele, Lea & Flood 2014): element q of stream
// `seed` is mix(seed + (q + 1) * 0x9E3779B97F4A7C15); uniform [-1, 1) from the
// top 53 bits.
__global__ void k_uniform(double* __restrict__ x, size_t n, uint64_t seed) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  uint64_t z = seed + (uint64_t)(q + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  const double u = (double)(z >> 11) * 0x1.0p-53;
  x[q] = 2.0 * u - 1.0;
}

__global__ void k_zero_walls(double* __restrict__ vel, int nx, int ny, int nz) {
  // one thread per (a, b) position on each of the six wall planes
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  const int which = blockIdx.z;  // 0: u walls, 1: v walls, 2: w walls
  const Idx I{nx, ny, nz};
  const size_t nu = (size_t)(nx + 1) * ny * nz, nv = (size_t)nx * (ny + 1) * nz;
  if (which == 0 && a < ny && b < nz) {
    vel[I.u(b, a, 0)] = 0.0;
    vel[I.u(b, a, nx)] = 0.0;
  } else if (which == 1 && a < nx && b < nz) {
    vel[nu + I.v(b, 0, a)] = 0.0;
    vel[nu + I.v(b, ny, a)] = 0.0;
  } else if (which == 2 && a < nx && b < ny) {
    vel[nu + nv + I.w(0, b, a)] = 0.0;
    vel[nu + nv + I.w(nz, b, a)] = 0.0;
  }
}

// --------------------------------------------------- tensor-product transforms
// Batched row-major GEMM C = A B on vector FMA units with LDS staging.  Thread
// (tx, ty) owns rows ty + RM*q and columns tx + RN*q (q < TM, TN) of the tile, so
// that LDS reads are broadcasts (A) or consecutive (B) and the stores coalesce.
template <typename T, int BM, int BN, int BK, int TM, int TN>
__global__ void __launch_bounds__((BM / TM) * (BN / TN))
    k_gemm(int M, int N, int K, const T* __restrict__ A, long lda, long sA, const T* __restrict__ B,
           long ldb, long sB, T* __restrict__ C, long ldc, long sC) {
  constexpr int RM = BM / TM, RN = BN / TN, NT = RM * RN;
  __shared__ T As[BK][BM + 1];
  __shared__ T Bs[BK][BN];
  const int tid = threadIdx.x;
  const int tx = tid % RN, ty = tid / RN;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const long b = blockIdx.z;
  A += b * sA;
  B += b * sB;
  C += b * sC;
  T acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int c = 0; c < TN; ++c) acc[a][c] = T(0);
  for (int k0 = 0; k0 < K; k0 += BK) {
    // A tile BM x BK, k contiguous in memory
    for (int e = tid; e < BM * BK; e += NT) {
      const int mm = e / BK, kk = e % BK;
      const int gm = m0 + mm, gk = k0 + kk;
      As[kk][mm] = (gm < M && gk < K) ? A[(long)gm * lda + gk] : T(0);
    }
    // B tile BK x BN, n contiguous
    for (int e = tid; e < BK * BN; e += NT) {
      const int kk = e / BN, nn = e % BN;
      const int gk = k0 + kk, gn = n0 + nn;
      Bs[kk][nn] = (gk < K && gn < N) ? B[(long)gk * ldb + gn] : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; ++kk) {
      T av[TM], bv[TN];
#pragma unroll
      for (int a = 0; a < TM; ++a) av[a] = As[kk][ty + RM * a];
#pragma unroll
      for (int c = 0; c < TN; ++c) bv[c] = Bs[kk][tx + RN * c];
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int c = 0; c < TN; ++c) acc[a][c] = fma(av[a], bv[c], acc[a][c]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < TM; ++a) {
    const int gm = m0 + ty + RM * a;
    if (gm >= M) continue;
#pragma unroll
    for (int c = 0; c < TN; ++c) {
      const int gn = n0 + tx + RN * c;
      if (gn < N) C[(long)gm * ldc + gn] = acc[a][c];
    }
  }
}

template <typename T>
__global__ void k_eigscale(T* __restrict__ x, const double* __restrict__ lx, const double* __restrict__ ly,
                           const double* __restrict__ lz, int nx, int ny, int nz, int zi, int zj, int zk) {
  const size_t n = (size_t)nx * ny * nz;
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int i = (int)(q % nx), j = (int)((q / nx) % ny), k = (int)(q / ((size_t)nx * ny));
  if (i == zi && j == zj && k == zk) {
    x[q] = T(0);
  } else {
    x[q] = (T)((double)x[q] / (lx[i] + ly[j] + lz[k]));
  }
}

inline unsigned blocks_for(size_t n, unsigned bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

// ==================================================================== launchers
hipError_t launch_momentum(const GridDev& g, const double* a, const double* b, double* out, double rre,
                           double s, bool lid, double lid_u, double lid_v, hipStream_t st) {
  const int nx = g.x.n, ny = g.y.n, nz = g.z.n;
  const VelLayout L = vel_layout(nx, ny, nz);
  const Idx I{nx, ny, nz};
  Vel A{a, a + L.ov(), a + L.ow(), I};
  Vel B{b, b + L.ov(), b + L.ow(), I};
  dim3 block(64, 4, 1);
  dim3 grid(blocks_for(nx + 1, 64), blocks_for(ny + 1, 4), nz + 1);
  if (lid)
    hipLaunchKernelGGL(k_momentum<true>, grid, block, 0, st, g, A, B, out, out + L.ov(), out + L.ow(), rre,
                       s, lid_u, lid_v);
  else
    hipLaunchKernelGGL(k_momentum<false>, grid, block, 0, st, g, A, B, out, out + L.ov(), out + L.ow(), rre,
                       s, 0.0, 0.0);
  return hipGetLastError();
}

hipError_t launch_divergence(const GridDev& g, const double* v, double* r, double* partials, int* nparts,
                             hipStream_t st) {
  const int nx = g.x.n, ny = g.y.n, nz = g.z.n;
  const VelLayout L = vel_layout(nx, ny, nz);
  Vel V{v, v + L.ov(), v + L.ow(), Idx{nx, ny, nz}};
  const size_t ncell = (size_t)nx * ny * nz;
  const unsigned nb = blocks_for(ncell, kReduceBlock);
  if (nparts) *nparts = (int)nb;
  hipLaunchKernelGGL(k_divergence, dim3(nb), dim3(kReduceBlock), 0, st, g, V, r, partials);
  return hipGetLastError();
}

hipError_t launch_correct(const GridDev& g, const double* w, const double* phi, double* v, double* p,
                          bool accumulate, hipStream_t st) {
  const int nx = g.x.n, ny = g.y.n, nz = g.z.n;
  dim3 block(64, 4, 1);
  dim3 grid(blocks_for(nx + 1, 64), blocks_for(ny + 1, 4), nz + 1);
  hipLaunchKernelGGL(k_correct, grid, block, 0, st, g, w, phi, v, p, accumulate ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_sum(const double* partials, int n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(1024), 0, st, partials, n, out);
  return hipGetLastError();
}

hipError_t launch_dot_partials(const double* a, const double* b, size_t n, double* partials, int* nparts,
                               hipStream_t st) {
  unsigned nb = blocks_for(n, kReduceBlock);
  if (nb > 4096) nb = 4096;
  if (nparts) *nparts = (int)nb;
  hipLaunchKernelGGL(k_dot, dim3(nb), dim3(kReduceBlock), 0, st, a, b, n, partials);
  return hipGetLastError();
}

hipError_t launch_axpy(size_t n, double a, const double* x, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_axpy, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, a, x, y);
  return hipGetLastError();
}

hipError_t launch_scale(size_t n, double a, double* x, hipStream_t st) {
  hipLaunchKernelGGL(k_scale, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, a, x);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gemm(int M, int N, int K, const T* A, long lda, long sA, const T* B, long ldb, long sB, T* C,
                       long ldc, long sC, int batch, hipStream_t st) {
  constexpr int BM = 64, BN = 64, BK = 16, TM = 4, TN = 4;
  dim3 grid(blocks_for(N, BN), blocks_for(M, BM), batch);
  hipLaunchKernelGGL((k_gemm<T, BM, BN, BK, TM, TN>), grid, dim3((BM / TM) * (BN / TN)), 0, st, M, N, K, A,
                     lda, sA, B, ldb, sB, C, ldc, sC);
  return hipGetLastError();
}
template hipError_t launch_gemm<double>(int, int, int, const double*, long, long, const double*, long, long,
                                        double*, long, long, int, hipStream_t);
template hipError_t launch_gemm<float>(int, int, int, const float*, long, long, const float*, long, long,
                                       float*, long, long, int, hipStream_t);

template <typename T>
hipError_t launch_eigscale(T* x, const double* lx, const double* ly, const double* lz, int nx, int ny, int nz,
                           int zi, int zj, int zk, hipStream_t st) {
  const size_t n = (size_t)nx * ny * nz;
  hipLaunchKernelGGL(k_eigscale<T>, dim3(blocks_for(n, 256)), dim3(256), 0, st, x, lx, ly, lz, nx, ny, nz, zi,
                     zj, zk);
  return hipGetLastError();
}
template hipError_t launch_eigscale<double>(double*, const double*, const double*, const double*, int, int, int,
                                            int, int, int, hipStream_t);
template hipError_t launch_eigscale<float>(float*, const double*, const double*, const double*, int, int, int,
                                           int, int, int, hipStream_t);

hipError_t launch_d2f(size_t n, const double* in, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_d2f, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, in, out);
  return hipGetLastError();
}

hipError_t launch_f2d(size_t n, const float* in, double* out, bool accumulate, hipStream_t st) {
  hipLaunchKernelGGL(k_f2d, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, in, out, accumulate ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_uniform(double* x, size_t n, uint64_t seed, hipStream_t st) {
  hipLaunchKernelGGL(k_uniform, dim3(blocks_for(n, 256)), dim3(256), 0, st, x, n, seed);
  return hipGetLastError();
}

hipError_t launch_zero_walls(double* vel, int nx, int ny, int nz, hipStream_t st) {
  const int amax = (nx > ny ? nx : ny) + 1;
  const int bmax = (ny > nz ? ny : nz) + 1;
  dim3 grid(blocks_for(amax, 64), bmax, 3);
  hipLaunchKernelGGL(k_zero_walls, grid, dim3(64), 0, st, vel, nx, ny, nz);
  return hipGetLastError();
}

}  // namespace lk
