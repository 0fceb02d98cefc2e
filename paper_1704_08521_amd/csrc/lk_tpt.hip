// Tridiagonal solves along x in (y, z) mode space: the x step of the pressure-correction
// Poisson solve by the TPT route of Section 3 (mode transforms in two directions, a
// tridiagonal solve in the third).  For every x-line (k, j) of the transformed field,
// (L_x + ly[j] + lz[k]) phi = rhs, with L_x = D_x G_x on the cells of the line (zero flux
// through the walls), by parallel cyclic reduction in LDS, one block per line.  The line
// whose shift is zero (the zero modes of y and z) is singular: its first equation is
// replaced by phi_0 = 0 and the solution is re-centred to zero d-weighted mean, which
// sets the constant mode to zero as the transform route does.
#include <hip/hip_runtime.h>

#include "lk_device.h"
#include "lk_internal.h"

namespace lk {
namespace {

template <int B>
__device__ __forceinline__ double block_total(double x, double* red) {
  // every thread gets the block sum (B threads, B / 64 waves)
  x = wave_sum(x);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = x;
  __syncthreads();
  double t = 0.0;
  for (int q = 0; q < B / 64; ++q) t += red[q];
  __syncthreads();
  return t;
}

// 1 / a to FP64 accuracy: the hardware reciprocal refined by two Newton steps
__device__ __forceinline__ double rcp64(double a) {
  double y = __builtin_amdgcn_rcp(a);
  double e = fma(-a, y, 1.0);
  y = fma(e, y, y);
  e = fma(-a, y, 1.0);
  return fma(e, y, y);
}

template <int B>
__global__ void __launch_bounds__(B) k_tridiag_x(const double* __restrict__ rd, const double* __restrict__ rdd,
                                                 const double* __restrict__ dx, int n, int ny,
                                                 const double* __restrict__ ly, const double* __restrict__ lz,
                                                 int zj, int zk, const double* __restrict__ in,
                                                 double* __restrict__ out) {
  __shared__ double sa[B], srb[B], sc[B], sd[B];  // srb: reciprocals of the diagonal
  __shared__ double red[B / 64];
  const long line = blockIdx.x;  // k * ny + j
  const int j = (int)(line % ny), k = (int)(line / ny);
  const int i = threadIdx.x;
  const double shift = ly[j] + lz[k];
  const bool sing = (j == zj) && (k == zk);
  // rows i >= n are the identity with a zero right side, coupled to nothing
  double a = 0.0, b = 1.0, c = 0.0, d = 0.0;
  if (i < n) {
    const double lo = (i > 0) ? rdd[i] * rd[i] : 0.0;
    const double up = (i + 1 < n) ? rdd[i + 1] * rd[i] : 0.0;
    a = lo;
    c = up;
    b = shift - (lo + up);
    d = in[(size_t)line * n + i];
    if (sing && i == 0) {
      a = 0.0;
      b = 1.0;
      c = 0.0;
      d = 0.0;
    }
  }
  // after the steps with strides 1, 2, 4, ... < n every row couples only to rows at least
  // n away: all rows are decoupled.  A row's diagonal enters its neighbours only through
  // its reciprocal.
  for (int s = 1; s < n; s <<= 1) {
    sa[i] = a;
    srb[i] = rcp64(b);
    sc[i] = c;
    sd[i] = d;
    __syncthreads();
    const int im = i - s, ip = i + s;
    double an = 0.0, cn = 0.0, bn = b, dn = d;
    if (im >= 0) {
      const double k1 = a * srb[im];
      an = -sa[im] * k1;
      bn -= sc[im] * k1;
      dn -= sd[im] * k1;
    }
    if (ip < B) {
      const double k2 = c * srb[ip];
      cn = -sc[ip] * k2;
      bn -= sa[ip] * k2;
      dn -= sd[ip] * k2;
    }
    __syncthreads();
    a = an;
    b = bn;
    c = cn;
    d = dn;
  }
  double x = d / b;
  if (sing) {  // block-uniform branch
    const double w = (i < n) ? dx[i] : 0.0;
    const double mean = block_total<B>(w * x, red) / block_total<B>(w, red);
    x -= mean;
  }
  if (i < n) out[(size_t)line * n + i] = x;
}

}  // namespace

int tridiag_x_max() { return 1024; }

hipError_t launch_tridiag_x(const GridDev& g, const double* ly, const double* lz, int zj, int zk, const double* in,
                            double* out, hipStream_t st) {
  const int n = g.x.n, ny = g.y.n, nz = g.z.n;
  const unsigned lines = (unsigned)((long)ny * nz);
  if (n <= 64)
    hipLaunchKernelGGL(k_tridiag_x<64>, dim3(lines), dim3(64), 0, st, g.x.rd, g.x.rdd, g.x.d, n, ny, ly, lz, zj, zk, in,
                       out);
  else if (n <= 128)
    hipLaunchKernelGGL(k_tridiag_x<128>, dim3(lines), dim3(128), 0, st, g.x.rd, g.x.rdd, g.x.d, n, ny, ly, lz, zj, zk,
                       in, out);
  else if (n <= 256)
    hipLaunchKernelGGL(k_tridiag_x<256>, dim3(lines), dim3(256), 0, st, g.x.rd, g.x.rdd, g.x.d, n, ny, ly, lz, zj, zk,
                       in, out);
  else if (n <= 512)
    hipLaunchKernelGGL(k_tridiag_x<512>, dim3(lines), dim3(512), 0, st, g.x.rd, g.x.rdd, g.x.d, n, ny, ly, lz, zj, zk,
                       in, out);
  else if (n <= 1024)
    hipLaunchKernelGGL(k_tridiag_x<1024>, dim3(lines), dim3(1024), 0, st, g.x.rd, g.x.rdd, g.x.d, n, ny, ly, lz, zj, zk,
                       in, out);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace lk
