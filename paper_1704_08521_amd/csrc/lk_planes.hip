// Divergence-free projections onto the coordinate planes and their vector potentials
// (Section 4, eqs. 11-17).  Projection P keeps two velocity components and removes the
// gradient of a plane pressure phi that solves the two-dimensional Poisson problem
// D2 G2 phi = D2 b in every plane normal to the third axis:
//   P = 1: (u, w), planes y = const;  P = 2: (v, w), planes x = const;
//   P = 3: (u, v), planes z = const.
// The plane solve itself reuses the per-axis transforms of the 3D solver (only the two
// in-plane axes are transformed); the kernels here are the right-hand side, the
// division by the in-plane eigenvalue sums, the correction and the potentials.
#include <hip/hip_runtime.h>

#include "lk_device.h"
#include "lk_internal.h"

namespace lk {
namespace {

constexpr int kPlaneBlock = 256;

template <int P>
struct Keep {
  static constexpr bool u = P != 2, v = P != 1, w = P != 3;
};

// r = D2 b, one thread per cell (grid: x tiles of the row, y = j, z = k): b is the input
// with the dropped component and the wall-normal faces set to zero.
template <int P>
__global__ void __launch_bounds__(kPlaneBlock) k_plane_rhs(GridDev g, const double* __restrict__ vel,
                                                            double* __restrict__ r) {
  const int nx = g.x.n, ny = g.y.n, nz = g.z.n;
  const int i = blockIdx.x * kPlaneBlock + threadIdx.x, j = blockIdx.y, k = blockIdx.z;
  if (i >= nx) return;
  const Idx I{nx, ny, nz};
  const size_t nu = (size_t)(nx + 1) * ny * nz, nv = (size_t)nx * (ny + 1) * nz;
  double s = 0.0;
  if (Keep<P>::u) {
    const double ue = (i + 1 < nx) ? vel[I.u(k, j, i + 1)] : 0.0, uw = (i > 0) ? vel[I.u(k, j, i)] : 0.0;
    s += (ue - uw) * g.x.rd[i];
  }
  if (Keep<P>::v) {
    const double vn = (j + 1 < ny) ? vel[nu + I.v(k, j + 1, i)] : 0.0, vs = (j > 0) ? vel[nu + I.v(k, j, i)] : 0.0;
    s += (vn - vs) * g.y.rd[j];
  }
  if (Keep<P>::w) {
    const double wt = (k + 1 < nz) ? vel[nu + nv + I.w(k + 1, j, i)] : 0.0;
    const double wb = (k > 0) ? vel[nu + nv + I.w(k, j, i)] : 0.0;
    s += (wt - wb) * g.z.rd[k];
  }
  r[I.c(k, j, i)] = s;
}

// Mode space: t /= (lx[i] + ly[j] + lz[k]) over the two in-plane axes (the normal
// axis's array is null and contributes nothing); the modes whose in-plane indices are
// both zero modes (one per plane: the plane's constant) are set to zero.  A negative
// zero-mode index stands for the normal axis, where every index matches.  Grid as the
// right side.
__global__ void __launch_bounds__(kPlaneBlock) k_plane_scale(double* __restrict__ t, int nx, int ny,
                                                              const double* __restrict__ lx,
                                                              const double* __restrict__ ly,
                                                              const double* __restrict__ lz, int zx, int zy, int zz) {
  const int i = blockIdx.x * kPlaneBlock + threadIdx.x, j = blockIdx.y, k = blockIdx.z;
  if (i >= nx) return;
  const size_t q = ((size_t)k * ny + j) * nx + i;
  const double lam = (lx ? lx[i] : 0.0) + (ly ? ly[j] : 0.0) + (lz ? lz[k] : 0.0);
  const bool zero = (zx < 0 || i == zx) && (zy < 0 || j == zy) && (zz < 0 || k == zz);
  t[q] = zero ? 0.0 : t[q] / lam;
}

// out = b - G2 phi on the interior faces of the kept components, zero on the walls and
// for the dropped component.  One thread per face position (i, j, k), i <= nx, j <= ny,
// k <= nz, writing the u, v and w faces that exist there.
template <int P>
__global__ void __launch_bounds__(kPlaneBlock) k_plane_correct(GridDev g, const double* __restrict__ vel,
                                                                const double* __restrict__ phi,
                                                                double* __restrict__ out) {
  const int nx = g.x.n, ny = g.y.n, nz = g.z.n;
  const int i = blockIdx.x * kPlaneBlock + threadIdx.x, j = blockIdx.y, k = blockIdx.z;
  if (i > nx) return;
  const Idx I{nx, ny, nz};
  const size_t nu = (size_t)(nx + 1) * ny * nz, nv = (size_t)nx * (ny + 1) * nz;
  if (j < ny && k < nz) {
    const size_t q = I.u(k, j, i);
    double val = 0.0;
    if (Keep<P>::u && i > 0 && i < nx) val = vel[q] - (phi[I.c(k, j, i)] - phi[I.c(k, j, i - 1)]) * g.x.rdd[i];
    out[q] = val;
  }
  if (i < nx && k < nz) {
    const size_t q = nu + I.v(k, j, i);
    double val = 0.0;
    if (Keep<P>::v && j > 0 && j < ny) val = vel[q] - (phi[I.c(k, j, i)] - phi[I.c(k, j - 1, i)]) * g.y.rdd[j];
    out[q] = val;
  }
  if (i < nx && j < ny) {
    const size_t q = nu + nv + I.w(k, j, i);
    double val = 0.0;
    if (Keep<P>::w && k > 0 && k < nz) val = vel[q] - (phi[I.c(k, j, i)] - phi[I.c(k - 1, j, i)]) * g.z.rdd[k];
    out[q] = val;
  }
}

// Row prefix sums for the potentials of P = 1 and P = 3: one wave per row of n source
// values src[row][i]; psi[row][0] = 0 and psi[row][i + 1] = psi[row][i] + sgn d[i] src[row][i].
// The wave scans 64 values at a time (shuffle scan) and carries the running total.
__global__ void __launch_bounds__(kPlaneBlock) k_row_scan(const double* __restrict__ src, const double* __restrict__ d,
                                                           double sgn, int n, long rows, double* __restrict__ psi) {
  const int lane = (int)(threadIdx.x % 64);
  const long row = (long)blockIdx.x * (kPlaneBlock / 64) + (long)(threadIdx.x / 64);
  if (row >= rows) return;  // uniform per wave
  const double* s = src + (size_t)row * n;
  double* o = psi + (size_t)row * (n + 1);
  if (lane == 0) o[0] = 0.0;
  double carry = 0.0;
  for (int base = 0; base < n; base += 64) {
    const int i = base + lane;
    double x = (i < n) ? sgn * d[i] * s[i] : 0.0;
    for (int off = 1; off < 64; off <<= 1) {
      const double y = __shfl_up(x, off);
      if (lane >= off) x += y;
    }
    x += carry;
    if (i < n) o[i + 1] = x;
    carry = __shfl(x, 63);
  }
}

// Column prefix sums for the potential of P = 2:
// psi[k][0][i] = 0, psi[k][j + 1][i] = psi[k][j][i] - dy[j] w[k][j][i].
// Block: 64 columns i x kColSeg segments of the j range (one wave per segment); each
// wave sums its segment, the segment offsets go through LDS, then each wave writes its
// running sums.  Loads are batched kColBatch at a time, each from an in-range row (the
// segment's last for the batch's surplus), so a batch's loads are in flight together.
constexpr int kColSeg = 8, kColBatch = 8;

__global__ void __launch_bounds__(64 * kColSeg) k_col_scan(const double* __restrict__ w,
                                                            const double* __restrict__ dy, int nx, int ny,
                                                            double* __restrict__ psi) {
  __shared__ double part[kColSeg][64];
  const int lane = (int)(threadIdx.x % 64), seg = (int)(threadIdx.x / 64);
  const int i = blockIdx.x * 64 + lane, k = blockIdx.y;
  const int len = (ny + kColSeg - 1) / kColSeg, j0 = min(seg * len, ny), j1 = min(j0 + len, ny);
  const bool col = i < nx;
  const double* src = w + (size_t)k * ny * nx + (col ? i : 0);
  double* dst = psi + (size_t)k * (ny + 1) * nx + (col ? i : 0);
  double s = 0.0;
  for (int jb = j0; jb < j1; jb += kColBatch) {
    double x[kColBatch];
#pragma unroll
    for (int t = 0; t < kColBatch; ++t) {
      // in range, and masked by a product rather than a select (a select of a loaded value
      // is turned back into a branch around the load): the batch's loads all go out
      // before the sum waits
      const int jr = min(jb + t, j1 - 1);
      x[t] = dy[jr] * src[(size_t)jr * nx] * ((col && jb + t < j1) ? 1.0 : 0.0);
    }
#pragma unroll
    for (int t = 0; t < kColBatch; ++t) s += x[t];
  }
  part[seg][lane] = s;
  __syncthreads();
  double acc = 0.0;
  for (int t = 0; t < seg; ++t) acc += part[t][lane];
  if (!col) return;
  if (seg == 0) dst[0] = 0.0;
  for (int jb = j0; jb < j1; jb += kColBatch) {
    double x[kColBatch];
#pragma unroll
    for (int t = 0; t < kColBatch; ++t) {
      const int jr = min(jb + t, j1 - 1);
      x[t] = dy[jr] * src[(size_t)jr * nx] * ((jb + t < j1) ? 1.0 : 0.0);
    }
#pragma unroll
    for (int t = 0; t < kColBatch; ++t) {
      acc += x[t];
      if (jb + t < j1) dst[(size_t)(jb + t + 1) * nx] = -acc;
    }
  }
}

}  // namespace

hipError_t launch_plane_rhs(const GridDev& g, int P, const double* vel, double* r, hipStream_t st) {
  const dim3 grid(blocks_for(g.x.n, kPlaneBlock), g.y.n, g.z.n), block(kPlaneBlock);
  if (P == 1)
    hipLaunchKernelGGL(k_plane_rhs<1>, grid, block, 0, st, g, vel, r);
  else if (P == 2)
    hipLaunchKernelGGL(k_plane_rhs<2>, grid, block, 0, st, g, vel, r);
  else
    hipLaunchKernelGGL(k_plane_rhs<3>, grid, block, 0, st, g, vel, r);
  return hipGetLastError();
}

hipError_t launch_plane_scale(double* t, int nx, int ny, int nz, const double* lx, const double* ly, const double* lz,
                              int zx, int zy, int zz, hipStream_t st) {
  hipLaunchKernelGGL(k_plane_scale, dim3(blocks_for(nx, kPlaneBlock), ny, nz), dim3(kPlaneBlock), 0, st, t, nx, ny, lx,
                     ly, lz, zx, zy, zz);
  return hipGetLastError();
}

hipError_t launch_plane_correct(const GridDev& g, int P, const double* vel, const double* phi, double* out,
                                hipStream_t st) {
  const dim3 grid(blocks_for(g.x.n + 1, kPlaneBlock), g.y.n + 1, g.z.n + 1), block(kPlaneBlock);
  if (P == 1)
    hipLaunchKernelGGL(k_plane_correct<1>, grid, block, 0, st, g, vel, phi, out);
  else if (P == 2)
    hipLaunchKernelGGL(k_plane_correct<2>, grid, block, 0, st, g, vel, phi, out);
  else
    hipLaunchKernelGGL(k_plane_correct<3>, grid, block, 0, st, g, vel, phi, out);
  return hipGetLastError();
}

hipError_t launch_plane_potential(const GridDev& g, int P, const double* vel, double* psi, hipStream_t st) {
  const int nx = g.x.n, ny = g.y.n, nz = g.z.n;
  const VelLayout L = vel_layout(nx, ny, nz);
  if (P == 2) {  // Psi_x from w2, columns in y, planes k = 0..nz
    hipLaunchKernelGGL(k_col_scan, dim3(blocks_for(nx, 64), nz + 1), dim3(64 * kColSeg), 0, st, vel + L.ow(), g.y.d,
                       nx, ny, psi);
  } else {  // Psi_y from w1 (rows (k, j), k up to nz) or Psi_z from v3 (rows (k, j), j up to ny)
    const long rows = (P == 1) ? (long)(nz + 1) * ny : (long)nz * (ny + 1);
    const double* src = (P == 1) ? vel + L.ow() : vel + L.ov();
    const double sgn = (P == 1) ? 1.0 : -1.0;
    const unsigned nb = (unsigned)((rows + kPlaneBlock / 64 - 1) / (kPlaneBlock / 64));
    hipLaunchKernelGGL(k_row_scan, dim3(nb), dim3(kPlaneBlock), 0, st, src, g.x.d, sgn, nx, rows, psi);
  }
  return hipGetLastError();
}

}  // namespace lk
