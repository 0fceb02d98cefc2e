// Tridiagonal solves along x in (y, z) mode space: the x step of the pressure-correction
// Poisson solve by the TPT route of Section 3 (mode transforms in two directions, a
// tridiagonal solve in the third).  For every x-line (k, j) of the transformed field,
// (L_x + ly[j] + lz[k]) phi = rhs, with L_x = D_x G_x on the cells of the line (zero flux
// through the walls).  One wave per line, by the partition method: lane p owns the M
// consecutive rows of segment p and eliminates its interior rows in registers (one
// Thomas sweep with three right sides), which leaves one unknown per segment, its last
// row; those form a tridiagonal system (the Schur complement, diagonally dominant like
// the line's own matrix) solved by cyclic reduction across the lanes with shuffles; each
// lane then recovers its interior rows.  The line whose shift is zero (the zero modes of
// y and z) is singular: its first equation is replaced by phi_0 = 0 and the solution is
// re-centred to zero d-weighted mean, which sets the constant mode to zero as the
// transform route does.  The plane projections use the same pass with one shift array
// null (adding nothing) and a negative zero-mode index matching every index.
#include <hip/hip_runtime.h>

#include "lk_device.h"
#include "lk_internal.h"

namespace lk {
namespace {

constexpr int kTriLinesPerBlock = 4;  // one wave per line

// 1 / a to the type's accuracy: the hardware reciprocal refined by Newton steps (two in
// FP64, one in FP32)
__device__ __forceinline__ double rcpx(double a) {
  double y = __builtin_amdgcn_rcp(a);
  double e = fma(-a, y, 1.0);
  y = fma(e, y, y);
  e = fma(-a, y, 1.0);
  return fma(e, y, y);
}
__device__ __forceinline__ float rcpx(float a) {
  const float y = __builtin_amdgcn_rcpf(a);
  return fmaf(fmaf(-a, y, 1.0f), y, y);
}

template <typename T, int M>
__global__ void __launch_bounds__(64 * kTriLinesPerBlock) k_tridiag_x(
    const double* __restrict__ rd, const double* __restrict__ rdd, const double* __restrict__ dx, int n, int ny,
    long lines, const double* __restrict__ ly, const double* __restrict__ lz, int zj, int zk,
    const T* __restrict__ in, T* __restrict__ out) {
  const int lane = (int)(threadIdx.x & 63);
  const long line = (long)blockIdx.x * kTriLinesPerBlock + (long)(threadIdx.x >> 6);
  if (line >= lines) return;  // uniform per wave
  const int j = (int)(line % ny), k = (int)(line / ny);
  const T shift = (T)((ly ? ly[j] : 0.0) + (lz ? lz[k] : 0.0));
  const bool sing = (zj < 0 || j == zj) && (zk < 0 || k == zk);
  const int P = (n + M - 1) / M;  // segments (lanes in use)
  const int s0 = lane * M;
  const int L = (lane < P) ? min(M, n - s0) : 0;  // rows of this lane's segment
  const T* src = in + (size_t)line * n;
  // the segment's rows: a x_{r-1} + b x_r + c x_{r+1} = d (identity rows beyond L); the
  // coefficients are formed in FP64 and rounded to T.  Every lane loads from an in-range
  // row (rows past the line re-read its last one) and selects afterwards, so all the
  // loads are in flight together instead of one branch and wait per row.
  T ra[M], rb[M], rc[M], rv[M];
#pragma unroll
  for (int t = 0; t < M; ++t) {
    const int r = s0 + t, rr = min(r, n - 1);
    const double rdr = rd[rr], rdd0 = rdd[rr], rdd1 = rdd[rr + 1];  // rdd has n + 1 entries
    const T dr = src[rr];
    const bool in = t < L;
    const bool pin = sing && r == 0;
    const double a64 = (in && r > 0) ? rdd0 * rdr : 0.0;
    const double c64 = (in && r + 1 < n) ? rdd1 * rdr : 0.0;
    ra[t] = pin ? T(0) : (T)a64;
    rc[t] = pin ? T(0) : (T)c64;
    rb[t] = (in && !pin) ? shift - (T)(a64 + c64) : T(1);
    rv[t] = (in && !pin) ? dr : T(0);
  }
  // interior rows 0 .. q-1 in terms of the two segment ends z_{p-1} (previous lane's last
  // row) and z_p (own last row): x = Y - V z_{p-1} - W z_p
  const int q = L - 1;
  T Y[M], V[M], W[M], cp[M];
#pragma unroll
  for (int i = 0; i < M; ++i) {
    Y[i] = 0;
    V[i] = 0;
    W[i] = 0;
    cp[i] = 0;
  }
#pragma unroll
  for (int i = 0; i < M - 1; ++i) {
    if (i < q) {
      const T sub = (i > 0) ? ra[i] : T(0);
      const T den = rb[i] - ((i > 0) ? sub * cp[i - 1] : T(0));
      const T r = rcpx(den);
      cp[i] = ((i < q - 1) ? rc[i] : T(0)) * r;
      Y[i] = (rv[i] - ((i > 0) ? sub * Y[i - 1] : T(0))) * r;
      V[i] = (((i == 0) ? ra[0] : T(0)) - ((i > 0) ? sub * V[i - 1] : T(0))) * r;
      W[i] = (((i == q - 1) ? rc[i] : T(0)) - ((i > 0) ? sub * W[i - 1] : T(0))) * r;
    }
  }
#pragma unroll
  for (int i = M - 3; i >= 0; --i) {
    if (i < q - 1) {
      Y[i] -= cp[i] * Y[i + 1];
      V[i] -= cp[i] * V[i + 1];
      W[i] -= cp[i] * W[i + 1];
    }
  }
  // the segment's first row and the row before its last, as (Y, V, W) of the ends; with no
  // interior rows the first row is z_p itself and the row before the last is z_{p-1}
  T Yf = 0, Vf = 0, Wf = 0, Yl = 0, Vl = 0, Wl = 0;
  T ae = 0, be = 1, ce = 0, de = 0;
  if (q >= 1) {
    Yf = Y[0];
    Vf = V[0];
    Wf = W[0];
  } else if (q == 0) {
    Wf = -1;
    Vl = -1;
  }
#pragma unroll
  for (int i = 0; i < M; ++i) {
    if (i == q - 1) {
      Yl = Y[i];
      Vl = V[i];
      Wl = W[i];
    }
    if (i == L - 1) {
      ae = ra[i];
      be = rb[i];
      ce = rc[i];
      de = rv[i];
    }
  }
  // the last row's equation in the segment ends: al z_{p-1} + bt z_p + ga z_{p+1} = dl
  const T Yn = __shfl_down(Yf, 1), Vn = __shfl_down(Vf, 1), Wn = __shfl_down(Wf, 1);
  T al = 0, bt = 1, ga = 0, dl = 0;
  if (L > 0) {
    al = -ae * Vl;
    bt = be - ae * Wl - ce * Vn;
    ga = -ce * Wn;
    dl = de - ae * Yl - ce * Yn;
  }
  // cyclic reduction across the lanes (identity rows beyond P couple to nothing).  At step
  // st a row couples to rows st below and above it; the lower coupling al is exactly zero
  // on lanes below st and the upper one ga on lanes with no row st above (initially from
  // the zero coefficients of the line's first and last rows, then because each update
  // multiplies by them), so the products with the values a shuffle returns past the wave's
  // ends vanish and the updates need no lane conditions.
  for (int st = 1; st < P; st <<= 1) {
    const T rbt = rcpx(bt);
    T an, gn, bn = bt, dn = dl;
    if constexpr (sizeof(T) == 8) {
      // each lane sends its row divided by its own diagonal: three values per direction
      // (12 LDS permutes per step instead of 16)
      const T as = al * rbt, gs = ga * rbt, ds = dl * rbt;
      const T am = __shfl_up(as, st), gm = __shfl_up(gs, st), dm = __shfl_up(ds, st);
      const T ap = __shfl_down(as, st), gp = __shfl_down(gs, st), dp = __shfl_down(ds, st);
      an = -al * am;
      bn -= al * gm;
      dn -= al * dm;
      gn = -ga * gp;
      bn -= ga * ap;
      dn -= ga * dp;
    } else {
      // FP32: the neighbour's reciprocal travels separately, which keeps the mixed form's
      // solves as accurate as before the FP64 change (the sender-side products lost a factor
      // of about 1.5 in the first-pass divergence)
      const T am = __shfl_up(al, st), gm = __shfl_up(ga, st), dm = __shfl_up(dl, st), rm = __shfl_up(rbt, st);
      const T ap = __shfl_down(al, st), gp = __shfl_down(ga, st), dp = __shfl_down(dl, st), rp = __shfl_down(rbt, st);
      const T k1 = al * rm, k2 = ga * rp;
      an = -am * k1;
      bn -= gm * k1;
      dn -= dm * k1;
      gn = -gp * k2;
      bn -= ap * k2;
      dn -= dp * k2;
    }
    al = an;
    bt = bn;
    ga = gn;
    dl = dn;
  }
  const T z = dl / bt;
  const T zu = __shfl_up(z, 1);  // every lane takes part in the shuffle
  const T zl = (lane > 0) ? zu : T(0);
  T x[M];
#pragma unroll
  for (int i = 0; i < M; ++i) x[i] = (i < q) ? Y[i] - V[i] * zl - W[i] * z : (i == q ? z : T(0));
  if (sing) {  // uniform per wave
    double sw = 0.0, swx = 0.0;
#pragma unroll
    for (int i = 0; i < M; ++i) {
      if (i < L) {
        const double w = dx[s0 + i];
        sw += w;
        swx += w * (double)x[i];
      }
    }
    // (the wave sums are complete in lane 0: broadcast them)
    const double mean = __shfl(wave_sum(swx), 0) / __shfl(wave_sum(sw), 0);
#pragma unroll
    for (int i = 0; i < M; ++i) x[i] -= (T)mean;
  }
  T* dst = out + (size_t)line * n;
#pragma unroll
  for (int i = 0; i < M; ++i)
    if (i < L) dst[s0 + i] = x[i];
}

}  // namespace

int tridiag_x_max() { return 64 * 16; }

template <typename T>
hipError_t launch_tridiag_x(const GridDev& g, const double* ly, const double* lz, int zj, int zk, const T* in, T* out,
                            hipStream_t st) {
  const int n = g.x.n, ny = g.y.n, nz = g.z.n;
  const long lines = (long)ny * nz;
  const dim3 grid((unsigned)((lines + kTriLinesPerBlock - 1) / kTriLinesPerBlock)), block(64 * kTriLinesPerBlock);
  const double *rd = g.x.rd, *rdd = g.x.rdd, *dx = g.x.d;
  if (n <= 64)
    hipLaunchKernelGGL((k_tridiag_x<T, 1>), grid, block, 0, st, rd, rdd, dx, n, ny, lines, ly, lz, zj, zk, in, out);
  else if (n <= 128)
    hipLaunchKernelGGL((k_tridiag_x<T, 2>), grid, block, 0, st, rd, rdd, dx, n, ny, lines, ly, lz, zj, zk, in, out);
  else if (n <= 256)
    hipLaunchKernelGGL((k_tridiag_x<T, 4>), grid, block, 0, st, rd, rdd, dx, n, ny, lines, ly, lz, zj, zk, in, out);
  else if (n <= 512)
    hipLaunchKernelGGL((k_tridiag_x<T, 8>), grid, block, 0, st, rd, rdd, dx, n, ny, lines, ly, lz, zj, zk, in, out);
  else if (n <= 1024)
    hipLaunchKernelGGL((k_tridiag_x<T, 16>), grid, block, 0, st, rd, rdd, dx, n, ny, lines, ly, lz, zj, zk, in, out);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template hipError_t launch_tridiag_x<double>(const GridDev&, const double*, const double*, int, int, const double*,
                                             double*, hipStream_t);
template hipError_t launch_tridiag_x<float>(const GridDev&, const double*, const double*, int, int, const float*,
                                            float*, hipStream_t);

}  // namespace lk
