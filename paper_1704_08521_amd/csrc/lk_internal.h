// Internal declarations shared by the kernel file and the host API.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace lk {

// One axis of the stretched staggered grid, device arrays.
//   d[n]    cell widths             rd[n]  = 1/d
//   dd[n+1] centre distances across faces (half widths at the walls), rdd = 1/dd
//   th[n+1] interpolation weight of face i between centres i-1 and i
struct AxisDev {
  const double* rd;
  const double* rdd;
  const double* th;
  const double* d;
  int n;
};

struct GridDev {
  AxisDev x, y, z;
};

// Offsets of u, v, w inside a packed velocity.
struct VelLayout {
  size_t nu, nv, nw;  // element counts
  size_t ou() const { return 0; }
  size_t ov() const { return nu; }
  size_t ow() const { return nu + nv; }
  size_t total() const { return nu + nv + nw; }
};

inline VelLayout vel_layout(int nx, int ny, int nz) {
  VelLayout L;
  L.nu = (size_t)(nx + 1) * ny * nz;
  L.nv = (size_t)nx * (ny + 1) * nz;
  L.nw = (size_t)nx * ny * (nz + 1);
  return L;
}

// ------------------------------------------------------------ launchers
// All launchers enqueue on `s` and return the launch status.

// out = rre * Lap_g(b) - s * [C(a, b) + C(b, a)], lid only if `lid` is set.
// Jacobian: a = U, b = v, s = 1, lid off.  Residual: a = b = U, s = 1/2, lid on.
hipError_t launch_momentum(const GridDev& g, const double* a, const double* b, double* out,
                           double rre, double s, bool lid, double lid_u, double lid_v,
                           hipStream_t st);

// r = D v (cell), and per-block partial sums of V r^2 into `partials`
// (nblocks returned through *nparts; partials may be null).
hipError_t launch_divergence(const GridDev& g, const double* v, double* r, double* partials,
                             int* nparts, hipStream_t st);

// v = w - G phi (interior faces), zero on walls; p = phi if p != null.
// If accumulate: v -= G phi in place on v (w ignored) and p += phi.
hipError_t launch_correct(const GridDev& g, const double* w, const double* phi, double* v,
                          double* p, bool accumulate, hipStream_t st);

// Fixed-order sum of n partials into out[0] (one block).
hipError_t launch_sum(const double* partials, int n, double* out, hipStream_t st);

// Per-block partial dot products of two arrays of length n.
hipError_t launch_dot_partials(const double* a, const double* b, size_t n, double* partials,
                               int* nparts, hipStream_t st);

// Fixed-order max of n partials into out[0]; per-block partial max |a|.
hipError_t launch_max(const double* partials, int n, double* out, hipStream_t st);
hipError_t launch_maxabs_partials(const double* a, size_t n, double* partials, int* nparts, hipStream_t st);


// y += sign * a_dev[0] / d_dev[0] * x (d_dev may be null): scalars from device memory.
hipError_t launch_axpy_dev(size_t n, const double* a_dev, const double* d_dev, double sign, const double* x,
                           double* y, hipStream_t st);

// out[c] = sum_i V[i] Q[i][c] for c < nc (<= 48), i < nv; vectors ld / ldo apart.
hipError_t launch_combine(const double* V, long ld, int nv, const double* Q, int nc, double* out, long ldo, size_t n,
                          hipStream_t st);

// y = a*x + y ; x *= a ; y = x
hipError_t launch_axpy(size_t n, double a, const double* x, double* y, hipStream_t st);
hipError_t launch_scale(size_t n, double a, double* x, hipStream_t st);

// Tensor-product line transform along a strided axis: C[m][n] = sum_k A[m][k] B[k][n]
// with A the K x K (= M x K) mode matrix and B/C data whose column n starts at
// (n / nseg) * seg_stride + n % nseg with rows kstride apart.  If lm is set the
// result is divided by lm[m] + ly[n / nxs] + lx[n % nxs] (mode (zm, zj, zi) -> 0).
template <typename T>
hipError_t launch_tp_left(int M, int N, int K, const T* A, const T* B, T* C, int nseg, long seg_stride,
                          long kstride, const double* lm, const double* ly, const double* lx, int nxs, int zm,
                          int zj, int zi, hipStream_t st);

// Line transform along the contiguous axis: C (M x N) = A (M x K data) * B (K x N).
template <typename T>
hipError_t launch_tp_right(int M, int N, int K, const T* A, const T* B, T* C, hipStream_t st);

// Mirror-symmetric axes (parity-sorted modes, he = ceil(n/2) even, ho = floor(n/2) odd):
// forward transforms fold line values on load and use the half matrices Ae (he x he) /
// Ao (ho x ho) (left) or their transposes Be / Bo (right); backward transforms use
// Se (he x he), So (he x ho) (left) or SeT (he x he), SoT (ho x he) (right) and unfold.
// Layout and scaling arguments as launch_tp_left / launch_tp_right.
template <typename T>
hipError_t launch_tpf_left(int n, int N, const T* Ae, const T* Ao, const T* B, T* C, int nseg, long seg_stride,
                           long kstride, const double* lm, const double* ly, const double* lx, int nxs, int zm, int zj,
                           int zi, hipStream_t st);
template <typename T>
hipError_t launch_tpu_left(int n, int N, const T* Se, const T* So, const T* B, T* C, int nseg, long seg_stride,
                           long kstride, hipStream_t st);
template <typename T>
hipError_t launch_tpf_right(int n, int Mlines, const T* A, const T* Be, const T* Bo, T* C, hipStream_t st);
template <typename T>
hipError_t launch_tpu_right(int n, int Mlines, const T* A, const T* SeT, const T* SoT, T* C, hipStream_t st);

// The same four transforms on the matrix cores, for he = ceil(n/2) <= 128 (kMfMaxHalf).
// The half matrices are passed as fragment packs: Pe, Po packs of Ae, Ao (forward), Pse,
// Pso packs of Se, So (backward), for the left and the right kernels alike
// (fragment (kq, t, l) = Mat[16 t + l % 16][4 kq + l / 16], RT = ceil(he / 16),
// kq < mf_steps(he), zero outside the matrix: the contraction steps of 4 are padded to a
// multiple of the kernels' prefetch depth kMfPD; layout mf_pack_index).  Here the eigenvalue scaling (lm, ly,
// lx, zero mode) belongs to the backward left transform: its input modes are scaled on
// load.
constexpr int kMfMaxHalf = 128;
constexpr int kMfPD = 1;
__host__ __device__ constexpr int mf_steps(int he, int pd = kMfPD) { return ((he + 3) / 4 + pd - 1) / pd * pd; }
// Fragments are grouped fg = 16 / sizeof(element) per lane (one 16-byte load fetches fg
// consecutive row tiles): fragment (kq, t, lane) sits at mf_pack_index(kq, t, lane, RT, fg).
__host__ __device__ constexpr int mf_tile_groups(int RT, int fg) { return (RT + fg - 1) / fg; }
__host__ __device__ constexpr long mf_pack_index(int kq, int t, int lane, int RT, int fg) {
  return ((long)(kq * mf_tile_groups(RT, fg) + t / fg) * 64 + lane) * fg + t % fg;
}
__host__ __device__ constexpr long mf_pack_size(int he, int fg) {
  return (long)mf_steps(he) * mf_tile_groups((he + 15) / 16, fg) * 64 * fg;
}
template <typename T>
hipError_t launch_mff_left(int n, int N, const T* Pe, const T* Po, const T* B, T* C, int nseg, long seg_stride,
                           long kstride, hipStream_t st);
template <typename T>
hipError_t launch_mfu_left(int n, int N, const T* Pse, const T* Pso, const T* B, T* C, int nseg, long seg_stride,
                           long kstride, const double* lm, const double* ly, const double* lx, int nxs, int zm, int zj,
                           int zi, hipStream_t st);
template <typename T>
hipError_t launch_mff_right(int n, int Mlines, const T* A, const T* Pe, const T* Po, T* C, hipStream_t st);
template <typename T>
hipError_t launch_mfu_right(int n, int Mlines, const T* A, const T* Pse, const T* Pso, T* C, hipStream_t st);

// Precision casts.
hipError_t launch_d2f(size_t n, const double* in, float* out, hipStream_t st);
// out = in (float -> double), or out += in when accumulate
hipError_t launch_f2d(size_t n, const float* in, double* out, bool accumulate, hipStream_t st);

// Fill with the counter-based SplitMix64 uniform [-1, 1) stream `seed`.
hipError_t launch_uniform(double* x, size_t n, uint64_t seed, hipStream_t st);

// Streaming probe: kind 0 copies a to c, 1 writes c = a + 1.5 b, 2 reads a; n2 16-byte
// elements.  sink: one device double (written only by a never-taken branch).
hipError_t launch_probe(int kind, const double* a, const double* b, double* c, size_t n2, double* sink,
                        hipStream_t st);

// Zero the wall-normal faces of a packed velocity.
hipError_t launch_zero_walls(double* vel, int nx, int ny, int nz, hipStream_t st);

// ---------------------------------------------------- TPT tridiagonal x step
// For every x-line (k, j) of a (y, z)-transformed cell field: (D_x G_x + ly[j] + lz[k]) out
// = in (a null array adds nothing); the lines with j = zj and k = zk are the singular ones
// (solutions with zero d-weighted mean), a negative index matching every j or k.
// Lines of up to tridiag_x_max() cells.
int tridiag_x_max();
template <typename T>
hipError_t launch_tridiag_x(const GridDev& g, const double* ly, const double* lz, int zj, int zk, const T* in, T* out,
                            hipStream_t st);

// ---------------------------------------------------- plane projections
// P = 1 keeps (u, w) (planes y = const), 2 keeps (v, w) (x = const), 3 keeps (u, v)
// (z = const).
// r = D2 b, b = the kept components of vel with the wall-normal faces zero.
hipError_t launch_plane_rhs(const GridDev& g, int P, const double* vel, double* r, hipStream_t st);
// t /= lx[i] + ly[j] + lz[k] (a null array adds nothing); zero where every index equals
// its zero mode, a negative zero mode matching every index.
hipError_t launch_plane_scale(double* t, int nx, int ny, int nz, const double* lx, const double* ly, const double* lz,
                              int zx, int zy, int zz, hipStream_t st);
// out = b - G2 phi on interior faces of the kept components, zero elsewhere.
hipError_t launch_plane_correct(const GridDev& g, int P, const double* vel, const double* phi, double* out,
                                hipStream_t st);
// The potential of a projection by prefix sums from the walls.
hipError_t launch_plane_potential(const GridDev& g, int P, const double* vel, double* psi, hipStream_t st);

constexpr int kReduceBlock = 256;
// Classical Gram-Schmidt: h[i] = V_i . w (i < nv; basis vectors ld apart; h on the device,
// fixed-order sums), then w -= sum_i h[i] V_i.  partials holds kGsBlocks * kGsChunk doubles.
constexpr int kGsBlocks = 2048, kGsChunk = 8;
hipError_t launch_gs_dot(const double* V, long ld, int nv, const double* w, size_t n, double* partials,
                         double* h, hipStream_t st);
hipError_t launch_gs_update(const double* V, long ld, int nv, const double* h, double* w, size_t n, hipStream_t st);

}  // namespace lk
