// Staggered finite-volume stencils: linearized momentum / residual (eq. 10,
// eq. 2), cell divergence (eq. 1) and the projection correction (Section 3,
// step 2).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "lk_device.h"

namespace lk {
namespace {

// ------------------------------------------------------------------ momentum
// One block owns a TX x TY column of (i, j) positions and marches along z over
// a chunk of planes.  For each of the six input fields (advecting a = U and
// advected b, components u, v, w) the planes k and k+1 with a one-cell x/y halo live
// in LDS (17 KB); the few plane k-1 values a step needs are carried in registers from
// the step before, and so are the products on the level between two planes (the edge
// fluxes at (x_i, z_k) and (y_j, z_k), the z-momentum's centre product), which two
// consecutive steps share.  Positions outside a field's stored range are
// filled with the wall value of that position: 0 on wall-normal faces, beyond
// tangential walls 0 or, for the advected field of the nonlinear residual, the
// lid velocity at z = 1 (eq. 4).  With these ghosts the wall fluxes of the
// Laplacian ((first - wall)/half width) and the vanishing edge fluxes on walls
// follow from the interior formulas, so the compute has no wall branches.

// Block id -> tile: workgroups are dispatched round-robin over the 8 XCDs, so
// consecutive ids land on different L2s.  Renumber so that each XCD receives a
// contiguous range of tiles (x fastest, then y, then z chunk): neighbouring tiles
// share their halo rows and overlap planes through the same L2.
__device__ __forceinline__ int xcd_tile(int bid, int nb) {
  constexpr int NX = 8;
  const int xcd = bid % NX, local = bid / NX;
  const int per = nb / NX, rem = nb % NX;
  return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

template <bool LID, int TX, int TY>
__global__ void __launch_bounds__(TX* TY) k_momentum(GridDev g, const double* __restrict__ a,
                                                    const double* __restrict__ b, double* __restrict__ out, double rre,
                                                    double s, double lid_u, double lid_v, int kchunk, int nbx,
                                                    int nby) {
  constexpr int MPX = TX + 2, MPY = TY + 2, MPS = MPX * MPY;
  __shared__ double sm[6][2][MPS];  // 0..2: a (u, v, w); 3..5: b (u, v, w); planes k, k+1
  const int nx = g.x.n, ny = g.y.n, nz = g.z.n;
  const size_t nu = (size_t)(nx + 1) * ny * nz, nv = (size_t)nx * (ny + 1) * nz;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int bx = tile % nbx, by = (tile / nbx) % nby, bz = tile / (nbx * nby);
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX, tid = threadIdx.x;
  const int i0 = bx * TX, j0 = by * TY;
  const int kb = bz * kchunk;
  const int ke = min(kb + kchunk, nz + 1);
  const int i = i0 + tx, j = j0 + ty;
  const double* src[6] = {a, a + nu, a + nu + nv, b, b + nu, b + nu + nv};

  // Halo positions of this thread (fixed along the march): in-plane byte offset per
  // component, kGhost for a ghost position.  The loads are raw buffer loads, which return 0
  // at or past a component's size, so a ghost (or a plane outside the field) costs no
  // select; a plane adds k * (plane stride).  The host keeps every component below 2^31
  // bytes, so an in-range offset plus kGhost cannot wrap.
  constexpr unsigned kGhost = 1u << 31;
  constexpr int NT = TX * TY;
  constexpr int PER = (MPS + NT - 1) / NT;
  unsigned col[3][PER];
  bool xy[3][PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = min(tid + q * NT, MPS - 1);  // the surplus threads re-read the last entry
    const int jj = j0 - 1 + e / MPX, ii = i0 - 1 + e % MPX;
    const bool in_i = (ii >= 0) & (ii < nx), in_j = (jj >= 0) & (jj < ny);
    xy[0][q] = (ii > 0) & (ii < nx) & in_j;
    xy[1][q] = (jj > 0) & (jj < ny) & in_i;
    xy[2][q] = in_i & in_j;
    col[0][q] = xy[0][q] ? 8u * (unsigned)(jj * (nx + 1) + ii) : kGhost;
    col[1][q] = xy[1][q] ? 8u * (unsigned)(jj * nx + ii) : kGhost;
    col[2][q] = xy[2][q] ? 8u * (unsigned)(jj * nx + ii) : kGhost;
  }
  const unsigned pstride[3] = {8u * (unsigned)(ny * (nx + 1)), 8u * (unsigned)((ny + 1) * nx),
                               8u * (unsigned)(ny * nx)};
  const unsigned nbytes[3] = {(unsigned)(8 * nu), (unsigned)(8 * nv), (unsigned)(8 * (size_t)nx * ny * (nz + 1))};
  __amdgpu_buffer_rsrc_t rs[6];
#pragma unroll
  for (int arr = 0; arr < 6; ++arr)  // raw buffer (stride 0), 32-bit data format
    rs[arr] = __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(src[arr]), (short)0, (int)nbytes[arr % 3],
                                                0x00020000);

  // Plane loads go to registers first and are written to LDS one step later, so
  // the next plane is in flight while the current one is computed.
  double r0[6][PER];
  auto load = [&](double(&reg)[6][PER], int k) {
    const bool kin_uv = (k >= 0) & (k < nz), kin_w = (k > 0) & (k < nz);
#pragma unroll
    for (int arr = 0; arr < 6; ++arr) {
      const int comp = arr % 3;
      const bool kin = comp == 2 ? kin_w : kin_uv;
      const unsigned kofs = (unsigned)k * pstride[comp];
      const double lid = comp == 0 ? lid_u : lid_v;
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const unsigned off = kin ? col[comp][q] + kofs : kGhost;
        const double x = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs[arr], off, 0, 0));
        // the advected field of the nonlinear residual carries the lid velocity above z = 1
        reg[arr][q] = (LID && arr >= 3 && comp < 2 && xy[comp][q] && k == nz) ? lid : x;
      }
    }
  };
  auto store = [&](const double(&reg)[6][PER], int k) {
    const int slot = (k + 2) & 1;
#pragma unroll
    for (int arr = 0; arr < 6; ++arr) {
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int e = tid + q * NT;
        if (e < MPS) sm[arr][slot][e] = reg[arr][q];
      }
    }
  };

  // per-thread x and y metrics (fixed along the march); out-of-range entries unused
  const double thx0 = (i <= nx) ? g.x.th[i] : 0.0, thx1 = (i + 1 <= nx) ? g.x.th[i + 1] : 0.0;
  const double rdx0 = (i < nx) ? g.x.rd[i] : 0.0, rdxm = (i >= 1 && i - 1 < nx) ? g.x.rd[i - 1] : 0.0;
  const double rddx0 = (i <= nx) ? g.x.rdd[i] : 0.0, rddx1 = (i + 1 <= nx) ? g.x.rdd[i + 1] : 0.0;
  const double thy0 = (j <= ny) ? g.y.th[j] : 0.0, thy1 = (j + 1 <= ny) ? g.y.th[j + 1] : 0.0;
  const double rdy0 = (j < ny) ? g.y.rd[j] : 0.0, rdym = (j >= 1 && j - 1 < ny) ? g.y.rd[j - 1] : 0.0;
  const double rddy0 = (j <= ny) ? g.y.rdd[j] : 0.0, rddy1 = (j + 1 <= ny) ? g.y.rdd[j + 1] : 0.0;

  double cm[6], c0[6], cp[6];
  double exz0, eyz0, czc0;  // the zf[k] level products (see compute)
  double nm0, nm3, nm1, nm4;  // plane k-1: u-fields at (0, +1), v-fields at (+1, 0)
  auto compute = [&](int k) {
    const int p0 = (k + 2) & 1, pp = (k + 3) & 1;  // planes k, k+1
    // S(arr, plane, dj, di)
#define S(arr, pl, dj, di) sm[arr][pl][(ty + 1 + (dj)) * MPX + (tx + 1 + (di))]
    // own-column values of planes k-1 and k, and the four plane k-1 neighbours the z-momentum
    // edges need, are carried in registers from the previous steps; only plane k+1's own
    // column is read here
#pragma unroll
    for (int arr = 0; arr < 6; ++arr) cp[arr] = S(arr, pp, 0, 0);

    const double thz0 = g.z.th[k], thz1 = (k + 1 <= nz) ? g.z.th[k + 1] : 0.0;
    const double rdz0 = (k < nz) ? g.z.rd[k] : 0.0, rdzm = (k >= 1) ? g.z.rd[k - 1] : 0.0;
    const double rddz0 = g.z.rdd[k], rddz1 = (k + 1 <= nz) ? g.z.rdd[k + 1] : 0.0;
    // products on the level zf[k + 1] between planes k and k + 1, used again (as the level
    // zf[k]) by the next step: the edge fluxes at (xf[i], zf[k + 1]) and (yf[j], zf[k + 1]),
    // and the z-momentum's centre product of cell k
    double exz1, eyz1, czc1;
    {
      const double aw = lerp(S(2, pp, 0, -1), cp[2], thx0);
      const double bw = lerp(S(5, pp, 0, -1), cp[5], thx0);
      const double au = lerp(c0[0], cp[0], thz1);
      const double bu = lerp(c0[3], cp[3], thz1);
      exz1 = aw * bu + bw * au;
    }
    {
      const double aw = lerp(S(2, pp, -1, 0), cp[2], thy0);
      const double bw = lerp(S(5, pp, -1, 0), cp[5], thy0);
      const double av = lerp(c0[1], cp[1], thz1);
      const double bv = lerp(c0[4], cp[4], thz1);
      eyz1 = aw * bv + bw * av;
    }
    {
      const double ap = 0.5 * (c0[2] + cp[2]), bp = 0.5 * (c0[5] + cp[5]);
      czc1 = ap * bp;
    }

    // ---- x-momentum at the x-face (i, j, k)
    if (k < nz && j < ny && i <= nx) {
      double val = 0.0;
      if (i >= 1 && i <= nx - 1) {
        const double bc = c0[3];
        double lap = ((S(3, p0, 0, 1) - bc) * rdx0 - (bc - S(3, p0, 0, -1)) * rdxm) * rddx0;
        lap += ((S(3, p0, 1, 0) - bc) * rddy1 - (bc - S(3, p0, -1, 0)) * rddy0) * rdy0;
        lap += ((cp[3] - bc) * rddz1 - (bc - cm[3]) * rddz0) * rdz0;
        const double ac = c0[0];
        const double am = 0.5 * (S(0, p0, 0, -1) + ac), ap = 0.5 * (ac + S(0, p0, 0, 1));
        const double bm = 0.5 * (S(3, p0, 0, -1) + bc), bp = 0.5 * (bc + S(3, p0, 0, 1));
        double conv = 2.0 * (ap * bp - am * bm) * rddx0;
        // edges (xf[i], yf[j + dj])
        double e0, e1;
        {
          const double av = lerp(S(1, p0, 0, -1), c0[1], thx0);
          const double bv = lerp(S(4, p0, 0, -1), c0[4], thx0);
          const double au = lerp(S(0, p0, -1, 0), c0[0], thy0);
          const double bu = lerp(S(3, p0, -1, 0), c0[3], thy0);
          e0 = av * bu + bv * au;
        }
        {
          const double av = lerp(S(1, p0, 1, -1), S(1, p0, 1, 0), thx0);
          const double bv = lerp(S(4, p0, 1, -1), S(4, p0, 1, 0), thx0);
          const double au = lerp(c0[0], S(0, p0, 1, 0), thy1);
          const double bu = lerp(c0[3], S(3, p0, 1, 0), thy1);
          e1 = av * bu + bv * au;
        }
        conv += (e1 - e0) * rdy0;
        // edges (xf[i], zf[k]) and (xf[i], zf[k + 1]): the first carried from the step before
        conv += (exz1 - exz0) * rdz0;
        val = rre * lap - s * conv;
      }
      out[((size_t)k * ny + j) * (nx + 1) + i] = val;
    }

    // ---- y-momentum at the y-face (i, j, k)
    if (k < nz && j <= ny && i < nx) {
      double val = 0.0;
      if (j >= 1 && j <= ny - 1) {
        const double bc = c0[4];
        double lap = ((S(4, p0, 1, 0) - bc) * rdy0 - (bc - S(4, p0, -1, 0)) * rdym) * rddy0;
        lap += ((S(4, p0, 0, 1) - bc) * rddx1 - (bc - S(4, p0, 0, -1)) * rddx0) * rdx0;
        lap += ((cp[4] - bc) * rddz1 - (bc - cm[4]) * rddz0) * rdz0;
        double e0, e1;
        // edges (xf[i + di], yf[j])
        {
          const double au = lerp(S(0, p0, -1, 0), c0[0], thy0);
          const double bu = lerp(S(3, p0, -1, 0), c0[3], thy0);
          const double av = lerp(S(1, p0, 0, -1), c0[1], thx0);
          const double bv = lerp(S(4, p0, 0, -1), c0[4], thx0);
          e0 = au * bv + bu * av;
        }
        {
          const double au = lerp(S(0, p0, -1, 1), S(0, p0, 0, 1), thy0);
          const double bu = lerp(S(3, p0, -1, 1), S(3, p0, 0, 1), thy0);
          const double av = lerp(c0[1], S(1, p0, 0, 1), thx1);
          const double bv = lerp(c0[4], S(4, p0, 0, 1), thx1);
          e1 = au * bv + bu * av;
        }
        double conv = (e1 - e0) * rdx0;
        const double ac = c0[1];
        const double am = 0.5 * (S(1, p0, -1, 0) + ac), ap = 0.5 * (ac + S(1, p0, 1, 0));
        const double bm = 0.5 * (S(4, p0, -1, 0) + bc), bp = 0.5 * (bc + S(4, p0, 1, 0));
        conv += 2.0 * (ap * bp - am * bm) * rddy0;
        // edges (yf[j], zf[k]) and (yf[j], zf[k + 1]): the first carried from the step before
        conv += (eyz1 - eyz0) * rdz0;
        val = rre * lap - s * conv;
      }
      out[nu + ((size_t)k * (ny + 1) + j) * nx + i] = val;
    }

    // ---- z-momentum at the z-face (i, j, k)
    if (k <= nz && j < ny && i < nx) {
      double val = 0.0;
      if (k >= 1 && k <= nz - 1) {
        const double bc = c0[5];
        double lap = ((cp[5] - bc) * rdz0 - (bc - cm[5]) * rdzm) * rddz0;
        lap += ((S(5, p0, 0, 1) - bc) * rddx1 - (bc - S(5, p0, 0, -1)) * rddx0) * rdx0;
        lap += ((S(5, p0, 1, 0) - bc) * rddy1 - (bc - S(5, p0, -1, 0)) * rddy0) * rdy0;
        double e0, e1;
        // edges (xf[i + di], zf[k]); the one at xf[i] is the x-momentum's, carried
        e0 = exz0;
        {
          const double au = lerp(nm0, S(0, p0, 0, 1), thz0);
          const double bu = lerp(nm3, S(3, p0, 0, 1), thz0);
          const double aw = lerp(c0[2], S(2, p0, 0, 1), thx1);
          const double bw = lerp(c0[5], S(5, p0, 0, 1), thx1);
          e1 = au * bw + bu * aw;
        }
        double conv = (e1 - e0) * rdx0;
        // edges (yf[j + dj], zf[k]); the one at yf[j] is the y-momentum's, carried
        e0 = eyz0;
        {
          const double av = lerp(nm1, S(1, p0, 1, 0), thz0);
          const double bv = lerp(nm4, S(4, p0, 1, 0), thz0);
          const double aw = lerp(c0[2], S(2, p0, 1, 0), thy1);
          const double bw = lerp(c0[5], S(5, p0, 1, 0), thy1);
          e1 = av * bw + bv * aw;
        }
        conv += (e1 - e0) * rdy0;
        conv += 2.0 * (czc1 - czc0) * rddz0;
        val = rre * lap - s * conv;
      }
      out[nu + nv + ((size_t)k * ny + j) * nx + i] = val;
    }
    nm0 = S(0, p0, 0, 1);
    nm3 = S(3, p0, 0, 1);
    nm1 = S(1, p0, 1, 0);
    nm4 = S(4, p0, 1, 0);
#undef S
#pragma unroll
    for (int arr = 0; arr < 6; ++arr) {
      cm[arr] = c0[arr];
      c0[arr] = cp[arr];
    }
    exz0 = exz1;
    eyz0 = eyz1;
    czc0 = czc1;
  };

  // LDS holds planes k and k+1 (two slots); plane kb - 1 passes through once for the values
  // carried in registers.  The next plane is loaded into registers during a step and
  // written to the freed slot after it.
#define S(arr, pl, dj, di) sm[arr][pl][(ty + 1 + (dj)) * MPX + (tx + 1 + (di))]
  {
    const int sl = (kb + 1) & 1;  // plane kb - 1
    load(r0, kb - 1);
    store(r0, kb - 1);
    __syncthreads();
#pragma unroll
    for (int arr = 0; arr < 6; ++arr) cm[arr] = S(arr, sl, 0, 0);
    nm0 = S(0, sl, 0, 1);
    nm3 = S(3, sl, 0, 1);
    nm1 = S(1, sl, 1, 0);
    nm4 = S(4, sl, 1, 0);
    __syncthreads();
  }
  load(r0, kb);
  store(r0, kb);
  load(r0, kb + 1);
  store(r0, kb + 1);
  __syncthreads();
#pragma unroll
  for (int arr = 0; arr < 6; ++arr) c0[arr] = S(arr, kb & 1, 0, 0);
  {
    // the zf[kb] level products from planes kb - 1 (registers) and kb
    const int p0 = kb & 1;
    const double thz0 = g.z.th[kb];
    {
      const double aw = lerp(S(2, p0, 0, -1), c0[2], thx0);
      const double bw = lerp(S(5, p0, 0, -1), c0[5], thx0);
      const double au = lerp(cm[0], c0[0], thz0);
      const double bu = lerp(cm[3], c0[3], thz0);
      exz0 = aw * bu + bw * au;
    }
    {
      const double aw = lerp(S(2, p0, -1, 0), c0[2], thy0);
      const double bw = lerp(S(5, p0, -1, 0), c0[5], thy0);
      const double av = lerp(cm[1], c0[1], thz0);
      const double bv = lerp(cm[4], c0[4], thz0);
      eyz0 = aw * bv + bw * av;
    }
    {
      const double am = 0.5 * (cm[2] + c0[2]), bm = 0.5 * (cm[5] + c0[5]);
      czc0 = am * bm;
    }
  }
#undef S
  if (kb + 2 <= ke) load(r0, kb + 2);
  for (int k = kb; k < ke; ++k) {
    compute(k);
    __syncthreads();
    if (k + 2 <= ke) store(r0, k + 2);
    __syncthreads();
    if (k + 3 <= ke) load(r0, k + 3);
  }
}

// ---------------------------------------------------------------- divergence
// One thread per (i, j) column of cells marching over KZ planes, so the w face
// between two cells is read once (carried in a register); tiles are grouped per XCD.
constexpr int kDivTX = 64, kDivTY = 4, kDivKZ = 4;

template <int KZ>
__global__ void __launch_bounds__(kDivTX* kDivTY) k_divergence(GridDev g, Vel V, double* __restrict__ r,
                                                               double* __restrict__ partials, int nbx, int nby) {
  const int nx = g.x.n, ny = g.y.n, nz = g.z.n;
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  const int i = (t % nbx) * kDivTX + (int)(threadIdx.x % kDivTX);
  const int j = ((t / nbx) % nby) * kDivTY + (int)(threadIdx.x / kDivTX);
  const int k0 = (t / (nbx * nby)) * KZ, k1 = min(k0 + KZ, nz);
  double contrib = 0.0;
  if (i < nx && j < ny) {
    const double rdx = g.x.rd[i], rdy = g.y.rd[j], dxy = g.x.d[i] * g.y.d[j];
    double wlo = V.W(k0, j, i);
    for (int k = k0; k < k1; ++k) {
      const double whi = V.W(k + 1, j, i);
      const double dv = (V.U(k, j, i + 1) - V.U(k, j, i)) * rdx + (V.V(k, j + 1, i) - V.V(k, j, i)) * rdy +
                        (whi - wlo) * g.z.rd[k];
      if (r) r[((size_t)k * ny + j) * nx + i] = dv;
      contrib += dxy * g.z.d[k] * dv * dv;
      wlo = whi;
    }
  }
  if (partials) {
    const double s = block_sum(contrib);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
  }
}

// ---------------------------------------------------------------- correction
// One thread per (i, j) face column marching over KZ planes (phi of the plane
// below carried in a register); tiles grouped per XCD.
constexpr int kCorTX = 64, kCorTY = 4, kCorKZ = 2;

template <int KZ>
__global__ void __launch_bounds__(kCorTX* kCorTY) k_correct(GridDev g, const double* __restrict__ w,
                                                            const double* __restrict__ phi, double* __restrict__ v,
                                                            double* __restrict__ p, int accumulate, int nbx, int nby) {
  const int nx = g.x.n, ny = g.y.n, nz = g.z.n;
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  const int i = (t % nbx) * kCorTX + (int)(threadIdx.x % kCorTX);
  const int j = ((t / nbx) % nby) * kCorTY + (int)(threadIdx.x / kCorTX);
  const int k0 = (t / (nbx * nby)) * KZ, k1 = min(k0 + KZ, nz + 1);
  if (i > nx || j > ny) return;
  const Idx I{nx, ny, nz};
  const size_t nu = (size_t)(nx + 1) * ny * nz, nv = (size_t)nx * (ny + 1) * nz;
  const double* src = accumulate ? v : w;
  // branch-free loads: in-range clamped cell indices, wall faces selected to 0
  const int ic = min(i, nx - 1), jc = min(j, ny - 1);
  const double rddx = g.x.rdd[i], rddy = g.y.rdd[j];
  double pb = phi[I.c(max(k0 - 1, 0), jc, ic)];  // phi below the first plane
  for (int k = k0; k < k1; ++k) {
    // every load of the plane from an in-range (clamped) position, before any store, so
    // that they are in flight together; only the stores depend on the face being stored
    const int kc = min(k, nz - 1);
    const double pc = phi[I.c(kc, jc, ic)];
    const double pw = phi[I.c(kc, jc, max(ic - 1, 0))], ps = phi[I.c(kc, max(jc - 1, 0), ic)];
    const size_t qu = I.u(kc, jc, i), qv = nu + I.v(kc, j, ic), qw = nu + nv + I.w(k, jc, ic);
    const double su = src[qu], sv = src[qv], sw = src[qw];
    const double pold = (p && accumulate) ? p[I.c(kc, jc, ic)] : 0.0;
    if (j < ny && k < nz) {
      const bool in = (i > 0) & (i < nx);
      const double val = su - (pc - pw) * rddx;
      v[qu] = in ? val : 0.0;
    }
    if (i < nx && k < nz) {
      const bool in = (j > 0) & (j < ny);
      const double val = sv - (pc - ps) * rddy;
      v[qv] = in ? val : 0.0;
    }
    if (i < nx && j < ny) {
      const bool in = (k > 0) & (k < nz);
      const double val = sw - (pc - pb) * g.z.rdd[k];
      v[qw] = in ? val : 0.0;
      if (p && k < nz) p[I.c(k, j, i)] = accumulate ? pold + pc : pc;
    }
    pb = pc;
  }
}

}  // namespace

// ==================================================================== launchers
// Tile of the momentum stencil: TX x TY threads; the nz + 1 planes are split into the
// nearest whole number of kMomChunk-plane chunks, ceil((nz + 1) / that number) planes each
// (the last takes the rest), one chunk per block.  Measured at
// 200^3 (201 planes, same bits for every length): 12 planes 191-192 us, 14 196-198, 17
// 193-195, 24 197-199, 29 197-198, 41 218; 8 and 10 (a last chunk of one plane) 197-201.
constexpr int kMomTX = 16, kMomTY = 8, kMomChunk = 12;

hipError_t launch_momentum(const GridDev& g, const double* a, const double* b, double* out, double rre, double s,
                           bool lid, double lid_u, double lid_v, hipStream_t st) {
  const int nx = g.x.n, ny = g.y.n, nz = g.z.n;
  const VelLayout L = vel_layout(nx, ny, nz);
  if (8 * std::max(L.nu, std::max(L.nv, L.nw)) >= (size_t(1) << 31)) return hipErrorInvalidValue;
  const int nbx = (int)blocks_for(nx + 1, kMomTX), nby = (int)blocks_for(ny + 1, kMomTY);
  const int nch = std::max(1, (nz + 1 + kMomChunk / 2) / kMomChunk);
  const int kchunk = (int)blocks_for(nz + 1, nch);
  const int nbz = (int)blocks_for(nz + 1, kchunk);
  const dim3 grid(nbx * nby * nbz), block(kMomTX * kMomTY);
  if (lid)
    hipLaunchKernelGGL((k_momentum<true, kMomTX, kMomTY>), grid, block, 0, st, g, a, b, out, rre, s, lid_u, lid_v,
                       kchunk, nbx, nby);
  else
    hipLaunchKernelGGL((k_momentum<false, kMomTX, kMomTY>), grid, block, 0, st, g, a, b, out, rre, s, 0.0, 0.0,
                       kchunk, nbx, nby);
  return hipGetLastError();
}

hipError_t launch_divergence(const GridDev& g, const double* v, double* r, double* partials, int* nparts,
                             hipStream_t st) {
  const int nx = g.x.n, ny = g.y.n, nz = g.z.n;
  const VelLayout L = vel_layout(nx, ny, nz);
  Vel V{v, v + L.ov(), v + L.ow(), Idx{nx, ny, nz}};
  const int nbx = (int)blocks_for(nx, kDivTX), nby = (int)blocks_for(ny, kDivTY);
  const unsigned nb = (unsigned)(nbx * nby * (int)blocks_for(nz, kDivKZ));
  if (nparts) *nparts = (int)nb;
  hipLaunchKernelGGL(k_divergence<kDivKZ>, dim3(nb), dim3(kDivTX * kDivTY), 0, st, g, V, r, partials, nbx, nby);
  return hipGetLastError();
}

hipError_t launch_correct(const GridDev& g, const double* w, const double* phi, double* v, double* p,
                          bool accumulate, hipStream_t st) {
  const int nx = g.x.n, ny = g.y.n, nz = g.z.n;
  const int nbx = (int)blocks_for(nx + 1, kCorTX), nby = (int)blocks_for(ny + 1, kCorTY);
  const unsigned nb = (unsigned)(nbx * nby * (int)blocks_for(nz + 1, kCorKZ));
  hipLaunchKernelGGL(k_correct<kCorKZ>, dim3(nb), dim3(kCorTX * kCorTY), 0, st, g, w, phi, v, p, accumulate ? 1 : 0, nbx,
                     nby);
  return hipGetLastError();
}

}  // namespace lk
