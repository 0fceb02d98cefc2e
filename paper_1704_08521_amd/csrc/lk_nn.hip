// Kernels of the learned pressure-correction guess: a 3-level 3D U-Net (3x3x3
// convolutions, 2x2x2 average pooling, nearest upsampling with skip
// concatenation, 1x1x1 head) in BF16 with FP32 accumulation on the CDNA4 matrix
// cores, its backward pass, Adam, and the conversions between the FP64 fields of
// the SIMPLE loop and the network tensors.
//
// Network tensors are channels-last, [D][H][W][C] (z, y, x, channel), BF16,
// C a multiple of 8 so that one lane's 8 reduction values are one 16-byte load.
// A 3x3x3 convolution is an implicit GEMM: rows = output voxels, columns = output
// channels, reduction index k = tap * CIN + ci (tap = (dz+1)*9 + (dy+1)*3 + (dx+1)),
// padded to a multiple of 32 with zero weights.  v_mfma_f32_16x16x32_bf16 lane
// layout (lane l, g = l / 16): A row l%16, k = 8g..8g+7; B column l%16, same k;
// result rows 4g..4g+3 of column l%16.
#include <hip/hip_runtime.h>

#include "lk_nn.h"

namespace lk {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kBlock = 256;

__device__ __forceinline__ bf16x8 load8(const bf16* p, bool ok) {
  // branch-free guarded 16-byte load: the address is valid whenever ok is false
  const u32x4 v = *reinterpret_cast<const u32x4*>(p);
  u32x4 s;
  s.x = ok ? v.x : 0u;
  s.y = ok ? v.y : 0u;
  s.z = ok ? v.z : 0u;
  s.w = ok ? v.w : 0u;
  return __builtin_bit_cast(bf16x8, s);
}

__device__ __forceinline__ float bf2f(bf16 h) { return static_cast<float>(h); }
__device__ __forceinline__ bf16 f2bf(float f) { return static_cast<bf16>(f); }

// Workgroups are dispatched round-robin over the 8 XCDs; renumber so that each XCD
// receives a contiguous range of tiles and neighbouring tiles share an L2.
__device__ __forceinline__ int xcd_tile(int bid, int nb) {
  constexpr int NX = 8;
  const int xcd = bid % NX, local = bid / NX;
  const int per = nb / NX, rem = nb % NX;
  return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

// ------------------------------------------------------------------ convolution
// out[p][co] = sum_k W[co][k] X_k[p] for the D x H x W voxel grid.  The input is
// either one tensor (CA = 0) or the concatenation of a half-resolution tensor A
// (CA channels, read at (z>>1, y>>1, x>>1): nearest upsampling) and a
// full-resolution tensor B (CIN - CA channels).  OUTF = false: out = relu(acc +
// bias) in BF16; OUTF = true: out = acc in FP32 (backward data pass).
//
// A block computes a 16 x 4 x 4 (x, y, z) brick of output voxels, one z-plane per
// wave, four 16-voxel rows per wave.  The 18 x 6 x 6 input brick is staged in LDS
// CC channels at a time (channel-group major, so the 16 lanes of one MFMA row group
// read one contiguous 256-byte LDS line), and all 27 taps read their A fragments from it: each
// input value is fetched from memory about 2.5 times instead of 27.  The weights
// are ordered (channel chunk, tap, channel) to match: one 32-wide k step covers
// 32 / CC taps of one chunk.
constexpr int kCTX = 16, kCTY = 4, kCTZ = 4;

template <int CIN, int COUT, int CA, bool OUTF>
__global__ __launch_bounds__(kBlock) void k_conv(const bf16* __restrict__ srcA, const bf16* __restrict__ srcB,
                                                 const bf16* __restrict__ wt, const float* __restrict__ bias,
                                                 void* __restrict__ out, int D, int H, int W) {
  constexpr int CC = conv_cc(CIN), NCH = CIN / CC, KPC = conv_kpc(CIN), KP = conv_kp(CIN);
  constexpr int NB = COUT / 16, CB = CIN - CA;
  constexpr int PX = kCTX + 2, PY = kCTY + 2, PZ = kCTZ + 2, NV = PX * PY * PZ;
  constexpr int C8 = CC / 8;
  // staged brick, channel-group major: [CC / 8][voxel][8], so 16 consecutive voxels of
  // one channel group are 256 contiguous bytes (one conflict-free LDS read)
  __shared__ __attribute__((aligned(16))) bf16 tile[C8 * NV * 8];
  const int nbx = (W + kCTX - 1) / kCTX, nby = (H + kCTY - 1) / kCTY;
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  const int x0 = (t % nbx) * kCTX, y0 = ((t / nbx) % nby) * kCTY, z0 = (t / (nbx * nby)) * kCTZ;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63, g = lane >> 4, r16 = lane & 15;
  const int H2 = H >> 1, W2 = W >> 1;
  floatx4 acc[4][NB];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[rb][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int ch = 0; ch < NCH; ++ch) {
    // stage the input brick of this channel chunk, 8 channels (16 bytes) per load
    for (int e = tid; e < NV * C8; e += kBlock) {
      const int c8 = e / NV, v = e - (e / NV) * NV;
      const int vx = v % PX, vy = (v / PX) % PY, vz = v / (PX * PY);
      const int gx = x0 - 1 + vx, gy = y0 - 1 + vy, gz = z0 - 1 + vz;
      const bool ok = (unsigned)gx < (unsigned)W && (unsigned)gy < (unsigned)H && (unsigned)gz < (unsigned)D;
      const int xc = ok ? gx : 0, yc = ok ? gy : 0, zc = ok ? gz : 0;
      const int ci = ch * CC + 8 * c8;
      const bf16* ptr;
      if (CA > 0 && ci < CA)
        ptr = srcA + (((long)(zc >> 1) * H2 + (yc >> 1)) * W2 + (xc >> 1)) * CA + ci;
      else
        ptr = srcB + (((long)zc * H + yc) * W + xc) * CB + (ci - CA);
      *reinterpret_cast<bf16x8*>(&tile[(c8 * NV + v) * 8]) = load8(ptr, ok);
    }
    __syncthreads();
    const bf16* wch = wt + (long)r16 * KP + ch * KPC + 8 * g;
    // A fragments (LDS) of step s + 1 and B fragments (weights, from L1/L2) of step
    // s + 3 are fetched while step s's MFMAs run
    constexpr int NS = KPC / 32, BD = 4;
    auto fetch_a = [&](int s, bf16x8 (&a)[4]) {
      // padding steps (tap >= 27) read tap 0: their weights are zero and staged values finite
      const int k = 32 * s + 8 * g;
      const int tap = k / CC, ci = k - (k / CC) * CC;
      const int tc = tap < 27 ? tap : 0;
      const int dz = tc / 9, dy = (tc / 3) % 3, dx = tc % 3;  // offsets + 1 into the padded brick
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) {
        const int v = ((wv + dz) * PY + (rb + dy)) * PX + (r16 + dx);
        a[rb] = *reinterpret_cast<const bf16x8*>(&tile[((ci >> 3) * NV + v) * 8]);
      }
    };
    bf16x8 bq[BD][NB];
#pragma unroll
    for (int s = 0; s < BD - 1; ++s)
      if (s < NS)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) bq[s][nb] = *reinterpret_cast<const bf16x8*>(wch + (long)nb * 16 * KP + 32 * s);
    bf16x8 a0[4], a1[4];
    fetch_a(0, a0);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      bf16x8(&ac)[4] = (s & 1) ? a1 : a0;
      bf16x8(&an)[4] = (s & 1) ? a0 : a1;
      if (s + 1 < NS) fetch_a(s + 1, an);
      if (s + BD - 1 < NS)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          bq[(s + BD - 1) % BD][nb] = *reinterpret_cast<const bf16x8*>(wch + (long)nb * 16 * KP + 32 * (s + BD - 1));
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
          acc[rb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ac[rb], bq[s % BD][nb], acc[rb][nb], 0, 0, 0);
    }
    __syncthreads();
  }
  // result rows 4g + j of a 16-voxel row are x0 + 4g + j; columns are channels
  const int z = z0 + wv;
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    const int y = y0 + rb;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int x = x0 + 4 * g + j;
      if (x >= W || y >= H || z >= D) continue;
      const long p = ((long)z * H + y) * W + x;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int co = nb * 16 + r16;
        if (OUTF) {
          static_cast<float*>(out)[p * COUT + co] = acc[rb][nb][j];
        } else {
          const float val = acc[rb][nb][j] + bias[co];
          static_cast<bf16*>(out)[p * COUT + co] = f2bf(val > 0.f ? val : 0.f);
        }
      }
    }
  }
}

// ------------------------------------------------ convolution, input rows shared by taps
// The same implicit GEMM for layers with at least 32 input channels, ordered so that one
// A fragment (16 consecutive input voxels of one (y, z) row, 32 channels) feeds every
// output row of the wave that reads it through some tap (dy, dz): a block computes a
// 16 x 4 x 4 TZW (x, y, z) brick, wave w the planes TZW w .. TZW w + TZW - 1, and for each
// x offset of the taps the wave keeps the 9 (dy, dz) weight fragments of that offset in
// registers and walks the (TZW + 2) x 6 input rows once, issuing up to 3 TZW MFMAs per
// fragment it reads from LDS (k_conv reads one fragment per MFMA).  The reduction index
// is (chunk of 32 channels, tap, channel), channels padded with zeros to a multiple of 32
// (CINP); weights [chunk][tap][co][32] (k_prep_rows).  Sources and output as in k_conv.
template <int CINP, int CREAL, int COUT, int CA, int TZW>
__global__ __launch_bounds__(kBlock) void k_conv_rows(const bf16* __restrict__ srcA, const bf16* __restrict__ srcB,
                                                      const bf16* __restrict__ wt, const float* __restrict__ bias,
                                                      bf16* __restrict__ out, int D, int H, int W) {
  constexpr int TX = 16, TY = 4, TZ = 4 * TZW;
  constexpr int PX = TX + 2, PY = TY + 2, PZ = TZ + 2, NV = PX * PY * PZ;
  constexpr int NB = COUT / 16, NCH = CINP / 32, CB = CREAL - CA;
  static_assert(CINP % 32 == 0 && CREAL <= CINP && COUT % 16 == 0, "channel layout");
  // staged brick of one 32-channel chunk, channel-group major ([4][voxel][8]) as in k_conv
  __shared__ __attribute__((aligned(16))) bf16 tile[4 * NV * 8];
  const int nbx = (W + TX - 1) / TX, nby = (H + TY - 1) / TY;
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  const int x0 = (t % nbx) * TX, y0 = ((t / nbx) % nby) * TY, z0 = (t / (nbx * nby)) * TZ;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63, g = lane >> 4, r16 = lane & 15;
  const int H2 = H >> 1, W2 = W >> 1;
  floatx4 acc[TZW][4][NB];
#pragma unroll
  for (int a = 0; a < TZW; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[a][b][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int ch = 0; ch < NCH; ++ch) {
    for (int e = tid; e < NV * 4; e += kBlock) {
      const int c8 = e / NV, v = e - c8 * NV;
      const int vx = v % PX, vy = (v / PX) % PY, vz = v / (PX * PY);
      const int gx = x0 - 1 + vx, gy = y0 - 1 + vy, gz = z0 - 1 + vz;
      const int ci = ch * 32 + 8 * c8;
      // outside the grid, and the padding channels, stage zeros (read from a valid address)
      const bool ok = (unsigned)gx < (unsigned)W && (unsigned)gy < (unsigned)H && (unsigned)gz < (unsigned)D &&
                      ci < CREAL;
      const int xc = ok ? gx : 0, yc = ok ? gy : 0, zc = ok ? gz : 0;
      const bf16* ptr;
      if (CA > 0 && ci < CA)
        ptr = srcA + (((long)(zc >> 1) * H2 + (yc >> 1)) * W2 + (xc >> 1)) * CA + ci;
      else
        ptr = srcB + (((long)zc * H + yc) * W + xc) * CB + (ok ? ci - CA : 0);
      *reinterpret_cast<bf16x8*>(&tile[(c8 * NV + v) * 8]) = load8(ptr, ok);
    }
    __syncthreads();
#pragma unroll
    for (int dxi = 0; dxi < 3; ++dxi) {
      bf16x8 bq[9][NB];  // taps (dz, dy) at x offset dxi - 1, q = 3 dz + dy (offsets + 1)
#pragma unroll
      for (int q = 0; q < 9; ++q)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          bq[q][nb] = *reinterpret_cast<const bf16x8*>(wt + ((long)(ch * 27 + 3 * q + dxi) * COUT + nb * 16 + r16) * 32 +
                                                       8 * g);
#pragma unroll
      for (int zz = 0; zz < TZW + 2; ++zz) {
#pragma unroll
        for (int yy = 0; yy < PY; ++yy) {
          const int v = ((TZW * wv + zz) * PY + yy) * PX + r16 + dxi;
          const bf16x8 a = *reinterpret_cast<const bf16x8*>(&tile[(g * NV + v) * 8]);
#pragma unroll
          for (int oz = 0; oz < TZW; ++oz) {
            const int dz = zz - oz;
            if (dz < 0 || dz > 2) continue;
#pragma unroll
            for (int oy = 0; oy < 4; ++oy) {
              const int dy = yy - oy;
              if (dy < 0 || dy > 2) continue;
#pragma unroll
              for (int nb = 0; nb < NB; ++nb)
                acc[oz][oy][nb] =
                    __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bq[3 * dz + dy][nb], acc[oz][oy][nb], 0, 0, 0);
            }
          }
        }
      }
    }
    __syncthreads();
  }
  // result rows 4g + j of a 16-voxel row are x0 + 4g + j; columns are channels
#pragma unroll
  for (int oz = 0; oz < TZW; ++oz) {
    const int z = z0 + TZW * wv + oz;
#pragma unroll
    for (int oy = 0; oy < 4; ++oy) {
      const int y = y0 + oy;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int x = x0 + 4 * g + j;
        if (x >= W || y >= H || z >= D) continue;
        const long p = ((long)z * H + y) * W + x;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const int co = nb * 16 + r16;
          const float val = acc[oz][oy][nb][j] + bias[co];
          out[p * COUT + co] = f2bf(val > 0.f ? val : 0.f);
        }
      }
    }
  }
}

// --------------------------------------------------------------- weight gradient
// part[blk][tap][co][CIN] = sum over the block's voxels p of dy[p][co] X_tap[p][ci],
// X_tap[p] = input at p + offset(tap) (zero outside), sources as in k_conv.
// Grid (nblk, 27).  Each wave reduces over 32-voxel slices (MFMA k = voxel), the
// four waves of a block are summed in LDS; the host sums the blocks in order.
template <int CIN, int COUT, int CA>
__global__ __launch_bounds__(kBlock) void k_wgrad(const bf16* __restrict__ srcA, const bf16* __restrict__ srcB,
                                                  const bf16* __restrict__ dy, float* __restrict__ part, int D, int H,
                                                  int W, long vox_per_block) {
  constexpr int MB = COUT / 16;
  constexpr int NC = (CIN + 15) / 16;
  constexpr int CB = CIN - CA;
  __shared__ float red[4][MB * NC * 256];
  const long P = (long)D * H * W;
  const int tap = blockIdx.y;
  const int dz = tap / 9 - 1, ddy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4;
  const int r16 = lane & 15;
  const int H2 = H >> 1, W2 = W >> 1;
  const long p_begin = (long)blockIdx.x * vox_per_block;
  const long p_end = p_begin + vox_per_block < P ? p_begin + vox_per_block : P;
  floatx4 acc[MB][NC];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nc = 0; nc < NC; ++nc) acc[mb][nc] = floatx4{0.f, 0.f, 0.f, 0.f};
  for (long p0 = p_begin + 32 * wave; p0 < p_end; p0 += 128) {
    bf16x8 a[MB], b[NC];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const long p = p0 + 8 * g + j;
      const bool vin = p < p_end;
      const long q = vin ? p : p_begin;
      const int x = (int)(q % W), y = (int)((q / W) % H), z = (int)(q / ((long)W * H));
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        const bf16 v = dy[q * COUT + mb * 16 + r16];
        a[mb][j] = vin ? v : f2bf(0.f);
      }
      const int zz = z + dz, yy = y + ddy, xx = x + dx;
      const bool ok = vin && (unsigned)zz < (unsigned)D && (unsigned)yy < (unsigned)H && (unsigned)xx < (unsigned)W;
      const int zc = ok ? zz : 0, yc = ok ? yy : 0, xc = ok ? xx : 0;
#pragma unroll
      for (int nc = 0; nc < NC; ++nc) {
        const int ci = nc * 16 + r16;
        const bool cok = ok && ci < CIN;
        const int cc = ci < CIN ? ci : 0;
        const bf16* ptr;
        if (CA > 0 && cc < CA)
          ptr = srcA + (((long)(zc >> 1) * H2 + (yc >> 1)) * W2 + (xc >> 1)) * CA + cc;
        else
          ptr = srcB + (((long)zc * H + yc) * W + xc) * CB + (cc - CA);
        const bf16 v = *ptr;
        b[nc][j] = cok ? v : f2bf(0.f);
      }
    }
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nc = 0; nc < NC; ++nc) acc[mb][nc] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mb], b[nc], acc[mb][nc], 0, 0, 0);
  }
  // result tile (mb, nc): lane holds rows co = mb*16 + 4g + j, column ci = nc*16 + r16
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nc = 0; nc < NC; ++nc)
#pragma unroll
      for (int j = 0; j < 4; ++j) red[wave][(mb * NC + nc) * 256 + (4 * g + j) * 16 + r16] = acc[mb][nc][j];
  __syncthreads();
  float* dst = part + ((long)blockIdx.x * 27 + tap) * COUT * CIN;
  for (int e = threadIdx.x; e < MB * NC * 256; e += kBlock) {
    const int tile = e >> 8, within = e & 255;
    const int mb = tile / NC, nc = tile % NC;
    const int co = mb * 16 + (within >> 4), ci = nc * 16 + (within & 15);
    if (ci < CIN) dst[co * CIN + ci] = red[0][e] + red[1][e] + red[2][e] + red[3][e];
  }
}

// grad[(co*27 + tap)*cin_real + ci] = sum_b part[b][tap][co][ci] (fixed order)
__global__ void k_wgrad_reduce(const float* __restrict__ part, float* __restrict__ grad, int nblk, int cout, int cin,
                               int cin_real) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= cout * 27 * cin_real) return;
  const int ci = e % cin_real;
  const int tap = (e / cin_real) % 27;
  const int co = e / (cin_real * 27);
  float s = 0.f;
  for (int b = 0; b < nblk; ++b) s += part[(((long)b * 27 + tap) * cout + co) * cin + ci];
  grad[e] = s;
}

// per-block channel sums of a [P][C] BF16 tensor (C divides 256)
__global__ __launch_bounds__(kBlock) void k_colsum(const bf16* __restrict__ x, float* __restrict__ part, long P, int C,
                                                   long vox_per_block) {
  __shared__ float sm[kBlock];
  const long e0 = (long)blockIdx.x * vox_per_block * C;
  long e1 = e0 + vox_per_block * C;
  if (e1 > P * C) e1 = P * C;
  float s = 0.f;
  for (long e = e0 + threadIdx.x; e < e1; e += kBlock) s += bf2f(x[e]);
  sm[threadIdx.x] = s;
  __syncthreads();
  if ((int)threadIdx.x < C) {
    float t = 0.f;
    for (int q = threadIdx.x; q < kBlock; q += C) t += sm[q];
    part[(long)blockIdx.x * C + threadIdx.x] = t;
  }
}

// dst[c] = sum_b part[b][c]
__global__ void k_part_reduce(const float* __restrict__ part, float* __restrict__ dst, int nblk, int C) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  float s = 0.f;
  for (int b = 0; b < nblk; ++b) s += part[(long)b * C + c];
  dst[c] = s;
}

// ------------------------------------------------------------ pooling, skips
__global__ void k_pool(const bf16* __restrict__ x, bf16* __restrict__ y, int D, int H, int W, int C) {
  // y [D/2][H/2][W/2][C] = 2x2x2 mean of x [D][H][W][C]
  const long n = (long)(D / 2) * (H / 2) * (W / 2) * C;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int c = (int)(e % C);
  const long q = e / C;
  const int W2 = W / 2, H2 = H / 2;
  const int x2 = (int)(q % W2), y2 = (int)((q / W2) % H2), z2 = (int)(q / ((long)W2 * H2));
  float s = 0.f;
#pragma unroll
  for (int o = 0; o < 8; ++o) {
    const int z = 2 * z2 + (o >> 2), yy = 2 * y2 + ((o >> 1) & 1), xx = 2 * x2 + (o & 1);
    s += bf2f(x[(((long)z * H + yy) * W + xx) * C + c]);
  }
  y[e] = f2bf(0.125f * s);
}

// dd[q][c] = (sum of dc[child][c] over the 8 children of half-res voxel q) * (act[q][c] > 0),
// c < CA; dc is [D][H][W][CT] FP32 (full resolution), dd and act [D/2][H/2][W/2][CA].
__global__ void k_upback_mask(const float* __restrict__ dc, const bf16* __restrict__ act, bf16* __restrict__ dd, int D,
                              int H, int W, int CT, int CA) {
  const long n = (long)(D / 2) * (H / 2) * (W / 2) * CA;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int c = (int)(e % CA);
  const long q = e / CA;
  const int W2 = W / 2, H2 = H / 2;
  const int x2 = (int)(q % W2), y2 = (int)((q / W2) % H2), z2 = (int)(q / ((long)W2 * H2));
  float s = 0.f;
#pragma unroll
  for (int o = 0; o < 8; ++o) {
    const int z = 2 * z2 + (o >> 2), yy = 2 * y2 + ((o >> 1) & 1), xx = 2 * x2 + (o & 1);
    s += dc[(((long)z * H + yy) * W + xx) * CT + c];
  }
  dd[e] = f2bf(bf2f(act[e]) > 0.f ? s : 0.f);
}

// de[p][c] = (dc[p][CA + c] + dp[parent(p)][c] / 8) * (act[p][c] > 0): the skip branch
// plus the backward of the average pooling, masked by the encoder activation.
__global__ void k_skip_mask(const float* __restrict__ dc, const float* __restrict__ dp, const bf16* __restrict__ act,
                            bf16* __restrict__ de, int D, int H, int W, int CT, int CA, int CB) {
  const long n = (long)D * H * W * CB;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int c = (int)(e % CB);
  const long p = e / CB;
  const int x = (int)(p % W), y = (int)((p / W) % H), z = (int)(p / ((long)W * H));
  const long par = (((long)(z >> 1) * (H >> 1) + (y >> 1)) * (W >> 1) + (x >> 1)) * CB + c;
  const float s = dc[p * CT + CA + c] + 0.125f * dp[par];
  de[e] = f2bf(bf2f(act[e]) > 0.f ? s : 0.f);
}

// ------------------------------------------------------------------ head, loss
// y[p] = b + sum_c w[c] d1[p][c]   (16 channels)
__global__ void k_head_fwd(const bf16* __restrict__ d1, const float* __restrict__ wb, float* __restrict__ y, long P) {
  const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const u32x4* src = reinterpret_cast<const u32x4*>(d1 + p * 16);
  const bf16x8 a = __builtin_bit_cast(bf16x8, src[0]);
  const bf16x8 b = __builtin_bit_cast(bf16x8, src[1]);
  float s = wb[16];
#pragma unroll
  for (int c = 0; c < 8; ++c) s += wb[c] * bf2f(a[c]) + wb[8 + c] * bf2f(b[c]);
  y[p] = s;
}

// dy[p] = 2 (y - t) / P; per-block partial sums of (y - t)^2
__global__ __launch_bounds__(kBlock) void k_loss(const float* __restrict__ y, const float* __restrict__ t,
                                                 float* __restrict__ dy, double* __restrict__ part, long P) {
  __shared__ double sm[kBlock];
  double s = 0.0;
  for (long p = (long)blockIdx.x * kBlock + threadIdx.x; p < P; p += (long)gridDim.x * kBlock) {
    const float d = y[p] - t[p];
    dy[p] = 2.f * d / (float)P;
    s += (double)d * d;
  }
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

// dd1[p][c] = dy[p] w[c] (d1[p][c] > 0); per-block partials of dy*d1 (16) and dy (1)
__global__ __launch_bounds__(kBlock) void k_head_bwd(const bf16* __restrict__ d1, const float* __restrict__ wb,
                                                     const float* __restrict__ dy, bf16* __restrict__ dd1,
                                                     float* __restrict__ part, long P) {
  __shared__ float sm[17][kBlock];
  float s[17];
#pragma unroll
  for (int c = 0; c < 17; ++c) s[c] = 0.f;
  for (long p = (long)blockIdx.x * kBlock + threadIdx.x; p < P; p += (long)gridDim.x * kBlock) {
    const float g = dy[p];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      const float a = bf2f(d1[p * 16 + c]);
      s[c] += g * a;
      dd1[p * 16 + c] = f2bf(a > 0.f ? g * wb[c] : 0.f);
    }
    s[16] += g;
  }
#pragma unroll
  for (int c = 0; c < 17; ++c) sm[c][threadIdx.x] = s[c];
  __syncthreads();
  if ((int)threadIdx.x < 17) {
    float t = 0.f;
    for (int q = 0; q < kBlock; ++q) t += sm[threadIdx.x][q];
    part[(long)blockIdx.x * 17 + threadIdx.x] = t;
  }
}

// -------------------------------------------------------------------- Adam
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, long n, float lr, float b1, float b2, float eps, float bc1, float bc2) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// BF16 GEMM weights of a 3x3x3 layer from its FP32 master W[co][27][cin_real], in
// the (channel chunk, tap, channel) order of k_conv: forward [cout][conv_kp(cinp)] (the
// layers with fewer than 32 input channels; k_prep_rows makes the others');
// transposed-flipped for the backward data pass [cin][conv_kp(cout)] holding
// W[co][26 - tap][ci] at (chunk of co, tap, co).
__global__ void k_prep_fwd(const float* __restrict__ w, bf16* __restrict__ out, int cout, int cinp, int cin_real) {
  const int CC = conv_cc(cinp), KPC = conv_kpc(cinp), KP = conv_kp(cinp);
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)cout * KP) return;
  const int k = (int)(e % KP), co = (int)(e / KP);
  const int ch = k / KPC, r = k % KPC;
  const int tap = r / CC, ci = ch * CC + r % CC;
  out[e] = f2bf(tap < 27 && ci < cin_real ? w[((long)co * 27 + tap) * cin_real + ci] : 0.f);
}

// BF16 weights of k_conv_rows: [chunk][tap][co][32] holding W[co][tap][32 chunk + c]
// (zero for padding channels).
__global__ void k_prep_rows(const float* __restrict__ w, bf16* __restrict__ out, int cout, int cinp, int cin_real) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= conv_wf_elems(cout, cinp)) return;
  const int c = (int)(e % 32), co = (int)((e / 32) % cout), tap = (int)((e / (32L * cout)) % 27);
  const int ch = (int)(e / (32L * cout * 27));
  const int ci = ch * 32 + c;
  out[e] = f2bf(ci < cin_real ? w[((long)co * 27 + tap) * cin_real + ci] : 0.f);
}

__global__ void k_prep_bwd(const float* __restrict__ w, bf16* __restrict__ out, int cout, int cin) {
  const int CC = conv_cc(cout), KPC = conv_kpc(cout), KP = conv_kp(cout);
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)cin * KP) return;
  const int k = (int)(e % KP), ci = (int)(e / KP);
  const int ch = k / KPC, r = k % KPC;
  const int tap = r / CC, co = ch * CC + r % CC;
  out[e] = f2bf(tap < 27 ? w[((long)co * 27 + (26 - tap)) * cin + ci] : 0.f);
}

// ------------------------------------------------------- fields <-> network
__device__ __forceinline__ double cell_vol(const GridDev& g, int i, int j, int k) {
  return g.x.d[i] * g.y.d[j] * g.z.d[k];
}

// per-block partials of sum V |w at centre|^2 and sum V r^2
__global__ __launch_bounds__(kBlock) void k_feat_sums(GridDev g, const double* __restrict__ w,
                                                      const double* __restrict__ r, double* __restrict__ part) {
  __shared__ double sa[kBlock], sb[kBlock];
  const int nx = g.x.n, ny = g.y.n, nz = g.z.n;
  const long n = (long)nx * ny * nz;
  const double* u = w;
  const double* v = w + (long)(nx + 1) * ny * nz;
  const double* ww = v + (long)nx * (ny + 1) * nz;
  double a = 0.0, b = 0.0;
  for (long e = (long)blockIdx.x * kBlock + threadIdx.x; e < n; e += (long)gridDim.x * kBlock) {
    const int i = (int)(e % nx), j = (int)((e / nx) % ny), k = (int)(e / ((long)nx * ny));
    const double cx = 0.5 * (u[((long)k * ny + j) * (nx + 1) + i] + u[((long)k * ny + j) * (nx + 1) + i + 1]);
    const double cy = 0.5 * (v[((long)k * (ny + 1) + j) * nx + i] + v[((long)k * (ny + 1) + j + 1) * nx + i]);
    const double cz = 0.5 * (ww[((long)k * ny + j) * nx + i] + ww[((long)(k + 1) * ny + j) * nx + i]);
    const double V = cell_vol(g, i, j, k);
    a += V * (cx * cx + cy * cy + cz * cz);
    b += V * r[e] * r[e];
  }
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sa[threadIdx.x] += sa[threadIdx.x + o];
      sb[threadIdx.x] += sb[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sa[0];
    part[2 * blockIdx.x + 1] = sb[0];
  }
}

// x[Dp][Hp][Wp][8] = (w_x, w_y, w_z) / sw, r / sr, 0, 0, 0, 0 on cells; zeros in the padding
__global__ void k_feat_pack(GridDev g, const double* __restrict__ w, const double* __restrict__ r, bf16* __restrict__ x,
                            int Dp, int Hp, int Wp, double isw, double isr) {
  const int nx = g.x.n, ny = g.y.n, nz = g.z.n;
  const long P = (long)Dp * Hp * Wp;
  const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const int i = (int)(p % Wp), j = (int)((p / Wp) % Hp), k = (int)(p / ((long)Wp * Hp));
  bf16x8 o;
#pragma unroll
  for (int c = 0; c < 8; ++c) o[c] = f2bf(0.f);
  if (i < nx && j < ny && k < nz) {
    const double* u = w;
    const double* v = w + (long)(nx + 1) * ny * nz;
    const double* ww = v + (long)nx * (ny + 1) * nz;
    const double cx = 0.5 * (u[((long)k * ny + j) * (nx + 1) + i] + u[((long)k * ny + j) * (nx + 1) + i + 1]);
    const double cy = 0.5 * (v[((long)k * (ny + 1) + j) * nx + i] + v[((long)k * (ny + 1) + j + 1) * nx + i]);
    const double cz = 0.5 * (ww[((long)k * ny + j) * nx + i] + ww[((long)(k + 1) * ny + j) * nx + i]);
    o[0] = f2bf((float)(cx * isw));
    o[1] = f2bf((float)(cy * isw));
    o[2] = f2bf((float)(cz * isw));
    o[3] = f2bf((float)(r[((long)k * ny + j) * nx + i] * isr));
  }
  *reinterpret_cast<u32x4*>(x + p * 8) = __builtin_bit_cast(u32x4, o);
}

// x8[p][0..7] = (x4[p][0..3], 0, 0, 0, 0) in BF16
__global__ void k_x4_to_x8(const float* __restrict__ x4, bf16* __restrict__ x8, long P) {
  const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  bf16x8 o;
#pragma unroll
  for (int c = 0; c < 8; ++c) o[c] = f2bf(c < 4 ? x4[p * 4 + c] : 0.f);
  *reinterpret_cast<u32x4*>(x8 + p * 8) = __builtin_bit_cast(u32x4, o);
}

// physical cells of the network output, times s: phi[k][j][i] = s y[k][j][i]
__global__ void k_unpack(const float* __restrict__ y, double* __restrict__ phi, int nx, int ny, int nz, int Hp, int Wp,
                         double s) {
  const long n = (long)nx * ny * nz;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int i = (int)(e % nx), j = (int)((e / nx) % ny), k = (int)(e / ((long)nx * ny));
  phi[e] = s * (double)y[((long)k * Hp + j) * Wp + i];
}

// training target t = phi * s on cells, 0 in the padding
__global__ void k_target(const double* __restrict__ phi, float* __restrict__ t, int nx, int ny, int nz, int Dp, int Hp,
                         int Wp, double s) {
  const long P = (long)Dp * Hp * Wp;
  const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const int i = (int)(p % Wp), j = (int)((p / Wp) % Hp), k = (int)(p / ((long)Wp * Hp));
  t[p] = (i < nx && j < ny && k < nz) ? (float)(s * phi[((long)k * ny + j) * nx + i]) : 0.f;
}

// per-block partials of sum V a^2, sum V a b, sum V b^2 over cells
__global__ __launch_bounds__(kBlock) void k_vdot3(GridDev g, const double* __restrict__ a,
                                                  const double* __restrict__ b, double* __restrict__ part) {
  __shared__ double s[3][kBlock];
  const int nx = g.x.n, ny = g.y.n, nz = g.z.n;
  const long n = (long)nx * ny * nz;
  double aa = 0.0, ab = 0.0, bb = 0.0;
  for (long e = (long)blockIdx.x * kBlock + threadIdx.x; e < n; e += (long)gridDim.x * kBlock) {
    const int i = (int)(e % nx), j = (int)((e / nx) % ny), k = (int)(e / ((long)nx * ny));
    const double V = cell_vol(g, i, j, k);
    aa += V * a[e] * a[e];
    ab += V * a[e] * b[e];
    bb += V * b[e] * b[e];
  }
  s[0][threadIdx.x] = aa;
  s[1][threadIdx.x] = ab;
  s[2][threadIdx.x] = bb;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int q = 0; q < 3; ++q) s[q][threadIdx.x] += s[q][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int q = 0; q < 3; ++q) part[3 * blockIdx.x + q] = s[q][0];
}

unsigned blocks(long n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

}  // namespace

// ------------------------------------------------------------------ launchers
hipError_t nn_conv(int layer, bool backward, const bf16* a, const bf16* b, const bf16* wt, const float* bias, void* out,
                   int D, int H, int W, hipStream_t st) {
  const long tiles = (long)((W + kCTX - 1) / kCTX) * ((H + kCTY - 1) / kCTY) * ((D + kCTZ - 1) / kCTZ);
  const dim3 grid((unsigned)tiles), blk(kBlock);  // one 16 x 4 x 4 output brick per block
#define CONV(CIN, COUT, CA, OUTF) \
  hipLaunchKernelGGL((k_conv<CIN, COUT, CA, OUTF>), grid, blk, 0, st, a, b, wt, bias, out, D, H, W)
  // k_conv_rows bricks: 16 x 4 x 4 TZW voxels per block
  auto rows_grid = [&](int tzw) {
    return dim3((unsigned)((long)((W + 15) / 16) * ((H + 3) / 4) * ((D + 4 * tzw - 1) / (4 * tzw))));
  };
#define ROWS(CINP, CREAL, COUT, CA, TZW)                                                                          \
  hipLaunchKernelGGL((k_conv_rows<CINP, CREAL, COUT, CA, TZW>), rows_grid(TZW), blk, 0, st, a, b, wt, bias, \
                     static_cast<bf16*>(out), D, H, W)
  if (!backward) {
    switch (layer) {
      case 0: CONV(8, 16, 0, false); break;
      case 1: CONV(16, 32, 0, false); break;
      case 2: ROWS(32, 32, 64, 0, 1); break;  // quarter resolution: the smaller brick keeps more blocks
      case 3: ROWS(96, 96, 32, 64, 2); break;
      case 4: ROWS(64, 48, 16, 32, 2); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (layer) {
      case 1: CONV(32, 16, 0, true); break;
      case 2: CONV(64, 32, 0, true); break;
      case 3: CONV(32, 96, 0, true); break;
      case 4: CONV(16, 48, 0, true); break;
      default: return hipErrorInvalidValue;
    }
  }
#undef CONV
#undef ROWS
  return hipGetLastError();
}

hipError_t nn_wgrad(int layer, const bf16* a, const bf16* b, const bf16* dy, float* part, int nblk, int D, int H, int W,
                    hipStream_t st) {
  const long P = (long)D * H * W;
  const long vpb = ((P + nblk - 1) / nblk + 31) / 32 * 32;
  const dim3 grid(nblk, 27), blk(kBlock);
#define WG(CIN, COUT, CA) hipLaunchKernelGGL((k_wgrad<CIN, COUT, CA>), grid, blk, 0, st, a, b, dy, part, D, H, W, vpb)
  switch (layer) {
    case 0: WG(8, 16, 0); break;
    case 1: WG(16, 32, 0); break;
    case 2: WG(32, 64, 0); break;
    case 3: WG(96, 32, 64); break;
    case 4: WG(48, 16, 32); break;
    default: return hipErrorInvalidValue;
  }
#undef WG
  return hipGetLastError();
}

hipError_t nn_wgrad_reduce(const float* part, float* grad, int nblk, int cout, int cin, int cin_real, hipStream_t st) {
  hipLaunchKernelGGL(k_wgrad_reduce, dim3(blocks((long)cout * 27 * cin_real)), dim3(kBlock), 0, st, part, grad, nblk,
                     cout, cin, cin_real);
  return hipGetLastError();
}

hipError_t nn_colsum(const bf16* x, float* part, float* dst, long P, int C, int nblk, hipStream_t st) {
  const long vpb = (P + nblk - 1) / nblk;
  hipLaunchKernelGGL(k_colsum, dim3(nblk), dim3(kBlock), 0, st, x, part, P, C, vpb);
  hipLaunchKernelGGL(k_part_reduce, dim3(1), dim3(64), 0, st, part, dst, nblk, C);
  return hipGetLastError();
}

hipError_t nn_pool(const bf16* x, bf16* y, int D, int H, int W, int C, hipStream_t st) {
  hipLaunchKernelGGL(k_pool, dim3(blocks((long)(D / 2) * (H / 2) * (W / 2) * C)), dim3(kBlock), 0, st, x, y, D, H, W, C);
  return hipGetLastError();
}

hipError_t nn_upback_mask(const float* dc, const bf16* act, bf16* dd, int D, int H, int W, int CT, int CA,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_upback_mask, dim3(blocks((long)(D / 2) * (H / 2) * (W / 2) * CA)), dim3(kBlock), 0, st, dc, act,
                     dd, D, H, W, CT, CA);
  return hipGetLastError();
}

hipError_t nn_skip_mask(const float* dc, const float* dp, const bf16* act, bf16* de, int D, int H, int W, int CT, int CA,
                        int CB, hipStream_t st) {
  hipLaunchKernelGGL(k_skip_mask, dim3(blocks((long)D * H * W * CB)), dim3(kBlock), 0, st, dc, dp, act, de, D, H, W, CT,
                     CA, CB);
  return hipGetLastError();
}

hipError_t nn_head_fwd(const bf16* d1, const float* wb, float* y, long P, hipStream_t st) {
  hipLaunchKernelGGL(k_head_fwd, dim3(blocks(P)), dim3(kBlock), 0, st, d1, wb, y, P);
  return hipGetLastError();
}

hipError_t nn_loss(const float* y, const float* t, float* dy, double* part, int nblk, long P, hipStream_t st) {
  hipLaunchKernelGGL(k_loss, dim3(nblk), dim3(kBlock), 0, st, y, t, dy, part, P);
  return hipGetLastError();
}

hipError_t nn_head_bwd(const bf16* d1, const float* wb, const float* dy, bf16* dd1, float* part, float* gdst, int nblk,
                       long P, hipStream_t st) {
  hipLaunchKernelGGL(k_head_bwd, dim3(nblk), dim3(kBlock), 0, st, d1, wb, dy, dd1, part, P);
  hipLaunchKernelGGL(k_part_reduce, dim3(1), dim3(64), 0, st, part, gdst, nblk, 17);
  return hipGetLastError();
}

hipError_t nn_adam(float* w, const float* g, float* m, float* v, long n, float lr, float b1, float b2, float eps,
                   float bc1, float bc2, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3(blocks(n)), dim3(kBlock), 0, st, w, g, m, v, n, lr, b1, b2, eps, bc1, bc2);
  return hipGetLastError();
}

hipError_t nn_prep(const float* w, bf16* fwd, bf16* bwd, int cout, int cinp, int cin_real, hipStream_t st) {
  if (conv_rows(cinp))
    hipLaunchKernelGGL(k_prep_rows, dim3(blocks(conv_wf_elems(cout, cinp))), dim3(kBlock), 0, st, w, fwd, cout, cinp,
                       cin_real);
  else
    hipLaunchKernelGGL(k_prep_fwd, dim3(blocks(conv_wf_elems(cout, cinp))), dim3(kBlock), 0, st, w, fwd, cout, cinp,
                       cin_real);
  if (bwd) {
    const int KPt = conv_kp(cout);
    hipLaunchKernelGGL(k_prep_bwd, dim3(blocks((long)cin_real * KPt)), dim3(kBlock), 0, st, w, bwd, cout, cin_real);
  }
  return hipGetLastError();
}

hipError_t nn_feat_sums(const GridDev& g, const double* w, const double* r, double* part, int nblk, hipStream_t st) {
  hipLaunchKernelGGL(k_feat_sums, dim3(nblk), dim3(kBlock), 0, st, g, w, r, part);
  return hipGetLastError();
}

hipError_t nn_feat_pack(const GridDev& g, const double* w, const double* r, bf16* x, int Dp, int Hp, int Wp, double isw,
                        double isr, hipStream_t st) {
  hipLaunchKernelGGL(k_feat_pack, dim3(blocks((long)Dp * Hp * Wp)), dim3(kBlock), 0, st, g, w, r, x, Dp, Hp, Wp, isw,
                     isr);
  return hipGetLastError();
}

hipError_t nn_x4_to_x8(const float* x4, bf16* x8, long P, hipStream_t st) {
  hipLaunchKernelGGL(k_x4_to_x8, dim3(blocks(P)), dim3(kBlock), 0, st, x4, x8, P);
  return hipGetLastError();
}

hipError_t nn_unpack(const float* y, double* phi, int nx, int ny, int nz, int Hp, int Wp, double s, hipStream_t st) {
  hipLaunchKernelGGL(k_unpack, dim3(blocks((long)nx * ny * nz)), dim3(kBlock), 0, st, y, phi, nx, ny, nz, Hp, Wp, s);
  return hipGetLastError();
}

hipError_t nn_target(const double* phi, float* t, int nx, int ny, int nz, int Dp, int Hp, int Wp, double s,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_target, dim3(blocks((long)Dp * Hp * Wp)), dim3(kBlock), 0, st, phi, t, nx, ny, nz, Dp, Hp, Wp, s);
  return hipGetLastError();
}

hipError_t nn_vdot3(const GridDev& g, const double* a, const double* b, double* part, int nblk, hipStream_t st) {
  hipLaunchKernelGGL(k_vdot3, dim3(nblk), dim3(kBlock), 0, st, g, a, b, part);
  return hipGetLastError();
}

}  // namespace lk
