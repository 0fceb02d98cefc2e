// Launchers of the network kernels (lk_nn.hip) used by the host driver (lk_nn_host.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include "lk_internal.h"

namespace lk {

typedef __bf16 bf16;

// GEMM reduction layout of a 3x3x3 convolution with cin input channels: chunks of
// conv_cc(cin) channels, each holding (tap, channel) pairs padded to a multiple of 32.
__host__ __device__ constexpr int conv_cc(int cin) { return cin <= 16 ? cin : (cin % 32 == 0 ? 32 : 16); }
__host__ __device__ constexpr int conv_kpc(int cin) { return (27 * conv_cc(cin) + 31) / 32 * 32; }
__host__ __device__ constexpr int conv_kp(int cin) { return cin / conv_cc(cin) * conv_kpc(cin); }
// Forward layers with at least 32 input channels run k_conv_rows: reduction index (chunk of
// 32 channels, tap, channel), the channels zero-padded to a multiple of 32.
__host__ __device__ constexpr bool conv_rows(int cin) { return cin >= 32; }
// elements of a layer's forward BF16 weights in the layout of its kernel
__host__ __device__ constexpr long conv_wf_elems(int cout, int cin) {
  return conv_rows(cin) ? 27L * cout * ((cin + 31) / 32 * 32) : (long)cout * conv_kp(cin);
}

// 3x3x3 convolution of layer `layer` (0 enc1, 1 enc2, 2 bottleneck, 3 dec2, 4 dec1).
// Forward: out = relu(conv(in) + bias) in BF16; `a` is the half-resolution source of
// a decoder's concatenated input (nullptr otherwise), `b` the full-resolution one.
// Backward (layers 1-4): the data gradient, conv with transposed-flipped weights, in
// FP32; the input is the masked output gradient passed as `b`.
hipError_t nn_conv(int layer, bool backward, const bf16* a, const bf16* b, const bf16* wt, const float* bias, void* out,
                   int D, int H, int W, hipStream_t st);
// per-block partial weight gradients of layer `layer` ([nblk][27][cout][cin])
hipError_t nn_wgrad(int layer, const bf16* a, const bf16* b, const bf16* dy, float* part, int nblk, int D, int H, int W,
                    hipStream_t st);
hipError_t nn_wgrad_reduce(const float* part, float* grad, int nblk, int cout, int cin, int cin_real, hipStream_t st);
// channel sums of a [P][C] tensor into dst (C divides 256); part holds nblk*C floats
hipError_t nn_colsum(const bf16* x, float* part, float* dst, long P, int C, int nblk, hipStream_t st);
hipError_t nn_pool(const bf16* x, bf16* y, int D, int H, int W, int C, hipStream_t st);
hipError_t nn_upback_mask(const float* dc, const bf16* act, bf16* dd, int D, int H, int W, int CT, int CA,
                          hipStream_t st);
hipError_t nn_skip_mask(const float* dc, const float* dp, const bf16* act, bf16* de, int D, int H, int W, int CT, int CA,
                        int CB, hipStream_t st);
hipError_t nn_head_fwd(const bf16* d1, const float* wb, float* y, long P, hipStream_t st);
hipError_t nn_loss(const float* y, const float* t, float* dy, double* part, int nblk, long P, hipStream_t st);
// gdst receives the 16 weight gradients and the bias gradient of the head
hipError_t nn_head_bwd(const bf16* d1, const float* wb, const float* dy, bf16* dd1, float* part, float* gdst, int nblk,
                       long P, hipStream_t st);
hipError_t nn_adam(float* w, const float* g, float* m, float* v, long n, float lr, float b1, float b2, float eps,
                   float bc1, float bc2, hipStream_t st);
// BF16 GEMM weights (forward and, if bwd != nullptr, backward-data) from FP32 master weights
hipError_t nn_prep(const float* w, bf16* fwd, bf16* bwd, int cout, int cinp, int cin_real, hipStream_t st);
hipError_t nn_feat_sums(const GridDev& g, const double* w, const double* r, double* part, int nblk, hipStream_t st);
hipError_t nn_feat_pack(const GridDev& g, const double* w, const double* r, bf16* x, int Dp, int Hp, int Wp, double isw,
                        double isr, hipStream_t st);
hipError_t nn_x4_to_x8(const float* x4, bf16* x8, long P, hipStream_t st);
hipError_t nn_unpack(const float* y, double* phi, int nx, int ny, int nz, int Hp, int Wp, double s, hipStream_t st);
hipError_t nn_target(const double* phi, float* t, int nx, int ny, int nz, int Dp, int Hp, int Wp, double s,
                     hipStream_t st);
// per-block partials (3 per block) of sum V a^2, sum V a b, sum V b^2 over cells
hipError_t nn_vdot3(const GridDev& g, const double* a, const double* b, double* part, int nblk, hipStream_t st);

}  // namespace lk
