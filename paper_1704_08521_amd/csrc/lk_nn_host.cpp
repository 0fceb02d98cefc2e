// Host driver of the learned pressure-correction guess: the network object
// (FP32 master parameters, Adam moments, BF16 GEMM weights, activations), its
// forward and backward passes on the stream of the caller, training on the
// corrections the SIMPLE projection computes, and the learned start of the
// SIMPLE loop with its least-squares scaling and plain fallback.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "lk_ctx.h"
#include "lk_nn.h"

namespace {

struct LayerDesc {
  int cin, cinp, cout, taps;
};

// enc1, enc2, bottleneck, dec2, dec1, head; master layout per layer: W[cout][taps][cin], b[cout]
constexpr LayerDesc kLayers[6] = {{4, 8, 16, 27},   {16, 16, 32, 27}, {32, 32, 64, 27},
                                  {96, 96, 32, 27}, {48, 48, 16, 27}, {16, 16, 1, 1}};
constexpr int kPartBlocks = 256;   // partial-sum blocks of the small reductions
constexpr int kWgradBlocks = 128;  // voxel chunks of the weight gradient

long woff(int l) {
  long o = 0;
  for (int q = 0; q < l; ++q) o += (long)kLayers[q].cout * kLayers[q].taps * kLayers[q].cin + kLayers[q].cout;
  return o;
}
long boff(int l) { return woff(l) + (long)kLayers[l].cout * kLayers[l].taps * kLayers[l].cin; }
long nparams() { return woff(6); }

uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace

struct lc_net {
  std::string err;
  long np = 0;
  float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;  // device, np each
  lk::bf16* wf[5] = {};                                          // forward GEMM weights
  lk::bf16* wb[5] = {};                                          // backward-data weights (layers 1-4)
  void* wmem = nullptr;
  long step = 0;
  // activations, sized for `cap` full-resolution voxels
  long cap = 0;
  bool cap_train = false;
  void* amem = nullptr;
  lk::bf16 *x8 = nullptr, *e1 = nullptr, *p1 = nullptr, *e2 = nullptr, *p2 = nullptr, *bt = nullptr, *d2 = nullptr,
           *d1 = nullptr;
  float *y = nullptr, *t = nullptr, *dy = nullptr;
  lk::bf16 *dd1 = nullptr, *dd2 = nullptr, *dbt = nullptr, *de2 = nullptr, *de1 = nullptr;
  float *dc1 = nullptr, *dc2 = nullptr, *dp2 = nullptr, *dp1 = nullptr, *part = nullptr;
  double* dpart = nullptr;  // kPartBlocks * 3 doubles
  double* hpart = nullptr;  // pinned mirror
};

namespace lk {
namespace {

int nfail(lc_net* n, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (n) n->err = buf;
  return code;
}

#define NCHK(n, expr)                                                                              \
  do {                                                                                             \
    hipError_t e_ = (expr);                                                                        \
    if (e_ != hipSuccess) return nfail((n), LC_EHIP, "%s: %s", #expr, hipGetErrorString(e_));     \
  } while (0)

size_t al(size_t bytes) { return (bytes + 255) / 256 * 256; }

// (Re)allocate activation buffers for P full-resolution voxels (forward, plus backward if train).
int ensure(lc_net* n, long P, bool train) {
  if (P <= n->cap && (!train || n->cap_train)) return LC_OK;
  if (n->amem) NCHK(n, hipFree(n->amem));
  n->amem = nullptr;
  n->cap = 0;
  const long P2 = P / 8, P4 = P / 64 + 1;
  const size_t B = sizeof(bf16), F = sizeof(float);
  struct Item {
    void** dst;
    size_t bytes;
  };
  std::vector<Item> items = {{(void**)&n->x8, P * 8 * B},  {(void**)&n->e1, P * 16 * B},  {(void**)&n->p1, P2 * 16 * B},
                             {(void**)&n->e2, P2 * 32 * B}, {(void**)&n->p2, P4 * 32 * B}, {(void**)&n->bt, P4 * 64 * B},
                             {(void**)&n->d2, P2 * 32 * B}, {(void**)&n->d1, P * 16 * B},  {(void**)&n->y, P * F}};
  if (train) {
    const size_t wpart = (size_t)kWgradBlocks * 27 * 96 * 32;
    std::vector<Item> more = {{(void**)&n->t, P * F},         {(void**)&n->dy, P * F},
                              {(void**)&n->dd1, P * 16 * B},  {(void**)&n->dc1, P * 48 * F},
                              {(void**)&n->dd2, P2 * 32 * B}, {(void**)&n->dc2, P2 * 96 * F},
                              {(void**)&n->dbt, P4 * 64 * B}, {(void**)&n->dp2, P4 * 32 * F},
                              {(void**)&n->de2, P2 * 32 * B}, {(void**)&n->dp1, P2 * 16 * F},
                              {(void**)&n->de1, P * 16 * B},  {(void**)&n->part, wpart * F}};
    items.insert(items.end(), more.begin(), more.end());
  }
  size_t total = 0;
  for (auto& it : items) total += al(it.bytes);
  if (hipMalloc(&n->amem, total) != hipSuccess) {
    n->amem = nullptr;
    return nfail(n, LC_ENOMEM, "cannot allocate %zu bytes of network activations", total);
  }
  char* p = static_cast<char*>(n->amem);
  for (auto& it : items) {
    *it.dst = p;
    p += al(it.bytes);
  }
  n->cap = P;
  n->cap_train = train;
  return LC_OK;
}

int prep_weights(lc_net* n, hipStream_t st) {
  for (int l = 0; l < 5; ++l) {
    const LayerDesc& L = kLayers[l];
    NCHK(n, nn_prep(n->w + woff(l), n->wf[l], l > 0 ? n->wb[l] : nullptr, L.cout, L.cinp, L.cin, st));
  }
  return LC_OK;
}

// Forward pass over x8 (D x H x W, multiples of 4) into y.
int forward(lc_net* n, int D, int H, int W, hipStream_t st) {
  const int D2 = D / 2, H2 = H / 2, W2 = W / 2, D4 = D / 4, H4 = H / 4, W4 = W / 4;
  const float* w = n->w;
  NCHK(n, nn_conv(0, false, nullptr, n->x8, n->wf[0], w + boff(0), n->e1, D, H, W, st));
  NCHK(n, nn_pool(n->e1, n->p1, D, H, W, 16, st));
  NCHK(n, nn_conv(1, false, nullptr, n->p1, n->wf[1], w + boff(1), n->e2, D2, H2, W2, st));
  NCHK(n, nn_pool(n->e2, n->p2, D2, H2, W2, 32, st));
  NCHK(n, nn_conv(2, false, nullptr, n->p2, n->wf[2], w + boff(2), n->bt, D4, H4, W4, st));
  NCHK(n, nn_conv(3, false, n->bt, n->e2, n->wf[3], w + boff(3), n->d2, D2, H2, W2, st));
  NCHK(n, nn_conv(4, false, n->d2, n->e1, n->wf[4], w + boff(4), n->d1, D, H, W, st));
  NCHK(n, nn_head_fwd(n->d1, w + woff(5), n->y, (long)D * H * W, st));
  return LC_OK;
}

int small_blocks(long P) {
  long b = (P + 1023) / 1024;
  return (int)(b < 1 ? 1 : (b > kPartBlocks ? kPartBlocks : b));
}

// Loss against n->t and the gradient of every parameter into n->g.
int backward(lc_net* n, int D, int H, int W, double* loss, hipStream_t st) {
  const long P = (long)D * H * W, P2 = P / 8, P4 = P / 64;
  const int D2 = D / 2, H2 = H / 2, W2 = W / 2, D4 = D / 4, H4 = H / 4, W4 = W / 4;
  const int nb = small_blocks(P);
  NCHK(n, nn_loss(n->y, n->t, n->dy, n->dpart, nb, P, st));
  float* g = n->g;
  NCHK(n, nn_head_bwd(n->d1, n->w + woff(5), n->dy, n->dd1, n->part, g + woff(5), nb, P, st));
  auto wg = [&](int l, const bf16* a, const bf16* b, const bf16* dy, int d, int h, int w_) -> int {
    const long Pl = (long)d * h * w_;
    long nbw = (Pl + 255) / 256;
    if (nbw > kWgradBlocks) nbw = kWgradBlocks;
    const LayerDesc& L = kLayers[l];
    NCHK(n, nn_wgrad(l, a, b, dy, n->part, (int)nbw, d, h, w_, st));
    NCHK(n, nn_wgrad_reduce(n->part, g + woff(l), (int)nbw, L.cout, L.cinp, L.cin, st));
    NCHK(n, nn_colsum(dy, n->part, g + boff(l), Pl, L.cout, small_blocks(Pl), st));
    return LC_OK;
  };
  int rc;
  if ((rc = wg(4, n->d2, n->e1, n->dd1, D, H, W))) return rc;
  NCHK(n, nn_conv(4, true, nullptr, n->dd1, n->wb[4], nullptr, n->dc1, D, H, W, st));
  NCHK(n, nn_upback_mask(n->dc1, n->d2, n->dd2, D, H, W, 48, 32, st));
  if ((rc = wg(3, n->bt, n->e2, n->dd2, D2, H2, W2))) return rc;
  NCHK(n, nn_conv(3, true, nullptr, n->dd2, n->wb[3], nullptr, n->dc2, D2, H2, W2, st));
  NCHK(n, nn_upback_mask(n->dc2, n->bt, n->dbt, D2, H2, W2, 96, 64, st));
  if ((rc = wg(2, nullptr, n->p2, n->dbt, D4, H4, W4))) return rc;
  NCHK(n, nn_conv(2, true, nullptr, n->dbt, n->wb[2], nullptr, n->dp2, D4, H4, W4, st));
  NCHK(n, nn_skip_mask(n->dc2, n->dp2, n->e2, n->de2, D2, H2, W2, 96, 64, 32, st));
  if ((rc = wg(1, nullptr, n->p1, n->de2, D2, H2, W2))) return rc;
  NCHK(n, nn_conv(1, true, nullptr, n->de2, n->wb[1], nullptr, n->dp1, D2, H2, W2, st));
  NCHK(n, nn_skip_mask(n->dc1, n->dp1, n->e1, n->de1, D, H, W, 48, 32, 16, st));
  if ((rc = wg(0, nullptr, n->x8, n->de1, D, H, W))) return rc;
  (void)P2;
  (void)P4;
  if (loss) {
    NCHK(n, hipMemcpyAsync(n->hpart, n->dpart, nb * sizeof(double), hipMemcpyDeviceToHost, st));
    NCHK(n, hipStreamSynchronize(st));
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += n->hpart[b];
    *loss = s / (double)P;
  }
  return LC_OK;
}

int adam(lc_net* n, double lr, hipStream_t st) {
  n->step += 1;
  const double b1 = 0.9, b2 = 0.999;
  const float bc1 = (float)(1.0 - std::pow(b1, (double)n->step));
  const float bc2 = (float)(1.0 - std::pow(b2, (double)n->step));
  NCHK(n, nn_adam(n->w, n->g, n->m, n->v, n->np, (float)lr, (float)b1, (float)b2, 1e-8f, bc1, bc2, st));
  return prep_weights(n, st);
}

bool dims_ok(int D, int H, int W) { return D >= 4 && H >= 4 && W >= 4 && D % 4 == 0 && H % 4 == 0 && W % 4 == 0; }

int pad4(int n) { return (n + 3) / 4 * 4; }

// host sums of the k interleaved per-block partials in n->dpart
int host_sums(lc_net* n, int nb, int k, double* out, hipStream_t st) {
  NCHK(n, hipMemcpyAsync(n->hpart, n->dpart, (size_t)nb * k * sizeof(double), hipMemcpyDeviceToHost, st));
  NCHK(n, hipStreamSynchronize(st));
  for (int q = 0; q < k; ++q) out[q] = 0.0;
  for (int b = 0; b < nb; ++b)
    for (int q = 0; q < k; ++q) out[q] += n->hpart[b * k + q];
  return LC_OK;
}

int net_to_ctx(lc_ctx* c, lc_net* n, int rc) {
  if (rc < 0 && rc != LC_ENOTCONV) return fail(c, rc, "network: %s", n->err.c_str());
  return rc;
}

// Features of the momentum update w (with r = D w already in c->r) into net->x8.
int pack_features(lc_ctx* c, lc_net* n, const double* w) {
  const int nb = small_blocks((long)c->ncell);
  KLAUNCH(c, LC_K_NN_MISC, nn_feat_sums(c->g, w, c->r, n->dpart, nb, c->stream));
  double s[2];
  int rc = host_sums(n, nb, 2, s, c->stream);
  if (rc) return net_to_ctx(c, n, rc);
  double vol = 1.0;
  for (int a = 0; a < 3; ++a) vol *= c->ax[a].xf.back() - c->ax[a].xf.front();
  const double sw = std::sqrt(s[0] / (3.0 * vol)), sr = std::sqrt(s[1] / vol);
  if (!std::isfinite(sw) || !std::isfinite(sr)) return fail(c, LC_EINVAL, "non-finite network input");
  KLAUNCH(c, LC_K_NN_MISC,
          nn_feat_pack(c->g, w, c->r, n->x8, pad4(c->nz), pad4(c->ny), pad4(c->nx), sw > 0 ? 1.0 / sw : 0.0,
                       sr > 0 ? 1.0 / sr : 0.0, c->stream));
  return LC_OK;
}

int run_forward(lc_ctx* c, lc_net* n) {
  const bool prof = c->prof;
  hipEvent_t a = nullptr;
  if (prof && (a = take_event(c))) (void)hipEventRecord(a, c->stream);
  int rc = forward(n, pad4(c->nz), pad4(c->ny), pad4(c->nx), c->stream);
  if (rc) return net_to_ctx(c, n, rc);
  if (prof && a) {
    hipEvent_t b = take_event(c);
    if (b) {
      (void)hipEventRecord(b, c->stream);
      c->recs.push_back({LC_K_NN_FORWARD, a, b});
    }
  }
  return LC_OK;
}

}  // namespace

// Learned start of the SIMPLE loop for the momentum update w (c->r = D w, |D w|_V = n0):
// phi0 = s y with y the network output and s minimising |r - s D G y|_V; on success
// v = w - G phi0, p = phi0 and *used = true.  c->phi, c->t1 are clobbered; c->r is kept.
int learned_start(lc_ctx* c, const double* w, double* v, double* p, bool* used, double* eps_fit) {
  lc_net* n = c->net;
  *used = false;
  *eps_fit = 1.0;
  const long P = (long)pad4(c->nz) * pad4(c->ny) * pad4(c->nx);
  int rc = ensure(n, P, false);
  if (rc) return net_to_ctx(c, n, rc);
  if ((rc = pack_features(c, n, w))) return rc;
  if ((rc = run_forward(c, n))) return rc;
  KLAUNCH(c, LC_K_NN_MISC, nn_unpack(n->y, c->phi, c->nx, c->ny, c->nz, pad4(c->ny), pad4(c->nx), 1.0, c->stream));
  KLAUNCH(c, LC_K_CORRECT, launch_correct(c->g, w, c->phi, v, nullptr, false, c->stream));
  int np = 0;
  KLAUNCH(c, LC_K_DIVERGENCE, launch_divergence(c->g, v, c->t1, nullptr, &np, c->stream));
  // t1 = D(w - G y) - D w = -D G y
  KLAUNCH(c, LC_K_VECTOR, launch_axpy(c->ncell, -1.0, c->r, c->t1, c->stream));
  const int nb = small_blocks((long)c->ncell);
  KLAUNCH(c, LC_K_NN_MISC, nn_vdot3(c->g, c->r, c->t1, n->dpart, nb, c->stream));
  double s[3];
  if ((rc = host_sums(n, nb, 3, s, c->stream))) return net_to_ctx(c, n, rc);
  const double rr = s[0], rz = -s[1], zz = s[2];
  if (!(rr > 0.0) || !(zz > 0.0) || !std::isfinite(rz) || !std::isfinite(zz)) return LC_OK;
  const double scale = rz / zz;
  const double e2 = 1.0 - rz * rz / (rr * zz);
  *eps_fit = std::sqrt(e2 > 0.0 ? e2 : 0.0);
  if (!(*eps_fit < 0.999)) return LC_OK;  // no gain: plain SIMPLE from v = w, p = 0
  KLAUNCH(c, LC_K_NN_MISC, nn_unpack(n->y, c->phi, c->nx, c->ny, c->nz, pad4(c->ny), pad4(c->nx), scale, c->stream));
  KLAUNCH(c, LC_K_CORRECT, launch_correct(c->g, w, c->phi, v, p, false, c->stream));
  *used = true;
  return LC_OK;
}

bool has_net(const lc_ctx* c) { return c->net != nullptr; }

}  // namespace lk

using namespace lk;

extern "C" {

long lc_net_param_count(void) { return nparams(); }

const char* lc_net_last_error(const lc_net* n) { return n ? n->err.c_str() : "null network"; }

int lc_net_create(lc_net** out, uint64_t seed) {
  if (!out) return LC_EINVAL;
  *out = nullptr;
  lc_net* n = new lc_net();
  n->np = nparams();
  const size_t pbytes = al(n->np * sizeof(float));
  size_t wbytes = 0;
  for (int l = 0; l < 5; ++l) {
    wbytes += al((size_t)lk::conv_wf_elems(kLayers[l].cout, kLayers[l].cinp) * sizeof(bf16));
    if (l > 0) wbytes += al((size_t)kLayers[l].cin * lk::conv_kp(kLayers[l].cout) * sizeof(bf16));
  }
  if (hipMalloc(&n->wmem, 4 * pbytes + wbytes) != hipSuccess || hipMalloc(&n->dpart, kPartBlocks * 3 * sizeof(double)) ||
      hipHostMalloc(&n->hpart, kPartBlocks * 3 * sizeof(double), 0) != hipSuccess) {
    if (n->wmem) (void)hipFree(n->wmem);
    if (n->dpart) (void)hipFree(n->dpart);
    delete n;
    return LC_ENOMEM;
  }
  char* p = static_cast<char*>(n->wmem);
  n->w = reinterpret_cast<float*>(p);
  n->g = reinterpret_cast<float*>(p + pbytes);
  n->m = reinterpret_cast<float*>(p + 2 * pbytes);
  n->v = reinterpret_cast<float*>(p + 3 * pbytes);
  p += 4 * pbytes;
  for (int l = 0; l < 5; ++l) {
    n->wf[l] = reinterpret_cast<bf16*>(p);
    p += al((size_t)lk::conv_wf_elems(kLayers[l].cout, kLayers[l].cinp) * sizeof(bf16));
    if (l > 0) {
      n->wb[l] = reinterpret_cast<bf16*>(p);
      p += al((size_t)kLayers[l].cin * lk::conv_kp(kLayers[l].cout) * sizeof(bf16));
    }
  }
  // He-normal weights (Box-Muller on a SplitMix64 stream), zero biases
  std::vector<float> h(n->np, 0.0f);
  uint64_t s = seed;
  for (int l = 0; l < 6; ++l) {
    const LayerDesc& L = kLayers[l];
    const double sd = std::sqrt(2.0 / (L.taps * L.cin));
    for (long e = woff(l); e < boff(l); ++e) {
      const double u1 = ((splitmix(s) >> 11) + 1.0) * 0x1.0p-53, u2 = (splitmix(s) >> 11) * 0x1.0p-53;
      h[e] = (float)(sd * std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2));
    }
  }
  int rc = lc_net_set_params(n, h.data());
  if (rc) {
    lc_net_destroy(n);
    return rc;
  }
  *out = n;
  return LC_OK;
}

int lc_net_destroy(lc_net* n) {
  if (!n) return LC_OK;
  (void)hipDeviceSynchronize();
  if (n->amem) (void)hipFree(n->amem);
  if (n->wmem) (void)hipFree(n->wmem);
  if (n->dpart) (void)hipFree(n->dpart);
  if (n->hpart) (void)hipHostFree(n->hpart);
  delete n;
  return LC_OK;
}

int lc_net_get_params(lc_net* n, float* host) {
  if (!n || !host) return LC_EINVAL;
  NCHK(n, hipMemcpy(host, n->w, n->np * sizeof(float), hipMemcpyDeviceToHost));
  return LC_OK;
}

int lc_net_set_params(lc_net* n, const float* host) {
  if (!n || !host) return LC_EINVAL;
  for (long e = 0; e < n->np; ++e)
    if (!std::isfinite(host[e])) return nfail(n, LC_EINVAL, "non-finite parameter %ld", e);
  NCHK(n, hipMemcpy(n->w, host, n->np * sizeof(float), hipMemcpyHostToDevice));
  NCHK(n, hipMemset(n->m, 0, n->np * sizeof(float)));
  NCHK(n, hipMemset(n->v, 0, n->np * sizeof(float)));
  NCHK(n, hipMemset(n->g, 0, n->np * sizeof(float)));
  n->step = 0;
  int rc = prep_weights(n, nullptr);
  if (rc) return rc;
  NCHK(n, hipDeviceSynchronize());
  return LC_OK;
}

int lc_net_save(lc_net* n, const char* path) {
  if (!n || !path) return LC_EINVAL;
  std::vector<float> h(n->np);
  int rc = lc_net_get_params(n, h.data());
  if (rc) return rc;
  FILE* f = std::fopen(path, "wb");
  if (!f) return nfail(n, LC_EINVAL, "cannot open %s for writing", path);
  const uint32_t count = (uint32_t)n->np;
  unsigned char head[12] = {'L', 'K', 'N', 'E', 'T', '0', '0', '1'};
  for (int b = 0; b < 4; ++b) head[8 + b] = (unsigned char)(count >> (8 * b));
  bool ok = std::fwrite(head, 1, 12, f) == 12;
  for (size_t q = 0; ok && q < h.size(); ++q) {
    uint32_t u;
    std::memcpy(&u, &h[q], 4);
    const unsigned char le[4] = {(unsigned char)u, (unsigned char)(u >> 8), (unsigned char)(u >> 16),
                                 (unsigned char)(u >> 24)};
    ok = std::fwrite(le, 1, 4, f) == 4;
  }
  ok = (std::fclose(f) == 0) && ok;
  return ok ? LC_OK : nfail(n, LC_EINVAL, "write failed: %s", path);
}

int lc_net_load(lc_net* n, const char* path) {
  if (!n || !path) return LC_EINVAL;
  FILE* f = std::fopen(path, "rb");
  if (!f) return nfail(n, LC_EINVAL, "cannot open %s", path);
  unsigned char head[12];
  const bool got = std::fread(head, 1, 12, f) == 12;
  if (!got || std::memcmp(head, "LKNET001", 8) != 0) {
    std::fclose(f);
    return nfail(n, LC_EINVAL, "not a network parameter file: %s", path);
  }
  uint32_t count = 0;
  for (int b = 0; b < 4; ++b) count |= (uint32_t)head[8 + b] << (8 * b);
  if ((long)count != n->np) {
    std::fclose(f);
    return nfail(n, LC_EINVAL, "parameter count %u differs from this network's %ld: %s", count, n->np, path);
  }
  std::vector<float> h(n->np);
  bool ok = true;
  for (size_t q = 0; ok && q < h.size(); ++q) {
    unsigned char le[4];
    ok = std::fread(le, 1, 4, f) == 4;
    const uint32_t u = (uint32_t)le[0] | ((uint32_t)le[1] << 8) | ((uint32_t)le[2] << 16) | ((uint32_t)le[3] << 24);
    std::memcpy(&h[q], &u, 4);
  }
  unsigned char extra;
  ok = ok && std::fread(&extra, 1, 1, f) == 0;  // exactly the declared length
  std::fclose(f);
  if (!ok) return nfail(n, LC_EINVAL, "file length does not match its parameter count: %s", path);
  return lc_net_set_params(n, h.data());
}

int lc_net_forward(lc_net* n, void* stream, const float* x4, float* y, int D, int H, int W) {
  if (!n || !x4 || !y) return LC_EINVAL;
  if (!dims_ok(D, H, W)) return nfail(n, LC_EINVAL, "network sizes must be positive multiples of 4");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const long P = (long)D * H * W;
  int rc = ensure(n, P, false);
  if (rc) return rc;
  NCHK(n, nn_x4_to_x8(x4, n->x8, P, st));
  if ((rc = forward(n, D, H, W, st))) return rc;
  NCHK(n, hipMemcpyAsync(y, n->y, P * sizeof(float), hipMemcpyDeviceToDevice, st));
  NCHK(n, hipStreamSynchronize(st));
  return LC_OK;
}

int lc_net_step(lc_net* n, void* stream, const float* x4, const float* t, int D, int H, int W, double lr, double* loss,
                float* grad_host) {
  if (!n || !x4 || !t) return LC_EINVAL;
  if (!dims_ok(D, H, W)) return nfail(n, LC_EINVAL, "network sizes must be positive multiples of 4");
  if (!(lr >= 0.0)) return nfail(n, LC_EINVAL, "bad learning rate");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const long P = (long)D * H * W;
  int rc = ensure(n, P, true);
  if (rc) return rc;
  NCHK(n, nn_x4_to_x8(x4, n->x8, P, st));
  NCHK(n, hipMemcpyAsync(n->t, t, P * sizeof(float), hipMemcpyDeviceToDevice, st));
  if ((rc = forward(n, D, H, W, st))) return rc;
  double l = 0.0;
  if ((rc = backward(n, D, H, W, &l, st))) return rc;
  if (grad_host) {
    NCHK(n, hipMemcpyAsync(grad_host, n->g, n->np * sizeof(float), hipMemcpyDeviceToHost, st));
    NCHK(n, hipStreamSynchronize(st));
  }
  if (lr > 0.0 && (rc = adam(n, lr, st))) return rc;
  NCHK(n, hipStreamSynchronize(st));
  if (loss) *loss = l;
  return LC_OK;
}

int lc_set_net(lc_ctx* c, lc_net* n) {
  if (!c) return LC_EINVAL;
  c->net = n;
  return LC_OK;
}

int lc_net_train(lc_ctx* c, lc_net* n, int steps, double lr, uint64_t seed, double* loss_hist) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (!n || steps < 0 || !(lr > 0.0)) return fail(c, LC_EINVAL, "bad network, step count or learning rate");
  const int D = pad4(c->nz), H = pad4(c->ny), W = pad4(c->nx);
  const long P = (long)D * H * W;
  if ((rc = ensure(n, P, true))) return net_to_ctx(c, n, rc);
  double* rs = nullptr;  // two velocities of the Krylov workspace: the random field and its projection
  long ld = 0;
  if ((rc = krylov_ws(c, 2, &rs, &ld))) return rc;
  double* v = rs + ld;
  auto body = [&]() -> int {
    for (int s = 0; s < steps; ++s) {
      // a pair of the method: v = P(r_s), w = L_U v, phi = first SIMPLE correction of w
      HIPCHK(c, launch_uniform(rs, c->nvel, seed * 1000003ull + (uint64_t)s, c->stream));
      HIPCHK(c, launch_zero_walls(rs, c->nx, c->ny, c->nz, c->stream));
      int r2 = lc_project(c, rs, v, nullptr, LC_FP64, 1e-10, 3, nullptr);
      if (r2 < 0) return r2;
      KLAUNCH(c, LC_K_MOMENTUM, launch_momentum(c->g, c->U, v, c->w, 1.0 / c->re, 1.0, false, 0, 0, c->stream));
      double n0 = 0.0;
      if ((r2 = vnorm_div(c, c->w, c->r, &n0))) return r2;
      if ((r2 = poisson(c, c->r, c->phi, LC_FP64))) return r2;
      if ((r2 = pack_features(c, n, c->w))) return r2;
      const int nb = small_blocks((long)c->ncell);
      KLAUNCH(c, LC_K_NN_MISC, nn_vdot3(c->g, c->phi, c->phi, n->dpart, nb, c->stream));
      double q[3];
      if ((r2 = host_sums(n, nb, 3, q, c->stream))) return net_to_ctx(c, n, r2);
      double vol = 1.0;
      for (int a = 0; a < 3; ++a) vol *= c->ax[a].xf.back() - c->ax[a].xf.front();
      const double sphi = std::sqrt(q[0] / vol);
      KLAUNCH(c, LC_K_NN_MISC,
              nn_target(c->phi, n->t, c->nx, c->ny, c->nz, D, H, W, sphi > 0 ? 1.0 / sphi : 0.0, c->stream));
      if ((r2 = forward(n, D, H, W, c->stream))) return net_to_ctx(c, n, r2);
      double l = 0.0;
      if ((r2 = backward(n, D, H, W, &l, c->stream))) return net_to_ctx(c, n, r2);
      if ((r2 = adam(n, lr, c->stream))) return net_to_ctx(c, n, r2);
      if (loss_hist) loss_hist[s] = l;
      if (!std::isfinite(l)) return fail(c, LC_EINVAL, "training loss is not finite at step %d", s);
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LC_OK;
  };
  rc = body();
  (void)hipStreamSynchronize(c->stream);
  return rc;
}

int lc_learned_guess(lc_ctx* c, const double* w, double* phi0, double* eps) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (!c->net) return fail(c, LC_ESTATE, "no network attached");
  if (!aligned(w) || !aligned(phi0)) return fail(c, LC_EINVAL, "bad pointers");
  double n0 = 0.0;
  if ((rc = vnorm_div(c, w, c->r, &n0))) return rc;
  if (!std::isfinite(n0)) return fail(c, LC_EINVAL, "non-finite input");
  double* v = nullptr;  // the guessed start velocity (discarded): one vector of the Krylov workspace
  long ld = 0;
  if ((rc = krylov_ws(c, 1, &v, &ld))) return rc;
  bool used = false;
  double e = 1.0;
  rc = n0 > 0.0 ? learned_start(c, w, v, phi0, &used, &e) : LC_OK;
  if (!rc && !used) rc = hipMemsetAsync(phi0, 0, c->ncell * sizeof(double), c->stream) ? LC_EHIP : LC_OK;
  (void)hipStreamSynchronize(c->stream);
  if (eps) *eps = used ? e : 1.0;
  return rc;
}

}  // extern "C"
