// C ABI of lidkrylov: context, grid, stencils, Poisson solve, SIMPLE projection.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "lk_ctx.h"
#include "lk_internal.h"
#include "lk_linalg.h"
#include "lk_modes.h"

using namespace lk;

namespace {
std::string g_create_error;
}  // namespace

namespace lk {

int fail(lc_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  else g_create_error = buf;
  return code;
}



hipEvent_t take_event(lc_ctx* c) {
  if (c->ev_used < c->ev_pool.size()) return c->ev_pool[c->ev_used++];
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  c->ev_pool.push_back(e);
  c->ev_used++;
  return e;
}



constexpr size_t kArenaAlign = 256;

size_t arena_next(const lc_ctx* c) { return (c->arena_used + kArenaAlign - 1) / kArenaAlign * kArenaAlign; }

hipError_t ctx_alloc(lc_ctx* c, void** p, size_t bytes) {
  if (c->dry) {
    *p = nullptr;
    c->arena_used = arena_next(c) + bytes;
    return hipSuccess;
  }
  if (!c->arena) return hipMalloc(p, bytes);
  const size_t at = arena_next(c);
  if (at + bytes > c->arena_size) return hipErrorOutOfMemory;
  *p = c->arena + at;
  c->arena_used = at + bytes;
  return hipSuccess;
}

int krylov_ws(lc_ctx* c, int nvec, double** p, long* ld) {
  *ld = ((long)c->nvel + 63) / 64 * 64;
  const size_t need = (size_t)nvec * *ld;
  if (need > c->kws_n) {
    if (c->arena)
      return fail(c, LC_ENOMEM, "workspace too small: %d Krylov vectors need %zu bytes, %zu remain", nvec,
                  need * sizeof(double), c->kws_n * sizeof(double));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (c->kws) (void)hipFree(c->kws);
    c->kws = nullptr;
    c->kws_n = 0;
    if (hipMalloc((void**)&c->kws, need * sizeof(double)) != hipSuccess)
      return fail(c, LC_ENOMEM, "cannot allocate %d Krylov vectors (%.1f GB)", nvec, need * 8e-9);
    c->kws_n = need;
  }
  *p = c->kws;
  return LC_OK;
}

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// Fixed-order reduction of partials on the device, then one scalar to the host.
int reduce_to_host(lc_ctx* c, int nparts, double* out) {
  KLAUNCH(c, LC_K_REDUCE, launch_sum(c->partials, nparts, c->dsum, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->hsum, c->dsum, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  *out = *c->hsum;
  return LC_OK;
}

int vnorm_div(lc_ctx* c, const double* v, double* r, double* out) {
  int np = 0;
  KLAUNCH(c, LC_K_DIVERGENCE, launch_divergence(c->g, v, r, c->partials, &np, c->stream));
  double s2 = 0.0;
  int rc = reduce_to_host(c, np, &s2);
  if (rc) return rc;
  *out = std::sqrt(s2);
  return LC_OK;
}

int upload_grid(lc_ctx* c) {
  const int n[3] = {c->nx, c->ny, c->nz};
  // metrics: per axis rd (n), rdd (n+1), th (n+1), d (n)
  const size_t total = metric_doubles(n[0], n[1], n[2]);
  if (!c->metric) HIPCHK(c, dalloc(c, &c->metric, total));
  std::vector<double> host(total);
  size_t off = 0;
  AxisDev* dst[3] = {&c->g.x, &c->g.y, &c->g.z};
  for (int a = 0; a < 3; ++a) {
    const AxisHost& A = c->ax[a];
    double* base = c->metric + off;
    std::copy(A.rd.begin(), A.rd.end(), host.begin() + off);
    dst[a]->rd = base;
    off += n[a];
    std::copy(A.rdd.begin(), A.rdd.end(), host.begin() + off);
    dst[a]->rdd = c->metric + off;
    off += n[a] + 1;
    std::copy(A.th.begin(), A.th.end(), host.begin() + off);
    dst[a]->th = c->metric + off;
    off += n[a] + 1;
    std::copy(A.d.begin(), A.d.end(), host.begin() + off);
    dst[a]->d = c->metric + off;
    off += n[a];
    dst[a]->n = n[a];
  }
  HIPCHK(c, hipMemcpyAsync(c->metric, host.data(), total * sizeof(double), hipMemcpyHostToDevice, c->stream));

  // tensor-product factorization of each axis (full matrices, plus the parity-sorted
  // half matrices of mirror-symmetric axes, in both precisions)
  size_t mbytes = 0;
  for (int a = 0; a < 3; ++a) mbytes += mode_bytes(n[a]);
  if (!c->modes_mem) HIPCHK(c, ctx_alloc(c, &c->modes_mem, mbytes));
  Stager st(mbytes, c->modes_mem);
  for (int a = 0; a < 3; ++a) {
    const int m = n[a];
    const AxisHost& AH = c->ax[a];
    // mirror symmetry: widths and centre distances equal under i -> m-1-i
    bool sym = m >= 2;
    double wmax = 0.0;
    for (int i = 0; i < m; ++i) wmax = std::max(wmax, AH.d[i]);
    for (int i = 0; i < m && sym; ++i) sym = std::fabs(AH.d[i] - AH.d[m - 1 - i]) <= 1e-12 * wmax;
    for (int i = 0; i <= m && sym; ++i) sym = std::fabs(AH.dd[i] - AH.dd[m - i]) <= 1e-12 * wmax;
    c->axis_sym[a] = sym;
    std::vector<double> kd, ko;
    neumann_operator(m, AH.dd.data(), kd, ko);
    ModeHost H;
    if (!compute_modes(m, kd, ko, AH.d, sym, H))
      return fail(c, LC_EINVAL, "tridiagonal eigen-solver did not converge on axis %d", a);
    place_modes(H, c->modes[a], st);
    // ascending; the Neumann null mode is the largest (~0), last of the even modes when folded
    c->zero_mode[a] = sym ? (m + 1) / 2 - 1 : m - 1;
  }
  if (st.overflow) return fail(c, LC_ENOMEM, "mode storage sized too small (internal)");
  HIPCHK(c, hipMemcpyAsync(c->modes_mem, st.host.data(), st.used, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->stokes_ready = false;  // the viscous-step factors belong to the previous grid
  c->grid_ready = true;
  return LC_OK;
}

// (D G) phi = r by transforming with S^T M along x, y, z, dividing by the sums of
// the axis eigenvalues (constant mode set to zero) and transforming back with S.
template <typename T>
int tp_solve(lc_ctx* c, const T* r, T* phi, T* t1, T* t2) {
  const int nx = c->nx, ny = c->ny, nz = c->nz;
  const long pl = (long)nx * ny;
  auto pick = [](const AxisModes& M, int which) -> const T* {
    if constexpr (sizeof(T) == sizeof(double)) {
      const double* a[4] = {M.F, M.Bk, M.FT, M.BkT};
      return (const T*)a[which];
    } else {
      const float* a[4] = {M.F32, M.Bk32, M.FT32, M.BkT32};
      return (const T*)a[which];
    }
  };
  auto half = [](const AxisModes& M, int which) -> const T* {
    if constexpr (sizeof(T) == sizeof(double))
      return (const T*)M.h64[which];
    else
      return (const T*)M.h32[which];
  };
  auto packs = [](const AxisModes& M, int which) -> const T* {
    if constexpr (sizeof(T) == sizeof(double))
      return (const T*)M.p64[which];
    else
      return (const T*)M.p32[which];
  };
  auto lams = [](const AxisModes& M) { return M.sym ? M.lam_s : M.lam; };
  const AxisModes &X = c->modes[0], &Y = c->modes[1], &Z = c->modes[2];
  hipStream_t s = c->stream;
  const int n_yz = ny * nz, n_xz = nx * nz;
  const double* nul = nullptr;
  {
    if (c->poisson_method == LC_POISSON_TPT && nx <= tridiag_x_max()) {
      // TPT: forward y and z, tridiagonal solves along x, backward z and y
      if (Y.mf)
        KLAUNCH(c, LC_K_TP_Y, launch_mff_left<T>(ny, n_xz, packs(Y, 0), packs(Y, 1), r, t1, nx, pl, nx, s));
      else if (Y.sym)
        KLAUNCH(c, LC_K_TP_Y, launch_tpf_left<T>(ny, n_xz, half(Y, 0), half(Y, 1), r, t1, nx, pl, nx, nul, nul, nul, 1,
                                                 0, 0, 0, s));
      else
        KLAUNCH(c, LC_K_TP_Y, launch_tp_left<T>(ny, n_xz, ny, pick(Y, 0), r, t1, nx, pl, nx, nul, nul, nul, 1, 0, 0, 0,
                                                s));
      if (Z.mf)
        KLAUNCH(c, LC_K_TP_Z, launch_mff_left<T>(nz, (int)pl, packs(Z, 0), packs(Z, 1), t1, t2, (int)pl, 0, pl, s));
      else if (Z.sym)
        KLAUNCH(c, LC_K_TP_Z, launch_tpf_left<T>(nz, (int)pl, half(Z, 0), half(Z, 1), t1, t2, (int)pl, 0, pl, nul, nul,
                                                 nul, 1, 0, 0, 0, s));
      else
        KLAUNCH(c, LC_K_TP_Z, launch_tp_left<T>(nz, (int)pl, nz, pick(Z, 0), t1, t2, (int)pl, 0, pl, nul, nul, nul, 1, 0,
                                                0, 0, s));
      KLAUNCH(c, LC_K_TRIDIAG,
              launch_tridiag_x<T>(c->g, lams(Y), lams(Z), c->zero_mode[1], c->zero_mode[2], t2, t1, s));
      if (Z.mf)
        KLAUNCH(c, LC_K_TP_Z, launch_mfu_left<T>(nz, (int)pl, packs(Z, 2), packs(Z, 3), t1, t2, (int)pl, 0, pl, nul,
                                                 nul, nul, 1, 0, 0, 0, s));
      else if (Z.sym)
        KLAUNCH(c, LC_K_TP_Z, launch_tpu_left<T>(nz, (int)pl, half(Z, 2), half(Z, 3), t1, t2, (int)pl, 0, pl, s));
      else
        KLAUNCH(c, LC_K_TP_Z, launch_tp_left<T>(nz, (int)pl, nz, pick(Z, 1), t1, t2, (int)pl, 0, pl, nul, nul, nul, 1, 0,
                                                0, 0, s));
      if (Y.mf)
        KLAUNCH(c, LC_K_TP_Y, launch_mfu_left<T>(ny, n_xz, packs(Y, 2), packs(Y, 3), t2, phi, nx, pl, nx, nul, nul, nul,
                                                 1, 0, 0, 0, s));
      else if (Y.sym)
        KLAUNCH(c, LC_K_TP_Y, launch_tpu_left<T>(ny, n_xz, half(Y, 2), half(Y, 3), t2, phi, nx, pl, nx, s));
      else
        KLAUNCH(c, LC_K_TP_Y, launch_tp_left<T>(ny, n_xz, ny, pick(Y, 1), t2, phi, nx, pl, nx, nul, nul, nul, 1, 0, 0, 0,
                                                s));
      return LC_OK;
    }
  }
  // forward: x (contiguous lines), y (columns (k, i), rows nx apart), z (rows nx*ny apart),
  // the division by lam_x + lam_y + lam_z fused into the z transform; a mirror-symmetric
  // axis uses the folded half-size transforms (modes parity-sorted)
  // (mirror-symmetric axes with he <= kMfMaxHalf run on the matrix cores)
  if (X.mf)
    KLAUNCH(c, LC_K_TP_X, launch_mff_right<T>(nx, n_yz, r, packs(X, 0), packs(X, 1), t1, s));
  else if (X.sym)
    KLAUNCH(c, LC_K_TP_X, launch_tpf_right<T>(nx, n_yz, r, half(X, 4), half(X, 5), t1, s));
  else
    KLAUNCH(c, LC_K_TP_X, launch_tp_right<T>(n_yz, nx, nx, r, pick(X, 2), t1, s));
  if (Y.mf)
    KLAUNCH(c, LC_K_TP_Y, launch_mff_left<T>(ny, n_xz, packs(Y, 0), packs(Y, 1), t1, t2, nx, pl, nx, s));
  else if (Y.sym)
    KLAUNCH(c, LC_K_TP_Y, launch_tpf_left<T>(ny, n_xz, half(Y, 0), half(Y, 1), t1, t2, nx, pl, nx, nul, nul, nul, 1, 0, 0,
                                             0, s));
  else
    KLAUNCH(c, LC_K_TP_Y, launch_tp_left<T>(ny, n_xz, ny, pick(Y, 0), t1, t2, nx, pl, nx, nul, nul, nul, 1, 0, 0, 0, s));
  if (Z.mf)  // (the eigenvalue division then happens in the backward z transform)
    KLAUNCH(c, LC_K_TP_Z, launch_mff_left<T>(nz, (int)pl, packs(Z, 0), packs(Z, 1), t2, t1, (int)pl, 0, pl, s));
  else if (Z.sym)
    KLAUNCH(c, LC_K_TP_Z, launch_tpf_left<T>(nz, (int)pl, half(Z, 0), half(Z, 1), t2, t1, (int)pl, 0, pl, lams(Z),
                                             lams(Y), lams(X), nx, c->zero_mode[2], c->zero_mode[1], c->zero_mode[0], s));
  else
    KLAUNCH(c, LC_K_TP_Z, launch_tp_left<T>(nz, (int)pl, nz, pick(Z, 0), t2, t1, (int)pl, 0, pl, lams(Z), lams(Y),
                                            lams(X), nx, c->zero_mode[2], c->zero_mode[1], c->zero_mode[0], s));
  // backward: z, y, x
  if (Z.mf)
    KLAUNCH(c, LC_K_TP_Z, launch_mfu_left<T>(nz, (int)pl, packs(Z, 2), packs(Z, 3), t1, t2, (int)pl, 0, pl, lams(Z),
                                             lams(Y), lams(X), nx, c->zero_mode[2], c->zero_mode[1], c->zero_mode[0], s));
  else if (Z.sym)
    KLAUNCH(c, LC_K_TP_Z, launch_tpu_left<T>(nz, (int)pl, half(Z, 2), half(Z, 3), t1, t2, (int)pl, 0, pl, s));
  else
    KLAUNCH(c, LC_K_TP_Z, launch_tp_left<T>(nz, (int)pl, nz, pick(Z, 1), t1, t2, (int)pl, 0, pl, nul, nul, nul, 1, 0, 0,
                                            0, s));
  if (Y.mf)
    KLAUNCH(c, LC_K_TP_Y, launch_mfu_left<T>(ny, n_xz, packs(Y, 2), packs(Y, 3), t2, t1, nx, pl, nx, nul, nul, nul, 1, 0,
                                             0, 0, s));
  else if (Y.sym)
    KLAUNCH(c, LC_K_TP_Y, launch_tpu_left<T>(ny, n_xz, half(Y, 2), half(Y, 3), t2, t1, nx, pl, nx, s));
  else
    KLAUNCH(c, LC_K_TP_Y, launch_tp_left<T>(ny, n_xz, ny, pick(Y, 1), t2, t1, nx, pl, nx, nul, nul, nul, 1, 0, 0, 0, s));
  if (X.mf)
    KLAUNCH(c, LC_K_TP_X, launch_mfu_right<T>(nx, n_yz, t1, packs(X, 2), packs(X, 3), phi, s));
  else if (X.sym)
    KLAUNCH(c, LC_K_TP_X, launch_tpu_right<T>(nx, n_yz, t1, half(X, 6), half(X, 7), phi, s));
  else
    KLAUNCH(c, LC_K_TP_X, launch_tp_right<T>(n_yz, nx, nx, t1, pick(X, 3), phi, s));
  return LC_OK;
}

int poisson(lc_ctx* c, const double* r, double* phi, int precision) {
  if (precision == LC_FP64) return tp_solve<double>(c, r, phi, c->t1, c->t2);
  KLAUNCH(c, LC_K_CAST, launch_d2f(c->ncell, r, c->r32, c->stream));
  int rc = tp_solve<float>(c, c->r32, c->r32, c->t1_32, c->t2_32);
  if (rc) return rc;
  KLAUNCH(c, LC_K_CAST, launch_f2d(c->ncell, c->r32, phi, false, c->stream));
  return LC_OK;
}

int check_ready(lc_ctx* c) {
  if (!c) return LC_EINVAL;
  if (!c->grid_ready) return fail(c, LC_ESTATE, "grid not set");
  return LC_OK;
}

bool aligned(const void* p) { return p && ((uintptr_t)p % 8 == 0); }

int reduce_max_to_host(lc_ctx* c, int nparts, double* out) {
  KLAUNCH(c, LC_K_REDUCE, launch_max(c->partials, nparts, c->dsum, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->hsum, c->dsum, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  *out = *c->hsum;
  return LC_OK;
}

int vdot(lc_ctx* c, const double* a, const double* b, double* out) {
  int np = 0;
  KLAUNCH(c, LC_K_VECTOR, launch_dot_partials(a, b, c->nvel, c->partials, &np, c->stream));
  return reduce_to_host(c, np, out);
}

int vmaxabs(lc_ctx* c, const double* a, double* out) {
  int np = 0;
  KLAUNCH(c, LC_K_VECTOR, launch_maxabs_partials(a, c->nvel, c->partials, &np, c->stream));
  return reduce_max_to_host(c, np, out);
}

}  // namespace lk

extern "C" {

const char* lc_version(void) { return "lidkrylov 0.1 (gfx950)"; }

const char* lc_last_error(const lc_ctx* c) { return c ? c->err.c_str() : g_create_error.c_str(); }

size_t lc_vel_size(const lc_ctx* c) { return c ? c->nvel : 0; }
size_t lc_cell_size(const lc_ctx* c) { return c ? c->ncell : 0; }

}  // extern "C"

namespace lk {

size_t metric_doubles(int nx, int ny, int nz) { return 4 * ((size_t)nx + ny + nz) + 6; }

size_t viscous_bytes(int nx, int ny, int nz) {
  size_t b = 0;
  for (int n : {nx, ny, nz}) b += mode_bytes(n) + mode_bytes(n + 1);
  return b;
}

size_t component_max(int nx, int ny, int nz) {
  return std::max({(size_t)(nx + 1) * ny * nz, (size_t)nx * (ny + 1) * nz, (size_t)nx * ny * (nz + 1)});
}

// Krylov vectors the drivers use with basis or restart length m: Arnoldi 2 (m + 1), Newton
// max(m + 1, 8) + 4 (GMRES basis, BiCGstab(2) vectors, right side, correction, spares).
int krylov_vectors(int m) { return std::max(2 * (m + 1), std::max(m + 1, 8) + 4); }

namespace {

void init_dims(lc_ctx* c, int nx, int ny, int nz) {
  c->nx = nx;
  c->ny = ny;
  c->nz = nz;
  c->nvel = vel_layout(nx, ny, nz).total();
  c->ncell = (size_t)nx * ny * nz;
  c->max_parts = (int)((c->ncell + kReduceBlock - 1) / kReduceBlock) + kGsBlocks * kGsChunk;
  // the divergence kernel: 64 x 4 cells x 4 planes per block
  const size_t nd = (size_t)((nx + 63) / 64) * ((ny + 3) / 4) * ((nz + 3) / 4);
  if (nd > (size_t)c->max_parts) c->max_parts = (int)nd;
}

// The context's device buffers, in a fixed order.  With a caller workspace (or a dry run)
// the buffers that are otherwise allocated on first use -- grid metrics and factors, the
// viscous-step factors, the critical-Re steady states -- are carved here as well, and the
// Krylov vectors get the remainder.
bool carve_all(lc_ctx* c) {
  bool ok = dalloc(c, &c->U, c->nvel) == hipSuccess && dalloc(c, &c->w, c->nvel) == hipSuccess &&
            dalloc(c, &c->r, c->ncell) == hipSuccess && dalloc(c, &c->phi, c->ncell) == hipSuccess &&
            dalloc(c, &c->t1, c->ncell) == hipSuccess && dalloc(c, &c->t2, c->ncell) == hipSuccess &&
            dalloc(c, &c->r32, c->ncell) == hipSuccess && dalloc(c, &c->t1_32, c->ncell) == hipSuccess &&
            dalloc(c, &c->t2_32, c->ncell) == hipSuccess && dalloc(c, &c->partials, c->max_parts) == hipSuccess &&
            dalloc(c, &c->dsum, 1) == hipSuccess && dalloc(c, &c->dsmall, kSmall) == hipSuccess;
  if (!ok || !(c->arena || c->dry)) return ok;
  const int nx = c->nx, ny = c->ny, nz = c->nz;
  size_t mbytes = 0;
  for (int n : {nx, ny, nz}) mbytes += mode_bytes(n);
  return dalloc(c, &c->metric, metric_doubles(nx, ny, nz)) == hipSuccess &&
         ctx_alloc(c, &c->modes_mem, mbytes) == hipSuccess &&
         ctx_alloc(c, &c->stokes_mem, viscous_bytes(nx, ny, nz)) == hipSuccess &&
         dalloc(c, &c->vscale, 2 * ((size_t)nx + ny + nz) + 3) == hipSuccess &&
         dalloc(c, &c->hs, component_max(nx, ny, nz)) == hipSuccess &&
         dalloc(c, &c->ucr, kCriticalVectors * c->nvel) == hipSuccess;
}

int create(lc_ctx** out, int nx, int ny, int nz, void* ws, size_t ws_bytes, void* hip_stream) {
  if (!out) return fail(nullptr, LC_EINVAL, "null output pointer");
  *out = nullptr;
  if (nx < 2 || ny < 2 || nz < 2 || nx > 4096 || ny > 4096 || nz > 4096)
    return fail(nullptr, LC_EINVAL, "grid size %dx%dx%d outside [2, 4096]", nx, ny, nz);
  {
    // the stencil kernels address each velocity component with 32-bit byte offsets
    const VelLayout L = vel_layout(nx, ny, nz);
    if (8 * std::max(L.nu, std::max(L.nv, L.nw)) >= (size_t(1) << 31))
      return fail(nullptr, LC_EINVAL, "grid %dx%dx%d: a velocity component exceeds 2^31 bytes", nx, ny, nz);
  }
  lc_ctx* c = new lc_ctx();
  init_dims(c, nx, ny, nz);
  c->stream = (hipStream_t)hip_stream;
  c->arena = (char*)ws;
  c->arena_size = ws ? ws_bytes : 0;
  bool ok = carve_all(c);
  if (ok && c->arena) {  // the Krylov vectors: the rest of the workspace
    const size_t at = (c->arena_used + 255) / 256 * 256;
    c->kws = (double*)(c->arena + std::min(at, c->arena_size));
    c->kws_n = at < c->arena_size ? (c->arena_size - at) / sizeof(double) : 0;
  }
  if (!ok) {
    lc_destroy(c);
    if (ws) {
      size_t need = 0;
      lc_workspace_query(nx, ny, nz, 0, &need);
      return fail(nullptr, LC_ENOMEM, "workspace of %zu bytes too small for a %dx%dx%d context (at least %zu)",
                  ws_bytes, nx, ny, nz, need);
    }
    return fail(nullptr, LC_ENOMEM, "device allocation failed for %dx%dx%d", nx, ny, nz);
  }
  ok = hipHostMalloc((void**)&c->hsmall, kSmall * sizeof(double), hipHostMallocDefault) == hipSuccess &&
       hipHostMalloc((void**)&c->hsum, sizeof(double), hipHostMallocDefault) == hipSuccess;
  if (!ok) {
    lc_destroy(c);
    return fail(nullptr, LC_ENOMEM, "pinned host allocation failed");
  }
  if (hipMemsetAsync(c->U, 0, c->nvel * sizeof(double), c->stream) != hipSuccess) {
    lc_destroy(c);
    return fail(nullptr, LC_EHIP, "hipMemsetAsync failed");
  }
  int rc = lc_set_stretching(c, LC_UNIFORM, 0.0);
  if (rc) {
    g_create_error = c->err;
    lc_destroy(c);
    return rc;
  }
  *out = c;
  return LC_OK;
}

}  // namespace
}  // namespace lk

extern "C" {

int lc_workspace_query(int nx, int ny, int nz, int m_max, size_t* bytes) {
  if (!bytes || nx < 2 || ny < 2 || nz < 2 || nx > 4096 || ny > 4096 || nz > 4096 || m_max < 0 || m_max > 400)
    return LC_EINVAL;
  const VelLayout L = vel_layout(nx, ny, nz);
  if (8 * std::max(L.nu, std::max(L.nv, L.nw)) >= (size_t(1) << 31)) return LC_EINVAL;
  lc_ctx c;
  init_dims(&c, nx, ny, nz);
  c.dry = true;
  carve_all(&c);
  const size_t at = (c.arena_used + 255) / 256 * 256;
  const size_t ld = (c.nvel + 63) / 64 * 64;
  *bytes = at + (size_t)krylov_vectors(m_max) * ld * sizeof(double);
  return LC_OK;
}

int lc_create(lc_ctx** out, int nx, int ny, int nz, void* hip_stream) {
  return create(out, nx, ny, nz, nullptr, 0, hip_stream);
}

int lc_create_in(lc_ctx** out, int nx, int ny, int nz, void* workspace, size_t bytes, void* hip_stream) {
  if (!workspace || (uintptr_t)workspace % 256) return fail(nullptr, LC_EINVAL, "workspace must be 256-byte aligned");
  return create(out, nx, ny, nz, workspace, bytes, hip_stream);
}

int lc_destroy(lc_ctx* c) {
  if (!c) return LC_OK;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  if (!c->arena) {  // carved buffers belong to the caller's workspace
    void* ptrs[] = {c->U, c->w, c->r, c->phi, c->t1, c->t2, c->r32, c->t1_32, c->t2_32, c->partials,
                    c->dsum, c->metric, c->modes_mem, c->dsmall, c->kws, c->ucr, c->stokes_mem, c->vscale, c->hs};
    for (void* p : ptrs)
      if (p) (void)hipFree(p);
  }
  if (c->hsum) (void)hipHostFree(c->hsum);
  if (c->hsmall) (void)hipHostFree(c->hsmall);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  delete c;
  return LC_OK;
}

int lc_set_stream(lc_ctx* c, void* s) {
  if (!c) return LC_EINVAL;
  c->stream = (hipStream_t)s;
  return LC_OK;
}

int lc_set_grid(lc_ctx* c, const double* xf, const double* yf, const double* zf) {
  if (!c || !xf || !yf || !zf) return fail(c, LC_EINVAL, "null argument");
  const double* f[3] = {xf, yf, zf};
  const int n[3] = {c->nx, c->ny, c->nz};
  for (int a = 0; a < 3; ++a) {
    if (f[a][0] != 0.0 || f[a][n[a]] != 1.0) return fail(c, LC_EINVAL, "axis %d faces must run from 0 to 1", a);
    for (int i = 0; i < n[a]; ++i)
      if (!(f[a][i + 1] > f[a][i]) || !std::isfinite(f[a][i + 1]))
        return fail(c, LC_EINVAL, "axis %d faces must increase strictly", a);
  }
  for (int a = 0; a < 3; ++a) c->ax[a].build(f[a], n[a]);
  return upload_grid(c);
}

int lc_set_stretching(lc_ctx* c, int kind, double param) {
  if (!c) return LC_EINVAL;
  if (kind == LC_TANH && !(param > 1.0)) return fail(c, LC_EINVAL, "tanh ratio must exceed 1");
  if (kind != LC_UNIFORM && kind != LC_SINE && kind != LC_TANH) return fail(c, LC_EINVAL, "unknown stretching");
  const int n[3] = {c->nx, c->ny, c->nz};
  std::vector<double> f[3];
  for (int a = 0; a < 3; ++a) {
    f[a].resize(n[a] + 1);
    for (int i = 0; i <= n[a]; ++i) {
      const double xi = (double)i / n[a];
      double x = xi;
      if (kind == LC_SINE) {
        x = xi - 0.0975 * std::sin(2.0 * M_PI * xi);  // Section 3, eq. 5
      } else if (kind == LC_TANH) {
        const double b = std::acosh(std::sqrt(param));
        x = 0.5 * (1.0 + std::tanh(b * (2.0 * xi - 1.0)) / std::tanh(b));
      }
      f[a][i] = x;
    }
    f[a][0] = 0.0;
    f[a][n[a]] = 1.0;
  }
  return lc_set_grid(c, f[0].data(), f[1].data(), f[2].data());
}

int lc_get_grid(const lc_ctx* c, double* xf, double* yf, double* zf) {
  if (!c || !xf || !yf || !zf) return LC_EINVAL;
  std::copy(c->ax[0].xf.begin(), c->ax[0].xf.end(), xf);
  std::copy(c->ax[1].xf.begin(), c->ax[1].xf.end(), yf);
  std::copy(c->ax[2].xf.begin(), c->ax[2].xf.end(), zf);
  return LC_OK;
}

int lc_set_poisson_method(lc_ctx* c, int method) {
  if (!c) return LC_EINVAL;
  if (method != LC_POISSON_TPF && method != LC_POISSON_TPT) return fail(c, LC_EINVAL, "unknown Poisson method %d", method);
  c->poisson_method = method;
  return LC_OK;
}

int lc_set_re(lc_ctx* c, double re) {
  if (!c) return LC_EINVAL;
  if (!(re > 0.0) || !std::isfinite(re)) return fail(c, LC_EINVAL, "Re must be positive and finite");
  c->re = re;
  return LC_OK;
}

int lc_set_lid(lc_ctx* c, double alpha) {
  if (!c) return LC_EINVAL;
  if (!std::isfinite(alpha)) return fail(c, LC_EINVAL, "lid angle must be finite");
  c->alpha = alpha;
  return LC_OK;
}

int lc_set_base_flow(lc_ctx* c, const double* U) {
  if (!c || !aligned(U)) return fail(c, LC_EINVAL, "null or misaligned base flow");
  HIPCHK(c, hipMemcpyAsync(c->U, U, c->nvel * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  KLAUNCH(c, LC_K_VECTOR, launch_zero_walls(c->U, c->nx, c->ny, c->nz, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LC_OK;
}

int lc_get_base_flow(lc_ctx* c, double* U, double* P) {
  if (!c || !aligned(U) || (P && !aligned(P))) return fail(c, LC_EINVAL, "bad pointers");
  HIPCHK(c, hipMemcpyAsync(U, c->U, c->nvel * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if (P) {
    // the pressure of the steady equations: R(U) - G P divergence-free, sum V P = 0 (at a
    // steady state R(U) = G P); the projection's velocity goes to one Krylov vector
    int rc = check_ready(c);
    if (rc) return rc;
    double* tmp = nullptr;
    long ld = 0;
    if ((rc = krylov_ws(c, 1, &tmp, &ld))) return rc;
    KLAUNCH(c, LC_K_RESIDUAL, launch_momentum(c->g, c->U, c->U, c->w, 1.0 / c->re, 0.5, true, std::cos(c->alpha),
                                              std::sin(c->alpha), c->stream));
    lc_stats st;
    rc = lc_project(c, c->w, tmp, P, LC_FP64, 1e-13, 4, &st);
    if (rc < 0) return rc;
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LC_OK;
}

int lc_jacobian_apply(lc_ctx* c, const double* v, double* w) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (!aligned(v) || !aligned(w) || v == w) return fail(c, LC_EINVAL, "bad or aliased velocity pointers");
  KLAUNCH(c, LC_K_MOMENTUM, launch_momentum(c->g, c->U, v, w, 1.0 / c->re, 1.0, false, 0, 0, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LC_OK;
}

int lc_residual(lc_ctx* c, const double* U, double* R) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (!aligned(U) || !aligned(R) || U == R) return fail(c, LC_EINVAL, "bad or aliased velocity pointers");
  KLAUNCH(c, LC_K_RESIDUAL, launch_momentum(c->g, U, U, R, 1.0 / c->re, 0.5, true, std::cos(c->alpha), std::sin(c->alpha),
                            c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LC_OK;
}

int lc_divergence(lc_ctx* c, const double* v, double* r, double* vn) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (!aligned(v) || !aligned(r)) return fail(c, LC_EINVAL, "bad pointers");
  double nrm = 0.0;
  rc = vnorm_div(c, v, r, &nrm);
  if (rc) return rc;
  if (vn) *vn = nrm;
  return LC_OK;
}

int lc_poisson_solve(lc_ctx* c, const double* r, double* phi, int precision) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (!aligned(r) || !aligned(phi)) return fail(c, LC_EINVAL, "bad pointers");
  if (precision != LC_FP64 && precision != LC_MIXED) return fail(c, LC_EINVAL, "unknown precision");
  rc = poisson(c, r, phi, precision);
  if (rc) return rc;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LC_OK;
}

int lc_correct(lc_ctx* c, const double* w, const double* phi, double* v, double* p) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (!aligned(w) || !aligned(phi) || !aligned(v) || (p && !aligned(p)) || v == w)
    return fail(c, LC_EINVAL, "bad pointers");
  KLAUNCH(c, LC_K_CORRECT, launch_correct(c->g, w, phi, v, p, false, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LC_OK;
}

}  // extern "C"

namespace {
// per-phase device time of the launches recorded since rec0 (profiling on), else -1
void fill_phases(lc_ctx* c, lc_stats* S, size_t rec0) {
  if (!S) return;
  S->ms_stencil = S->ms_poisson = S->ms_update = S->ms_network = -1.0;
  if (!c->prof || hipStreamSynchronize(c->stream) != hipSuccess) return;
  double t[4] = {0.0, 0.0, 0.0, 0.0};
  for (size_t q = rec0; q < c->recs.size(); ++q) {
    const int k = c->recs[q].kid;
    const int ph = (k == LC_K_MOMENTUM || k == LC_K_RESIDUAL || k == LC_K_DIVERGENCE) ? 0
                   : (k == LC_K_TP_X || k == LC_K_TP_Y || k == LC_K_TP_Z || k == LC_K_EIGSCALE ||
                      k == LC_K_TRIDIAG || k == LC_K_CAST)
                       ? 1
                   : k == LC_K_CORRECT                             ? 2
                   : (k == LC_K_NN_FORWARD || k == LC_K_NN_MISC) ? 3
                                                                   : -1;
    float ms = 0.f;
    if (ph >= 0 && hipEventElapsedTime(&ms, c->recs[q].a, c->recs[q].b) == hipSuccess) t[ph] += ms;
  }
  S->ms_stencil = t[0];
  S->ms_poisson = t[1];
  S->ms_update = t[2];
  S->ms_network = t[3];
}

int project_impl(lc_ctx* c, const double* w, double* v, double* p, int precision, double tol, int max_iter,
                 lc_stats* st) {
  const double t0 = now_ms();
  int rc = check_ready(c);
  if (rc) return rc;
  if (!aligned(w) || !aligned(v) || (p && !aligned(p)) || v == w || p == w || p == v)
    return fail(c, LC_EINVAL, "bad pointers");
  if (precision != LC_FP64 && precision != LC_MIXED && precision != LC_LEARNED)
    return fail(c, LC_EINVAL, "unknown precision");
  if (precision == LC_LEARNED && !c->net) return fail(c, LC_ESTATE, "no network attached for the learned form");
  if (!(tol >= 0.0) || max_iter < 1) return fail(c, LC_EINVAL, "bad tolerance or iteration cap");
  lc_stats local{};
  lc_stats& S = st ? *st : local;
  std::memset(&S, 0, sizeof S);
  S.guess_eps = 1.0;
  double n0 = 0.0;
  rc = vnorm_div(c, w, c->r, &n0);
  if (rc) return rc;
  if (!std::isfinite(n0)) return fail(c, LC_EINVAL, "non-finite input");
  S.rho0 = n0;
  if (n0 == 0.0) {
    // already divergence-free: v = w (walls zeroed), p = 0
    HIPCHK(c, hipMemsetAsync(c->phi, 0, c->ncell * sizeof(double), c->stream));
    KLAUNCH(c, LC_K_CORRECT, launch_correct(c->g, w, c->phi, v, p, false, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    S.ms_total = now_ms() - t0;
    return LC_OK;
  }
  // Learned form: the network's correction starts the loop (v = w - G phi0, p = phi0),
  // then mixed-precision passes; without gain it falls back to v = w, p = 0.
  bool started = false;
  const int pass_precision = precision == LC_LEARNED ? LC_MIXED : precision;
  if (precision == LC_LEARNED) {
    double fit = 1.0;
    rc = learned_start(c, w, v, p, &started, &fit);
    if (rc) return rc;
    if (started) {
      double nk = 0.0;
      rc = vnorm_div(c, v, c->r, &nk);
      if (rc) return rc;
      S.guess_used = 1;
      S.guess_eps = nk / n0;
      if (!std::isfinite(S.guess_eps)) return fail(c, LC_EINVAL, "non-finite divergence after the learned guess");
      S.rho = S.guess_eps;
      if (S.rho <= tol) {
        S.ms_total = now_ms() - t0;
        return LC_OK;
      }
    }
  }
  // SIMPLE loop (Section 3): v = w, p = 0; repeat {solve; v -= G phi; p += phi}
  // The certificate of an FP64 pass (exact solve: it nearly always ends the loop) only
  // reduces the norm; D v is then written again if another pass needs it.  FP32 passes
  // (one more always follows at tight tolerances) keep D v from the certificate.
  for (int it = 0; it < max_iter; ++it) {
    rc = poisson(c, c->r, c->phi, pass_precision);
    if (rc) return rc;
    KLAUNCH(c, LC_K_CORRECT, launch_correct(c->g, w, c->phi, v, p, started || it > 0, c->stream));
    double nk = 0.0;
    const bool keep_r = pass_precision != LC_FP64;
    rc = vnorm_div(c, v, keep_r ? c->r : nullptr, &nk);
    if (rc) return rc;
    if (!keep_r && nk / n0 > tol && it + 1 < max_iter) {
      rc = vnorm_div(c, v, c->r, &nk);
      if (rc) return rc;
    }
    S.iterations = it + 1;
    S.rho = nk / n0;
    if (it < 16) S.rho_hist[it] = S.rho;
    if (!std::isfinite(S.rho)) return fail(c, LC_EINVAL, "non-finite divergence during projection");
    if (S.rho <= tol) {
      S.ms_total = now_ms() - t0;
      return LC_OK;
    }
  }
  S.ms_total = now_ms() - t0;
  return LC_ENOTCONV;
}

}  // namespace

extern "C" {

int lc_project(lc_ctx* c, const double* w, double* v, double* p, int precision, double tol, int max_iter,
               lc_stats* st) {
  const size_t rec0 = c ? c->recs.size() : 0;
  const int rc = project_impl(c, w, v, p, precision, tol, max_iter, st);
  if (c && rc >= 0) fill_phases(c, st, rec0);
  return rc;
}

int lc_krylov_vector(lc_ctx* c, const double* vin, double* vout, double* pout, int precision, double tol,
                     int max_iter, lc_stats* st) {
  const double t0 = now_ms();
  int rc = check_ready(c);
  if (rc) return rc;
  if (!aligned(vin) || !aligned(vout) || vin == vout) return fail(c, LC_EINVAL, "bad or aliased pointers");
  const size_t rec0 = c->recs.size();
  KLAUNCH(c, LC_K_MOMENTUM, launch_momentum(c->g, c->U, vin, c->w, 1.0 / c->re, 1.0, false, 0, 0, c->stream));
  rc = project_impl(c, c->w, vout, pout, precision, tol, max_iter, st);
  if (rc >= 0) fill_phases(c, st, rec0);
  if (st) st->ms_total = now_ms() - t0;
  return rc;
}

int lc_dot(lc_ctx* c, const double* a, const double* b, double* out) {
  if (!c || !aligned(a) || !aligned(b) || !out) return fail(c, LC_EINVAL, "bad pointers");
  int np = 0;
  KLAUNCH(c, LC_K_VECTOR, launch_dot_partials(a, b, c->nvel, c->partials, &np, c->stream));
  return reduce_to_host(c, np, out);
}

}  // extern "C"

static const char* kKernelNames[LC_K_COUNT] = {"momentum", "residual", "divergence", "correct",  "tp_x",
                                                "tp_y",     "tp_z",     "eigscale",   "reduce",   "cast",
                                                "vector",   "nn_forward", "nn_misc",  "planes",  "tridiag"};

extern "C" const char* lc_profile_name(int k) { return (k >= 0 && k < LC_K_COUNT) ? kKernelNames[k] : nullptr; }

extern "C" int lc_profile_enable(lc_ctx* c, int on) {
  if (!c) return LC_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->recs.clear();
  c->ev_used = 0;
  c->prof = on != 0;
  return LC_OK;
}

extern "C" int lc_profile_read(lc_ctx* c, int k, double* total_ms, long* launches) {
  if (!c || k < 0 || k >= LC_K_COUNT || !total_ms || !launches) return LC_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double t = 0.0;
  long n = 0;
  for (const auto& r : c->recs) {
    if (r.kid != k) continue;
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, r.a, r.b));
    t += ms;
    ++n;
  }
  *total_ms = t;
  *launches = n;
  return LC_OK;
}

extern "C" int lc_stream_probe(int kind, size_t bytes, int reps, void* hip_stream, double* tbps, double* us) {
  if (kind < 0 || kind > 2 || bytes < 4096 || reps < 1 || !tbps) return LC_EINVAL;
  const size_t n2 = bytes / 16;
  hipStream_t st = (hipStream_t)hip_stream;
  double *a = nullptr, *b = nullptr, *c = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = LC_OK;
  if (hipMalloc((void**)&a, n2 * 16) != hipSuccess || hipMalloc((void**)&b, n2 * 16) != hipSuccess ||
      hipMalloc((void**)&c, n2 * 16 + 8) != hipSuccess) {
    rc = LC_ENOMEM;
  } else if (hipMemsetAsync(a, 0, n2 * 16, st) != hipSuccess || hipMemsetAsync(b, 0, n2 * 16, st) != hipSuccess ||
             hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    rc = LC_EHIP;
  } else {
    double* sink = c + 2 * n2;
    bool ok = true;
    for (int w = 0; w < 3 && ok; ++w) ok = launch_probe(kind, a, b, c, n2, sink, st) == hipSuccess;
    ok = ok && hipEventRecord(e0, st) == hipSuccess;
    for (int r = 0; r < reps && ok; ++r) ok = launch_probe(kind, a, b, c, n2, sink, st) == hipSuccess;
    ok = ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
    float ms = 0.f;
    ok = ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
    if (!ok) {
      rc = LC_EHIP;
    } else {
      const double moved = (kind == 0 ? 2.0 : kind == 1 ? 3.0 : 1.0) * (double)(n2 * 16);
      const double t = (double)ms * 1e-3 / reps;
      *tbps = moved / t / 1e12;
      if (us) *us = t * 1e6;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (a) (void)hipFree(a);
  if (b) (void)hipFree(b);
  if (c) (void)hipFree(c);
  return rc;
}

extern "C" int lc_axis_modes(int n, const double* faces, double* lam, double* S, double* Wf) {
  if (n < 1 || !faces || !lam || !S || !Wf) return LC_EINVAL;
  for (int i = 0; i < n; ++i)
    if (!(faces[i + 1] > faces[i])) return LC_EINVAL;
  AxisHost A;
  A.build(faces, n);
  std::vector<double> l, s, w;
  if (!neumann_modes(n, A.d.data(), A.dd.data(), l, s, w)) return LC_EINVAL;
  std::copy(l.begin(), l.end(), lam);
  std::copy(s.begin(), s.end(), S);
  std::copy(w.begin(), w.end(), Wf);
  return LC_OK;
}
