// Context of the C ABI and the helpers shared by the host-side drivers.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/lidkrylov.h"
#include "lk_internal.h"

namespace lk {

struct AxisHost {
  std::vector<double> xf, d, dd, th, rd, rdd;
  void build(const double* faces, int n) {
    xf.assign(faces, faces + n + 1);
    d.resize(n);
    for (int i = 0; i < n; ++i) d[i] = xf[i + 1] - xf[i];
    std::vector<double> c(n);
    for (int i = 0; i < n; ++i) c[i] = 0.5 * (xf[i] + xf[i + 1]);
    dd.resize(n + 1);
    dd[0] = 0.5 * d[0];
    dd[n] = 0.5 * d[n - 1];
    for (int i = 1; i < n; ++i) dd[i] = c[i] - c[i - 1];
    th.assign(n + 1, 0.5);
    for (int i = 1; i < n; ++i) th[i] = d[i - 1] / (2.0 * dd[i]);
    rd.resize(n);
    rdd.resize(n + 1);
    for (int i = 0; i < n; ++i) rd[i] = 1.0 / d[i];
    for (int i = 0; i <= n; ++i) rdd[i] = 1.0 / dd[i];
  }
};

// Tensor-product factorization of one axis, device copies in float64 and float32.
// On a mirror-symmetric axis the modes are also stored parity-sorted (he even modes,
// then ho odd ones) as half-size matrices for the folded transforms.
struct AxisModes {
  double* lam = nullptr;          // n eigenvalues
  double *F = nullptr, *Bk = nullptr, *FT = nullptr, *BkT = nullptr;
  float *F32 = nullptr, *Bk32 = nullptr, *FT32 = nullptr, *BkT32 = nullptr;
  bool sym = false;
  int he = 0, ho = 0;
  double* lam_s = nullptr;        // eigenvalues in parity-sorted order
  // [0] Ae (he x he), [1] Ao (ho x ho), [2] Se (he x he), [3] So (he x ho),
  // [4] FTe (he x he), [5] FTo (ho x ho), [6] SeT (he x he), [7] SoT (ho x he)
  double* h64[8] = {};
  float* h32[8] = {};
  // matrix-core fragment packs of Ae, Ao, Se, So (he <= kMfMaxHalf)
  bool mf = false;
  double* p64[4] = {};
  float* p32[4] = {};
};

}  // namespace lk

struct lc_ctx {
  using AxisHost = lk::AxisHost;
  using AxisModes = lk::AxisModes;
  using GridDev = lk::GridDev;
  int nx = 0, ny = 0, nz = 0;
  hipStream_t stream = nullptr;
  std::string err;
  double re = 1.0, alpha = 0.0;
  bool grid_ready = false;
  AxisHost ax[3];  // x, y, z
  double* metric = nullptr;  // device storage of rd, rdd, th, d for the three axes
  GridDev g{};
  AxisModes modes[3];
  void* modes_mem = nullptr;
  int zero_mode[3] = {0, 0, 0};
  int poisson_method = 1;  // LC_POISSON_TPT (default) or LC_POISSON_TPF
  // fields
  double* U = nullptr;   // base flow (velocity)
  double* w = nullptr;   // momentum work vector (velocity)
  double* r = nullptr;   // divergence (cell)
  double* phi = nullptr; // correction (cell)
  double* t1 = nullptr;  // transform temporaries (cell)
  double* t2 = nullptr;
  float *r32 = nullptr, *t1_32 = nullptr, *t2_32 = nullptr;
  double* partials = nullptr;
  int max_parts = 0;
  double* dsum = nullptr;   // device scalar
  double* hsum = nullptr;   // pinned host scalar
  size_t nvel = 0, ncell = 0;
  // profiling: event pairs around launches on `stream`
  struct Rec {
    int kid;
    hipEvent_t a, b;
  };
  // Krylov drivers: basis workspace (grown on demand), small device/host scalars
  double* kws = nullptr;
  size_t kws_n = 0;
  double* dsmall = nullptr;  // kSmall doubles
  double* hsmall = nullptr;  // kSmall doubles, pinned
  double* ucr = nullptr;     // critical-Re driver: two stored steady states + a residual
  lc_net* net = nullptr;     // learned guess (not owned)
  // Stokes-preconditioned vectors: the viscous step (I/dt - Re^-1 Lap_0)^-1 by the tensor
  // product of the Dirichlet factors of each axis (cell-centred: n points, faces: n + 1),
  // built on first use for the current grid
  bool axis_sym[3] = {false, false, false};
  bool stokes_ready = false;
  void* stokes_mem = nullptr;
  AxisModes vcell[3], vface[3];
  std::vector<double> vlam_cell[3], vlam_face[3];  // eigenvalues in kernel order (parity-sorted if folded)
  double* vscale = nullptr;   // device: scaled eigenvalues (cell x, face x, cell y, face y, cell z, face z)
  size_t vscale_off[6] = {};
  double vscale_re = 0.0, vscale_dt = -1.0;  // (Re, dt) vscale was built for
  double* hs = nullptr;       // component-sized transform temporary
  double stokes_dt = 0.0;     // Newton preconditioning by the viscous step (0: off)
  // Caller-provided workspace (lc_create_in): every device buffer of the context is carved
  // from it in a fixed order at creation, the Krylov vectors take what remains, and the
  // library allocates no device memory.  `dry` sizes the carve without memory (the query).
  char* arena = nullptr;
  size_t arena_size = 0, arena_used = 0;
  bool dry = false;
  bool prof = false;
  std::vector<Rec> recs;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
};


namespace lk {

constexpr int kSmall = 16384;

// Device memory of a context: carved from the caller's workspace when there is one (256-byte
// aligned; hipErrorOutOfMemory when it is exhausted), else hipMalloc'ed.  Freed by
// lc_destroy only in the second case.
hipError_t ctx_alloc(lc_ctx* c, void** p, size_t bytes);
template <typename T>
hipError_t dalloc(lc_ctx* c, T** p, size_t n) {
  return ctx_alloc(c, (void**)p, (n ? n : 1) * sizeof(T));
}
// Sizes of the lazily allocated buffers (doubles unless bytes): grid metrics, viscous-step
// factors, the largest velocity component; Krylov vectors of drivers with basis length m.
size_t metric_doubles(int nx, int ny, int nz);
size_t viscous_bytes(int nx, int ny, int nz);
size_t component_max(int nx, int ny, int nz);
int krylov_vectors(int m);
// Velocities the critical-Re driver keeps: two steady states, a residual, the last leading
// eigenvector (real, imaginary part) and the next Arnoldi start.
constexpr int kCriticalVectors = 6;
// Krylov vectors: `nvec` velocities ld = lc_vel_size rounded up to 64 apart (grown on demand,
// or the remainder of the caller's workspace: LC_ENOMEM when it holds fewer).
int krylov_ws(lc_ctx* c, int nvec, double** p, long* ld);

int fail(lc_ctx* c, int code, const char* fmt, ...);
hipEvent_t take_event(lc_ctx* c);
double now_ms();
bool aligned(const void* p);
int check_ready(lc_ctx* c);
// fixed-order device reduction of c->partials (sum or max) to a host scalar
int reduce_to_host(lc_ctx* c, int nparts, double* out);
int reduce_max_to_host(lc_ctx* c, int nparts, double* out);
// |D v|_V (r receives D v when not null)
int vnorm_div(lc_ctx* c, const double* v, double* r, double* out);
// pressure-correction solve in the given precision
int poisson(lc_ctx* c, const double* r, double* phi, int precision);
// Euclidean dot product / max |x| of velocity vectors, host results
int vdot(lc_ctx* c, const double* a, const double* b, double* out);
int vmaxabs(lc_ctx* c, const double* a, double* out);
// viscous step u = (I/dt - Re^-1 Lap_0)^-1 f (velocities, distinct; dt may be infinite),
// and the Stokes step u = P (viscous step of f) (lk_stokes.cpp; uses c->w)
int viscous_solve(lc_ctx* c, const double* f, double* u, double dt);
int stokes_step(lc_ctx* c, const double* f, double* u, double dt, int precision, double tol, int max_iter);
// learned start of the SIMPLE loop (see lk_nn_host.cpp); requires c->net
int learned_start(lc_ctx* c, const double* w, double* v, double* p, bool* used, double* eps_fit);

}  // namespace lk

#define HIPCHK(c, expr)                                                                           \
  do {                                                                                            \
    hipError_t e_ = (expr);                                                                       \
    if (e_ != hipSuccess) return lk::fail((c), LC_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// Launch with optional event timing (kernel class `kid`).
#define KLAUNCH(c, kid, expr)                                                        \
  do {                                                                               \
    hipEvent_t a_ = nullptr;                                                         \
    if ((c)->prof && (a_ = lk::take_event(c))) (void)hipEventRecord(a_, (c)->stream); \
    HIPCHK(c, expr);                                                                 \
    if ((c)->prof && a_) {                                                           \
      hipEvent_t b_ = lk::take_event(c);                                             \
      if (b_) {                                                                      \
        (void)hipEventRecord(b_, (c)->stream);                                       \
        (c)->recs.push_back({(kid), a_, b_});                                        \
      }                                                                              \
    }                                                                                \
  } while (0)
