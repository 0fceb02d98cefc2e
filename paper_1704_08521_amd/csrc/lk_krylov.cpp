// Krylov-subspace drivers on SIMPLE-evaluated Krylov vectors (Section 3):
// Newton steps whose corrections are solved by restarted GMRES with a
// BiCGstab(2) hand-off on saturation, and the leading eigenvalues of eq. 7 by
// implicitly restarted Arnoldi with classical Gram-Schmidt (repeated when the norm
// drops) in float64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "lk_ctx.h"
#include "lk_internal.h"
#include "lk_linalg.h"

using namespace lk;

namespace {

struct Basis {
  double* p;
  long ld;
  double* at(int i) const { return p + (size_t)i * ld; }
};

// Device workspace of `nvec` velocity vectors, ld apart.
int ensure_ws(lc_ctx* c, int nvec, Basis* B) { return krylov_ws(c, nvec, &B->p, &B->ld); }

struct KMap {
  int precision;
  double ptol;
  int pmax;
  long count = 0;
  double sdt = 0.0;      // > 0: right preconditioning by the viscous step with this time step
  double* z = nullptr;   // its output (velocity), when sdt > 0
};

bool verbose() {  // read on every call: callers may switch the trace on around one driver call
  const char* e = std::getenv("LK_VERBOSE");
  return e && e[0] && e[0] != '0';
}

// out = P L_U in (one Krylov vector), or with right preconditioning
// out = P L_U P (I/dt - Re^-1 Lap_0)^-1 in; a projection that misses its tolerance is an
// error here (the Krylov drivers need the divergence-free subspace).
int kmap(lc_ctx* c, KMap& K, const double* in, double* out) {
  lc_stats st;
  if (K.sdt > 0.0) {
    int rc = stokes_step(c, in, K.z, K.sdt, K.precision, K.ptol, K.pmax);
    if (rc == LC_ENOTCONV) return fail(c, LC_ENOTCONV, "preconditioner projection missed its tolerance");
    if (rc) return rc;
    in = K.z;
  }
  int rc = lc_krylov_vector(c, in, out, nullptr, K.precision, K.ptol, K.pmax, &st);
  K.count++;
  if (rc == LC_ENOTCONV) return fail(c, LC_ENOTCONV, "projection missed its tolerance (rho = %.3e)", st.rho);
  if (rc) {
    const std::string msg = c->err;
    return fail(c, rc, "Krylov vector %ld: %s", K.count, msg.c_str());
  }
  return LC_OK;
}

int vscale(lc_ctx* c, double a, double* x) {
  KLAUNCH(c, LC_K_VECTOR, launch_scale(c->nvel, a, x, c->stream));
  return LC_OK;
}

int vaxpy(lc_ctx* c, double a, const double* x, double* y) {
  KLAUNCH(c, LC_K_VECTOR, launch_axpy(c->nvel, a, x, y, c->stream));
  return LC_OK;
}

int vcopy(lc_ctx* c, const double* x, double* y) {
  HIPCHK(c, hipMemcpyAsync(y, x, c->nvel * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  return LC_OK;
}

double vnorm(double s) { return std::sqrt(std::max(s, 0.0)); }

// x <- P x (exact float64 projection; tmp is overwritten).  Removes the
// divergent part that residuals computed at the rounding floor carry: left in a
// Krylov basis it would let the solution pick up components in the null space
// of P L_U, which lies outside the divergence-free space.
int vproject(lc_ctx* c, double* x, double* tmp) {
  lc_stats st;
  const int rc = lc_project(c, x, tmp, nullptr, LC_FP64, 1e-13, 4, &st);
  if (rc < 0) return rc;
  return vcopy(c, tmp, x);
}

// Orthogonalizes w against the nv basis vectors of V: classical Gram-Schmidt (one
// block dot-product pass and one update pass over the basis, coefficients staying on the
// device), repeated once when the norm drops below 1/sqrt 2 of its value (the DGKS
// criterion; twice-classical Gram-Schmidt is orthogonal to working precision).  h[0..nv)
// receives the projections, h[nv] the final norm.
int mgs(lc_ctx* c, const Basis& V, int nv, double* w, double* h) {
  if (nv + 1 > kSmall) return fail(c, LC_EINVAL, "basis too large");
  double before = 0.0;
  int rc = vdot(c, w, w, &before);
  if (rc) return rc;
  before = vnorm(before);
  std::fill(h, h + nv + 1, 0.0);
  double after = before;
  for (int pass = 0; pass < 2; ++pass) {
    KLAUNCH(c, LC_K_VECTOR, launch_gs_dot(V.at(0), V.ld, nv, w, c->nvel, c->partials, c->dsmall, c->stream));
    KLAUNCH(c, LC_K_VECTOR, launch_gs_update(V.at(0), V.ld, nv, c->dsmall, w, c->nvel, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->hsmall, c->dsmall, nv * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    double a2 = 0.0;
    rc = vdot(c, w, w, &a2);  // synchronizes the stream
    if (rc) return rc;
    for (int i = 0; i < nv; ++i) h[i] += c->hsmall[i];
    after = vnorm(a2);
    if (!(after < 0.7071067811865476 * before)) break;
    before = after;
  }
  h[nv] = after;
  return LC_OK;
}

bool is_pair(cplx a, cplx b) {
  return std::fabs(a.imag()) > 0.0 && std::abs(a - std::conj(b)) <= 1e-8 * std::max(std::abs(a), 1e-300);
}

}  // namespace

extern "C" int lc_hessenberg_eigvals(int m, const double* H, double* re, double* im) {
  if (m < 1 || !H || !re || !im) return LC_EINVAL;
  std::vector<double> A((size_t)m * m);
  for (int r = 0; r < m; ++r)
    for (int col = 0; col < m; ++col) A[(size_t)r * m + col] = (r > col + 1) ? 0.0 : H[(size_t)r * m + col];
  std::vector<cplx> lam;
  if (!hess_eigvals(m, A, lam) || (int)lam.size() != m) return LC_EINVAL;
  for (int i = 0; i < m; ++i) {
    re[i] = lam[i].real();
    im[i] = lam[i].imag();
  }
  return LC_OK;
}

// ============================================================== Arnoldi
namespace {

// Implicitly restarted Arnoldi (see lc_arnoldi_leading); the first `nvec` Ritz vectors go
// to vec_re / vec_im (nvel apart).
int arnoldi_run(lc_ctx* c, int k, int m, double tol, int max_restarts, unsigned long long seed, const double* v0,
                int precision, double proj_tol, double* eig_re, double* eig_im, double* resid, double* vec_re,
                double* vec_im, int nvec, int* n_out, long* n_vectors) {
  KMap K{precision, proj_tol, 8};
  Basis V, W;
  int rc = ensure_ws(c, 2 * (m + 1), &V);
  if (rc) return rc;
  W.p = V.p + (size_t)(m + 1) * V.ld;
  W.ld = V.ld;
  // divergence scale of a vector with no solenoidal structure (a seeded uniform [-1, 1)
  // field): a Ritz vector whose relative divergence is a sizeable fraction of it is not an
  // eigenvector of eq. 7 (see `spurious` below)
  KLAUNCH(c, LC_K_VECTOR, launch_uniform(W.at(0), c->nvel, seed, c->stream));
  KLAUNCH(c, LC_K_VECTOR, launch_zero_walls(W.at(0), c->nx, c->ny, c->nz, c->stream));
  double dref = 0.0, wn = 0.0;
  if ((rc = vnorm_div(c, W.at(0), nullptr, &dref))) return rc;
  if ((rc = vdot(c, W.at(0), W.at(0), &wn))) return rc;
  dref /= std::max(vnorm(wn), 1e-300);
  // start vector: that random field, or the caller's, projected onto the divergence-free space
  if (v0) {
    if ((rc = vcopy(c, v0, W.at(0)))) return rc;
    KLAUNCH(c, LC_K_VECTOR, launch_zero_walls(W.at(0), c->nx, c->ny, c->nz, c->stream));
  }
  lc_stats st;
  rc = lc_project(c, W.at(0), V.at(0), nullptr, LC_FP64, 1e-13, 4, &st);
  if (rc < 0) return rc;
  double nrm = 0.0;
  if ((rc = vdot(c, V.at(0), V.at(0), &nrm))) return rc;
  if ((rc = vscale(c, 1.0 / vnorm(nrm), V.at(0)))) return rc;

  std::vector<double> H((size_t)(m + 1) * m, 0.0);  // (m+1) x m, row-major
  auto h = [&](int r, int col) -> double& { return H[(size_t)r * m + col]; };
  std::vector<double> hcol(m + 2);
  std::vector<cplx> theta, wanted;
  std::vector<double> res;
  std::vector<std::vector<cplx>> Y;
  int j0 = 0, kk = k, kc = k;
  double hnorm = 0.0;
  bool converged = false;
  for (int restart = 0; restart <= max_restarts; ++restart) {
    for (int j = j0; j < m; ++j) {
      if ((rc = kmap(c, K, V.at(j), V.at(j + 1)))) return rc;
      if ((rc = mgs(c, V, j + 1, V.at(j + 1), hcol.data()))) return rc;
      for (int i = 0; i <= j; ++i) h(i, j) = hcol[i];
      h(j + 1, j) = hcol[j + 1];
      if (hcol[j + 1] > 0.0 && (rc = vscale(c, 1.0 / hcol[j + 1], V.at(j + 1)))) return rc;
    }
    // Ritz values of H_m, largest real part first; near-zero values (components
    // outside the divergence-free space grown by rounding) count as unwanted
    std::vector<double> Hm((size_t)m * m);
    for (int r = 0; r < m; ++r)
      for (int col = 0; col < m; ++col) Hm[(size_t)r * m + col] = h(r, col);
    hnorm = 0.0;
    for (double x : Hm) hnorm = std::max(hnorm, std::fabs(x));
    if (!hess_eigvals(m, Hm, theta)) return fail(c, LC_EINVAL, "Hessenberg QR did not converge");
    double tmax = 0.0;
    for (const cplx& t : theta) tmax = std::max(tmax, std::abs(t));
    // P L_U is zero on the gradient directions, to the right of the wanted
    // eigenvalues; rounding-level components there grow under the restart filter
    // and show up as Ritz values near 0.  Sorting those among the unwanted makes
    // them exact shifts, which removes them when (and only when) they appear.  A
    // genuine eigenvalue can be near 0 too (a real eigenvalue crossing the imaginary
    // axis), so a near-zero Ritz value that would be kept is judged by its Ritz
    // vector: spurious when that vector is far from divergence-free.
    auto by_real = [](const cplx& a, const cplx& b) {
      if (a.real() != b.real()) return a.real() > b.real();
      return a.imag() > b.imag();
    };
    // Ritz values whose residual, recomputed with the Krylov map itself, failed (see below)
    std::vector<cplx> rejected;
    auto is_rejected = [&](const cplx& t) {  // the value or its conjugate
      for (const cplx& r : rejected) {
        const double close = 1e-12 * std::abs(r);
        if (std::abs(t - r) <= close || std::abs(t - std::conj(r)) <= close) return true;
      }
      return false;
    };
    for (int pass = 0; pass < 4; ++pass) {
      std::stable_sort(theta.begin(), theta.end(), by_real);
      std::vector<char> spur(m, 0);
      for (int i = 0; i < m; ++i) spur[i] = is_rejected(theta[i]);
      const int front = std::min(m, k + std::max(1, (m - k) / 3) + 2);
      for (int i = 0; i < front; ++i) {
        if (spur[i] || !(std::abs(theta[i]) < 1e-5 * tmax)) continue;
        std::vector<cplx> y;
        if (!hess_eigvec(m, Hm, theta[i], y)) return fail(c, LC_EINVAL, "Ritz vector failed");
        std::vector<double> Qy((size_t)m * 2);
        for (int r = 0; r < m; ++r) {
          Qy[(size_t)r * 2] = y[r].real();
          Qy[(size_t)r * 2 + 1] = y[r].imag();
        }
        std::memcpy(c->hsmall, Qy.data(), Qy.size() * sizeof(double));
        HIPCHK(c, hipMemcpyAsync(c->dsmall, c->hsmall, Qy.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
        KLAUNCH(c, LC_K_VECTOR, launch_combine(V.p, V.ld, m, c->dsmall, 2, W.p, W.ld, c->nvel, c->stream));
        double d0 = 0.0, d1 = 0.0, n0 = 0.0, n1 = 0.0;
        if ((rc = vnorm_div(c, W.at(0), nullptr, &d0)) || (rc = vnorm_div(c, W.at(1), nullptr, &d1)) ||
            (rc = vdot(c, W.at(0), W.at(0), &n0)) || (rc = vdot(c, W.at(1), W.at(1), &n1)))
          return rc;
        const double rel = std::hypot(d0, d1) / std::max(vnorm(n0 + n1), 1e-300) / std::max(dref, 1e-300);
        spur[i] = rel > 1e-6;
        if (verbose())
          std::fprintf(stderr, "[lk arnoldi] near-zero Ritz value %.3e%+.3ei: relative divergence %.2e (%s)\n",
                       theta[i].real(), theta[i].imag(), rel, spur[i] ? "spurious" : "kept");
      }
      {
        std::vector<std::pair<cplx, char>> tv(m);
        for (int i = 0; i < m; ++i) tv[i] = {theta[i], spur[i]};
        std::stable_sort(tv.begin(), tv.end(), [&](const std::pair<cplx, char>& a, const std::pair<cplx, char>& b) {
          if (a.second != b.second) return b.second != 0;
          return by_real(a.first, b.first);
        });
        for (int i = 0; i < m; ++i) theta[i] = tv[i].first;
      }
      for (int i = 0; i + 1 < m; ++i)  // within a conjugate pair: positive imaginary part first
        if (is_pair(theta[i], theta[i + 1])) {
          if (theta[i].imag() < theta[i + 1].imag()) std::swap(theta[i], theta[i + 1]);
          ++i;
        }
      kc = k;  // values tested and returned (a conjugate pair is not split)
      if (kc < m && is_pair(theta[kc - 1], theta[kc])) ++kc;
      // the restart keeps more vectors than requested: a wanted eigenvalue whose
      // early Ritz approximation falls among the unwanted would otherwise be
      // filtered out by its own exact shift
      kk = std::min(m - 3, std::max(kc, k + std::max(1, (m - k) / 3)));
      if (kk < m && is_pair(theta[kk - 1], theta[kk])) ++kk;
      // residual estimates |h_{m+1,m}| |e_m^T y|
      converged = true;
      res.assign(kc, 0.0);
      Y.assign(kc, {});
      for (int i = 0; i < kc; ++i) {
        if (!hess_eigvec(m, Hm, theta[i], Y[i])) return fail(c, LC_EINVAL, "Ritz vector failed");
        res[i] = std::fabs(h(m, m - 1)) * std::abs(Y[i][m - 1]);
        if (res[i] > tol * std::max(std::abs(theta[i]), 1e-14 * hnorm)) converged = false;
      }
      if (!converged) break;
      // The estimates say converged: recompute each wanted pair's residual |K x - theta x| with
      // the Krylov map itself (two vectors per pair).  A Ritz value whose basis has drifted from
      // the Arnoldi relation -- seen as a real value near the gradient directions' zeros with a
      // tiny estimate -- has a residual of order one; it is then treated as unwanted (an exact
      // shift) and the selection is redone.  A genuine pair passes: the map's own error (an
      // inexact projection in the mixed form, relative to |L_U x| rather than |theta|) keeps its
      // recomputed residual above the estimate but orders of magnitude below the threshold.
      bool all_ok = true;
      for (int i = 0; i < kc; ++i) {
        std::vector<double> Qy((size_t)m * 2);
        for (int r = 0; r < m; ++r) {
          Qy[(size_t)r * 2] = Y[i][r].real();
          Qy[(size_t)r * 2 + 1] = Y[i][r].imag();
        }
        std::memcpy(c->hsmall, Qy.data(), Qy.size() * sizeof(double));
        HIPCHK(c, hipMemcpyAsync(c->dsmall, c->hsmall, Qy.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
        KLAUNCH(c, LC_K_VECTOR, launch_combine(V.p, V.ld, m, c->dsmall, 2, W.p, W.ld, c->nvel, c->stream));
        const double tr = theta[i].real(), ti = theta[i].imag();
        double r2 = 0.0, i2 = 0.0, x2 = 0.0, y2 = 0.0;
        if ((rc = kmap(c, K, W.at(0), W.at(2))) || (rc = vaxpy(c, -tr, W.at(0), W.at(2)))) return rc;
        if (ti != 0.0) {
          // (K - theta)(xr + i xi): real part K xr - tr xr + ti xi, imaginary part K xi - tr xi - ti xr
          if ((rc = kmap(c, K, W.at(1), W.at(3))) || (rc = vaxpy(c, ti, W.at(1), W.at(2))) ||
              (rc = vaxpy(c, -tr, W.at(1), W.at(3))) || (rc = vaxpy(c, -ti, W.at(0), W.at(3))) ||
              (rc = vdot(c, W.at(3), W.at(3), &i2)) || (rc = vdot(c, W.at(1), W.at(1), &y2)))
            return rc;
        }
        if ((rc = vdot(c, W.at(2), W.at(2), &r2)) || (rc = vdot(c, W.at(0), W.at(0), &x2))) return rc;
        const double rel = vnorm(r2 + i2) / std::max(std::abs(theta[i]) * vnorm(x2 + y2), 1e-300);
        constexpr double kSpurious = 1e-3;
        if (verbose())
          std::fprintf(stderr, "[lk arnoldi] verify %.10f%+.10fi: estimate %.2e, recomputed %.2e%s\n", tr, ti,
                       res[i] / std::max(std::abs(theta[i]), 1e-300), rel, rel > kSpurious ? " (rejected)" : "");
        if (rel > kSpurious) {
          rejected.push_back(theta[i]);
          all_ok = false;
        }
      }
      if (all_ok) break;
      converged = false;
    }  // selection passes
    if (verbose())
      std::fprintf(stderr, "[lk arnoldi] restart %d: theta0 = %.10f%+.10fi  resid0 = %.3e  vectors %ld\n", restart,
                   theta[0].real(), theta[0].imag(), res[0], K.count);
    if (converged || restart == max_restarts) break;
    // Implicit restart with the unwanted Ritz values as exact shifts (complex
    // pairs as real double shifts).
    struct Shift {
      double re, im;
      bool pair;
    };
    std::vector<Shift> shifts;
    for (int i = kk; i < m; ++i) {
      const cplx t = theta[i];
      if (std::fabs(t.imag()) > 0.0 && i + 1 < m && is_pair(t, theta[i + 1])) {
        shifts.push_back({t.real(), t.imag(), true});
        ++i;
      } else {
        shifts.push_back({t.real(), 0.0, false});
      }
    }
    std::vector<double> Q((size_t)m * m, 0.0), Hs(Hm);
    for (int r = 0; r < m; ++r) Q[(size_t)r * m + r] = 1.0;
    for (const Shift& sh : shifts) shifted_qr_step(m, Hs, Q, sh.re, sh.im, sh.pair);
    const double beta = Hs[(size_t)kk * m + (kk - 1)];
    const double sigma = Q[(size_t)(m - 1) * m + (kk - 1)];
    const double hm = h(m, m - 1);
    // new basis: W[c] = sum_r V[r] Qext[r][c], c <= kk (column kk is the new residual)
    const int nc = kk + 1;
    std::vector<double> Qext((size_t)(m + 1) * nc, 0.0);
    for (int r = 0; r < m; ++r) {
      for (int col = 0; col < kk; ++col) Qext[(size_t)r * nc + col] = Q[(size_t)r * m + col];
      Qext[(size_t)r * nc + kk] = Q[(size_t)r * m + kk] * beta;
    }
    Qext[(size_t)m * nc + kk] = hm * sigma;
    std::memcpy(c->hsmall, Qext.data(), Qext.size() * sizeof(double));
    HIPCHK(c, hipMemcpyAsync(c->dsmall, c->hsmall, Qext.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    KLAUNCH(c, LC_K_VECTOR, launch_combine(V.p, V.ld, m + 1, c->dsmall, nc, W.p, W.ld, c->nvel, c->stream));
    std::swap(V, W);
    if ((rc = vdot(c, V.at(kk), V.at(kk), &nrm))) return rc;
    nrm = vnorm(nrm);
    std::fill(H.begin(), H.end(), 0.0);
    for (int r = 0; r < kk; ++r)
      for (int col = 0; col < kk; ++col) h(r, col) = Hs[(size_t)r * m + col];
    h(kk, kk - 1) = nrm;
    if (nrm > 0.0 && (rc = vscale(c, 1.0 / nrm, V.at(kk)))) return rc;
    j0 = kk;
  }
  *n_out = kc;
  for (int i = 0; i < kc; ++i) {
    eig_re[i] = theta[i].real();
    eig_im[i] = theta[i].imag();
    if (resid) resid[i] = res[i];
  }
  if (vec_re || vec_im) {  // Ritz vectors x_i = V_m y_i (unit norm)
    for (int i = 0; i < std::min(kc, nvec); ++i) {
      std::vector<double> Qy((size_t)m * 2);
      for (int r = 0; r < m; ++r) {
        Qy[(size_t)r * 2] = Y[i][r].real();
        Qy[(size_t)r * 2 + 1] = Y[i][r].imag();
      }
      std::memcpy(c->hsmall, Qy.data(), Qy.size() * sizeof(double));
      HIPCHK(c, hipMemcpyAsync(c->dsmall, c->hsmall, Qy.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
      KLAUNCH(c, LC_K_VECTOR, launch_combine(V.p, V.ld, m, c->dsmall, 2, W.p, W.ld, c->nvel, c->stream));
      if (vec_re) HIPCHK(c, hipMemcpyAsync(vec_re + (size_t)i * c->nvel, W.at(0), c->nvel * sizeof(double),
                                           hipMemcpyDeviceToDevice, c->stream));
      if (vec_im) HIPCHK(c, hipMemcpyAsync(vec_im + (size_t)i * c->nvel, W.at(1), c->nvel * sizeof(double),
                                           hipMemcpyDeviceToDevice, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
    }
  }
  if (n_vectors) *n_vectors = K.count;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return converged ? LC_OK : LC_ENOTCONV;
}

}  // namespace

extern "C" int lc_arnoldi_leading(lc_ctx* c, int k, int m, double tol, int max_restarts, unsigned long long seed,
                                  const double* v0, int precision, double proj_tol, double* eig_re, double* eig_im,
                                  double* resid, double* vec_re, double* vec_im, int* n_out, long* n_vectors) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (k < 1 || m < k + 3 || m > 100 || k + 2 > 48 || !eig_re || !eig_im || !n_out)
    return fail(c, LC_EINVAL, "need 1 <= k, k + 3 <= m <= 100, k <= 46 and output arrays");
  if ((vec_re && !aligned(vec_re)) || (vec_im && !aligned(vec_im)) || (v0 && !aligned(v0)) || !(tol > 0.0) ||
      max_restarts < 0)
    return fail(c, LC_EINVAL, "bad argument");
  return arnoldi_run(c, k, m, tol, max_restarts, seed, v0, precision, proj_tol, eig_re, eig_im, resid, vec_re, vec_im,
                     k + 1, n_out, n_vectors);
}

// ================================================================ Newton
namespace {

// BiCGstab(2) for A x = b from the current x (Sleijpen & Fokkema's BiCGstab(l)
// with l = 2); vectors r0..r2, u0..u2, the shadow rh and a spare.
int bicgstab2(lc_ctx* c, KMap& K, const double* b, double* x, const Basis& S, double bnorm, double tol,
              long max_vectors, double* final_res) {
  double *r0 = S.at(0), *r1 = S.at(1), *r2 = S.at(2), *u0 = S.at(3), *u1 = S.at(4), *u2 = S.at(5), *rh = S.at(6);
  double* xbest = S.at(7);  // iterate with the smallest residual so far
  double* r[3] = {r0, r1, r2};
  double* u[3] = {u0, u1, u2};
  int rc;
  if ((rc = kmap(c, K, x, r0))) return rc;  // r0 = b - A x
  if ((rc = vscale(c, -1.0, r0))) return rc;
  if ((rc = vaxpy(c, 1.0, b, r0))) return rc;
  if ((rc = vproject(c, r0, u1))) return rc;
  if ((rc = vcopy(c, r0, rh))) return rc;
  HIPCHK(c, hipMemsetAsync(u0, 0, c->nvel * sizeof(double), c->stream));
  double rho0 = 1.0, alpha = 0.0, omega = 1.0, rn = 0.0;
  if ((rc = vdot(c, r0, r0, &rn))) return rc;
  rn = vnorm(rn);
  double best = rn;
  if ((rc = vcopy(c, x, xbest))) return rc;
  // a zero or non-finite denominator is a breakdown: stop with the current x
  auto usable = [](double d) { return std::isfinite(d) && d != 0.0; };
  bool broke = false;
  while (rn > tol * bnorm && K.count + 4 <= max_vectors && !broke) {
    rho0 = -omega * rho0;
    for (int j = 0; j < 2 && !broke; ++j) {
      double rho1 = 0.0;
      if ((rc = vdot(c, rh, r[j], &rho1))) return rc;
      if (!usable(rho0) || !std::isfinite(rho1)) {
        broke = true;
        break;
      }
      const double beta = alpha * rho1 / rho0;
      rho0 = rho1;
      for (int i = 0; i <= j; ++i) {  // u_i = r_i - beta u_i
        if ((rc = vscale(c, -beta, u[i]))) return rc;
        if ((rc = vaxpy(c, 1.0, r[i], u[i]))) return rc;
      }
      if ((rc = kmap(c, K, u[j], u[j + 1]))) return rc;
      double gamma = 0.0;
      if ((rc = vdot(c, rh, u[j + 1], &gamma))) return rc;
      if (!usable(gamma)) {
        broke = true;
        break;
      }
      alpha = rho0 / gamma;
      for (int i = 0; i <= j; ++i)
        if ((rc = vaxpy(c, -alpha, u[i + 1], r[i]))) return rc;
      if ((rc = kmap(c, K, r[j], r[j + 1]))) return rc;
      if ((rc = vaxpy(c, alpha, u0, x))) return rc;
    }
    if (broke) break;
    // minimal-residual part, l = 2
    double s1 = 0.0, t01 = 0.0, t21 = 0.0, s2 = 0.0, t02 = 0.0;
    if ((rc = vdot(c, r1, r1, &s1))) return rc;
    if ((rc = vdot(c, r0, r1, &t01))) return rc;
    if ((rc = vdot(c, r2, r1, &t21))) return rc;
    if (!usable(s1)) break;
    const double gp1 = t01 / s1, tau12 = t21 / s1;
    if ((rc = vaxpy(c, -tau12, r1, r2))) return rc;
    if ((rc = vdot(c, r2, r2, &s2))) return rc;
    if ((rc = vdot(c, r0, r2, &t02))) return rc;
    if (!usable(s2)) break;
    const double gp2 = t02 / s2;
    const double g2 = gp2, g1 = gp1 - tau12 * g2, gpp1 = g2;
    omega = g2;
    if ((rc = vaxpy(c, g1, r0, x))) return rc;
    if ((rc = vaxpy(c, -gp2, r2, r0))) return rc;
    if ((rc = vaxpy(c, -g2, u2, u0))) return rc;
    if ((rc = vaxpy(c, -g1, u1, u0))) return rc;
    if ((rc = vaxpy(c, gpp1, r1, x))) return rc;
    if ((rc = vaxpy(c, -gp1, r1, r0))) return rc;
    if ((rc = vdot(c, r0, r0, &rn))) return rc;
    rn = vnorm(rn);
    if (verbose()) std::fprintf(stderr, "[lk bicgstab2] |res| = %.3e (rel %.3e)\n", rn, rn / bnorm);
    // The residual of BiCGstab(2) is not monotone: on these convection-dominated systems it
    // rises by 1e2-1e3 for hundreds of iterations before falling (measured at 100^3 near
    // Re_cr), so only a non-finite residual ends the iteration; the best iterate is kept.
    if (std::isfinite(rn) && rn < best) {
      best = rn;
      if ((rc = vcopy(c, x, xbest))) return rc;
    } else if (!std::isfinite(rn)) {
      break;
    }
  }
  if ((rc = vcopy(c, xbest, x))) return rc;
  *final_res = best;
  return LC_OK;
}

}  // namespace

extern "C" int lc_newton_residual(lc_ctx* c, double* F, double* res_inf) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (!F || !aligned(F) || !res_inf) return fail(c, LC_EINVAL, "bad pointers");
  KLAUNCH(c, LC_K_RESIDUAL, launch_momentum(c->g, c->U, c->U, c->w, 1.0 / c->re, 0.5, true, std::cos(c->alpha),
                                            std::sin(c->alpha), c->stream));
  lc_stats st;
  rc = lc_project(c, c->w, F, nullptr, LC_FP64, 1e-13, 4, &st);
  if (rc < 0) return rc;
  // R(U) carries an O(1) pressure gradient, so the first projection leaves a
  // divergent residue of ~1e-13 of that size -- as large as F itself near
  // convergence, where Krylov solves cannot reduce it.  A second projection
  // (the residue's divergence is rounding noise) removes it.
  if ((rc = vproject(c, F, c->w))) return rc;
  return vmaxabs(c, F, res_inf);
}

extern "C" int lc_newton_step(lc_ctx* c, double lin_tol, int gmres_m, long max_vectors, int precision,
                              double proj_tol, double* res_inf, double* corr_inf, long* n_vectors, int* used_bicgstab) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (gmres_m < 0 || gmres_m > 400 || max_vectors < 1 || !(lin_tol > 0.0))
    return fail(c, LC_EINVAL, "bad Newton arguments");
  Basis B;
  const int nbasis = std::max(gmres_m + 1, 8);
  if ((rc = ensure_ws(c, nbasis + 4, &B))) return rc;
  double* F = B.at(nbasis);      // right side P R(U)
  double* x = B.at(nbasis + 1);  // the correction (preconditioned: its preimage y, x = M^-1 y)
  double* t = B.at(nbasis + 2);  // spare
  // steps 2-3 of Section 3: residual, then the Jacobian system on the divergence-free space
  double rinf = 0.0;
  if ((rc = lc_newton_residual(c, F, &rinf))) return rc;
  if (res_inf) *res_inf = rinf;
  if (used_bicgstab) *used_bicgstab = 0;
  KMap K{precision, proj_tol, 8};
  K.sdt = c->stokes_dt;
  K.z = B.at(nbasis + 3);
  HIPCHK(c, hipMemsetAsync(x, 0, c->nvel * sizeof(double), c->stream));
  double bnorm = 0.0;
  if ((rc = vdot(c, F, F, &bnorm))) return rc;
  bnorm = vnorm(bnorm);
  bool solved = bnorm == 0.0;
  double beta = bnorm, prev = bnorm;
  if ((rc = vcopy(c, F, B.at(0)))) return rc;  // r0 = F (x = 0)
  std::vector<double> hcol(gmres_m + 2), g(gmres_m + 1), cs(gmres_m), sn(gmres_m);
  std::vector<double> R((size_t)gmres_m * gmres_m);
  bool saturated = gmres_m == 0;  // gmres_m = 0: BiCGstab(2) alone
  while (!solved && !saturated && K.count < max_vectors) {
    if ((rc = vscale(c, 1.0 / beta, B.at(0)))) return rc;
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int used = 0;
    for (int j = 0; j < gmres_m && K.count < max_vectors; ++j) {
      if ((rc = kmap(c, K, B.at(j), B.at(j + 1)))) return rc;
      if ((rc = mgs(c, B, j + 1, B.at(j + 1), hcol.data()))) return rc;
      const double hnext = hcol[j + 1];
      for (int i = 0; i < j; ++i) {  // previous rotations
        const double a = hcol[i], b2 = hcol[i + 1];
        hcol[i] = cs[i] * a + sn[i] * b2;
        hcol[i + 1] = -sn[i] * a + cs[i] * b2;
      }
      const double r = std::hypot(hcol[j], hnext);
      cs[j] = r > 0 ? hcol[j] / r : 1.0;
      sn[j] = r > 0 ? hnext / r : 0.0;
      hcol[j] = r;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      for (int i = 0; i <= j; ++i) R[(size_t)i * gmres_m + j] = hcol[i];
      used = j + 1;
      if (verbose())
        std::fprintf(stderr, "[lk gmres] j=%d h_{j+1,j}=%.3e |res|=%.3e (rel %.3e)\n", j, hnext, std::fabs(g[j + 1]),
                     std::fabs(g[j + 1]) / bnorm);
      if (hnext > 0.0 && (rc = vscale(c, 1.0 / hnext, B.at(j + 1)))) return rc;
      if (std::fabs(g[j + 1]) <= lin_tol * bnorm || hnext == 0.0) break;
    }
    // y = R^-1 g, x += V y
    std::vector<double> y(used);
    for (int i = used - 1; i >= 0; --i) {
      double s = g[i];
      for (int q = i + 1; q < used; ++q) s -= R[(size_t)i * gmres_m + q] * y[q];
      const double d = R[(size_t)i * gmres_m + i];
      y[i] = (d != 0.0 && std::isfinite(d)) ? s / d : 0.0;
    }
    std::memcpy(c->hsmall, y.data(), used * sizeof(double));
    HIPCHK(c, hipMemcpyAsync(c->dsmall, c->hsmall, used * sizeof(double), hipMemcpyHostToDevice, c->stream));
    KLAUNCH(c, LC_K_VECTOR, launch_combine(B.p, B.ld, used, c->dsmall, 1, t, B.ld, c->nvel, c->stream));
    if ((rc = vaxpy(c, 1.0, t, x))) return rc;
    // true residual of the restart
    if ((rc = kmap(c, K, x, t))) return rc;
    if ((rc = vcopy(c, F, B.at(0)))) return rc;
    if ((rc = vaxpy(c, -1.0, t, B.at(0)))) return rc;
    if ((rc = vproject(c, B.at(0), t))) return rc;
    if ((rc = vdot(c, B.at(0), B.at(0), &beta))) return rc;
    beta = vnorm(beta);
    if (verbose()) std::fprintf(stderr, "[lk gmres] restart: true |res| = %.3e (rel %.3e)\n", beta, beta / bnorm);
    if (beta <= lin_tol * bnorm) {
      solved = true;
      break;
    }
    // the cycle's estimate met the tolerance but the true residual did not: the
    // rounding floor of the Krylov map is reached; a residual within
    // sqrt(lin_tol) is accepted rather than restarting from rounding noise
    const bool est_met = used > 0 && std::fabs(g[used]) <= lin_tol * bnorm;
    if (est_met && beta <= std::sqrt(lin_tol) * bnorm) {
      solved = true;
      break;
    }
    if (beta > 0.9 * prev) {  // a restart that gains less than 10%: GMRES saturated
      // near the rounding floor of the Krylov map (late Newton steps) a residual
      // within sqrt(lin_tol) is accepted; otherwise BiCGstab(2) takes over
      if (beta <= std::sqrt(lin_tol) * bnorm) solved = true;
      else saturated = true;
      break;
    }
    prev = beta;
  }
  if (!solved && saturated) {
    if (used_bicgstab) *used_bicgstab = 1;
    Basis S{B.p, B.ld};
    double fr = 0.0;
    if ((rc = bicgstab2(c, K, F, x, S, bnorm, lin_tol, max_vectors, &fr))) return rc;
    solved = fr <= lin_tol * bnorm;
  }
  // right preconditioning: the Krylov solve was for y with (P L_U M^-1) y = F; x = M^-1 y
  if (K.sdt > 0.0) {
    if ((rc = stokes_step(c, x, t, K.sdt, LC_FP64, 1e-13, 4)) < 0) return rc;
    if ((rc = vcopy(c, t, x))) return rc;
  }
  // step 4: U <- U - x, with x kept in the divergence-free space
  if ((rc = vproject(c, x, t))) return rc;
  if ((rc = vaxpy(c, -1.0, x, c->U))) return rc;
  KLAUNCH(c, LC_K_VECTOR, launch_zero_walls(c->U, c->nx, c->ny, c->nz, c->stream));
  double cinf = 0.0;
  if ((rc = vmaxabs(c, x, &cinf))) return rc;
  if (corr_inf) *corr_inf = cinf;
  if (n_vectors) *n_vectors = K.count;
  return solved ? LC_OK : LC_ENOTCONV;
}

// ================================================================ critical Reynolds number
extern "C" int lc_critical_re(lc_ctx* c, double re0, double re1, const lc_critical_opts* o, double* re_cr,
                              double* omega_cr, double* hist, int* n_evals) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (!o || !re_cr || !omega_cr || !n_evals) return fail(c, LC_EINVAL, "null argument");
  if (!(re0 > 0.0) || !(re1 > 0.0) || re0 == re1 || !std::isfinite(re0) || !std::isfinite(re1))
    return fail(c, LC_EINVAL, "need two distinct positive starting Reynolds numbers");
  if (o->max_evals < 2 || o->newton_steps < 0 || !(o->re_tol > 0.0) || !(o->newton_tol > 0.0))
    return fail(c, LC_EINVAL, "bad critical-Re options");
  *n_evals = 0;
  if (!c->ucr && dalloc(c, &c->ucr, kCriticalVectors * c->nvel) != hipSuccess)
    return fail(c, LC_ENOMEM, "cannot allocate the stored steady states");
  double* Us[2] = {c->ucr, c->ucr + c->nvel};  // the last two steady states, oldest first
  double* Fr = c->ucr + 2 * c->nvel;            // projected residual (scratch)
  // the last leading eigenvector (real, imaginary part) and the next Arnoldi start
  double *xr = c->ucr + 3 * c->nvel, *xi = c->ucr + 4 * c->nvel, *v0 = c->ucr + 5 * c->nvel;
  bool have_vec = false;
  double Re_s[2] = {0.0, 0.0};
  int nstored = 0;
  std::vector<double> R, F, W;  // evaluations: Re, Re Lambda, |Im Lambda|
  const int kk = std::max(o->k, 1);
  std::vector<double> er(kk + 1), ei(kk + 1), res(kk + 1);
  auto evaluate = [&](double re) -> int {
    if (nstored == 2) {  // U = U_b + (U_b - U_a) (re - re_b) / (re_b - re_a)
      const double t = (re - Re_s[1]) / (Re_s[1] - Re_s[0]);
      int r2;
      if ((r2 = vcopy(c, Us[1], c->U))) return r2;
      if ((r2 = vscale(c, 1.0 + t, c->U))) return r2;
      if ((r2 = vaxpy(c, -t, Us[0], c->U))) return r2;
    } else if (nstored == 1) {
      int r2;
      if ((r2 = vcopy(c, Us[1], c->U))) return r2;
    }
    c->re = re;
    double rinf = 0.0;
    int r2;
    for (int s = 0;; ++s) {
      if ((r2 = lc_newton_residual(c, Fr, &rinf))) return r2;
      if (rinf <= o->newton_tol || s >= o->newton_steps) break;
      double ri, ci;
      long nv;
      int bi;
      r2 = lc_newton_step(c, o->lin_tol, o->gmres_m, o->max_vectors, LC_FP64, 1e-12, &ri, &ci, &nv, &bi);
      if (r2 < 0) return r2;
    }
    // keep this steady state (oldest dropped)
    std::swap(Us[0], Us[1]);
    Re_s[0] = Re_s[1];
    if ((r2 = vcopy(c, c->U, Us[1]))) return r2;
    Re_s[1] = re;
    nstored = std::min(nstored + 1, 2);
    int nout = 0;
    long nvec = 0;
    // warm start after the first evaluation: the leading eigenvector changes little between
    // nearby Re, so Arnoldi starts from its real plus imaginary part (spanning the pair's
    // invariant subspace) plus a seeded random part of relative size 1e-3 that keeps every
    // other direction present
    const double* start = nullptr;
    if (have_vec && o->warm_start) {
      KLAUNCH(c, LC_K_VECTOR, launch_uniform(v0, c->nvel, o->seed + 7919ull * R.size(), c->stream));
      if ((r2 = vscale(c, 1e-3 * std::sqrt(3.0 / (double)c->nvel), v0))) return r2;
      if ((r2 = vaxpy(c, 1.0, xr, v0)) || (r2 = vaxpy(c, 1.0, xi, v0))) return r2;
      start = v0;
    }
    r2 = arnoldi_run(c, o->k, o->m, o->eig_tol, o->max_restarts, o->seed, start, LC_FP64, 1e-12, er.data(),
                     ei.data(), res.data(), xr, xi, 1, &nout, &nvec);
    if (r2 < 0) return r2;
    if (nout < 1) return fail(c, LC_ENOTCONV, "no Ritz values at Re = %g", re);
    have_vec = true;
    // the largest real part among the Ritz values within 1e-3 of convergence (a value far
    // from it -- such as a transient real one near zero, pulled from the gradient directions
    // on which P L_U vanishes -- is not yet an eigenvalue); among all of them if none is
    int lead = -1;
    for (int i = 0; i < nout; ++i)
      if (res[i] <= 1e-3 * std::hypot(er[i], ei[i]) && (lead < 0 || er[i] > er[lead])) lead = i;
    if (lead < 0) {
      lead = 0;
      for (int i = 1; i < nout; ++i)
        if (er[i] > er[lead]) lead = i;
    }
    if (hist && (int)R.size() < o->max_evals) {
      double* h = hist + 4 * R.size();
      h[0] = re;
      h[1] = er[lead];
      h[2] = std::fabs(ei[lead]);
      h[3] = rinf;
    }
    R.push_back(re);
    F.push_back(er[lead]);
    W.push_back(std::fabs(ei[lead]));
    *n_evals = (int)R.size();
    if (verbose())
      std::fprintf(stderr, "[lk critical] Re %.8f: Lambda %+.10e %+.10ei, |F| %.2e\n", re, er[lead], ei[lead], rinf);
    return LC_OK;
  };
  if ((rc = evaluate(re0))) return rc;
  if ((rc = evaluate(re1))) return rc;
  bool converged = false;
  double rn = R.back();
  while (true) {
    const size_t b = R.size() - 1, a = b - 1;
    if (F[b] == F[a]) break;
    rn = R[b] - F[b] * (R[b] - R[a]) / (F[b] - F[a]);
    if (!std::isfinite(rn) || !(rn > 0.0)) return fail(c, LC_ENOTCONV, "secant left the positive axis");
    if (std::fabs(rn - R[b]) <= o->re_tol * std::fabs(R[b])) {
      converged = true;
      break;
    }
    if ((int)R.size() >= o->max_evals) break;
    if ((rc = evaluate(rn))) return rc;
  }
  size_t b = R.size() - 1, a = b - 1;
  if (!converged) {
    // noisy or slow: the linear root between the evaluations closest to zero on either
    // side of it (largest negative and smallest positive Re Lambda), if they exist
    int lo = -1, hi = -1;
    for (size_t i = 0; i < R.size(); ++i) {
      if (F[i] < 0.0 && (lo < 0 || F[i] > F[lo])) lo = (int)i;
      if (F[i] > 0.0 && (hi < 0 || F[i] < F[hi])) hi = (int)i;
    }
    if (lo >= 0 && hi >= 0) {
      a = lo;
      b = hi;
      rn = R[a] - F[a] * (R[b] - R[a]) / (F[b] - F[a]);
    }
  }
  *re_cr = rn;
  *omega_cr = W[b] + (W[b] - W[a]) * (rn - R[b]) / (R[b] - R[a]);
  return converged ? LC_OK : LC_ENOTCONV;
}
