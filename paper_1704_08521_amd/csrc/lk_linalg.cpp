// Small dense host linear algebra (float64) for set-up and Krylov drivers.
#include "lk_linalg.h"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace lk {

// Implicit symmetric QR with Wilkinson shifts on the unreduced trailing block;
// each step chases the bulge with plane rotations J = [[c, -s], [s, c]] applied
// as T <- J^T T J on indices (k, k+1) and accumulated into Q <- Q J.
bool sym_tridiag_eig(int n, std::vector<double> a, std::vector<double> b, std::vector<double>& lam,
                     std::vector<double>& Q) {
  Q.assign((size_t)n * n, 0.0);
  for (int r = 0; r < n; ++r) Q[(size_t)r * n + r] = 1.0;
  b.resize(std::max(n, 1), 0.0);
  const double eps = 2.220446049250313e-16;
  int hi = n - 1;
  long budget = 60L * n + 100;
  while (hi > 0) {
    if (std::fabs(b[hi - 1]) <= eps * (std::fabs(a[hi - 1]) + std::fabs(a[hi]))) {
      b[hi - 1] = 0.0;
      --hi;
      continue;
    }
    if (--budget < 0) return false;
    int lo = hi - 1;
    while (lo > 0 && std::fabs(b[lo - 1]) > eps * (std::fabs(a[lo - 1]) + std::fabs(a[lo]))) --lo;
    // Wilkinson shift: eigenvalue of the trailing 2x2 block nearer to a[hi]
    const double d = 0.5 * (a[hi - 1] - a[hi]);
    const double bh = b[hi - 1];
    const double den = d + std::copysign(std::hypot(d, bh), d);
    const double mu = (den != 0.0) ? a[hi] - bh * bh / den : a[hi];
    double x = a[lo] - mu, z = b[lo];
    double bulge = 0.0;
    for (int k = lo; k < hi; ++k) {
      double r = std::hypot(x, z);
      double c = 1.0, s = 0.0;
      if (r != 0.0) {
        c = x / r;
        s = z / r;
      }
      if (k > lo) b[k - 1] = r;  // the bulge at (k-1, k+1) is annihilated
      const double ak = a[k], ak1 = a[k + 1], bk = b[k];
      a[k] = c * c * ak + 2.0 * c * s * bk + s * s * ak1;
      a[k + 1] = s * s * ak - 2.0 * c * s * bk + c * c * ak1;
      b[k] = c * s * (ak1 - ak) + (c * c - s * s) * bk;
      if (k + 1 < hi) {
        bulge = s * b[k + 1];
        b[k + 1] = c * b[k + 1];
        x = b[k];
        z = bulge;
      }
      for (int row = 0; row < n; ++row) {
        double* q = &Q[(size_t)row * n];
        const double qk = q[k], qk1 = q[k + 1];
        q[k] = c * qk + s * qk1;
        q[k + 1] = -s * qk + c * qk1;
      }
    }
  }
  // sort ascending
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int p, int q) { return a[p] < a[q]; });
  lam.resize(n);
  std::vector<double> Qs((size_t)n * n);
  for (int m = 0; m < n; ++m) {
    lam[m] = a[idx[m]];
    for (int row = 0; row < n; ++row) Qs[(size_t)row * n + m] = Q[(size_t)row * n + idx[m]];
  }
  Q.swap(Qs);
  return true;
}

bool hess_eigvals(int m, const std::vector<double>& H, std::vector<cplx>& lam) {
  std::vector<cplx> A(H.begin(), H.begin() + (size_t)m * m);
  auto at = [&](int r, int c) -> cplx& { return A[(size_t)r * m + c]; };
  const double eps = 2.220446049250313e-16;
  double hnorm = 0.0;
  for (double x : H) hnorm = std::max(hnorm, std::fabs(x));
  lam.clear();
  int hi = m - 1, iter = 0, total = 0;
  while (hi >= 0) {
    if (hi == 0) {
      lam.push_back(at(0, 0));
      break;
    }
    int l = hi;
    while (l > 0) {
      double s = std::abs(at(l, l)) + std::abs(at(l - 1, l - 1));
      if (s == 0.0) s = hnorm;
      if (std::abs(at(l, l - 1)) <= eps * s) {
        at(l, l - 1) = 0.0;
        break;
      }
      --l;
    }
    if (l == hi) {
      lam.push_back(at(hi, hi));
      --hi;
      iter = 0;
      continue;
    }
    if (++iter > 60 || ++total > 60 * m) return false;
    // Wilkinson shift: eigenvalue of the trailing 2x2 block nearer to its last entry
    const cplx a = at(hi - 1, hi - 1), b = at(hi - 1, hi), c = at(hi, hi - 1), d = at(hi, hi);
    const cplx half_tr = 0.5 * (a + d);
    const cplx disc = std::sqrt(half_tr * half_tr - (a * d - b * c));
    const cplx mu1 = half_tr + disc, mu2 = half_tr - disc;
    cplx mu = (std::abs(mu1 - d) < std::abs(mu2 - d)) ? mu1 : mu2;
    if (iter % 11 == 10) mu = d + 0.75 * std::abs(c);  // exceptional shift
    for (int k = l; k <= hi; ++k) at(k, k) -= mu;
    std::vector<cplx> cs(hi - l), sn(hi - l);
    for (int k = l; k < hi; ++k) {  // R = [[conj c, conj s], [-s, c]] zeroes (k+1, k)
      const cplx x = at(k, k), y = at(k + 1, k);
      const double r = std::sqrt(std::norm(x) + std::norm(y));
      const cplx cc = r > 0 ? x / r : cplx(1.0), ss = r > 0 ? y / r : cplx(0.0);
      cs[k - l] = cc;
      sn[k - l] = ss;
      for (int col = k; col <= hi; ++col) {
        const cplx p = at(k, col), q = at(k + 1, col);
        at(k, col) = std::conj(cc) * p + std::conj(ss) * q;
        at(k + 1, col) = -ss * p + cc * q;
      }
    }
    for (int k = l; k < hi; ++k) {  // right-multiply by R^H on columns (k, k+1)
      const cplx cc = cs[k - l], ss = sn[k - l];
      for (int row = l; row <= std::min(k + 1, hi); ++row) {
        const cplx p = at(row, k), q = at(row, k + 1);
        at(row, k) = p * cc + q * ss;
        at(row, k + 1) = -p * std::conj(ss) + q * std::conj(cc);
      }
    }
    for (int k = l; k <= hi; ++k) at(k, k) += mu;
  }
  return true;
}

bool hess_eigvec(int m, const std::vector<double>& H, cplx lam, std::vector<cplx>& y) {
  double hnorm = 0.0;
  for (double x : H) hnorm = std::max(hnorm, std::fabs(x));
  const cplx shift = lam + cplx(1e-13 * std::max(hnorm, 1.0), 0.0);
  std::vector<cplx> A((size_t)m * m);
  for (int r = 0; r < m; ++r)
    for (int c = 0; c < m; ++c) A[(size_t)r * m + c] = H[(size_t)r * m + c] - (r == c ? shift : cplx(0.0));
  std::vector<int> piv(m);
  for (int k = 0; k < m; ++k) {  // LU with partial pivoting
    int p = k;
    for (int r = k + 1; r < m; ++r)
      if (std::abs(A[(size_t)r * m + k]) > std::abs(A[(size_t)p * m + k])) p = r;
    piv[k] = p;
    if (p != k)
      for (int c = 0; c < m; ++c) std::swap(A[(size_t)k * m + c], A[(size_t)p * m + c]);
    if (std::abs(A[(size_t)k * m + k]) == 0.0) A[(size_t)k * m + k] = 1e-300;
    for (int r = k + 1; r < m; ++r) {
      const cplx f = A[(size_t)r * m + k] / A[(size_t)k * m + k];
      A[(size_t)r * m + k] = f;
      for (int c = k + 1; c < m; ++c) A[(size_t)r * m + c] -= f * A[(size_t)k * m + c];
    }
  }
  y.assign(m, cplx(1.0));
  for (int it = 0; it < 3; ++it) {
    std::vector<cplx> z(y);
    for (int k = 0; k < m; ++k) std::swap(z[k], z[piv[k]]);
    for (int r = 0; r < m; ++r)
      for (int c = 0; c < r; ++c) z[r] -= A[(size_t)r * m + c] * z[c];
    for (int r = m - 1; r >= 0; --r) {
      for (int c = r + 1; c < m; ++c) z[r] -= A[(size_t)r * m + c] * z[c];
      z[r] /= A[(size_t)r * m + r];
    }
    double nrm = 0.0;
    for (const cplx& v : z) nrm += std::norm(v);
    nrm = std::sqrt(nrm);
    if (!(nrm > 0.0) || !std::isfinite(nrm)) return false;
    for (int r = 0; r < m; ++r) y[r] = z[r] / nrm;
  }
  int big = 0;
  for (int r = 1; r < m; ++r)
    if (std::abs(y[r]) > std::abs(y[big])) big = r;
  const cplx ph = std::conj(y[big]) / std::abs(y[big]);
  for (cplx& v : y) v *= ph;
  return true;
}

void shifted_qr_step(int m, std::vector<double>& H, std::vector<double>& Q, double re, double im, bool pair) {
  auto h = [&](int r, int c) -> double& { return H[(size_t)r * m + c]; };
  std::vector<double> M((size_t)m * m);
  for (int r = 0; r < m; ++r)
    for (int c = 0; c < m; ++c) {
      double v = 0.0;
      if (pair) {
        for (int t = 0; t < m; ++t) v += h(r, t) * h(t, c);
        v -= 2.0 * re * h(r, c);
        if (r == c) v += re * re + im * im;
      } else {
        v = h(r, c) - (r == c ? re : 0.0);
      }
      M[(size_t)r * m + c] = v;
    }
  // Householder QR of M, accumulating Qs (m x m)
  std::vector<double> Qs((size_t)m * m, 0.0);
  for (int r = 0; r < m; ++r) Qs[(size_t)r * m + r] = 1.0;
  std::vector<double> v(m);
  for (int k = 0; k < m - 1; ++k) {
    double nrm = 0.0;
    for (int r = k; r < m; ++r) nrm += M[(size_t)r * m + k] * M[(size_t)r * m + k];
    nrm = std::sqrt(nrm);
    if (nrm == 0.0) continue;
    const double x0 = M[(size_t)k * m + k];
    const double alpha = (x0 >= 0.0) ? -nrm : nrm;
    double vv = 0.0;
    for (int r = k; r < m; ++r) {
      v[r] = M[(size_t)r * m + k] - (r == k ? alpha : 0.0);
      vv += v[r] * v[r];
    }
    if (vv == 0.0) continue;
    for (int c = k; c < m; ++c) {  // M <- (I - 2 v v^T / v^T v) M
      double s = 0.0;
      for (int r = k; r < m; ++r) s += v[r] * M[(size_t)r * m + c];
      s *= 2.0 / vv;
      for (int r = k; r < m; ++r) M[(size_t)r * m + c] -= s * v[r];
    }
    for (int r = 0; r < m; ++r) {  // Qs <- Qs (I - 2 v v^T / v^T v)
      double s = 0.0;
      for (int c = k; c < m; ++c) s += Qs[(size_t)r * m + c] * v[c];
      s *= 2.0 / vv;
      for (int c = k; c < m; ++c) Qs[(size_t)r * m + c] -= s * v[c];
    }
  }
  // H <- Qs^T H Qs ; Q <- Q Qs
  std::vector<double> T((size_t)m * m, 0.0), Hn((size_t)m * m, 0.0), Qn((size_t)m * m, 0.0);
  for (int r = 0; r < m; ++r)
    for (int c = 0; c < m; ++c) {
      double s = 0.0;
      for (int t = 0; t < m; ++t) s += h(r, t) * Qs[(size_t)t * m + c];
      T[(size_t)r * m + c] = s;
    }
  for (int r = 0; r < m; ++r)
    for (int c = 0; c < m; ++c) {
      double s = 0.0;
      for (int t = 0; t < m; ++t) s += Qs[(size_t)t * m + r] * T[(size_t)t * m + c];
      Hn[(size_t)r * m + c] = (r > c + 1) ? 0.0 : s;
    }
  for (int r = 0; r < m; ++r)
    for (int c = 0; c < m; ++c) {
      double s = 0.0;
      for (int t = 0; t < m; ++t) s += Q[(size_t)r * m + t] * Qs[(size_t)t * m + c];
      Qn[(size_t)r * m + c] = s;
    }
  H.swap(Hn);
  Q.swap(Qn);
}

bool tridiag_modes(int n, const double* kd, const double* ko, const double* m, std::vector<double>& lam,
                   std::vector<double>& S, std::vector<double>& Wf) {
  // T = M^-1/2 K M^-1/2 is symmetric tridiagonal; its eigenvectors q give s = M^-1/2 q.
  std::vector<double> a(n, 0.0), b(std::max(n - 1, 1), 0.0);
  for (int i = 0; i < n; ++i) a[i] = kd[i] / m[i];
  for (int i = 0; i + 1 < n; ++i) b[i] = ko[i] / std::sqrt(m[i] * m[i + 1]);
  std::vector<double> Q;
  if (!sym_tridiag_eig(n, a, b, lam, Q)) return false;
  S.resize((size_t)n * n);
  Wf.resize((size_t)n * n);
  for (int i = 0; i < n; ++i) {
    const double sq = std::sqrt(m[i]);
    for (int k = 0; k < n; ++k) {
      const double q = Q[(size_t)i * n + k];
      S[(size_t)i * n + k] = q / sq;   // S = M^-1/2 Q, S^T M S = I
      Wf[(size_t)k * n + i] = q * sq;  // S^T M
    }
  }
  return true;
}

// The operator restricted to the even or odd subspace of a mirror-symmetric problem
// (kd[i] = kd[n-1-i], ko[i] = ko[n-2-i], m[i] = m[n-1-i]).  Basis: e_p = (delta_p +
// delta_{n-1-p}) / sqrt2 (p < n/2) plus delta_mid for odd n (even), o_p = (delta_p -
// delta_{n-1-p}) / sqrt2 (odd).  The projected K and M are tridiagonal and diagonal, so
// the half problem is solved like the full one; its eigenvectors are exactly even / odd,
// which separates the nearly degenerate mirror pairs that wall-refined grids produce.
// Outputs: lam (h ascending), Sh (h x h, row-major [p][k]): the k-th mode in the basis,
// Sh^T Mh Sh = I.
bool tridiag_half_modes(int n, const double* kd, const double* ko, const double* m, bool odd,
                        std::vector<double>& lam, std::vector<double>& Sh) {
  const int he = (n + 1) / 2, ho = n / 2;
  const int h = odd ? ho : he;
  if (h == 0) {
    lam.clear();
    Sh.clear();
    return true;
  }
  const double r2 = std::sqrt(0.5);
  auto K = [&](int i, int j) -> double {
    if (j == i) return kd[i];
    if (j == i + 1) return ko[i];
    if (j == i - 1) return ko[j];
    return 0.0;
  };
  // basis column p: up to two (index, weight) entries
  auto col = [&](int p, int* idx, double* w) -> int {
    if (!odd && (n % 2 == 1) && p == he - 1) {
      idx[0] = p;
      w[0] = 1.0;
      return 1;
    }
    idx[0] = p;
    w[0] = r2;
    idx[1] = n - 1 - p;
    w[1] = odd ? -r2 : r2;
    return 2;
  };
  auto proj = [&](int p, int q) -> double {
    int ip[2], iq[2];
    double wp[2], wq[2];
    const int np = col(p, ip, wp), nq = col(q, iq, wq);
    double v = 0.0;
    for (int a = 0; a < np; ++a)
      for (int b = 0; b < nq; ++b) v += wp[a] * wq[b] * K(ip[a], iq[b]);
    return v;
  };
  std::vector<double> mh(h), a(h), b(std::max(h - 1, 1), 0.0);
  for (int p = 0; p < h; ++p) mh[p] = m[p];  // e_p^T M e_p = (m_p + m_{n-1-p}) / 2 = m_p
  for (int p = 0; p < h; ++p) a[p] = proj(p, p) / mh[p];
  for (int p = 0; p + 1 < h; ++p) b[p] = proj(p, p + 1) / std::sqrt(mh[p] * mh[p + 1]);
  std::vector<double> Q;
  if (!sym_tridiag_eig(h, a, b, lam, Q)) return false;
  Sh.resize((size_t)h * h);
  for (int p = 0; p < h; ++p) {
    const double sq = std::sqrt(mh[p]);
    for (int k = 0; k < h; ++k) Sh[(size_t)p * h + k] = Q[(size_t)p * h + k] / sq;
  }
  return true;
}

void neumann_operator(int n, const double* dd, std::vector<double>& kd, std::vector<double>& ko) {
  // couplings c_f = 1/dd[f] across the interior faces f = 1..n-1; none through the walls
  kd.assign(n, 0.0);
  ko.assign(std::max(n - 1, 1), 0.0);
  for (int i = 0; i < n; ++i) {
    double v = 0.0;
    if (i > 0) v -= 1.0 / dd[i];
    if (i < n - 1) v -= 1.0 / dd[i + 1];
    kd[i] = v;
  }
  for (int i = 0; i + 1 < n; ++i) ko[i] = 1.0 / dd[i + 1];
}

void dirichlet_cell_operator(int n, const double* dd, std::vector<double>& kd, std::vector<double>& ko) {
  // couplings c_f = 1/dd[f] across every face f = 0..n, the two walls (half widths) included
  kd.assign(n, 0.0);
  ko.assign(std::max(n - 1, 1), 0.0);
  for (int i = 0; i < n; ++i) kd[i] = -(1.0 / dd[i] + 1.0 / dd[i + 1]);
  for (int i = 0; i + 1 < n; ++i) ko[i] = 1.0 / dd[i + 1];
}

void dirichlet_face_operator(int n, const double* d, const double* dd, std::vector<double>& kd,
                             std::vector<double>& ko, std::vector<double>& m) {
  // n + 1 points (faces 0..n): interior face i couples to i -+ 1 through cells i-1, i
  // (1/d), mass dd[i]; the wall faces are decoupled points with K = -1, M = 1
  kd.assign(n + 1, -1.0);
  ko.assign(n, 0.0);
  m.assign(n + 1, 1.0);
  for (int i = 1; i < n; ++i) {
    kd[i] = -(1.0 / d[i - 1] + 1.0 / d[i]);
    m[i] = dd[i];
  }
  for (int i = 1; i + 1 < n; ++i) ko[i] = 1.0 / d[i];
}

bool neumann_modes(int n, const double* d, const double* dd, std::vector<double>& lam, std::vector<double>& S,
                   std::vector<double>& Wf) {
  std::vector<double> kd, ko;
  neumann_operator(n, dd, kd, ko);
  return tridiag_modes(n, kd.data(), ko.data(), d, lam, S, Wf);
}

bool neumann_half_modes(int n, const double* d, const double* dd, bool odd, std::vector<double>& lam,
                        std::vector<double>& Sh) {
  std::vector<double> kd, ko;
  neumann_operator(n, dd, kd, ko);
  return tridiag_half_modes(n, kd.data(), ko.data(), d, odd, lam, Sh);
}

}  // namespace lk
