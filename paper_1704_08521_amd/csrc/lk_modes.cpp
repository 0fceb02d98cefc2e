// Tensor-product factors of 1D operators: host eigen-decomposition and device placement.
#include "lk_modes.h"

#include <cmath>
#include <cstring>

#include "lk_internal.h"
#include "lk_linalg.h"

namespace lk {

bool compute_modes(int n, const std::vector<double>& kd, const std::vector<double>& ko, const std::vector<double>& m,
                   bool sym, ModeHost& H) {
  H.n = n;
  H.m = m;
  H.sym = sym;
  if (!tridiag_modes(n, kd.data(), ko.data(), m.data(), H.lam, H.S, H.Wf)) return false;
  if (sym && (!tridiag_half_modes(n, kd.data(), ko.data(), m.data(), false, H.lam_e, H.Sh_e) ||
              !tridiag_half_modes(n, kd.data(), ko.data(), m.data(), true, H.lam_o, H.Sh_o)))
    return false;
  return true;
}

size_t mode_bytes(int n) {
  const size_t nn = (size_t)n * n;
  const int he = (n + 1) / 2;
  return 2 * n * sizeof(double) + 4 * nn * sizeof(double) + 4 * nn * sizeof(float) +
         3 * nn * (sizeof(double) + sizeof(float)) +
         4 * (mf_pack_size(he, 2) * sizeof(double) + mf_pack_size(he, 4) * sizeof(float)) +
         64 * 16;  // alignment padding (at most 15 bytes for each of an operator's <= 34 arrays)
}

void* Stager::put(const void* src, size_t bytes) {
  const size_t pad = (16 - used % 16) % 16;
  if (used + pad + bytes > host.size()) {
    overflow = true;
    return nullptr;
  }
  used += pad;
  std::memcpy(host.data() + used, src, bytes);
  void* d = dev + used;
  used += bytes;
  return d;
}

double* Stager::put_d(const std::vector<double>& v) { return (double*)put(v.data(), v.size() * sizeof(double)); }

float* Stager::put_f(const std::vector<double>& v) {
  std::vector<float> f(v.begin(), v.end());
  return (float*)put(f.data(), f.size() * sizeof(float));
}

void place_modes(const ModeHost& H, AxisModes& M, Stager& st) {
  const int n = H.n;
  const size_t nn = (size_t)n * n;
  std::vector<double> FT(nn), BkT(nn);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      FT[(size_t)j * n + i] = H.Wf[(size_t)i * n + j];
      BkT[(size_t)j * n + i] = H.S[(size_t)i * n + j];
    }
  M.lam = st.put_d(H.lam);
  M.F = st.put_d(H.Wf);
  M.Bk = st.put_d(H.S);
  M.FT = st.put_d(FT);
  M.BkT = st.put_d(BkT);
  M.F32 = st.put_f(H.Wf);
  M.Bk32 = st.put_f(H.S);
  M.FT32 = st.put_f(FT);
  M.BkT32 = st.put_f(BkT);
  const int he = (n + 1) / 2, ho = n / 2;
  M.sym = H.sym;
  M.mf = false;
  M.he = he;
  M.ho = ho;
  if (!H.sym) return;
  // parity-sorted modes: the he even ones (ascending), then the odd ones
  const double r2 = std::sqrt(0.5);
  const bool mid = (n % 2) == 1;
  const std::vector<double>&Sh_e = H.Sh_e, &Sh_o = H.Sh_o, &m = H.m;
  std::vector<double> lam_s(H.lam_e), h[8];
  lam_s.insert(lam_s.end(), H.lam_o.begin(), H.lam_o.end());
  h[0].assign((size_t)he * he, 0.0);
  h[1].assign((size_t)ho * ho, 0.0);
  h[2].assign((size_t)he * he, 0.0);
  h[3].assign((size_t)he * ho, 0.0);
  // forward: c_k = sum_p A[k][p] fold(r)_p, fold = r_p + r_{n-1-p} (r_mid alone), r_p - r_{n-1-p}
  for (int k = 0; k < he; ++k)
    for (int p = 0; p < he; ++p) {
      const double wgt = (mid && p == he - 1) ? 1.0 : r2;
      h[0][(size_t)k * he + p] = Sh_e[(size_t)p * he + k] * m[p] * wgt;
      h[2][(size_t)p * he + k] = Sh_e[(size_t)p * he + k] * wgt;  // backward: values at p from even modes
    }
  for (int k = 0; k < ho; ++k)
    for (int p = 0; p < ho; ++p) {
      h[1][(size_t)k * ho + p] = Sh_o[(size_t)p * ho + k] * m[p] * r2;
      h[3][(size_t)p * ho + k] = Sh_o[(size_t)p * ho + k] * r2;  // rows p < ho; the middle row stays 0
    }
  h[4].resize((size_t)he * he);
  h[5].resize((size_t)ho * ho);
  h[6].resize((size_t)he * he);
  h[7].resize((size_t)ho * he);
  for (int r = 0; r < he; ++r)
    for (int i = 0; i < he; ++i) {
      h[4][(size_t)i * he + r] = h[0][(size_t)r * he + i];
      h[6][(size_t)r * he + i] = h[2][(size_t)i * he + r];
    }
  for (int r = 0; r < ho; ++r)
    for (int i = 0; i < ho; ++i) h[5][(size_t)i * ho + r] = h[1][(size_t)r * ho + i];
  for (int i = 0; i < he; ++i)
    for (int r = 0; r < ho; ++r) h[7][(size_t)r * he + i] = h[3][(size_t)i * ho + r];
  M.lam_s = st.put_d(lam_s);
  for (int q = 0; q < 8; ++q) M.h64[q] = st.put_d(h[q]);
  for (int q = 0; q < 8; ++q) M.h32[q] = st.put_f(h[q]);
  // fragment packs for the matrix-core transforms: fragment (kq, t, l) =
  // Mat[o = 16 t + l % 16][k = 4 kq + l / 16], zero outside the matrix, laid out by
  // mf_pack_index (two FP64 / four FP32 fragments per 16-byte lane load)
  M.mf = he <= kMfMaxHalf;
  if (!M.mf) return;
  const int RT = (he + 15) / 16, KQ = mf_steps(he);
  const int rows[4] = {he, ho, he, he}, cols[4] = {he, ho, he, ho};
  for (int q = 0; q < 4; ++q) {
    std::vector<double> P2(mf_pack_size(he, 2), 0.0), P4(mf_pack_size(he, 4), 0.0);
    for (int kq = 0; kq < KQ; ++kq)
      for (int t = 0; t < RT; ++t)
        for (int l = 0; l < 64; ++l) {
          const int o = 16 * t + l % 16, k = 4 * kq + l / 16;
          if (o < rows[q] && k < cols[q]) {
            const double v = h[q][(size_t)o * cols[q] + k];
            P2[mf_pack_index(kq, t, l, RT, 2)] = v;
            P4[mf_pack_index(kq, t, l, RT, 4)] = v;
          }
        }
    M.p64[q] = st.put_d(P2);
    M.p32[q] = st.put_f(P4);
  }
}

}  // namespace lk
