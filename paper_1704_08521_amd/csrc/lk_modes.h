// Tensor-product factors of 1D operators (host computation and device placement), shared by
// the pressure-correction solve and the viscous step of the Stokes-preconditioned vectors.
#pragma once

#include <cstddef>
#include <vector>

#include "lk_ctx.h"

namespace lk {

// Host results for one 1D operator K s = lam M s on n points.
struct ModeHost {
  int n = 0;
  std::vector<double> lam, S, Wf, m;  // full modes (S^T M S = I, Wf = S^T M) and the mass
  bool sym = false;                   // mirror-symmetric: the half problems below are set
  std::vector<double> lam_e, Sh_e, lam_o, Sh_o;
};

// Full modes, and the even / odd half modes when `sym` (the operator must then be
// mirror-symmetric).  False if an eigensolve fails.
bool compute_modes(int n, const std::vector<double>& kd, const std::vector<double>& ko, const std::vector<double>& m,
                   bool sym, ModeHost& H);

// Device bytes that place_modes needs for one operator of n points (alignment included).
size_t mode_bytes(int n);

// Writes arrays into a host staging buffer whose image is later copied to the device
// allocation `dev` in one transfer; device pointers are handed out as the arrays are
// placed.  Every array starts 16-byte aligned.
struct Stager {
  std::vector<char> host;
  char* dev = nullptr;
  size_t used = 0;
  bool overflow = false;
  Stager(size_t bytes, void* device) : host(bytes), dev((char*)device) {}
  void* put(const void* src, size_t bytes);
  double* put_d(const std::vector<double>& v);
  float* put_f(const std::vector<double>& v);  // rounded to float32
};

// Places the factors of one operator: the full matrices F = S^T M, Bk = S and their
// transposes (float64 and float32), and for a mirror-symmetric operator the
// parity-sorted eigenvalues, the half-size matrices and (half length <= kMfMaxHalf) the
// matrix-core fragment packs.
void place_modes(const ModeHost& H, AxisModes& M, Stager& st);

}  // namespace lk
