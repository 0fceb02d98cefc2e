// C ABI of the plane projections (Section 4, eqs. 11-17): the plane Poisson problems
// reuse the per-axis transforms of the pressure solver along the two in-plane axes, or,
// for the planes containing x with the TPT route selected, one transform pair and the
// tridiagonal x pass.
#include <hip/hip_runtime.h>

#include "lk_ctx.h"
#include "lk_internal.h"

using namespace lk;

namespace {

// One transform pass along `axis` (0 x, 1 y, 2 z), forward (S^T M) or backward (S),
// in the same variant the 3D solver picks for that axis: matrix cores, folded
// half-size transforms of a mirror-symmetric axis, or the full matrices.
int axis_pass(lc_ctx* c, int axis, bool fwd, const double* in, double* out) {
  const int nx = c->nx, ny = c->ny, nz = c->nz;
  const long pl = (long)nx * ny;
  const int n_yz = ny * nz, n_xz = nx * nz;
  const AxisModes& M = c->modes[axis];
  const double* nul = nullptr;
  hipStream_t s = c->stream;
  if (axis == 0) {
    if (M.mf) {
      if (fwd)
        KLAUNCH(c, LC_K_TP_X, launch_mff_right<double>(nx, n_yz, in, M.p64[0], M.p64[1], out, s));
      else
        KLAUNCH(c, LC_K_TP_X, launch_mfu_right<double>(nx, n_yz, in, M.p64[2], M.p64[3], out, s));
    } else if (M.sym) {
      if (fwd)
        KLAUNCH(c, LC_K_TP_X, launch_tpf_right<double>(nx, n_yz, in, M.h64[4], M.h64[5], out, s));
      else
        KLAUNCH(c, LC_K_TP_X, launch_tpu_right<double>(nx, n_yz, in, M.h64[6], M.h64[7], out, s));
    } else {
      KLAUNCH(c, LC_K_TP_X, launch_tp_right<double>(n_yz, nx, nx, in, fwd ? M.FT : M.BkT, out, s));
    }
    return LC_OK;
  }
  // left transforms: y runs over columns (k, i) with rows nx apart in segments of nx
  // columns, pl apart; z over the pl columns with rows pl apart
  const int kid = axis == 1 ? LC_K_TP_Y : LC_K_TP_Z;
  const int n = axis == 1 ? ny : nz, cols = axis == 1 ? n_xz : (int)pl;
  const int nseg = axis == 1 ? nx : (int)pl;
  const long sstride = axis == 1 ? pl : 0, rstride = axis == 1 ? (long)nx : pl;
  if (M.mf) {
    if (fwd)
      KLAUNCH(c, kid, launch_mff_left<double>(n, cols, M.p64[0], M.p64[1], in, out, nseg, sstride, rstride, s));
    else
      KLAUNCH(c, kid, launch_mfu_left<double>(n, cols, M.p64[2], M.p64[3], in, out, nseg, sstride, rstride, nul, nul, nul,
                                              1, 0, 0, 0, s));
  } else if (M.sym) {
    if (fwd)
      KLAUNCH(c, kid, launch_tpf_left<double>(n, cols, M.h64[0], M.h64[1], in, out, nseg, sstride, rstride, nul, nul, nul,
                                              1, 0, 0, 0, s));
    else
      KLAUNCH(c, kid, launch_tpu_left<double>(n, cols, M.h64[2], M.h64[3], in, out, nseg, sstride, rstride, s));
  } else {
    KLAUNCH(c, kid, launch_tp_left<double>(n, cols, n, fwd ? M.F : M.Bk, in, out, nseg, sstride, rstride, nul, nul, nul,
                                           1, 0, 0, 0, s));
  }
  return LC_OK;
}

}  // namespace

extern "C" int lc_plane_project(lc_ctx* c, const double* v, int which, double* out, double* psi) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (which < 1 || which > 3) return fail(c, LC_EINVAL, "plane projection must be 1, 2 or 3");
  if (!aligned(v) || !aligned(out) || (psi && !aligned(psi)) || out == v) return fail(c, LC_EINVAL, "bad pointers");
  // the two in-plane axes (a, b) and the normal one
  static const int kA[4] = {0, 0, 1, 0}, kB[4] = {0, 2, 2, 1}, kN[4] = {0, 1, 0, 2};
  const int a = kA[which], b = kB[which], nrm = kN[which];
  hipStream_t s = c->stream;
  KLAUNCH(c, LC_K_PLANES, launch_plane_rhs(c->g, which, v, c->r, s));
  if (a == 0 && c->poisson_method == LC_POISSON_TPT && c->nx <= tridiag_x_max()) {
    // planes containing x (P = 1, 3): transform along the other in-plane axis, one
    // tridiagonal solve per x-line shifted by that axis's eigenvalues, transform back
    const AxisModes& B = c->modes[b];
    const double* lb = B.sym ? B.lam_s : B.lam;
    rc = axis_pass(c, b, true, c->r, c->t1);
    if (rc) return rc;
    KLAUNCH(c, LC_K_TRIDIAG,
            launch_tridiag_x<double>(c->g, b == 1 ? lb : nullptr, b == 2 ? lb : nullptr, b == 1 ? c->zero_mode[1] : -1,
                             b == 2 ? c->zero_mode[2] : -1, c->t1, c->t2, s));
    rc = axis_pass(c, b, false, c->t2, c->phi);
    if (rc) return rc;
    KLAUNCH(c, LC_K_PLANES, launch_plane_correct(c->g, which, v, c->phi, out, s));
    if (psi) KLAUNCH(c, LC_K_PLANES, launch_plane_potential(c->g, which, out, psi, s));
    HIPCHK(c, hipStreamSynchronize(s));
    return LC_OK;
  }
  // forward along a then b, scale, backward along b then a
  rc = axis_pass(c, a, true, c->r, c->t1);
  if (!rc) rc = axis_pass(c, b, true, c->t1, c->t2);
  if (rc) return rc;
  const double* lam[3];
  int zm[3];
  for (int ax = 0; ax < 3; ++ax) {
    const AxisModes& M = c->modes[ax];
    lam[ax] = ax == nrm ? nullptr : (M.sym ? M.lam_s : M.lam);
    zm[ax] = ax == nrm ? -1 : c->zero_mode[ax];
  }
  KLAUNCH(c, LC_K_PLANES,
          launch_plane_scale(c->t2, c->nx, c->ny, c->nz, lam[0], lam[1], lam[2], zm[0], zm[1], zm[2], s));
  rc = axis_pass(c, b, false, c->t2, c->t1);
  if (!rc) rc = axis_pass(c, a, false, c->t1, c->phi);
  if (rc) return rc;
  KLAUNCH(c, LC_K_PLANES, launch_plane_correct(c->g, which, v, c->phi, out, s));
  if (psi) KLAUNCH(c, LC_K_PLANES, launch_plane_potential(c->g, which, out, psi, s));
  HIPCHK(c, hipStreamSynchronize(s));
  return LC_OK;
}
