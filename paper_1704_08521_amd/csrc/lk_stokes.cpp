// Stokes-preconditioned (time-stepper) Krylov vectors, the comparison variant of Section 3
// (Stokes preconditioning by time steps, refs. [35-37]): the viscous part of a linearized
// time step taken implicitly, u = (I/dt - Re^-1 Lap_0)^-1 f, followed by the projection.
//
// On the staggered tensor-product grid Lap_0 acts on each velocity component as a sum of
// three 1D operators: along the component's own axis the face operator (walls hold zero),
// along the two others the cell-centred operator whose wall value zero is reached over a
// half width.  Each is symmetric in its own mass (K s = lam M s, S^T M S = I), so the
// viscous step of a component is a full tensor-product factorization: transform with S^T M
// along x, y, z, divide by 1/dt - Re^-1 (lam_x + lam_y + lam_z), transform back with S --
// the pressure solve's transform kernels with other factors and another scaling.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "lk_ctx.h"
#include "lk_internal.h"
#include "lk_linalg.h"
#include "lk_modes.h"

using namespace lk;

namespace {

// Factors of the cell-centred and face operators of every axis, for the current grid.
int build_viscous_factors(lc_ctx* c) {
  const int n[3] = {c->nx, c->ny, c->nz};
  const size_t bytes = viscous_bytes(n[0], n[1], n[2]);
  if (!c->stokes_mem && ctx_alloc(c, &c->stokes_mem, bytes) != hipSuccess)
    return fail(c, LC_ENOMEM, "cannot allocate the viscous-step factors (%.1f MB)", bytes * 1e-6);
  HIPCHK(c, hipStreamSynchronize(c->stream));  // the factors may be in use by queued work
  Stager st(bytes, c->stokes_mem);
  for (int a = 0; a < 3; ++a) {
    const AxisHost& AH = c->ax[a];
    const bool sym = c->axis_sym[a];
    std::vector<double> kd, ko, m;
    ModeHost Hc, Hf;
    dirichlet_cell_operator(n[a], AH.dd.data(), kd, ko);
    if (!compute_modes(n[a], kd, ko, AH.d, sym, Hc))
      return fail(c, LC_EINVAL, "viscous factors: eigen-solver did not converge on axis %d (cells)", a);
    dirichlet_face_operator(n[a], AH.d.data(), AH.dd.data(), kd, ko, m);
    if (!compute_modes(n[a] + 1, kd, ko, m, sym, Hf))
      return fail(c, LC_EINVAL, "viscous factors: eigen-solver did not converge on axis %d (faces)", a);
    place_modes(Hc, c->vcell[a], st);
    place_modes(Hf, c->vface[a], st);
    auto order = [](const ModeHost& H) {
      if (!H.sym) return H.lam;
      std::vector<double> l(H.lam_e);
      l.insert(l.end(), H.lam_o.begin(), H.lam_o.end());
      return l;
    };
    c->vlam_cell[a] = order(Hc);
    c->vlam_face[a] = order(Hf);
  }
  if (st.overflow) return fail(c, LC_ENOMEM, "viscous factor storage sized too small (internal)");
  HIPCHK(c, hipMemcpy(c->stokes_mem, st.host.data(), st.used, hipMemcpyHostToDevice));
  size_t total = 0;
  for (int a = 0; a < 3; ++a) {
    c->vscale_off[2 * a] = total;
    total += n[a];
    c->vscale_off[2 * a + 1] = total;
    total += n[a] + 1;
  }
  if (!c->vscale && dalloc(c, &c->vscale, total) != hipSuccess)
    return fail(c, LC_ENOMEM, "cannot allocate the viscous-step eigenvalues");
  if (!c->hs && dalloc(c, &c->hs, component_max(n[0], n[1], n[2])) != hipSuccess)
    return fail(c, LC_ENOMEM, "cannot allocate the viscous-step temporary");
  c->vscale_dt = -1.0;
  c->stokes_ready = true;
  return LC_OK;
}

// Scaled eigenvalues for (Re, dt): -Re^-1 lam along x and y, -Re^-1 lam + 1/dt along z,
// so that the kernels' division by the sum is the division by 1/dt - Re^-1 (lam_x + lam_y
// + lam_z), the eigenvalue of I/dt - Re^-1 Lap_0 (lam <= 0; dt = inf gives 1/dt = 0).
int viscous_scales(lc_ctx* c, double dt) {
  if (c->vscale_dt == dt && c->vscale_re == c->re) return LC_OK;
  const double rre = 1.0 / c->re, rdt = std::isinf(dt) ? 0.0 : 1.0 / dt;
  std::vector<double> h;
  for (int a = 0; a < 3; ++a)
    for (const std::vector<double>* l : {&c->vlam_cell[a], &c->vlam_face[a]})
      for (double x : *l) h.push_back(-rre * x + (a == 2 ? rdt : 0.0));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(c->vscale, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice));
  c->vscale_dt = dt;
  c->vscale_re = c->re;
  return LC_OK;
}

// out = scaled tensor-product solve of one component stored [Lz][Ly][Lx] (x fastest):
// forward transforms along x, y, z with the factors' S^T M, division by lm_z[k] + l_y[j]
// + l_x[i], backward transforms with S.  in, out: distinct; tmp: one component of scratch.
int tp3(lc_ctx* c, const AxisModes& X, const AxisModes& Y, const AxisModes& Z, int Lx, int Ly, int Lz,
        const double* sx, const double* sy, const double* sz, const double* in, double* out, double* tmp) {
  const long pl = (long)Lx * Ly;
  const int n_yz = Ly * Lz, n_xz = Lx * Lz;
  hipStream_t s = c->stream;
  const double* nul = nullptr;
  // forward x: in -> tmp
  if (X.mf)
    KLAUNCH(c, LC_K_TP_X, launch_mff_right<double>(Lx, n_yz, in, X.p64[0], X.p64[1], tmp, s));
  else if (X.sym)
    KLAUNCH(c, LC_K_TP_X, launch_tpf_right<double>(Lx, n_yz, in, X.h64[4], X.h64[5], tmp, s));
  else
    KLAUNCH(c, LC_K_TP_X, launch_tp_right<double>(n_yz, Lx, Lx, in, X.FT, tmp, s));
  // forward y: tmp -> out
  if (Y.mf)
    KLAUNCH(c, LC_K_TP_Y, launch_mff_left<double>(Ly, n_xz, Y.p64[0], Y.p64[1], tmp, out, Lx, pl, Lx, s));
  else if (Y.sym)
    KLAUNCH(c, LC_K_TP_Y, launch_tpf_left<double>(Ly, n_xz, Y.h64[0], Y.h64[1], tmp, out, Lx, pl, Lx, nul, nul, nul,
                                                  1, 0, 0, 0, s));
  else
    KLAUNCH(c, LC_K_TP_Y,
            launch_tp_left<double>(Ly, n_xz, Ly, Y.F, tmp, out, Lx, pl, Lx, nul, nul, nul, 1, 0, 0, 0, s));
  // forward z: out -> tmp (the division here unless the backward matrix-core transform takes it)
  if (Z.mf)
    KLAUNCH(c, LC_K_TP_Z, launch_mff_left<double>(Lz, (int)pl, Z.p64[0], Z.p64[1], out, tmp, (int)pl, 0, pl, s));
  else if (Z.sym)
    KLAUNCH(c, LC_K_TP_Z, launch_tpf_left<double>(Lz, (int)pl, Z.h64[0], Z.h64[1], out, tmp, (int)pl, 0, pl, sz, sy,
                                                  sx, Lx, -1, -1, -1, s));
  else
    KLAUNCH(c, LC_K_TP_Z, launch_tp_left<double>(Lz, (int)pl, Lz, Z.F, out, tmp, (int)pl, 0, pl, sz, sy, sx, Lx, -1,
                                                 -1, -1, s));
  // backward z: tmp -> out
  if (Z.mf)
    KLAUNCH(c, LC_K_TP_Z, launch_mfu_left<double>(Lz, (int)pl, Z.p64[2], Z.p64[3], tmp, out, (int)pl, 0, pl, sz, sy,
                                                  sx, Lx, -1, -1, -1, s));
  else if (Z.sym)
    KLAUNCH(c, LC_K_TP_Z, launch_tpu_left<double>(Lz, (int)pl, Z.h64[2], Z.h64[3], tmp, out, (int)pl, 0, pl, s));
  else
    KLAUNCH(c, LC_K_TP_Z, launch_tp_left<double>(Lz, (int)pl, Lz, Z.Bk, tmp, out, (int)pl, 0, pl, nul, nul, nul, 1,
                                                 0, 0, 0, s));
  // backward y: out -> tmp
  if (Y.mf)
    KLAUNCH(c, LC_K_TP_Y, launch_mfu_left<double>(Ly, n_xz, Y.p64[2], Y.p64[3], out, tmp, Lx, pl, Lx, nul, nul, nul,
                                                  1, 0, 0, 0, s));
  else if (Y.sym)
    KLAUNCH(c, LC_K_TP_Y, launch_tpu_left<double>(Ly, n_xz, Y.h64[2], Y.h64[3], out, tmp, Lx, pl, Lx, s));
  else
    KLAUNCH(c, LC_K_TP_Y,
            launch_tp_left<double>(Ly, n_xz, Ly, Y.Bk, out, tmp, Lx, pl, Lx, nul, nul, nul, 1, 0, 0, 0, s));
  // backward x: tmp -> out
  if (X.mf)
    KLAUNCH(c, LC_K_TP_X, launch_mfu_right<double>(Lx, n_yz, tmp, X.p64[2], X.p64[3], out, s));
  else if (X.sym)
    KLAUNCH(c, LC_K_TP_X, launch_tpu_right<double>(Lx, n_yz, tmp, X.h64[6], X.h64[7], out, s));
  else
    KLAUNCH(c, LC_K_TP_X, launch_tp_right<double>(n_yz, Lx, Lx, tmp, X.BkT, out, s));
  return LC_OK;
}

}  // namespace

namespace lk {

// u = (I/dt - Re^-1 Lap_0)^-1 f, component by component (u, f: velocity, distinct).
int viscous_solve(lc_ctx* c, const double* f, double* u, double dt) {
  int rc;
  if (!c->stokes_ready && (rc = build_viscous_factors(c))) return rc;
  if ((rc = viscous_scales(c, dt))) return rc;
  const VelLayout L = vel_layout(c->nx, c->ny, c->nz);
  const int nx = c->nx, ny = c->ny, nz = c->nz;
  const double* sc[3];
  const double* sf[3];
  for (int a = 0; a < 3; ++a) {
    sc[a] = c->vscale + c->vscale_off[2 * a];
    sf[a] = c->vscale + c->vscale_off[2 * a + 1];
  }
  // u on x-faces [nz][ny][nx+1]: faces along x, cells along y and z
  if ((rc = tp3(c, c->vface[0], c->vcell[1], c->vcell[2], nx + 1, ny, nz, sf[0], sc[1], sc[2], f + L.ou(),
                u + L.ou(), c->hs)))
    return rc;
  // v on y-faces [nz][ny+1][nx]
  if ((rc = tp3(c, c->vcell[0], c->vface[1], c->vcell[2], nx, ny + 1, nz, sc[0], sf[1], sc[2], f + L.ov(),
                u + L.ov(), c->hs)))
    return rc;
  // w on z-faces [nz+1][ny][nx]
  if ((rc = tp3(c, c->vcell[0], c->vcell[1], c->vface[2], nx, ny, nz + 1, sc[0], sc[1], sf[2], f + L.ow(),
                u + L.ow(), c->hs)))
    return rc;
  // the decoupled wall points carry the zero they were given; make the walls exact zeros
  KLAUNCH(c, LC_K_VECTOR, launch_zero_walls(u, nx, ny, nz, c->stream));
  return LC_OK;
}

// u = P (I/dt - Re^-1 Lap_0)^-1 f: the viscous step, then the projection (precision and
// tolerance of the projection as for a Krylov vector).  u must not alias f; uses c->w.
int stokes_step(lc_ctx* c, const double* f, double* u, double dt, int precision, double tol, int max_iter) {
  int rc = viscous_solve(c, f, c->w, dt);
  if (rc) return rc;
  lc_stats st;
  rc = lc_project(c, c->w, u, nullptr, precision, tol, max_iter, &st);
  return rc;
}

}  // namespace lk

namespace {
int check_dt(lc_ctx* c, double dt) {
  if (!(dt > 0.0)) return fail(c, LC_EINVAL, "time step must be positive (or infinite)");
  return LC_OK;
}
}  // namespace

extern "C" int lc_viscous_solve(lc_ctx* c, const double* f, double* u, double dt) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (!aligned(f) || !aligned(u) || f == u) return fail(c, LC_EINVAL, "bad or aliased velocity pointers");
  if ((rc = check_dt(c, dt))) return rc;
  if ((rc = viscous_solve(c, f, u, dt))) return rc;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LC_OK;
}

extern "C" int lc_stokes_step(lc_ctx* c, const double* f, double* u, double dt, int precision, double tol,
                              int max_iter, lc_stats* st) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (!aligned(f) || !aligned(u) || f == u) return fail(c, LC_EINVAL, "bad or aliased velocity pointers");
  if ((rc = check_dt(c, dt))) return rc;
  if ((rc = viscous_solve(c, f, c->w, dt))) return rc;
  return lc_project(c, c->w, u, nullptr, precision, tol, max_iter, st);
}

extern "C" int lc_stokes_vector(lc_ctx* c, const double* v, double* out, double dt, int precision, double tol,
                                int max_iter, lc_stats* st) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (!aligned(v) || !aligned(out) || v == out) return fail(c, LC_EINVAL, "bad or aliased velocity pointers");
  if ((rc = check_dt(c, dt))) return rc;
  rc = lc_krylov_vector(c, v, out, nullptr, precision, tol, max_iter, st);
  if (rc) return rc;
  if ((rc = viscous_solve(c, out, c->w, dt))) return rc;
  return lc_project(c, c->w, out, nullptr, precision, tol, max_iter, st);
}

extern "C" int lc_set_stokes_precond(lc_ctx* c, double dt) {
  if (!c) return LC_EINVAL;
  if (!(dt >= 0.0)) return fail(c, LC_EINVAL, "time step must be >= 0 (0: off) or infinite");
  c->stokes_dt = dt;
  return LC_OK;
}
