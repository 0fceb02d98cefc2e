/*
 * lidkrylov -- SIMPLE-evaluated Krylov vectors for the linear stability of the
 * lid-driven flow in a cube (Gelfgat, "Linear instability of the lid-driven flow
 * in a cubic cavity"), on one AMD Instinct MI355X (gfx950).
 *
 * C ABI.  Every field argument is a caller-owned DEVICE pointer (e.g. the
 * data_ptr() of a contiguous torch tensor on the GPU), 8-byte aligned, holding
 * IEEE float64 values, unless a comment says "host".  Field layout, x fastest
 * (C order), for an Nx x Ny x Nz grid of finite volumes:
 *
 *   u : [Nz][Ny][Nx+1]   x-faces, i = 0 and i = Nx are walls
 *   v : [Nz][Ny+1][Nx]   y-faces, j = 0 and j = Ny are walls
 *   w : [Nz+1][Ny][Nx]   z-faces, k = 0 and k = Nz are walls
 *   p : [Nz][Ny][Nx]     cell centres
 *
 * A "velocity" argument is the packed vector u|v|w of
 * lc_vel_size() = (Nx+1)NyNz + Nx(Ny+1)Nz + NxNy(Nz+1) doubles; a "cell"
 * argument holds NxNyNz doubles.  Wall-normal faces of velocity inputs are
 * ignored (read as zero); every velocity output has exact zeros there.
 *
 * Execution: one context per stream; calls enqueue on the context's HIP stream
 * and return when their outputs are valid (convergence control reads scalar
 * reductions back to the host).  Contexts are not thread-safe.  Inputs and
 * outputs of one call must not alias unless a comment allows it.  A context made by
 * lc_create owns its scratch device memory (allocated in lc_create, lc_set_grid and
 * on first use of a driver, freed in lc_destroy); one made by lc_create_in carves it
 * from a caller-owned block sized by lc_workspace_query.
 *
 * Return codes: LC_OK = 0; LC_ENOTCONV = 1 (outputs valid, tolerance not met);
 * negative values are errors, the message is in lc_last_error().
 */
#ifndef LIDKRYLOV_H
#define LIDKRYLOV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LC_OK 0
#define LC_ENOTCONV 1
#define LC_EINVAL (-1)  /* bad size, pointer, value, or non-finite input      */
#define LC_ESTATE (-2)  /* grid, Re or base flow not set                      */
#define LC_EHIP (-3)    /* HIP runtime error                                  */
#define LC_ENOMEM (-4)  /* device allocation failed, or caller workspace too small */

/* Stretching kinds for lc_set_stretching. */
#define LC_UNIFORM 0 /* x_i = i/N                                             */
#define LC_SINE 1    /* Section 3, eq. 5: x_i -> x_i - 0.0975 sin(2 pi x_i)   */
#define LC_TANH 2    /* x = (1 + tanh(b(2xi-1))/tanh b)/2, cosh^2 b = param    */

/* Precision forms of the pressure-correction solve. */
#define LC_FP64 0  /* plain: every step in float64                            */
#define LC_MIXED 1 /* float32 tensor-product solves inside float64 refinement */
#define LC_LEARNED 2 /* network guess of the first correction, then LC_MIXED  */
                     /* passes (needs lc_set_net; plain fallback, see below) */

typedef struct lc_ctx lc_ctx;
typedef struct lc_net lc_net;

typedef struct {
  int iterations;     /* SIMPLE passes (projection corrections) performed      */
  double rho;         /* final |D v|_V / |D w|_V (volume-weighted L2)          */
  double rho0;        /* |D w|_V, the divergence of the uncorrected vector     */
  double rho_hist[16];/* rho after each pass                                   */
  double ms_total;    /* wall time of the call, host clock                     */
  int guess_used;     /* LC_LEARNED: 1 if the network guess started the loop,  */
                      /* 0 if it fell back to the plain start v = w, p = 0     */
  double guess_eps;   /* LC_LEARNED: rho right after the guess (1 on fallback) */
  /* Device time of the call per phase, from the profiling events (lc_profile_enable on;
   * -1 when profiling is off): momentum stencil and divergences, pressure-correction
   * solves (transforms, tridiagonal passes, precision casts), velocity/pressure
   * corrections, and the network's guess.  Reductions and vector operations are in
   * ms_total only. */
  double ms_stencil, ms_poisson, ms_update, ms_network;
} lc_stats;

/* Library version string (static storage). */
const char* lc_version(void);

/* Message of the last error on this context (or of the last failed lc_create
 * when ctx is NULL).  Static or context-owned storage. */
const char* lc_last_error(const lc_ctx* ctx);

/* Create a context for an nx x ny x nz grid (each >= 2, <= 4096, and each velocity
 * component below 2^31 bytes: about 640^3 for a cube) on the HIP
 * stream `hip_stream` (hipStream_t, NULL = default stream) of the current
 * device.  The grid starts uniform, Re = 1, lid angle 0, base flow zero. */
int lc_create(lc_ctx** out, int nx, int ny, int nz, void* hip_stream);
int lc_destroy(lc_ctx* ctx);

/* Caller-owned workspace.  lc_workspace_query gives the device bytes a context of an
 * nx x ny x nz grid needs when every buffer it uses -- work fields, grid factors,
 * viscous-step factors, reduction scratch, the critical-Re steady states, and the Krylov
 * vectors of Newton with gmres_m <= m_max and Arnoldi with m <= m_max (0 <= m_max <= 400)
 * -- comes from one block.  lc_create_in is lc_create with that block (device memory,
 * 256-byte aligned, `bytes` long, owned by the caller and untouched by lc_destroy): the
 * library then allocates no device memory of its own (small pinned host scalars and
 * events only).  A call that needs more Krylov vectors than the block holds fails with
 * LC_ENOMEM ("workspace too small"), as does lc_create_in when the block cannot hold the
 * fixed buffers.  The block must outlive the context. */
int lc_workspace_query(int nx, int ny, int nz, int m_max, size_t* bytes);
int lc_create_in(lc_ctx** out, int nx, int ny, int nz, void* workspace, size_t bytes, void* hip_stream);
int lc_set_stream(lc_ctx* ctx, void* hip_stream);

/* Number of doubles in a packed velocity / a cell field. */
size_t lc_vel_size(const lc_ctx* ctx);
size_t lc_cell_size(const lc_ctx* ctx);

/* Face coordinates (host arrays of nx+1, ny+1, nz+1 doubles, strictly
 * increasing from 0 to 1) -- the N+1 grid points per direction of Section 3.
 * Rebuilds the metrics and the tensor-product Poisson factorization. */
int lc_set_grid(lc_ctx* ctx, const double* xf, const double* yf, const double* zf);

/* Generate the faces of every axis with one stretching (LC_UNIFORM, LC_SINE,
 * LC_TANH with param = centre/wall spacing ratio > 1) and call lc_set_grid. */
int lc_set_stretching(lc_ctx* ctx, int kind, double param);

/* Copy the faces out (host arrays of nx+1, ny+1, nz+1 doubles). */
int lc_get_grid(const lc_ctx* ctx, double* xf, double* yf, double* zf);

/* Reynolds number Re = UL/nu (Section 2), re > 0. */
int lc_set_re(lc_ctx* ctx, double re);

/* Lid direction: u = cos(alpha), v = sin(alpha) at z = 1 (Section 2, eq. 4). */
int lc_set_lid(lc_ctx* ctx, double alpha_rad);

/* Base flow U (velocity, device) about which eq. 6 is linearized; copied.  The base-flow
 * pressure enters the equations linearly, so the linearized operator does not depend on
 * it and it is not an input; lc_get_base_flow computes it from U. */
int lc_set_base_flow(lc_ctx* ctx, const double* U);
/* Copy the base flow out (velocity, device).  P (cell, device, may be NULL) receives the
 * pressure of the steady equations at U: the P with R(U) - G P divergence-free and
 * sum V P = 0 (R the residual of lc_residual; at a steady state R(U) = G P), by one exact
 * projection (uses the work vector and one Krylov vector). */
int lc_get_base_flow(lc_ctx* ctx, double* U, double* P);

/* ---------------------------------------------------------------- stencils */

/* Right side of eq. 10, the linearized momentum (eq. 6) applied to v:
 * w = Re^-1 Lap v - (U.grad)v - (v.grad)U with homogeneous wall values, in the
 * conservative staggered form.  v, w: velocity. */
int lc_jacobian_apply(lc_ctx* ctx, const double* v, double* w);

/* Momentum residual of eq. 2 at steady state without pressure:
 * R(U) = Re^-1 Lap U - (U.grad)U with the lid of eq. 4.  U, R: velocity. */
int lc_residual(lc_ctx* ctx, const double* U, double* R);

/* Cell divergence (eq. 1) of a velocity; r: cell.  If vnorm is not NULL it
 * receives (host) the volume-weighted norm sqrt(sum V r^2). */
int lc_divergence(lc_ctx* ctx, const double* v, double* r, double* vnorm);

/* Pressure-solve route (Section 3: the paper's TPT and TPF tensor-product solvers),
 * for the FP64 and FP32 solves alike.  LC_POISSON_TPT (default): mode transforms along
 * y and z and, along x, one tridiagonal solve per line (a partition method: per-lane
 * segment elimination, cyclic reduction across the lanes), for nx up to 1024 (larger nx
 * uses TPF).  LC_POISSON_TPF: mode transforms along x, y and z and a division by the
 * eigenvalue sums.  Both give the same solution up to rounding.  LC_EINVAL for an
 * unknown method. */
#define LC_POISSON_TPF 0
#define LC_POISSON_TPT 1
int lc_set_poisson_method(lc_ctx* ctx, int method);

/* Pressure-correction Poisson solve (Section 3, step 1): (D G) phi = r with the
 * Neumann wall condition and sum V phi = 0.  r, phi: cell (may alias). */
int lc_poisson_solve(lc_ctx* ctx, const double* r, double* phi, int precision);

/* Velocity/pressure correction (Section 3, step 2): v = w - G phi on interior
 * faces (zero on walls) and p = phi.  w, v: velocity; phi, p: cell. */
int lc_correct(lc_ctx* ctx, const double* w, const double* phi, double* v, double* p);

/* ------------------------------------------------------------- hot path */

/* Divergence-free projection of w by the SIMPLE-like loop of Section 3:
 * v = w, p = 0; repeat { solve (D G) phi = D v; v -= G phi; p += phi } until
 * |D v|_V <= tol |D w|_V or max_iter passes.  v_out (velocity) is required; p_out
 * (cell) may be NULL, and then no pressure is written (the Krylov drivers use the
 * velocity only).  Neither may alias w.  stats may be NULL. */
int lc_project(lc_ctx* ctx, const double* w, double* v_out, double* p_out,
               int precision, double tol, int max_iter, lc_stats* stats);

/* The next Krylov vector (eqs. 8-10): v_out = P(L_U v_in), p_out its pressure (may be
 * NULL), by lc_jacobian_apply followed by lc_project. */
int lc_krylov_vector(lc_ctx* ctx, const double* v_in, double* v_out, double* p_out,
                     int precision, double tol, int max_iter, lc_stats* stats);

/* Host-only utility (no GPU needed): the modes of one axis used by the
 * tensor-product Poisson solve.  faces: host array of n+1 strictly increasing
 * doubles.  Solves K s = lam M s, with M = diag(cell widths) and K the Neumann
 * couplings 1/(centre distance) across interior faces (the 1D factor of D G).
 * Outputs (host): lam[n] ascending (the last is the Neumann null mode, ~0),
 * S[n*n] row-major with the modes as columns (S^T M S = I), Wf[n*n] = S^T M. */
int lc_axis_modes(int n, const double* faces, double* lam, double* S, double* Wf);

/* Host-only utility (no GPU needed): eigenvalues of a real m x m upper
 * Hessenberg matrix H (host, row-major; entries below the subdiagonal are
 * ignored), the eigensolve of the Arnoldi restarts.  re, im: m doubles each
 * (host), unordered.  LC_EINVAL if m < 1 or the QR iteration fails. */
int lc_hessenberg_eigvals(int m, const double* H, double* re, double* im);

/* -------------------------------------------------------- Krylov drivers */

/* Projected steady residual F = P R(U) of the context's base flow (Section 3,
 * Newton step 2): the residual of eqs. 1-4 with its pressure part removed by
 * the projection.  F: velocity (device); res_inf (host) = max |F|. */
int lc_newton_residual(lc_ctx* ctx, double* F, double* res_inf);

/* One Newton step of Section 3 on the context's base flow U: F = P R(U), solve
 * the Jacobian system (P L_U) d = F on the divergence-free space with restarted
 * GMRES(gmres_m) on SIMPLE-evaluated Krylov vectors (classical Gram-Schmidt in
 * float64, repeated when the norm drops); a restart that lowers the residual by
 * less than 10% counts as saturation and hands its iterate to BiCGstab(2)
 * (gmres_m = 0: BiCGstab(2)
 * alone, as Section 3 used it at 100^3); then U <- U - d (step 4).  A saturated
 * restart whose residual is already within sqrt(lin_tol) |F| (the rounding
 * floor of late Newton steps) is accepted as converged.
 * The linear solve stops at |res| <= lin_tol |F| or after max_vectors Krylov
 * vectors (then LC_ENOTCONV, U still updated).  precision / proj_tol: form and
 * divergence tolerance of each Krylov vector (max 8 SIMPLE passes).  Outputs
 * (host, each may be NULL): res_inf = max |F| before the step, corr_inf =
 * max |d|, n_vectors = Krylov vectors used, used_bicgstab = 1 if the hand-off
 * happened.  Workspace: max(gmres_m + 1, 8) + 3 velocity vectors (library-owned). */
int lc_newton_step(lc_ctx* ctx, double lin_tol, int gmres_m, long max_vectors, int precision, double proj_tol,
                   double* res_inf, double* corr_inf, long* n_vectors, int* used_bicgstab);

/* Leading eigenvalues of the stability problem (eq. 7): the k eigenvalues of
 * P L_U with largest real part, by implicitly restarted Arnoldi on
 * SIMPLE-evaluated Krylov vectors started from v0 (velocity, device; NULL: a seeded
 * SplitMix64 uniform field of stream `seed`) projected onto the divergence-free space.
 * A start close to the wanted eigenvectors (the last ones of a nearby Re) shortens the
 * iteration; the seeded field also sets the divergence scale of the test below.  Each extension
 * orthogonalizes by classical Gram-Schmidt in float64 (repeated once when the
 * norm drops below 1/sqrt 2 of its value); the m x m Hessenberg eigenproblem
 * is solved in float64 on the host and the m - k unwanted Ritz values serve as
 * exact shifts (complex pairs as real double shifts).  A kept Ritz value of
 * modulus below 1e-5 of the largest is treated as unwanted when its Ritz vector is
 * far from divergence-free (relative divergence above 1e-6 of a raw random
 * vector's): such values come from rounding-level components in the gradient
 * directions, where P L_U is zero; a genuine eigenvalue near 0 (a real eigenvalue
 * crossing the imaginary axis) is divergence-free and is kept.  Converged when every
 * wanted pair has |h_{m+1,m} e_m^T y| <= tol |theta| and, recomputed with the Krylov
 * map on the Ritz vector x, |P L_U x - theta x| <= 1e-3 |theta| |x|: a pair failing
 * the second test is spurious (a drifted basis), is moved among the exact shifts and
 * the restarts continue (two extra Krylov vectors per pair checked).  If the k-th and (k+1)-th
 * values are a conjugate pair both are returned.
 * Requirements: 1 <= k <= 46, k + 3 <= m <= 100.  Outputs (host): eig_re,
 * eig_im, resid (may be NULL): arrays of k+1 doubles, real part descending;
 * n_out = number returned.  vec_re, vec_im (device, may be NULL): k+1
 * velocity vectors each, the unit-norm Ritz vectors.  n_vectors (may be NULL):
 * Krylov vectors evaluated.  Returns LC_ENOTCONV after max_restarts restarts
 * without convergence (outputs hold the last Ritz values).  Workspace:
 * 2 (m + 1) velocity vectors (library-owned). */
int lc_arnoldi_leading(lc_ctx* ctx, int k, int m, double tol, int max_restarts, unsigned long long seed,
                       const double* v0, int precision, double proj_tol, double* eig_re, double* eig_im, double* resid,
                       double* vec_re, double* vec_im, int* n_out, long* n_vectors);

/* ------------------------------------ Stokes-preconditioned Krylov vectors */

/* The comparison variant of Section 3: Krylov vectors preconditioned by a time step
 * whose viscous part is implicit (Stokes preconditioning, the paper's refs. [35-37]).
 *
 * Viscous step: u = (I/dt - Re^-1 Lap_0)^-1 f, with Lap_0 the vector Laplacian of
 * eq. 2 with homogeneous wall values (the operator of lc_jacobian_apply's viscous
 * term), solved exactly per velocity component by a tensor-product factorization of
 * its 1D Dirichlet factors (faces along the component's own axis, cells along the
 * others).  dt > 0; dt = INFINITY gives the pure Stokes operator -Re^-1 Lap_0.
 * f, u: velocity (device), distinct; wall-normal faces of f are ignored, those of u are
 * zero.  LC_EINVAL for dt <= 0 or bad pointers.  The first call on a grid builds the
 * factors (library-owned device memory, about 2.5 (n+1)^2 doubles per axis). */
int lc_viscous_solve(lc_ctx* ctx, const double* f, double* u, double dt);

/* Stokes step: u = P (I/dt - Re^-1 Lap_0)^-1 f, the viscous step followed by the
 * divergence-free projection of lc_project (precision, tol, max_iter, stats as there;
 * LC_ENOTCONV likewise).  As a right preconditioner M^-1 of the Newton system it keeps
 * the solutions of (P L_U) d = F: M^-1 maps the divergence-free space onto itself and is
 * invertible there (P (I/dt - Re^-1 Lap_0)^-1 P is symmetric definite in the face-volume
 * inner product). */
int lc_stokes_step(lc_ctx* ctx, const double* f, double* u, double dt, int precision, double tol, int max_iter,
                   lc_stats* stats);

/* Stokes-preconditioned Krylov vector: out = P (I/dt - Re^-1 Lap_0)^-1 P L_U v, the
 * time-stepper form of the next Krylov vector (lc_krylov_vector followed by
 * lc_stokes_step).  Its eigenvalues are not those of eq. 7; Newton corrections solved on
 * it are.  v, out: velocity, distinct.  stats: those of the second projection. */
int lc_stokes_vector(lc_ctx* ctx, const double* v, double* out, double dt, int precision, double tol, int max_iter,
                     lc_stats* stats);

/* Newton preconditioning: dt > 0 (or INFINITY) makes lc_newton_step solve
 * (P L_U) M^-1 y = F with M^-1 = the Stokes step of time step dt and take d = M^-1 y
 * (right preconditioning: the residual GMRES and BiCGstab(2) minimise is the true one);
 * dt = 0 (the default) solves on the SIMPLE Krylov vectors alone.  Each preconditioned
 * Krylov vector costs one viscous step and two projections more. */
int lc_set_stokes_precond(lc_ctx* ctx, double dt);

/* ------------------------------------------------- critical Reynolds number */

/* Options of lc_critical_re. */
typedef struct {
  double re_tol;          /* stop when the secant update |dRe| <= re_tol * Re              */
  int max_evals;          /* steady-state + eigenvalue evaluations (>= 2)                  */
  double newton_tol;      /* steady state: max |P R(U)| <= newton_tol (lc_newton_residual) */
  int newton_steps;       /* at most this many Newton steps per evaluation                 */
  double lin_tol;         /* Newton linear solves, as in lc_newton_step                    */
  int gmres_m;
  long max_vectors;
  int k, m;               /* Arnoldi, as in lc_arnoldi_leading (float64 Krylov vectors)    */
  double eig_tol;
  int max_restarts;
  unsigned long long seed;
  int warm_start;         /* 1: Arnoldi after the first evaluation starts from the last     */
                          /* leading eigenvector (see below); 0: every one from `seed`      */
} lc_critical_opts;

/* Critical Reynolds number of the context's grid and lid direction (Section 2, the
 * paragraph after eq. 7): the Re at which the leading eigenvalue Lambda (largest
 * real part) of the stability problem crosses the imaginary axis, and the critical
 * frequency |Im Lambda| there.  The paper does not say how it located the root; this
 * driver uses the secant method on Re -> Re Lambda(Re) from re0 and re1.  Each
 * evaluation sets Re, starts from the context's base flow (first evaluation) or from
 * the linear extrapolation in Re of the last two steady states, runs Newton steps
 * (lc_newton_step, preconditioned as lc_set_stokes_precond says) until max |P R(U)| <=
 * newton_tol or newton_steps, then lc_arnoldi_leading (LC_ENOTCONV there is accepted: its
 * last Ritz values are used), from the seeded random field the first time and afterwards
 * (warm_start = 1)
 * from the previous leading eigenvector (real plus imaginary part) plus a seeded random
 * part of relative size 1e-3.
 * The context's base flow should be a steady state (or a good guess) at re0; on
 * return it holds the last steady state and Re the last evaluated value.
 * Outputs (host): re_cr, omega_cr (|Im Lambda| interpolated linearly in Re between the
 * last two evaluations); hist (NULL or 4 * max_evals doubles) rows (Re, Re Lambda,
 * |Im Lambda|, max |P R(U)| reached); n_evals.  Returns LC_ENOTCONV when max_evals
 * evaluations did not meet re_tol; re_cr and omega_cr then come from the linear root
 * between the evaluations closest to zero on either side (largest negative and
 * smallest positive Re Lambda) when both exist, else from the last secant iterate.
 * Workspace: six velocity vectors (the stored steady states, a residual, the leading
 * eigenvector and the next start) plus those of Newton and Arnoldi. */
int lc_critical_re(lc_ctx* ctx, double re0, double re1, const lc_critical_opts* opt, double* re_cr,
                   double* omega_cr, double* hist, int* n_evals);

/* ------------------------------------------ plane projections (Section 4) */

/* Divergence-free projection of a velocity onto one family of coordinate planes
 * (Section 4, eqs. 11-14) and its vector potential (eqs. 15-17).
 *   which = 1: v1 = (u1, 0, w1), planes y = const;
 *   which = 2: v2 = (0, v2, w2), planes x = const;
 *   which = 3: v3 = (u3, v3, 0), planes z = const.
 * out (velocity, packed u|v|w) receives the orthogonal projection, in the
 * face-volume inner product, of the input's two kept components (its wall-normal
 * faces taken as zero) onto the fields whose two-dimensional divergence vanishes
 * in every such plane and whose wall-normal components vanish; the third
 * component of out is zero.  The plane pressure solves D2 G2 phi = D2 b in each
 * plane by the per-axis transforms of the pressure solver (two in-plane axes,
 * FP64).  If psi is not NULL it receives the one non-zero component of the
 * potential whose discrete curl is out, zero on the walls, on the cell edges
 * normal to the planes, last index fastest:
 *   which 1: Psi_y[k][j][i], (nz+1) x ny x (nx+1)  (x-face i, z-face k);
 *   which 2: Psi_x[k][j][i], (nz+1) x (ny+1) x nx  (y-face j, z-face k);
 *   which 3: Psi_z[k][j][i], nz x (ny+1) x (nx+1)  (x-face i, y-face j).
 * v, out, psi: device, 8-byte aligned, caller-owned; out must not alias v.
 * Uses the context's cell work arrays.  LC_EINVAL for a bad `which` or pointer,
 * LC_ESTATE before a grid is set. */
int lc_plane_project(lc_ctx* ctx, const double* v, int which, double* out, double* psi);

/* ------------------------------------------------- learned correction guess */

/* Not part of the paper's method: a small 3D convolutional network (3-level
 * U-Net, 3x3x3 kernels, channels 4-16-32-64, 2x2x2 average pooling, nearest
 * upsampling with skip concatenation, ReLU, 1x1x1 head) that guesses the first
 * pressure correction of the SIMPLE loop (Section 3, step 1) from the momentum
 * update w.  Input channels on the cells: w averaged to cell centres (3) and
 * D w, each group divided by its volume-weighted RMS; the grid is zero-padded
 * to multiples of 4.  Weights and activations are BF16 on the matrix cores
 * with FP32 accumulation; FP32 master weights and Adam moments.
 *
 * In the LC_LEARNED form the output y is scaled by the s minimising
 * |D w - s D G y|_V, the loop starts from v = w - G (s y), p = s y and then
 * runs LC_MIXED passes to the tolerance.  If the scaled guess would not lower
 * the divergence by at least 0.1% (or the fit is void) the loop starts plainly
 * from v = w, p = 0 (stats.guess_used = 0): the network can cost time but never
 * changes the fixed point.
 *
 * Parameters (host order, float32): for each layer enc1, enc2, bottleneck,
 * dec2, dec1, head the weights W[cout][taps][cin] (taps 27, tap = (dz+1)*9 +
 * (dy+1)*3 + (dx+1), cross-correlation) then the biases b[cout];
 * lc_net_param_count() values in total.  A network is used on one stream at
 * a time; its activation memory grows on demand and is freed by lc_net_destroy. */
long lc_net_param_count(void);

/* Create a network with He-normal weights (SplitMix64 stream `seed`, Box-Muller)
 * and zero biases on the current device.  LC_ENOMEM on allocation failure. */
int lc_net_create(lc_net** out, uint64_t seed);
int lc_net_destroy(lc_net* net);
const char* lc_net_last_error(const lc_net* net);

/* Copy the float32 master parameters out of / into the network (host arrays of
 * lc_net_param_count() floats).  Setting resets the Adam state. */
int lc_net_get_params(lc_net* net, float* host);
int lc_net_set_params(lc_net* net, const float* host);

/* Save / load the master parameters to / from a file (path: NUL-terminated, host):
 * the 8 bytes "LKNET001", the parameter count as a little-endian uint32, then that many
 * little-endian float32 values in lc_net_get_params order.  Loading checks the tag, the
 * count and the length (LC_EINVAL with the reason in lc_net_last_error otherwise, the
 * network unchanged) and resets the Adam state, as lc_net_set_params does. */
int lc_net_save(lc_net* net, const char* path);
int lc_net_load(lc_net* net, const char* path);

/* Forward pass on a D x H x W grid (each a positive multiple of 4):
 * x (device float32 [D][H][W][4]) -> y (device float32 [D][H][W]).
 * hip_stream: hipStream_t (NULL = default).  Returns when y is valid. */
int lc_net_forward(lc_net* net, void* hip_stream, const float* x, float* y, int D, int H, int W);

/* Mean squared error of the output against t (device float32 [D][H][W]) and
 * its gradient; grad_host (may be NULL) receives the lc_net_param_count()
 * gradients in parameter order; if lr > 0 one Adam step (beta 0.9, 0.999,
 * eps 1e-8) follows.  loss (host, may be NULL). */
int lc_net_step(lc_net* net, void* hip_stream, const float* x, const float* t, int D, int H, int W, double lr,
                double* loss, float* grad_host);

/* Attach a network to a context for LC_LEARNED (NULL detaches; not owned). */
int lc_set_net(lc_ctx* ctx, lc_net* net);

/* Train on pairs the method generates on the context's grid, base flow and Re:
 * per step a seeded random velocity (SplitMix64 stream seed * 1000003 + step) is
 * projected (float64) to v, w = L_U v, and the target is the first SIMPLE
 * correction phi of w (the float64 tensor-product solve of (D G) phi = D w),
 * scaled by its volume-weighted RMS; one Adam step of learning rate lr.
 * loss_hist (host, may be NULL): `steps` losses. */
int lc_net_train(lc_ctx* ctx, lc_net* net, int steps, double lr, uint64_t seed, double* loss_hist);

/* The scaled network guess phi0 (cell, device) for the momentum update w
 * (velocity, device) with the attached network, and eps (host, may be NULL) =
 * |D w - D G phi0|_V / |D w|_V.  On fallback phi0 = 0 and eps = 1. */
int lc_learned_guess(lc_ctx* ctx, const double* w, double* phi0, double* eps);

/* ---------------------------------------------------------- vector helpers */

/* Euclidean dot product of two velocity vectors (host result). */
int lc_dot(lc_ctx* ctx, const double* a, const double* b, double* out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): lc_dot without a context.  out (host)
 * = sum a[i] b[i] over n doubles (device, 8-byte aligned), enqueued on hip_stream
 * (hipStream_t, NULL = default) and synchronized; bit-identical to lc_dot on a context
 * whose lc_vel_size() is n (same block partial sums, same fixed-order final sum).
 * Allocates nothing: the at most 4096 partial sums and the result live in a 33 KB
 * file-scope device array, one per GPU, held until the process ends.  Every call on a
 * GPU shares that array, so calls that overlap on one GPU (several streams or host
 * threads) race; serialize them.  LC_EINVAL for null or misaligned pointers, n < 1 or
 * n > LC_NOALLOC_MAX_N; LC_EHIP for a HIP error. */
#define LC_NOALLOC_MAX_N (1ull << 36)
int lc_dot_noalloc(const double* a, const double* b, size_t n, double* out, void* hip_stream);

/* ---------------------------------------------------------------- profiling */

/* Kernel classes timed by the profiling mode. */
#define LC_K_MOMENTUM 0   /* linearized momentum stencil (eq. 10)             */
#define LC_K_RESIDUAL 1   /* nonlinear momentum residual                     */
#define LC_K_DIVERGENCE 2 /* cell divergence + norm partials                 */
#define LC_K_CORRECT 3    /* velocity/pressure correction                    */
#define LC_K_TP_X 4       /* tensor-product transform along x                */
#define LC_K_TP_Y 5       /* tensor-product transform along y                */
#define LC_K_TP_Z 6       /* tensor-product transform along z                */
#define LC_K_EIGSCALE 7   /* division by the eigenvalue sums                 */
#define LC_K_REDUCE 8     /* fixed-order final reductions                    */
#define LC_K_CAST 9       /* float64 <-> float32 conversions                 */
#define LC_K_VECTOR 10    /* dot / axpy / scale / fill                       */
#define LC_K_NN_FORWARD 11 /* network forward pass (all layers)              */
#define LC_K_NN_MISC 12   /* network input/output conversions and fits       */
#define LC_K_PLANES 13    /* plane-projection right side, scaling, correction, potentials */
#define LC_K_TRIDIAG 14   /* TPT tridiagonal solves along x                  */
#define LC_K_COUNT 15

/* Enable (1) or disable (0) per-launch HIP-event timing on the context's
 * stream; enabling clears previous records.  Adds two event records per
 * kernel launch. */
int lc_profile_enable(lc_ctx* ctx, int on);

/* Summed device time (ms) and launch count of one kernel class since the last
 * enable.  Synchronizes the stream. */
int lc_profile_read(lc_ctx* ctx, int kernel_class, double* total_ms, long* launches);

/* Name of a kernel class (static storage), NULL if out of range. */
const char* lc_profile_name(int kernel_class);

/* Streaming ceiling of the current device, the reference the stencil kernels' bandwidth is
 * judged against: a plain kernel with 16-byte accesses over arrays of `bytes` each
 * (>= 4096), kind 0 copy (1 read + 1 write), 1 two reads + one write (the momentum
 * stencil's pattern), 2 read only; 3 warm-up launches, then `reps` timed by HIP events on
 * hip_stream (hipStream_t, NULL = default).  tbps (host) = bytes moved per launch / mean
 * launch time, in TB/s; us (host, may be NULL) the mean launch time.  Allocates (and frees)
 * three arrays.  LC_EINVAL for bad arguments, LC_ENOMEM, LC_EHIP. */
int lc_stream_probe(int kind, size_t bytes, int reps, void* hip_stream, double* tbps, double* us);

#ifdef __cplusplus
}
#endif

#endif /* LIDKRYLOV_H */
