"""SIMPLE-evaluated Krylov vectors for the lid-driven cube on one MI355X.

Python face of the C ABI in ``include/lidkrylov.h``.  PyTorch supplies device
memory and the stream; every step runs in the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import _lib
from ._lib import FP64, LEARNED, MIXED, SINE, TANH, UNIFORM, CriticalOpts, LidKrylovError, Stats  # noqa: F401

__all__ = ["Context", "Net", "FP64", "MIXED", "LEARNED", "UNIFORM", "SINE", "TANH", "LidKrylovError"]


def _torch():
    import torch
    return torch


class Context:
    """One grid, one Reynolds number / lid, one base flow, on one HIP stream."""

    def __init__(self, nx: int, ny: int | None = None, nz: int | None = None, stream=None, workspace=None):
        """workspace: None (the library allocates its device memory), or a contiguous CUDA
        tensor of at least ``Context.workspace_bytes(nx, ny, nz, m_max)`` bytes that holds all of
        it (kept referenced by the context)."""
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("lidkrylov needs a GPU (torch.cuda.is_available() is False)")
        self.lib = _lib.load()
        ny = nx if ny is None else ny
        nz = nx if nz is None else nz
        self.nx, self.ny, self.nz = nx, ny, nz
        self.device = torch.device("cuda", torch.cuda.current_device())
        s = stream if stream is not None else torch.cuda.current_stream()
        self.stream = s
        h = C.c_void_p()
        if workspace is None:
            rc = self.lib.lc_create(C.byref(h), nx, ny, nz, C.c_void_p(s.cuda_stream))
        else:
            if not workspace.is_cuda or not workspace.is_contiguous():
                raise ValueError("workspace: need a contiguous CUDA tensor")
            nbytes = workspace.numel() * workspace.element_size()
            rc = self.lib.lc_create_in(C.byref(h), nx, ny, nz, C.c_void_p(workspace.data_ptr()), C.c_size_t(nbytes),
                                       C.c_void_p(s.cuda_stream))
        self.workspace = workspace
        if rc != 0:
            raise LidKrylovError(rc, self.lib.lc_last_error(None).decode())
        self._h = h
        self.nvel = int(self.lib.lc_vel_size(h))
        self.ncell = int(self.lib.lc_cell_size(h))

    # ------------------------------------------------------------- helpers
    net = None

    @staticmethod
    def workspace_bytes(nx: int, ny: int, nz: int, m_max: int = 100) -> int:
        """Device bytes of a caller workspace for this grid and Krylov basis length m_max."""
        lib = _lib.load()
        b = C.c_size_t()
        rc = lib.lc_workspace_query(int(nx), int(ny), int(nz), int(m_max), C.byref(b))
        if rc != 0:
            raise LidKrylovError(rc, "bad workspace query arguments")
        return int(b.value)

    def _check(self, rc, allow_notconv=False):
        if rc == 0 or (allow_notconv and rc == _lib.LC_ENOTCONV):
            return rc
        raise LidKrylovError(rc, self.lib.lc_last_error(self._h).decode())

    def _ptr(self, t, n, name):
        torch = _torch()
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
            raise ValueError(f"{name}: need a contiguous float64 CUDA tensor of {n} elements")
        return C.c_void_p(t.data_ptr())

    def vel(self):
        return _torch().zeros(self.nvel, dtype=_torch().float64, device=self.device)

    def cells(self):
        return _torch().zeros(self.ncell, dtype=_torch().float64, device=self.device)

    def close(self):
        if getattr(self, "_h", None):
            self.lib.lc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------- set-up
    def set_stretching(self, kind, param=10.0):
        kinds = {"uniform": UNIFORM, "sine": SINE, "tanh": TANH}
        k = kinds[kind] if isinstance(kind, str) else int(kind)
        self._check(self.lib.lc_set_stretching(self._h, k, float(param)))

    def set_grid(self, xf, yf, zf):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (xf, yf, zf)]
        for a, n in zip(arrs, (self.nx, self.ny, self.nz)):
            if a.size != n + 1:
                raise ValueError("face arrays need n+1 entries")
        self._check(self.lib.lc_set_grid(self._h, *[a.ctypes.data_as(C.c_void_p) for a in arrs]))

    def get_grid(self):
        arrs = [np.zeros(n + 1) for n in (self.nx, self.ny, self.nz)]
        self._check(self.lib.lc_get_grid(self._h, *[a.ctypes.data_as(C.c_void_p) for a in arrs]))
        return arrs

    def set_re(self, re):
        self._check(self.lib.lc_set_re(self._h, float(re)))

    def set_lid(self, alpha):
        self._check(self.lib.lc_set_lid(self._h, float(alpha)))

    def set_poisson_method(self, method):
        """Pressure-solve route (FP64 and FP32 solves): "tpt" (the default: transforms
        along y, z and tridiagonal solves along x) or "tpf" (transforms along x, y, z)."""
        m = {"tpf": 0, "tpt": 1}[method]
        self._check(self.lib.lc_set_poisson_method(self._h, m))

    def set_base_flow(self, U):
        self._check(self.lib.lc_set_base_flow(self._h, self._ptr(U, self.nvel, "U")))

    def get_base_flow(self, out=None, pressure=False):
        """The base flow U (a copy); with pressure=True also (U, P), P the pressure of the
        steady equations at U (R(U) - G P divergence-free, volume mean zero)."""
        out = self.vel() if out is None else out
        P = self.cells() if pressure else None
        self._check(self.lib.lc_get_base_flow(self._h, self._ptr(out, self.nvel, "U"),
                                              None if P is None else self._ptr(P, self.ncell, "P")))
        return (out, P) if pressure else out

    # ------------------------------------------------------------ stencils
    def jacobian_apply(self, v, out=None):
        out = self.vel() if out is None else out
        self._check(self.lib.lc_jacobian_apply(self._h, self._ptr(v, self.nvel, "v"),
                                               self._ptr(out, self.nvel, "w")))
        return out

    def residual(self, U, out=None):
        out = self.vel() if out is None else out
        self._check(self.lib.lc_residual(self._h, self._ptr(U, self.nvel, "U"),
                                         self._ptr(out, self.nvel, "R")))
        return out

    def divergence(self, v, out=None):
        out = self.cells() if out is None else out
        nrm = C.c_double()
        self._check(self.lib.lc_divergence(self._h, self._ptr(v, self.nvel, "v"),
                                           self._ptr(out, self.ncell, "r"), C.byref(nrm)))
        return out, nrm.value

    def poisson_solve(self, r, out=None, precision=FP64):
        out = self.cells() if out is None else out
        self._check(self.lib.lc_poisson_solve(self._h, self._ptr(r, self.ncell, "r"),
                                              self._ptr(out, self.ncell, "phi"), int(precision)))
        return out

    def correct(self, w, phi, v=None, p=None):
        v = self.vel() if v is None else v
        p = self.cells() if p is None else p
        self._check(self.lib.lc_correct(self._h, self._ptr(w, self.nvel, "w"), self._ptr(phi, self.ncell, "phi"),
                                        self._ptr(v, self.nvel, "v"), self._ptr(p, self.ncell, "p")))
        return v, p

    def psi_size(self, which):
        """Entries of the vector potential of plane projection `which` (1, 2, 3)."""
        nx, ny, nz = self.nx, self.ny, self.nz
        return {1: (nz + 1) * ny * (nx + 1), 2: (nz + 1) * (ny + 1) * nx, 3: nz * (ny + 1) * (nx + 1)}[which]

    def plane_project(self, v, which, out=None, psi=None, potential=True):
        """Divergence-free projection of v onto the planes of family `which` (1: (u, w)
        in y = const, 2: (v, w) in x = const, 3: (u, v) in z = const) and, if potential,
        its vector potential (Section 4, eqs. 11-17).  Returns (out, psi or None)."""
        if which not in (1, 2, 3):
            raise ValueError("which must be 1, 2 or 3")
        out = self.vel() if out is None else out
        if potential and psi is None:
            psi = _torch().zeros(self.psi_size(which), dtype=_torch().float64, device=self.device)
        pp = self._ptr(psi, self.psi_size(which), "psi") if potential else None
        self._check(self.lib.lc_plane_project(self._h, self._ptr(v, self.nvel, "v"), int(which),
                                              self._ptr(out, self.nvel, "out"), pp))
        return out, (psi if potential else None)

    # ------------------------------------------------------------ hot path
    def project(self, w, v=None, p=None, precision=FP64, tol=1e-8, max_iter=8):
        v = self.vel() if v is None else v
        p = self.cells() if p is None else p
        st = Stats()
        rc = self._check(self.lib.lc_project(self._h, self._ptr(w, self.nvel, "w"), self._ptr(v, self.nvel, "v"),
                                             self._ptr(p, self.ncell, "p"), int(precision), float(tol),
                                             int(max_iter), C.byref(st)), allow_notconv=True)
        return v, p, dict(st.as_dict(), converged=(rc == 0))

    def krylov_vector(self, v_in, v=None, p=None, precision=FP64, tol=1e-8, max_iter=8):
        v = self.vel() if v is None else v
        p = self.cells() if p is None else p
        st = Stats()
        rc = self._check(self.lib.lc_krylov_vector(self._h, self._ptr(v_in, self.nvel, "v_in"),
                                                   self._ptr(v, self.nvel, "v"), self._ptr(p, self.ncell, "p"),
                                                   int(precision), float(tol), int(max_iter), C.byref(st)),
                         allow_notconv=True)
        return v, p, dict(st.as_dict(), converged=(rc == 0))

    # ---------------------------------------- Stokes-preconditioned vectors
    def viscous_solve(self, f, dt, out=None):
        """u = (I/dt - Re^-1 Lap_0)^-1 f (dt = float('inf'): the pure Stokes operator)."""
        out = self.vel() if out is None else out
        self._check(self.lib.lc_viscous_solve(self._h, self._ptr(f, self.nvel, "f"), self._ptr(out, self.nvel, "u"),
                                              float(dt)))
        return out

    def stokes_step(self, f, dt, out=None, precision=FP64, tol=1e-12, max_iter=8):
        """u = P (I/dt - Re^-1 Lap_0)^-1 f: the viscous step, then the projection."""
        out = self.vel() if out is None else out
        st = Stats()
        rc = self._check(self.lib.lc_stokes_step(self._h, self._ptr(f, self.nvel, "f"), self._ptr(out, self.nvel, "u"),
                                                 float(dt), int(precision), float(tol), int(max_iter), C.byref(st)),
                         allow_notconv=True)
        return out, dict(st.as_dict(), converged=(rc == 0))

    def stokes_vector(self, v, dt, out=None, precision=FP64, tol=1e-12, max_iter=8):
        """The Stokes-preconditioned Krylov vector P (I/dt - Re^-1 Lap_0)^-1 P L_U v."""
        out = self.vel() if out is None else out
        st = Stats()
        rc = self._check(self.lib.lc_stokes_vector(self._h, self._ptr(v, self.nvel, "v"),
                                                   self._ptr(out, self.nvel, "out"), float(dt), int(precision),
                                                   float(tol), int(max_iter), C.byref(st)), allow_notconv=True)
        return out, dict(st.as_dict(), converged=(rc == 0))

    def set_stokes_precond(self, dt):
        """Right-precondition Newton's linear solves by the Stokes step of time step dt (0: off)."""
        self._check(self.lib.lc_set_stokes_precond(self._h, float(dt)))

    # ------------------------------------------------------ Krylov drivers
    def newton_residual(self, out=None):
        """(F = P R(U), max |F|) for the context's base flow."""
        out = self.vel() if out is None else out
        r = C.c_double()
        self._check(self.lib.lc_newton_residual(self._h, self._ptr(out, self.nvel, "F"), C.byref(r)))
        return out, r.value

    def newton_step(self, lin_tol=1e-10, gmres_m=100, max_vectors=5000, precision=FP64, proj_tol=1e-12):
        """One Newton step on the context's base flow (updated in place)."""
        ri, ci, nv, bi = C.c_double(), C.c_double(), C.c_long(), C.c_int()
        rc = self._check(self.lib.lc_newton_step(self._h, float(lin_tol), int(gmres_m), int(max_vectors),
                                                 int(precision), float(proj_tol), C.byref(ri), C.byref(ci),
                                                 C.byref(nv), C.byref(bi)), allow_notconv=True)
        return {"res_inf": ri.value, "corr_inf": ci.value, "n_vectors": nv.value, "bicgstab": bool(bi.value),
                "converged": rc == 0}

    def newton(self, tol=1e-10, max_steps=12, **kw):
        """Newton iterations from the current base flow until max |P R(U)| <= tol."""
        hist = []
        for _ in range(max_steps):
            _, r = self.newton_residual()
            hist.append(r)
            if r <= tol:
                break
            self.newton_step(**kw)
        return hist

    def arnoldi_leading(self, k=4, m=20, tol=1e-10, max_restarts=200, seed=1, precision=FP64, proj_tol=1e-12,
                        vectors=False, start=None):
        """Leading eigenvalues (largest real part) of eq. 7 by implicitly restarted Arnoldi,
        started from the velocity `start` (projected) or from a seeded random field."""
        torch = _torch()
        re = np.zeros(k + 1); im = np.zeros(k + 1); res = np.zeros(k + 1)
        vre = vim = None
        if vectors:
            vre = torch.zeros((k + 1, self.nvel), dtype=torch.float64, device=self.device)
            vim = torch.zeros((k + 1, self.nvel), dtype=torch.float64, device=self.device)
        nout, nvec = C.c_int(), C.c_long()
        p = lambda a: a.ctypes.data_as(C.c_void_p)
        rc = self._check(self.lib.lc_arnoldi_leading(
            self._h, int(k), int(m), float(tol), int(max_restarts), C.c_ulonglong(seed),
            None if start is None else self._ptr(start, self.nvel, "start"), int(precision),
            float(proj_tol), p(re), p(im), p(res), C.c_void_p(vre.data_ptr()) if vectors else None,
            C.c_void_p(vim.data_ptr()) if vectors else None, C.byref(nout), C.byref(nvec)), allow_notconv=True)
        n = nout.value
        out = {"eig": re[:n] + 1j * im[:n], "resid": res[:n], "n_vectors": nvec.value, "converged": rc == 0}
        if vectors:
            out["vectors"] = (vre[:n], vim[:n])
        return out

    def critical_re(self, re0, re1, re_tol=1e-8, max_evals=12, newton_tol=1e-10, newton_steps=12, lin_tol=1e-10,
                    gmres_m=100, max_vectors=5000, k=6, m=40, eig_tol=1e-10, max_restarts=400, seed=1,
                    warm_start=False):
        """Critical Reynolds number and frequency: secant on the real part of the leading
        eigenvalue from re0, re1 (the base flow should be a steady state at re0)."""
        o = CriticalOpts(float(re_tol), int(max_evals), float(newton_tol), int(newton_steps), float(lin_tol),
                         int(gmres_m), int(max_vectors), int(k), int(m), float(eig_tol), int(max_restarts), int(seed),
                         int(bool(warm_start)))
        rc_, om = C.c_double(), C.c_double()
        ne = C.c_int()
        hist = np.zeros(4 * max(int(max_evals), 2))
        rc = self._check(self.lib.lc_critical_re(self._h, float(re0), float(re1), C.byref(o), C.byref(rc_),
                                                 C.byref(om), hist.ctypes.data_as(C.c_void_p), C.byref(ne)),
                         allow_notconv=True)
        n = ne.value
        return {"re_cr": rc_.value, "omega_cr": om.value, "converged": rc == 0,
                "history": [tuple(hist[4 * i:4 * i + 4]) for i in range(n)]}

    # ----------------------------------------------------------- profiling
    # ------------------------------------------------------ learned guess
    def set_net(self, net):
        """Attach a Net for the LEARNED form (None detaches)."""
        self._check(self.lib.lc_set_net(self._h, net._h if net is not None else None))
        self.net = net

    def learned_guess(self, w, out=None):
        """(phi0, eps): the scaled network guess of the first correction of w."""
        out = self.cells() if out is None else out
        eps = C.c_double()
        self._check(self.lib.lc_learned_guess(self._h, self._ptr(w, self.nvel, "w"),
                                              self._ptr(out, self.ncell, "phi0"), C.byref(eps)))
        return out, eps.value

    def profile(self, on=True):
        self._check(self.lib.lc_profile_enable(self._h, 1 if on else 0))

    def profile_read(self):
        """{kernel class: (total ms, launches)} since profiling was enabled."""
        out = {}
        for k, name in enumerate(_lib.KERNEL_CLASSES):
            ms, n = C.c_double(), C.c_long()
            self._check(self.lib.lc_profile_read(self._h, k, C.byref(ms), C.byref(n)))
            if n.value:
                out[name] = (ms.value, n.value)
        return out

    def dot(self, a, b):
        out = C.c_double()
        self._check(self.lib.lc_dot(self._h, self._ptr(a, self.nvel, "a"), self._ptr(b, self.nvel, "b"),
                                    C.byref(out)))
        return out.value


class Net:
    """The learned pressure-correction guess (3-level 3D U-Net, BF16 matrix cores)."""

    def __init__(self, seed: int = 0):
        self.lib = _lib.load()
        h = C.c_void_p()
        rc = self.lib.lc_net_create(C.byref(h), seed)
        if rc != 0:
            raise LidKrylovError(rc, "lc_net_create failed")
        self._h = h
        self.nparams = int(self.lib.lc_net_param_count())

    def _check(self, rc):
        if rc != 0:
            raise LidKrylovError(rc, self.lib.lc_net_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self.lib.lc_net_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        out = np.zeros(self.nparams, dtype=np.float32)
        self._check(self.lib.lc_net_get_params(self._h, out.ctypes.data_as(C.c_void_p)))
        return out

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != self.nparams:
            raise ValueError(f"need {self.nparams} parameters")
        self._check(self.lib.lc_net_set_params(self._h, p.ctypes.data_as(C.c_void_p)))

    def save(self, path):
        """Write the master parameters to `path` (lc_net_save's file format)."""
        self._check(self.lib.lc_net_save(self._h, os.fsencode(path)))

    def load(self, path):
        """Read the master parameters from `path`; resets the Adam state."""
        self._check(self.lib.lc_net_load(self._h, os.fsencode(path)))

    @staticmethod
    def _f32(t, shape, name):
        torch = _torch()
        if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name}: need a contiguous float32 CUDA tensor of shape {tuple(shape)}")
        return C.c_void_p(t.data_ptr())

    def forward(self, x, stream=None):
        """x: [D][H][W][4] float32 CUDA tensor -> y [D][H][W]."""
        torch = _torch()
        D, H, W, _ = x.shape
        y = torch.empty((D, H, W), dtype=torch.float32, device=x.device)
        s = stream if stream is not None else torch.cuda.current_stream()
        self._check(self.lib.lc_net_forward(self._h, C.c_void_p(s.cuda_stream), self._f32(x, (D, H, W, 4), "x"),
                                            C.c_void_p(y.data_ptr()), D, H, W))
        return y

    def step(self, x, t, lr=0.0, grads=False, stream=None):
        """MSE loss of forward(x) against t, optional gradients (host) and Adam step."""
        torch = _torch()
        D, H, W, _ = x.shape
        s = stream if stream is not None else torch.cuda.current_stream()
        g = np.zeros(self.nparams, dtype=np.float32) if grads else None
        loss = C.c_double()
        self._check(self.lib.lc_net_step(self._h, C.c_void_p(s.cuda_stream), self._f32(x, (D, H, W, 4), "x"),
                                         self._f32(t, (D, H, W), "t"), D, H, W, lr, C.byref(loss),
                                         g.ctypes.data_as(C.c_void_p) if grads else None))
        return (loss.value, g) if grads else loss.value

    def train(self, ctx: "Context", steps: int, lr: float = 1e-3, seed: int = 1):
        """Adam steps on pairs the method generates on ctx's grid; returns the losses."""
        hist = np.zeros(max(steps, 1), dtype=np.float64)
        ctx._check(self.lib.lc_net_train(ctx._h, self._h, steps, lr, seed, hist.ctypes.data_as(C.c_void_p)))
        return hist[:steps]

