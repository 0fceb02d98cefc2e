"""CPU checks of the C-ABI library: it loads, exports every declared entry point,
and its host-side tensor-product set-up matches the oracle's axis modes."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle.grid import Axis, faces
from oracle.poisson import axis_modes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lidkrylov.h")


def _lib():
    from paper_1704_08521_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("liblidkrylov.so is not built (run __graft_entry__.build())")
    return L.load()


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lc_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("lc_create", "lc_set_grid", "lc_set_stretching", "lc_set_re", "lc_set_lid",
                 "lc_krylov_vector", "lc_project", "lc_jacobian_apply", "lc_residual",
                 "lc_poisson_solve", "lc_correct", "lc_divergence"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = _lib()
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    from paper_1704_08521_amd import _lib as L
    assert set(L.exported_symbols()) >= set(declared())


@pytest.mark.parametrize("n,kind", [(2, "uniform"), (7, "tanh"), (64, "sine"), (200, "tanh")])
def test_axis_modes_match_oracle(n, kind):
    lib = _lib()
    xf = faces(n, kind)
    lam = np.zeros(n); S = np.zeros((n, n)); Wf = np.zeros((n, n))
    p = lambda a: a.ctypes.data_as(C.c_void_p)
    assert lib.lc_axis_modes(n, p(xf), p(lam), p(S), p(Wf)) == 0
    lo, So, M = axis_modes(Axis(xf))
    assert np.allclose(lam, lo, rtol=1e-12, atol=1e-10 * np.abs(lo).max())
    assert abs(lam[-1]) < 1e-9 * np.abs(lo).max()          # Neumann null mode last
    # S^T M S = I and Wf = S^T M, eigen-equation K S = M S diag(lam)
    assert np.allclose(S.T @ M @ S, np.eye(n), atol=1e-11)
    assert np.allclose(Wf, S.T @ M, atol=1e-12)
    ax = Axis(xf)
    K = np.zeros((n, n))
    for f in range(1, n):
        c = 1 / ax.dd[f]
        K[f - 1, f - 1] -= c; K[f, f] -= c; K[f - 1, f] += c; K[f, f - 1] += c
    assert np.max(np.abs(K @ S - M @ S * lam)) < 1e-10 * np.abs(lo).max()


def test_axis_modes_rejects_bad_faces():
    lib = _lib()
    xf = np.array([0.0, 0.5, 0.4, 1.0])
    out = np.zeros(9)
    p = lambda a: a.ctypes.data_as(C.c_void_p)
    assert lib.lc_axis_modes(3, p(xf), p(out), p(out), p(out)) == -1


@pytest.mark.parametrize("m,seed", [(1, 0), (5, 1), (20, 2), (60, 3)])
def test_hessenberg_eigvals_match_numpy(m, seed):
    lib = _lib()
    rng = np.random.default_rng(seed)
    H = np.triu(rng.standard_normal((m, m)), -1)
    re = np.zeros(m); im = np.zeros(m)
    p = lambda a: a.ctypes.data_as(C.c_void_p)
    assert lib.lc_hessenberg_eigvals(m, p(np.ascontiguousarray(H)), p(re), p(im)) == 0
    from oracle.eigen import match_distance
    assert match_distance(np.linalg.eigvals(H), re + 1j * im) < 1e-10 * max(1.0, np.abs(H).max())


def test_grid_size_limits_rejected_on_the_host():
    """Sizes the kernels cannot address (a velocity component of 2^31 bytes or more, an axis
    outside [2, 4096]) are refused before any device call."""
    from paper_1704_08521_amd import _lib as L
    lib = _lib()
    nbytes = C.c_size_t(0)
    assert lib.lc_workspace_query(200, 200, 200, 40, C.byref(nbytes)) == L.LC_OK and nbytes.value > 0
    for n in ((1, 8, 8), (8, 8, 4097), (650, 650, 650), (4096, 4096, 16)):
        assert lib.lc_workspace_query(*n, 40, C.byref(nbytes)) == L.LC_EINVAL, n
        ctx = C.c_void_p()
        assert lib.lc_create(C.byref(ctx), *n, None) == L.LC_EINVAL, n
        assert not ctx.value
