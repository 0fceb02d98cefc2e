"""Failure handling and reproducibility through the C ABI (conditions forced from the host:
every kernel still runs normally or is never launched).

* A device pointer that is not 8-byte aligned is refused on the host (LC_EINVAL), before
  any launch.
* The learned form without an attached network is a state error (LC_ESTATE).
* Reductions are fixed-order two-stage sums, so repeated calls are bitwise identical: a
  Krylov vector, the Newton residual and a whole Arnoldi run (same seed) are compared bit
  for bit (an LDS race or an order-dependent atomic would show here).
"""
import ctypes as C

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    import paper_1704_08521_amd as lk
    n = (20, 18, 16)
    c = lk.Context(*n)
    c.set_stretching("tanh", 10.0)
    c.set_re(800.0)
    c.set_lid(0.3)
    U = torch.from_numpy(synth.random_velocity(*n, 31)).cuda()
    U, _, _ = c.project(U, tol=1e-12, max_iter=4)
    c.set_base_flow(U / U.abs().max())
    v = torch.from_numpy(synth.random_velocity(*n, 32)).cuda()
    v, _, _ = c.project(v, tol=1e-12, max_iter=4)
    return lk, c, v


def test_misaligned_pointer_refused(setup):
    import torch
    lk, c, v = setup
    buf = torch.zeros(c.nvel + 1, dtype=torch.float64, device="cuda")
    out = c.vel()
    st = lk.Stats()
    rc = c.lib.lc_krylov_vector(c._h, C.c_void_p(buf.data_ptr() + 4), C.c_void_p(out.data_ptr()), None,
                                lk.FP64, C.c_double(1e-10), 4, C.byref(st))
    assert rc == lk._lib.LC_EINVAL
    assert "pointer" in c.lib.lc_last_error(c._h).decode()
    assert torch.count_nonzero(out) == 0  # nothing was written


def test_learned_without_network_is_state_error(setup):
    lk, c, v = setup
    with pytest.raises(lk.LidKrylovError) as e:
        c.krylov_vector(v, precision=lk.LEARNED, tol=1e-10)
    assert e.value.code == lk._lib.LC_ESTATE


def test_repeated_calls_are_bitwise_identical(setup):
    lk, c, v = setup
    a, _, _ = c.krylov_vector(v, tol=1e-12)
    b, _, _ = c.krylov_vector(v, tol=1e-12)
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
    F1, r1 = c.newton_residual()
    F2, r2 = c.newton_residual()
    assert r1 == r2 and np.array_equal(F1.cpu().numpy(), F2.cpu().numpy())
    e1 = c.arnoldi_leading(k=2, m=20, tol=1e-8, max_restarts=30, seed=7)
    e2 = c.arnoldi_leading(k=2, m=20, tol=1e-8, max_restarts=30, seed=7)
    assert np.array_equal(np.asarray(e1["eig"]), np.asarray(e2["eig"]))
    assert e1["n_vectors"] == e2["n_vectors"]
