"""Contexts inside a caller-owned workspace (lc_workspace_query / lc_create_in).

The library carves every device buffer from the caller's block; results must be
bit-identical to those of a context that allocates its own memory (same kernels, same
reduction order), and a block one byte smaller than the query fails with LC_ENOMEM when
the Krylov vectors are needed.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

DIMS = (16, 14, 12)
M = 20


def setup(ctx, U):
    ctx.set_stretching("tanh", 10.0)
    ctx.set_re(300.0)
    ctx.set_lid(0.3)
    ctx.set_base_flow(U)


def test_workspace_results_identical_and_one_byte_short():
    import torch
    import paper_1704_08521_amd as lk
    nbytes = lk.Context.workspace_bytes(*DIMS, m_max=M)
    print(f"[case] workspace {DIMS} m_max={M}: {nbytes} bytes", flush=True)
    U = torch.from_numpy(synth.random_velocity(*DIMS, 91)).cuda()
    U *= 0.5
    v = torch.from_numpy(synth.random_velocity(*DIMS, 92)).cuda()
    own = lk.Context(*DIMS)
    setup(own, U)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    ctx = lk.Context(*DIMS, workspace=ws)
    setup(ctx, U)
    for prec in (lk.FP64, lk.MIXED):
        a, pa, _ = own.krylov_vector(v, precision=prec, tol=1e-10)
        b, pb, _ = ctx.krylov_vector(v, precision=prec, tol=1e-10)
        assert torch.equal(a, b) and torch.equal(pa, pb)
    ra = own.arnoldi_leading(k=3, m=M, tol=1e-8, max_restarts=50, seed=2)
    rb = ctx.arnoldi_leading(k=3, m=M, tol=1e-8, max_restarts=50, seed=2)
    assert np.array_equal(ra["eig"], rb["eig"]) and ra["n_vectors"] == rb["n_vectors"]
    sa = own.newton_step(lin_tol=1e-8, gmres_m=M, max_vectors=400)
    sb = ctx.newton_step(lin_tol=1e-8, gmres_m=M, max_vectors=400)
    assert sa == sb and torch.equal(own.get_base_flow(), ctx.get_base_flow())
    fa, _ = own.stokes_step(v, 0.5)
    fb, _ = ctx.stokes_step(v, 0.5)
    assert torch.equal(fa, fb)
    ctx.close()
    del ws
    # one byte short: creation succeeds (the fixed buffers fit), the Krylov vectors do not
    short = torch.empty(nbytes - 1, dtype=torch.uint8, device="cuda")
    ctx2 = lk.Context(*DIMS, workspace=short)
    setup(ctx2, U)
    ctx2.krylov_vector(v, tol=1e-10)
    with pytest.raises(lk.LidKrylovError) as e:
        ctx2.arnoldi_leading(k=3, m=M, tol=1e-8, max_restarts=5, seed=2)
    assert e.value.code == lk._lib.LC_ENOMEM
    print("one byte short:", e.value)
    ctx2.close()


def test_workspace_too_small_for_fixed_buffers():
    import torch
    import paper_1704_08521_amd as lk
    tiny = torch.empty(4096, dtype=torch.uint8, device="cuda")
    with pytest.raises(lk.LidKrylovError) as e:
        lk.Context(*DIMS, workspace=tiny)
    assert e.value.code == lk._lib.LC_ENOMEM
