"""Per-phase device times in lc_stats: filled from the profiling events when profiling is
on (stencil, pressure solve, correction, network), -1 when it is off."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def test_phase_times():
    import torch
    import paper_1704_08521_amd as lk
    n = 24
    c = lk.Context(n)
    c.set_stretching("tanh", 10.0)
    c.set_re(500.0)
    U = torch.from_numpy(synth.random_velocity(n, n, n, 4)).cuda()
    U, _, _ = c.project(U, tol=1e-12, max_iter=4)
    c.set_base_flow(U)
    v = torch.from_numpy(synth.random_velocity(n, n, n, 5)).cuda()
    v, _, _ = c.project(v, tol=1e-12, max_iter=4)
    _, _, st = c.krylov_vector(v, tol=1e-10)
    assert st["ms_stencil"] == st["ms_poisson"] == st["ms_update"] == st["ms_network"] == -1.0
    c.profile(True)
    _, _, st = c.krylov_vector(v, tol=1e-10)
    prof = c.profile_read()
    c.profile(False)
    print(st)
    for key in ("ms_stencil", "ms_poisson", "ms_update"):
        assert st[key] > 0.0, key
    assert st["ms_network"] == 0.0
    assert st["ms_stencil"] + st["ms_poisson"] + st["ms_update"] <= st["ms_total"]
    # the call's phases are the profile's classes of this one call
    stencil = sum(prof[k][0] for k in ("momentum", "divergence") if k in prof)
    assert np.isclose(st["ms_stencil"], stencil, rtol=1e-6)
    assert np.isclose(st["ms_update"], prof["correct"][0], rtol=1e-6)
