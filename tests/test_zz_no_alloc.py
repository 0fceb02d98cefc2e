"""The allocation-free dot product (lc_dot_noalloc) against lc_dot through the C ABI.

Both run the same block partial sums and the same fixed-order final sum, so the results
must be bit-identical; two calls in a row on one device, the second on a smaller input,
check that the shared device scratch keeps no state between calls.
"""
import ctypes as C

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _dot_noalloc(lib, a, b, n, stream):
    out = C.c_double()
    rc = lib.lc_dot_noalloc(C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()), C.c_size_t(n), C.byref(out),
                            C.c_void_p(stream.cuda_stream))
    return rc, out.value


def test_dot_noalloc_matches_dot_two_calls():
    import torch
    import paper_1704_08521_amd as lk
    for dims, seeds in (((40, 36, 33), (1, 2)), ((9, 7, 5), (3, 4))):
        print(f"[case] dims {dims}", flush=True)
        ctx = lk.Context(*dims)
        a_h = synth.random_velocity(*dims, seeds[0])
        b_h = synth.random_velocity(*dims, seeds[1])
        a = torch.from_numpy(a_h).cuda()
        b = torch.from_numpy(b_h).cuda()
        ref = ctx.dot(a, b)
        rc, got = _dot_noalloc(ctx.lib, a, b, ctx.nvel, torch.cuda.current_stream())
        assert rc == 0
        print(f"  lc_dot {ref!r} lc_dot_noalloc {got!r}")
        assert got == ref
        assert abs(got - float(np.dot(a_h, b_h))) <= 1e-12 * float(np.dot(np.abs(a_h), np.abs(b_h)))


def test_dot_noalloc_rejects_bad_sizes():
    import torch
    import paper_1704_08521_amd as lk
    from paper_1704_08521_amd import _lib
    lib = _lib.load()
    a = torch.zeros(8, dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream()
    assert _dot_noalloc(lib, a, a, 0, s)[0] == lk._lib.LC_EINVAL
    out = C.c_double()
    rc = lib.lc_dot_noalloc(C.c_void_p(a.data_ptr()), C.c_void_p(a.data_ptr()),
                            C.c_size_t(_lib.NOALLOC_MAX_N + 1), C.byref(out), C.c_void_p(s.cuda_stream))
    assert rc == lk._lib.LC_EINVAL
