"""Pins of the FP64 network oracle (learned pressure-correction guess).

Each layer is checked against something other than itself: the convolution against
scipy.ndimage.correlate and a brute-force loop, backward passes against adjoint
identities and central finite differences, pooling/upsampling against closed forms,
Adam's first step against its closed form.
"""
import numpy as np
import pytest
from scipy import ndimage

from oracle import nn


def rnd(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def test_conv_matches_scipy_correlate():
    x = rnd((5, 6, 7, 3), 1)
    w = rnd((2, 27, 3), 2)
    b = rnd(2, 3)
    y = nn.conv(x, w, b)
    for co in range(2):
        ref = np.full(x.shape[:3], b[co])
        for ci in range(3):
            k = w[co, :, ci].reshape(3, 3, 3)  # tap = (dz+1)*9 + (dy+1)*3 + (dx+1)
            ref += ndimage.correlate(x[..., ci], k, mode="constant", cval=0.0)
        assert np.allclose(y[..., co], ref, rtol=0, atol=1e-12)


def test_conv_brute_force_tiny():
    x = rnd((3, 2, 4, 2), 4)
    w = rnd((3, 27, 2), 5)
    b = rnd(3, 6)
    y = nn.conv(x, w, b)
    D, H, W, C = x.shape
    for z in range(D):
        for yy in range(H):
            for xx in range(W):
                for co in range(3):
                    s = b[co]
                    for dz in (-1, 0, 1):
                        for dy in (-1, 0, 1):
                            for dx in (-1, 0, 1):
                                zz, y2, x2 = z + dz, yy + dy, xx + dx
                                if 0 <= zz < D and 0 <= y2 < H and 0 <= x2 < W:
                                    t = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)
                                    s += sum(w[co, t, ci] * x[zz, y2, x2, ci] for ci in range(C))
                    assert abs(y[z, yy, xx, co] - s) < 1e-12


def test_conv_delta_kernels_shift():
    x = rnd((4, 5, 6, 1), 7)
    for t, (dz, dy, dx) in enumerate(nn.TAPS):
        w = np.zeros((1, 27, 1))
        w[0, t, 0] = 1.0
        y = nn.conv(x, w, np.zeros(1))[..., 0]
        z0, y0, x0 = 1, 2, 3
        assert y[z0, y0, x0] == x[z0 + dz, y0 + dy, x0 + dx, 0]
    # a pointwise (1x1x1) conv is a channel matmul
    w1 = rnd((4, 1, 1), 8)
    assert np.allclose(nn.conv(x, w1, np.zeros(4)), x @ w1[:, 0, :].T)


def test_conv_backward_adjoint_and_linear():
    x = rnd((4, 5, 6, 3), 9)
    w = rnd((2, 27, 3), 10)
    dy = rnd((4, 5, 6, 2), 11)
    dx, dw, db = nn.conv_backward(x, w, dy)
    z = np.zeros(2)
    # <conv(x), dy> = <x, dx>: the data gradient is the adjoint of the convolution
    assert np.isclose(np.sum(nn.conv(x, w, z) * dy), np.sum(x * dx), rtol=1e-12)
    # conv is linear in w: <dw, E> = <conv(x, E), dy>
    E = rnd(w.shape, 12)
    assert np.isclose(np.sum(dw * E), np.sum(nn.conv(x, E, z) * dy), rtol=1e-12)
    assert np.allclose(db, dy.sum(axis=(0, 1, 2)))


def test_pool_up_closed_forms():
    a = rnd((2, 3, 2, 5), 13)
    assert np.allclose(nn.pool(nn.up(a)), a)
    c = np.full((4, 6, 8, 2), 3.5)
    assert np.allclose(nn.pool(c), 3.5)
    big = rnd((4, 6, 4, 5), 14)
    # adjoint pairs
    assert np.isclose(np.sum(nn.up(a) * big), np.sum(a * nn.up_backward(big)))
    assert np.isclose(np.sum(nn.pool(big) * a), np.sum(big * nn.pool_backward(a)))
    # explicit 2x2x2 mean of one block
    assert np.isclose(nn.pool(big)[1, 2, 0, 3], big[2:4, 4:6, 0:2, 3].mean())


def test_network_shapes_and_params():
    p = nn.init_params(0)
    assert p["enc1.w"].shape == (16, 27, 4) and p["dec2.w"].shape == (32, 27, 96)
    assert p["head.w"].shape == (1, 1, 16)
    assert sum(v.size for v in p.values()) == nn.param_count()
    y, _ = nn.forward(p, rnd((8, 4, 12, 4), 15))
    assert y.shape == (8, 4, 12, 1)


def _fd_check(p, x, t, key, idx, h=1e-6):
    q = {k: v.copy() for k, v in p.items()}
    q[key][idx] += h
    lp, _ = nn.loss_and_grad(q, x, t)
    q[key][idx] -= 2 * h
    lm, _ = nn.loss_and_grad(q, x, t)
    return (lp - lm) / (2 * h)


@pytest.mark.parametrize("key", ["enc1.w", "enc1.b", "enc2.w", "bott.w", "bott.b", "dec2.w",
                                 "dec1.w", "dec1.b", "head.w", "head.b"])
def test_loss_gradient_central_differences(key):
    p = nn.init_params(3)
    for k in p:
        if k.endswith(".b"):
            p[k] = 0.1 * rnd(p[k].shape, hash(k) % 1000)
    x = rnd((8, 8, 8, 4), 16)
    t = rnd((8, 8, 8, 1), 17)
    _, g = nn.loss_and_grad(p, x, t)
    rng = np.random.default_rng(18)
    for _ in range(4):
        idx = tuple(rng.integers(0, s) for s in p[key].shape)
        fd = _fd_check(p, x, t, key, idx)
        assert abs(fd - g[key][idx]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (key, idx, fd, g[key][idx])


def test_input_gradient_central_differences():
    p = nn.init_params(4)
    x = rnd((8, 8, 4, 4), 19)
    t = rnd((8, 8, 4, 1), 20)
    _, g = nn.loss_and_grad(p, x, t)
    h = 1e-6
    for idx in [(0, 0, 0, 0), (3, 5, 2, 3), (7, 7, 3, 1)]:
        xp = x.copy(); xp[idx] += h
        xm = x.copy(); xm[idx] -= h
        fd = (nn.loss_and_grad(p, xp, t)[0] - nn.loss_and_grad(p, xm, t)[0]) / (2 * h)
        assert abs(fd - g["x"][idx]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8


def test_head_bias_gradient_closed_form():
    p = nn.init_params(5)
    x = rnd((4, 4, 4, 4), 21)
    t = rnd((4, 4, 4, 1), 22)
    y, _ = nn.forward(p, x)
    _, g = nn.loss_and_grad(p, x, t)
    assert np.isclose(g["head.b"][0], 2.0 * np.mean(y - t), rtol=1e-12)


def test_adam_first_step_closed_form():
    p = {"a": np.array([1.0, -2.0, 0.5])}
    g = {"a": np.array([0.3, -4.0, 1e-9])}
    m = {"a": np.zeros(3)}
    v = {"a": np.zeros(3)}
    nn.adam(p, g, m, v, 1, lr=0.01)
    # bias-corrected moments are g and g^2 on the first step
    expect = np.array([1.0, -2.0, 0.5]) - 0.01 * g["a"] / (np.abs(g["a"]) + 1e-8)
    assert np.allclose(p["a"], expect, rtol=1e-14)


def test_features_brute_force_tiny():
    from oracle.grid import Grid
    import synth
    g = Grid.make(5, 4, 3, kind="tanh", ratio=4.0)
    w = synth.random_velocity(5, 4, 3, 31)
    x, r = nn.features(g, w)
    assert x.shape == (4, 4, 8, 4)
    u, v, ww = g.unpack(w)
    V = g.volumes()
    cen = np.zeros((3, 4, 5, 3))
    div = np.zeros((3, 4, 5))
    for k in range(3):
        for j in range(4):
            for i in range(5):
                cen[k, j, i] = [(u[k, j, i] + u[k, j, i + 1]) / 2, (v[k, j, i] + v[k, j + 1, i]) / 2,
                                (ww[k, j, i] + ww[k + 1, j, i]) / 2]
                div[k, j, i] = ((u[k, j, i + 1] - u[k, j, i]) / (g.X.xf[i + 1] - g.X.xf[i])
                                + (v[k, j + 1, i] - v[k, j, i]) / (g.Y.xf[j + 1] - g.Y.xf[j])
                                + (ww[k + 1, j, i] - ww[k, j, i]) / (g.Z.xf[k + 1] - g.Z.xf[k]))
    sw = np.sqrt(np.sum(V[..., None] * cen ** 2) / (3 * V.sum()))
    sr = np.sqrt(np.sum(V * div ** 2) / V.sum())
    assert np.allclose(x[:3, :4, :5, :3], cen / sw, atol=1e-13)
    assert np.allclose(x[:3, :4, :5, 3], div / sr, atol=1e-12)
    assert np.all(x[3:] == 0) and np.all(x[:, :, 5:] == 0)
    assert np.allclose(r, div, atol=1e-12)


def test_guess_fit_recovers_exact_solution(monkeypatch):
    """If the network returned any multiple of the exact correction, the fitted
    guess is that correction and the continuity residual vanishes; for any other
    output the fit is orthogonal and eps <= 1."""
    from oracle.grid import Grid
    from oracle.poisson import PoissonFD
    import synth
    g = Grid.make(6, 5, 4, kind="sine")
    w = synth.random_velocity(6, 5, 4, 32)
    _, r = nn.features(g, w)
    phi = PoissonFD(g).solve(r)
    scale = -2.5

    def fake(p, x, q=None):
        y = np.zeros(x.shape[:3] + (1,))
        y[:4, :5, :6, 0] = scale * phi
        return y, None
    monkeypatch.setattr(nn, "forward", fake)
    phi0, eps = nn.guess(g, None, w)
    assert eps < 1e-10
    assert np.allclose(phi0, phi, atol=1e-10 * np.abs(phi).max())
    monkeypatch.undo()
    p = nn.init_params(1)
    phi0, eps = nn.guess(g, p, w)
    assert 0.0 < eps <= 1.0


def test_bf16_rounding_closed_forms():
    # representable values stay, halfway cases go to even, one ulp of 1 is 2^-7
    vals = np.array([1.0, -2.5, 1.0 + 2 ** -7, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 3.0e38, 1e-40])
    r = nn.bf16(vals)
    assert r[0] == 1.0 and r[1] == -2.5 and r[2] == 1.0 + 2 ** -7
    assert r[3] == 1.0 and r[4] == 1.0 + 2 ** -6
    assert abs(r[5] - 3.0e38) / 3.0e38 < 2 ** -8
    x = rnd(1000, 23)
    assert np.max(np.abs(nn.bf16(x) - x) / np.abs(x)) <= 2 ** -8


def test_rounded_network_close_to_exact():
    """The rounding hook only perturbs: with BF16 storage the loss gradient stays
    within a few percent of the exact one, with the identity it is the same."""
    p = nn.init_params(6)
    x = rnd((8, 8, 8, 4), 24)
    t = rnd((8, 8, 8, 1), 25)
    l0, g0 = nn.loss_and_grad(p, x, t)
    l1, g1 = nn.loss_and_grad(p, x, t, q=lambda a: a)
    assert l0 == l1 and all(np.array_equal(g0[k], g1[k]) for k in g0)
    l2, g2 = nn.loss_and_grad(p, x, t, q=nn.bf16)
    assert abs(l2 - l0) < 1e-2 * l0
    for k in ("head.w", "dec1.w", "enc1.w"):
        assert np.linalg.norm(g2[k] - g0[k]) < 0.1 * np.linalg.norm(g0[k])
