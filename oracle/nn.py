"""FP64 reference of the learned pressure-correction guess (test infrastructure).

Not from the paper: a small 3-level 3D U-Net maps the (cell-centred) momentum update
w and its divergence D w to an initial guess of the pressure correction phi of the
SIMPLE loop (Section 3, step 1).  Tensors are channels-last, [D][H][W][C] (z, y, x,
channel).  Layers:

    e1 = relu(conv3(x,  4 -> 16))                 full resolution
    e2 = relu(conv3(pool(e1), 16 -> 32))          1/2
    b  = relu(conv3(pool(e2), 32 -> 64))          1/4
    d2 = relu(conv3(cat(up(b),  e2), 96 -> 32))   1/2
    d1 = relu(conv3(cat(up(d2), e1), 48 -> 16))   full
    y  = conv1(d1, 16 -> 1)

conv3: 3x3x3 cross-correlation with zero padding, weights W[co][tap][ci], tap =
(dz+1)*9 + (dy+1)*3 + (dx+1), plus a bias per output channel.  pool: 2x2x2 average;
up: nearest-neighbour 2x; cat: channel concatenation.  Loss: mean squared error.
Forward and backward are written out directly (loops over the 27 taps), in float64.
"""
from __future__ import annotations

import numpy as np

from . import fv
from .grid import Grid

LAYERS = [("enc1", 4, 16, 3), ("enc2", 16, 32, 3), ("bott", 32, 64, 3),
          ("dec2", 96, 32, 3), ("dec1", 48, 16, 3), ("head", 16, 1, 1)]
TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def param_count():
    return sum(co * (27 if k == 3 else 1) * ci + co for _, ci, co, k in LAYERS)


def init_params(seed=0):
    rng = np.random.default_rng(seed)
    p = {}
    for name, ci, co, k in LAYERS:
        taps = 27 if k == 3 else 1
        std = np.sqrt(2.0 / (taps * ci))
        p[name + ".w"] = rng.standard_normal((co, taps, ci)) * std
        p[name + ".b"] = np.zeros(co)
    return p


def _shift(x, dz, dy, dx):
    """x[z+dz, y+dy, x+dx] with zeros outside (x is [D][H][W][C])."""
    out = np.zeros_like(x)
    D, H, W = x.shape[:3]
    zs = slice(max(0, -dz), D - max(0, dz)); zd = slice(max(0, dz), D - max(0, -dz))
    ys = slice(max(0, -dy), H - max(0, dy)); yd = slice(max(0, dy), H - max(0, -dy))
    xs = slice(max(0, -dx), W - max(0, dx)); xd = slice(max(0, dx), W - max(0, -dx))
    out[zs, ys, xs] = x[zd, yd, xd]
    return out


def conv(x, w, b):
    """y[p][co] = b[co] + sum_tap sum_ci w[co][tap][ci] x[p + off(tap)][ci]."""
    co, taps, ci = w.shape
    y = np.zeros(x.shape[:3] + (co,)) + b
    offs = TAPS if taps == 27 else [(0, 0, 0)]
    for t, (dz, dy, dx) in enumerate(offs):
        y += _shift(x, dz, dy, dx) @ w[:, t, :].T
    return y


def conv_backward(x, w, dy):
    """(dx, dw, db) of conv for upstream gradient dy."""
    co, taps, ci = w.shape
    offs = TAPS if taps == 27 else [(0, 0, 0)]
    dx = np.zeros_like(x)
    dw = np.zeros_like(w)
    for t, (dz, dyy, dxx) in enumerate(offs):
        xs = _shift(x, dz, dyy, dxx)
        dw[:, t, :] = np.einsum("zyxo,zyxi->oi", dy, xs)
        dx += _shift(dy @ w[:, t, :], -dz, -dyy, -dxx)
    return dx, dw, dy.sum(axis=(0, 1, 2))


def pool(x):
    D, H, W, C = x.shape
    return x.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).mean(axis=(1, 3, 5))


def pool_backward(dy):
    return np.repeat(np.repeat(np.repeat(dy, 2, 0), 2, 1), 2, 2) / 8.0


def up(x):
    return np.repeat(np.repeat(np.repeat(x, 2, 0), 2, 1), 2, 2)


def up_backward(dy):
    D, H, W, C = dy.shape
    return dy.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).sum(axis=(1, 3, 5))


def relu(x):
    return np.maximum(x, 0.0)


def _ident(a):
    return a


def forward(p, x, q=None):
    """Network output y ([D][H][W][1]) and the cache for backward.  q (default:
    identity) is applied to every stored activation: passing a rounding to a
    narrower format reproduces a network that keeps its activations in it."""
    q = q or _ident
    c = {"x": x}
    c["e1"] = q(relu(conv(x, p["enc1.w"], p["enc1.b"])))
    c["p1"] = q(pool(c["e1"]))
    c["e2"] = q(relu(conv(c["p1"], p["enc2.w"], p["enc2.b"])))
    c["p2"] = q(pool(c["e2"]))
    c["bt"] = q(relu(conv(c["p2"], p["bott.w"], p["bott.b"])))
    c["c2"] = np.concatenate([up(c["bt"]), c["e2"]], axis=3)
    c["d2"] = q(relu(conv(c["c2"], p["dec2.w"], p["dec2.b"])))
    c["c1"] = np.concatenate([up(c["d2"]), c["e1"]], axis=3)
    c["d1"] = q(relu(conv(c["c1"], p["dec1.w"], p["dec1.b"])))
    y = conv(c["d1"], p["head.w"], p["head.b"])
    return y, c


def loss_and_grad(p, x, target, q=None):
    """Mean squared error and its gradient with respect to every parameter and x.
    q as in forward, applied also to the gradients that enter a convolution's
    backward pass (the masked output gradients)."""
    q = q or _ident
    y, c = forward(p, x, q)
    n = y.size
    loss = float(np.sum((y - target) ** 2) / n)
    dy = 2.0 * (y - target) / n
    g = {}
    dd1, g["head.w"], g["head.b"] = conv_backward(c["d1"], p["head.w"], dy)
    dd1 = q(dd1 * (c["d1"] > 0))
    dc1, g["dec1.w"], g["dec1.b"] = conv_backward(c["c1"], p["dec1.w"], dd1)
    dd2 = q(up_backward(dc1[..., :32]) * (c["d2"] > 0))
    de1 = dc1[..., 32:]
    dc2, g["dec2.w"], g["dec2.b"] = conv_backward(c["c2"], p["dec2.w"], dd2)
    dbt = q(up_backward(dc2[..., :64]) * (c["bt"] > 0))
    de2 = dc2[..., 64:]
    dp2, g["bott.w"], g["bott.b"] = conv_backward(c["p2"], p["bott.w"], dbt)
    de2 = q((de2 + pool_backward(dp2)) * (c["e2"] > 0))
    dp1, g["enc2.w"], g["enc2.b"] = conv_backward(c["p1"], p["enc2.w"], de2)
    de1 = q((de1 + pool_backward(dp1)) * (c["e1"] > 0))
    dx, g["enc1.w"], g["enc1.b"] = conv_backward(c["x"], p["enc1.w"], de1)
    g["x"] = dx
    return loss, g


def bf16(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64).reshape(np.shape(a))


def adam(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba) in place; t counts from 1."""
    for k in p:
        m[k] = b1 * m[k] + (1 - b1) * g[k]
        v[k] = b2 * v[k] + (1 - b2) * g[k] ** 2
        mh = m[k] / (1 - b1 ** t)
        vh = v[k] / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)


# ------------------------------------------------------------ use inside SIMPLE
def pad4(n):
    """Network domain size along an axis: two 2x poolings need a multiple of 4."""
    return (n + 3) // 4 * 4


def _vdot(g: Grid, a, b):
    return float(np.sum(g.volumes() * a * b))


def features(g: Grid, w):
    """Network input for a momentum update w (packed velocity): channels
    (w_x, w_y, w_z) averaged to cell centres and scaled by their common V-weighted
    RMS, and D w scaled by its V-weighted RMS, on the zero-padded domain
    [pad4(nz)][pad4(ny)][pad4(nx)][4].  Returns (x, D w)."""
    u, v, ww = g.unpack(w)
    c = [0.5 * (u[:, :, 1:] + u[:, :, :-1]), 0.5 * (v[:, 1:, :] + v[:, :-1, :]), 0.5 * (ww[1:] + ww[:-1])]
    r = fv.divergence(g, w)
    vol = float(np.sum(g.volumes()))
    sw = np.sqrt(sum(_vdot(g, a, a) for a in c) / (3.0 * vol))
    sr = np.sqrt(_vdot(g, r, r) / vol)
    nz, ny, nx = r.shape
    x = np.zeros((pad4(nz), pad4(ny), pad4(nx), 4))
    for ch in range(3):
        x[:nz, :ny, :nx, ch] = c[ch] / sw if sw > 0 else 0.0
    x[:nz, :ny, :nx, 3] = r / sr if sr > 0 else 0.0
    return x, r


def targets(g: Grid, phi):
    """Training target: the correction phi scaled by its V-weighted RMS, padded."""
    vol = float(np.sum(g.volumes()))
    s = np.sqrt(_vdot(g, phi, phi) / vol)
    nz, ny, nx = phi.shape
    t = np.zeros((pad4(nz), pad4(ny), pad4(nx), 1))
    t[:nz, :ny, :nx, 0] = phi / s if s > 0 else 0.0
    return t


def guess(g: Grid, p, w, q=None):
    """Learned initial correction phi0 = c y for SIMPLE's first pass, where y is
    the network output on the physical cells and c minimises the V-weighted
    continuity residual |r - c D G y| (r = D w).  Returns (phi0, eps) with
    eps = |r - D G phi0|_V / |r|_V <= 1; phi0 = 0 (eps = 1) when the fit is void.
    q: rounding of the network input and activations, as in forward."""
    x, r = features(g, w)
    nz, ny, nx = r.shape
    if q is not None:
        x = q(x)
    y = forward(p, x, q)[0][:nz, :ny, :nx, 0]
    z = fv.divergence(g, fv.gradient(g, y))
    zz = _vdot(g, z, z)
    rr = _vdot(g, r, r)
    if not (zz > 0 and rr > 0 and np.isfinite(zz)):
        return np.zeros_like(r), 1.0
    c = _vdot(g, r, z) / zz
    res = r - c * z
    return c * y, float(np.sqrt(_vdot(g, res, res) / rr))
