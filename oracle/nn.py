"""FP64 NumPy oracle of the learned CG warm start (TEST INFRASTRUCTURE ONLY).

The paper's method has no learned component; the warm start is an
extension of the CG initial guess (Eq. 9 is solved from it to the same
residual).  This module is the plain reference for the network, its
analytic backward pass and the Adam update, written from the definitions:

* conv3d: 3x3x3 kernels, stride 1, zero padding 1, weights w[o, c, kz, ky, kx],
  out[b, o] = bias[o] + sum_c sum_taps w[o, c, t] in[b, c, p + t - 1];
* avgpool2: mean over 2x2x2 blocks; up2: nearest-neighbour x2;
* the U-Net below; loss = mean squared error; Adam (beta1 0.9, beta2 0.999,
  eps 1e-8) with bias correction;
* trilinear resampling between an n^3 domain and an m^3 grid with the cube
  corners aligned (sample k of m sits at k (n-1)/(m-1)).

U-Net (16 channels; levels 32, 16, 8, 4 for a 32^3 input):
  e0a(1->16) e0b(16->16) -> s0, pool, e1a e1b -> s1, pool, e2a e2b -> s2,
  pool, e3a e3b, up, cat[up, s2] d2a(32->16) d2b, up, cat[up, s1] d1a d1b,
  up, cat[up, s0] d0a d0b, head(16->1).  Every conv but the head is
  followed by ReLU.  Inputs and outputs have shape (B, 1, D, D, D).

Pins: central finite differences for every gradient, SciPy correlate for the
single-channel convolution, exactness of trilinear resampling on affine
fields, constants through pooling/upsampling (tests/test_oracle_nn.py).
"""
from __future__ import annotations

import numpy as np

LAYERS = [  # name, c_in, c_out, relu
    ("e0a", 1, 16, True), ("e0b", 16, 16, True),
    ("e1a", 16, 16, True), ("e1b", 16, 16, True),
    ("e2a", 16, 16, True), ("e2b", 16, 16, True),
    ("e3a", 16, 16, True), ("e3b", 16, 16, True),
    ("d2a", 32, 16, True), ("d2b", 16, 16, True),
    ("d1a", 32, 16, True), ("d1b", 16, 16, True),
    ("d0a", 32, 16, True), ("d0b", 16, 16, True),
    ("head", 16, 1, False),
]


# ----------------------------------------------------------------- layers

def conv3d(x, w, b):
    """x (B, C, D, D, D), w (O, C, 3, 3, 3), b (O,) -> (B, O, D, D, D)."""
    B, C, D, H, W_ = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1), (1, 1)))
    out = np.zeros((B, w.shape[0], D, H, W_))
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                out += np.einsum("bczyx,oc->bozyx", xp[:, :, dz:dz + D, dy:dy + H, dx:dx + W_],
                                 w[:, :, dz, dy, dx])
    return out + b[None, :, None, None, None]


def conv3d_backward(x, w, g):
    """Gradients of sum(g * conv3d(x, w, b)) w.r.t. x, w, b."""
    B, C, D, H, W_ = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1), (1, 1)))
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w)
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                win = xp[:, :, dz:dz + D, dy:dy + H, dx:dx + W_]
                gw[:, :, dz, dy, dx] = np.einsum("bozyx,bczyx->oc", g, win)
                gxp[:, :, dz:dz + D, dy:dy + H, dx:dx + W_] += np.einsum("bozyx,oc->bczyx", g, w[:, :, dz, dy, dx])
    gb = g.sum(axis=(0, 2, 3, 4))
    return gxp[:, :, 1:-1, 1:-1, 1:-1], gw, gb


def avgpool2(x):
    B, C, D, H, W_ = x.shape
    return x.reshape(B, C, D // 2, 2, H // 2, 2, W_ // 2, 2).mean(axis=(3, 5, 7))


def avgpool2_backward(g):
    return np.repeat(np.repeat(np.repeat(g, 2, axis=2), 2, axis=3), 2, axis=4) / 8.0


def up2(x):
    return np.repeat(np.repeat(np.repeat(x, 2, axis=2), 2, axis=3), 2, axis=4)


def up2_backward(g):
    B, C, D, H, W_ = g.shape
    return g.reshape(B, C, D // 2, 2, H // 2, 2, W_ // 2, 2).sum(axis=(3, 5, 7))


# ----------------------------------------------------------------- model

def init_params(seed: int):
    """He-normal weights, zero biases (reference initialization)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, ci, co, _ in LAYERS:
        std = np.sqrt(2.0 / (ci * 27))
        p[name + ".w"] = rng.standard_normal((co, ci, 3, 3, 3)) * std
        p[name + ".b"] = np.zeros(co)
    return p


def forward(p, x):
    """Returns the output and the activations needed by backward()."""
    act = {"in": x}
    relu = {n: r for n, _, _, r in LAYERS}

    def layer(name, inp):
        z = conv3d(inp, p[name + ".w"], p[name + ".b"])
        y = np.maximum(z, 0.0) if relu[name] else z
        act[name + ".in"] = inp
        act[name + ".out"] = y
        return y

    s0 = layer("e0b", layer("e0a", x))
    s1 = layer("e1b", layer("e1a", avgpool2(s0)))
    s2 = layer("e2b", layer("e2a", avgpool2(s1)))
    bott = layer("e3b", layer("e3a", avgpool2(s2)))
    d2 = layer("d2b", layer("d2a", np.concatenate([up2(bott), s2], axis=1)))
    d1 = layer("d1b", layer("d1a", np.concatenate([up2(d2), s1], axis=1)))
    d0 = layer("d0b", layer("d0a", np.concatenate([up2(d1), s0], axis=1)))
    out = layer("head", d0)
    return out, act


def backward(p, act, g_out):
    """Gradients of sum(g_out * forward(p, x)) with respect to every parameter."""
    grads = {}
    relu = {n: r for n, _, _, r in LAYERS}

    def back(name, g):
        y = act[name + ".out"]
        if relu[name]:
            g = g * (y > 0.0)
        gx, gw, gb = conv3d_backward(act[name + ".in"], p[name + ".w"], g)
        grads[name + ".w"] = gw
        grads[name + ".b"] = gb
        return gx

    g = back("head", g_out)
    g = back("d0b", g)
    g = back("d0a", g)
    g_up, g_s0 = g[:, :16], g[:, 16:]
    g = up2_backward(g_up)
    g = back("d1b", g)
    g = back("d1a", g)
    g_up, g_s1 = g[:, :16], g[:, 16:]
    g = up2_backward(g_up)
    g = back("d2b", g)
    g = back("d2a", g)
    g_up, g_s2 = g[:, :16], g[:, 16:]
    g = up2_backward(g_up)
    g = back("e3b", g)
    g = back("e3a", g)
    g = avgpool2_backward(g) + g_s2
    g = back("e2b", g)
    g = back("e2a", g)
    g = avgpool2_backward(g) + g_s1
    g = back("e1b", g)
    g = back("e1a", g)
    g = avgpool2_backward(g) + g_s0
    g = back("e0b", g)
    grads["input"] = back("e0a", g)
    return grads


def mse(y, t):
    d = y - t
    return float(np.mean(d * d)), 2.0 * d / d.size


def adam_step(p, grads, state, lr, step, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update in place; state holds the m and v moments."""
    for k in p:
        g = grads[k]
        m = state.setdefault(k + ".m", np.zeros_like(g))
        v = state.setdefault(k + ".v", np.zeros_like(g))
        m[...] = b1 * m + (1 - b1) * g
        v[...] = b2 * v + (1 - b2) * g * g
        mh = m / (1 - b1 ** step)
        vh = v / (1 - b2 ** step)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)


# ----------------------------------------------------------------- resampling

def _lin_weights(n, m):
    """Sample positions k (n-1)/(m-1) of an m-grid on an n-grid: (i0, i1, t)."""
    u = np.arange(m) * ((n - 1) / (m - 1))
    i0 = np.minimum(np.floor(u).astype(int), n - 2)
    return i0, i0 + 1, u - i0


def resample(f, m):
    """Trilinear resampling of f (n, n, n) onto m^3, corners aligned."""
    out = f
    for ax in range(3):
        n = out.shape[ax]
        i0, i1, t = _lin_weights(n, m)
        a = np.take(out, i0, axis=ax)
        b = np.take(out, i1, axis=ax)
        shape = [1, 1, 1]
        shape[ax] = m
        t = t.reshape(shape)
        out = (1 - t) * a + t * b
    return out


def upsample_cubic(f, m):
    """Tricubic map of f (a 3-D array) onto m points per axis (an int, or
    one per axis in array order), corners aligned: the learned start's way
    back to the pair domain.  Fine point k of an axis sits at
    u = k (n-1)/(m-1) on the coarse axis of n points; with
    i = min(floor(u), n-2) and t = u - i the value is the 4-point Lagrange
    interpolant through the coarse points i-1, i, i+1, i+2, a point one
    beyond an end taking the linear extrapolation 2 f(end) - f(end -+ 1).
    One axis at a time."""
    out = np.asarray(f, dtype=np.float64)
    ms = (m,) * 3 if np.isscalar(m) else tuple(m)
    for ax in range(3):
        n, mm = out.shape[ax], ms[ax]
        u = np.arange(mm) * ((n - 1) / (mm - 1))
        i = np.minimum(np.floor(u).astype(int), n - 2)
        t = u - i
        # one ghost point on each side, by linear extrapolation
        a = np.moveaxis(out, ax, 0)
        ext = np.concatenate([(2 * a[0] - a[1])[None], a, (2 * a[-1] - a[-2])[None]], axis=0)
        res = 0.0
        for q in range(4):
            # Lagrange basis of node q over the nodes at offsets -1, 0, 1, 2
            lq = np.ones_like(t)
            for r in range(4):
                if r != q:
                    lq = lq * (t - (r - 1)) / ((q - 1) - (r - 1))
            vals = ext[i + q]            # ghost-shifted index of point i - 1 + q
            res = res + lq.reshape((mm,) + (1,) * (vals.ndim - 1)) * vals
        out = np.moveaxis(res, 0, ax)
    return out
