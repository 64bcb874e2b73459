"""Pins of the FP64 network oracle (oracle/nn.py): finite differences,
SciPy correlation, adjointness, exactness on affine fields, Adam closed form."""
import numpy as np
import pytest
from scipy.ndimage import correlate

from oracle import nn


def test_conv3d_single_channel_matches_scipy():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((1, 1, 6, 7, 5))
    w = rng.standard_normal((1, 1, 3, 3, 3))
    got = nn.conv3d(x, w, np.array([0.25]))[0, 0]
    want = correlate(x[0, 0], w[0, 0], mode="constant", cval=0.0) + 0.25
    assert np.max(np.abs(got - want)) < 1e-12


def _fd(f, arr, idx, h=1e-6):
    old = arr[idx]
    arr[idx] = old + h
    fp = f()
    arr[idx] = old - h
    fm = f()
    arr[idx] = old
    return (fp - fm) / (2 * h)


def test_conv3d_backward_finite_differences():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 2, 4, 4, 4))
    w = rng.standard_normal((3, 2, 3, 3, 3))
    b = rng.standard_normal(3)
    g = rng.standard_normal((2, 3, 4, 4, 4))
    loss = lambda: float(np.sum(g * nn.conv3d(x, w, b)))
    gx, gw, gb = nn.conv3d_backward(x, w, g)
    for idx in [(0, 0, 0, 0, 0), (1, 1, 2, 3, 1), (0, 1, 3, 3, 3)]:
        assert abs(_fd(loss, x, idx) - gx[idx]) < 1e-7
    for idx in [(0, 0, 0, 0, 0), (2, 1, 1, 2, 0), (1, 0, 2, 2, 2)]:
        assert abs(_fd(loss, w, idx) - gw[idx]) < 1e-7
    for k in range(3):
        assert abs(_fd(loss, b, (k,)) - gb[k]) < 1e-7


def test_pool_and_upsample_adjoint_and_constants():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 3, 4, 4, 4))
    y = rng.standard_normal((2, 3, 2, 2, 2))
    assert abs(np.sum(nn.avgpool2(x) * y) - np.sum(x * nn.avgpool2_backward(y))) < 1e-12
    assert abs(np.sum(nn.up2(y) * x) - np.sum(y * nn.up2_backward(x))) < 1e-12
    c = np.full((1, 1, 4, 4, 4), 3.5)
    assert np.all(nn.avgpool2(c) == 3.5) and np.all(nn.up2(nn.avgpool2(c)) == 3.5)


@pytest.fixture(scope="module")
def tiny_net():
    rng = np.random.default_rng(3)
    p = nn.init_params(7)
    for k in p:
        if k.endswith(".b"):
            p[k] = 0.1 * rng.standard_normal(p[k].shape)
    x = rng.standard_normal((2, 1, 8, 8, 8))
    t = rng.standard_normal((2, 1, 8, 8, 8))
    return p, x, t


def test_unet_backward_finite_differences(tiny_net):
    """P11: analytic gradients of the MSE loss through the whole U-Net."""
    p, x, t = tiny_net

    def loss():
        y, _ = nn.forward(p, x)
        return nn.mse(y, t)[0]

    y, act = nn.forward(p, x)
    L, gy = nn.mse(y, t)
    grads = nn.backward(p, act, gy)
    rng = np.random.default_rng(4)
    checked = 0
    for name, _, _, _ in nn.LAYERS:
        for suffix in (".w", ".b"):
            arr = p[name + suffix]
            for _ in range(2):
                idx = tuple(rng.integers(0, s) for s in arr.shape)
                fd = _fd(loss, arr, idx)
                an = grads[name + suffix][idx]
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (name, suffix, idx, fd, an)
                checked += 1
    for idx in [(0, 0, 1, 2, 3), (1, 0, 7, 0, 4)]:
        assert abs(_fd(loss, x, idx) - grads["input"][idx]) < 1e-6
    assert checked == 60


def test_mse_gradient():
    rng = np.random.default_rng(5)
    y = rng.standard_normal((3, 4))
    t = rng.standard_normal((3, 4))
    L, g = nn.mse(y, t)
    assert abs(L - np.mean((y - t) ** 2)) < 1e-15
    assert abs(_fd(lambda: nn.mse(y, t)[0], y, (1, 2)) - g[1, 2]) < 1e-9


def test_adam_first_step_closed_form():
    """From zero moments, the first bias-corrected step is -lr g/(|g| + eps)."""
    p = {"a": np.array([1.0, -2.0, 0.5])}
    g = {"a": np.array([0.3, -4.0, 1e-3])}
    st = {}
    nn.adam_step(p, g, st, lr=0.01, step=1)
    want = np.array([1.0, -2.0, 0.5]) - 0.01 * g["a"] / (np.abs(g["a"]) + 1e-8)
    assert np.max(np.abs(p["a"] - want)) < 1e-15


@pytest.mark.parametrize("n,m", [(63, 32), (29, 32), (32, 63)])
def test_resample_exact_on_affine_fields(n, m):
    ax = np.arange(n, dtype=float)
    f = 0.5 + 2.0 * ax[:, None, None] - 1.5 * ax[None, :, None] + 0.25 * ax[None, None, :]
    got = nn.resample(f, m)
    u = np.arange(m) * ((n - 1) / (m - 1))
    want = 0.5 + 2.0 * u[:, None, None] - 1.5 * u[None, :, None] + 0.25 * u[None, None, :]
    assert np.max(np.abs(got - want)) < 1e-11


def test_resample_63_to_32_is_subsampling():
    f = np.random.default_rng(6).standard_normal((63, 63, 63))
    assert np.array_equal(nn.resample(f, 32), f[::2, ::2, ::2])


def test_upsample_cubic_pins():
    """The learned start's tricubic map: coarse values kept where fine and
    coarse points coincide (63 = 2 x 32 - 1), affine fields exact everywhere
    (the ghost extrapolation is linear), cubic polynomials exact wherever the
    4-point stencil stays inside the coarse grid, and a coarse delta gives
    the textbook midpoint weights -1/16, 9/16, 9/16, -1/16."""
    rng = np.random.default_rng(3)
    f = rng.standard_normal((32, 32, 32))
    g = nn.upsample_cubic(f, 63)
    assert np.max(np.abs(g[::2, ::2, ::2] - f)) < 1e-13
    c = np.linspace(0.0, 1.0, 32)
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    fine = np.linspace(0.0, 1.0, 63)
    Zf, Yf, Xf = np.meshgrid(fine, fine, fine, indexing="ij")
    aff = nn.upsample_cubic(0.5 + 2 * X - 3 * Y + 0.25 * Z, 63)
    assert np.max(np.abs(aff - (0.5 + 2 * Xf - 3 * Yf + 0.25 * Zf))) < 1e-12
    cub = nn.upsample_cubic(X ** 3 - 2 * Y ** 2 * Z + X * Y * Z, 63)
    want = Xf ** 3 - 2 * Yf ** 2 * Zf + Xf * Yf * Zf
    inner = slice(2, 61)   # fine points whose stencil has no ghost node
    assert np.max(np.abs(cub[inner, inner, inner] - want[inner, inner, inner])) < 1e-12
    d = np.zeros((32, 32, 32))
    d[10, 10, 10] = 1.0
    u = nn.upsample_cubic(d, 63)
    line = u[20, 20, 15:26]   # fine points 15..25 along x at the delta's row and plane
    want_line = [0, 0, -1 / 16, 0, 9 / 16, 1, 9 / 16, 0, -1 / 16, 0, 0]   # fine 20 is coarse 10
    assert np.max(np.abs(line - np.array(want_line))) < 1e-14
    # non-cubic target shape
    h = nn.upsample_cubic(f[:8, :9, :10], (15, 17, 19))
    assert h.shape == (15, 17, 19) and np.max(np.abs(h[::2, ::2, ::2] - f[:8, :9, :10])) < 1e-13
