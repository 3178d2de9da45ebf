"""Pins of the network oracle (oracle/nnref.py) on the CPU.

The convolution is checked against scipy.ndimage.correlate in 'wrap' mode (an
independent library routine), its adjoint through the identity
<conv(x), z> = <x, conv^T(z)>, its weight gradient and the whole network's
chain rule through central finite differences.
"""
import numpy as np
import pytest
from scipy import ndimage

from oracle import nnref as N


def rng(seed):
    return np.random.default_rng(seed)


def test_conv3d_matches_scipy_wrap_correlate():
    r = rng(0)
    x = r.standard_normal((2, 3, 4, 6, 8))
    w = r.standard_normal((5, 3, 27))
    b = r.standard_normal(5)
    y = N.conv3d(x, w, b)
    for bb in range(2):
        for o in range(5):
            ref = b[o] + sum(ndimage.correlate(x[bb, i], w[o, i].reshape(3, 3, 3), mode="wrap")
                             for i in range(3))
            assert np.abs(y[bb, o] - ref).max() < 1e-12


def test_conv3d_tap_order_delta():
    # a delta input returns the kernel reflected: y[v] = w[t] at v = -d(t)
    x = np.zeros((1, 1, 4, 4, 4))
    x[0, 0, 0, 0, 0] = 1.0
    w = np.arange(27, dtype=float).reshape(1, 1, 27)
    y = N.conv3d(x, w)
    for t, (dx, dy, dz) in enumerate(N.TAPS):
        assert y[0, 0, (-dz) % 4, (-dy) % 4, (-dx) % 4] == t


def test_backward_data_is_adjoint():
    r = rng(1)
    x = r.standard_normal((2, 4, 4, 4, 8))
    w = r.standard_normal((3, 4, 27))
    z = r.standard_normal((2, 3, 4, 4, 8))
    lhs = np.vdot(N.conv3d(x, w), z)
    rhs = np.vdot(x, N.conv3d_backward_data(z, w))
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)


def test_backward_weight_finite_difference():
    r = rng(2)
    x = r.standard_normal((2, 2, 4, 4, 4))
    w = r.standard_normal((3, 2, 27))
    b = r.standard_normal(3)
    z = r.standard_normal((2, 3, 4, 4, 4))
    dw, db = N.conv3d_backward_weight(x, z)
    f = lambda w_, b_: np.vdot(N.conv3d(x, w_, b_), z)
    h = 1e-6
    for idx in [(0, 0, 0), (2, 1, 13), (1, 0, 26), (0, 1, 5)]:
        e = np.zeros_like(w)
        e[idx] = h
        assert abs((f(w + e, b) - f(w - e, b)) / (2 * h) - dw[idx]) < 1e-6 * max(1, abs(dw[idx]))
    e = np.zeros(3)
    e[1] = h
    assert abs((f(w, b + e) - f(w, b - e)) / (2 * h) - db[1]) < 1e-6 * max(1, abs(db[1]))


def test_pool_up_adjoints():
    r = rng(3)
    x = r.standard_normal((2, 3, 4, 4, 4))
    y = r.standard_normal((2, 3, 2, 2, 2))
    assert abs(np.vdot(N.pool2(x), y) - np.vdot(x, N.pool2_backward(y))) < 1e-12
    assert abs(np.vdot(N.up2(y), x) - np.vdot(y, N.up2_backward(x))) < 1e-12
    assert np.allclose(N.pool2(N.up2(y)), y)


def test_default_parameter_count():
    u = N.UNetRef()
    assert sum(co * ci * 27 for ci, co, _ in u.convs) == 368712
    assert u.nparam == 368712 + 370


@pytest.mark.parametrize("levels,base", [(1, 2), (2, 2), (3, 1)])
def test_unet_gradient_finite_difference(levels, base):
    r = rng(10 + levels)
    net = N.UNetRef(levels=levels, base=base, cin=1, cout=2)
    D = 2 << (levels - 1) if levels > 1 else 4
    D = max(D, 4)
    p = r.standard_normal(net.nparam) * 0.5
    x = r.standard_normal((2, 1, D, D, D))
    dy = r.standard_normal((2, 2, D, D, D))
    y, cache = net.forward(p, x)
    g, dx = net.backward(p, cache, dy)
    f = lambda pp, xx: np.vdot(net.forward(pp, xx)[0], dy)
    h = 1e-6
    picks = r.choice(net.nparam, size=min(25, net.nparam), replace=False)
    for k in picks:
        e = np.zeros_like(p)
        e[k] = h
        fd = (f(p + e, x) - f(p - e, x)) / (2 * h)
        assert abs(fd - g[k]) < 1e-5 * max(1.0, abs(g[k])), (k, fd, g[k])
    for idx in [(0, 0, 0, 1, 2), (1, 0, D - 1, 0, 1)]:
        e = np.zeros_like(x)
        e[idx] = h
        fd = (f(p, x + e) - f(p, x - e)) / (2 * h)
        assert abs(fd - dx[idx]) < 1e-5 * max(1.0, abs(dx[idx]))


def test_round_bf16_matches_torch_and_bounds():
    import torch
    r = rng(20)
    a = r.standard_normal(10000) * 10.0 ** r.integers(-6, 6, 10000)
    ref = torch.from_numpy(a.astype(np.float32)).to(torch.bfloat16).double().numpy()
    assert np.array_equal(N.round_bf16(a), ref)
    f = a.astype(np.float32).astype(np.float64)
    assert np.all(np.abs(N.round_bf16(a) - f) <= 2.0 ** -8 * np.abs(f))
    # exact ties (low half 0x8000) round to the even bf16, for even and odd upper
    # halves and both signs; random values almost never hit a tie
    hi = np.arange(0x3F00, 0x3F40, dtype=np.uint32)
    ties = ((hi << 16) | 0x8000).view(np.float32)
    ties = np.concatenate([ties, -ties])
    ref = torch.from_numpy(ties).to(torch.bfloat16).double().numpy()
    assert np.array_equal(N.round_bf16(ties.astype(np.float64)), ref)
    up = ties.view(np.uint32) >> 16
    assert np.array_equal(ref.astype(np.float32).view(np.uint32) >> 16,
                          np.where(up & 1, up + 1, up).astype(np.uint32))
