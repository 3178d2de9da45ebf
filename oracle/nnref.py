"""FP64 CPU oracle of the learned warm-start network (test infrastructure only).

Only tests/, the benchmark's CPU baseline and the smoke check may import this
module; the product path never does.  Everything here is the plain definition,
written with numpy in float64:

* 3x3x3 convolution with periodic padding and stride 1,
  y[b, o, v] = bias[o] + sum_{i, t} w[o, i, t] x[b, i, v + d(t)],
  tap t = (dx+1) + 3 (dy+1) + 9 (dz+1), tensors [batch][channel][z][y][x];
* its adjoint with respect to x (backward data) and its gradient with respect
  to w and bias (backward weight);
* 2x average pooling, nearest-neighbour 2x upsampling, ReLU;
* the encoder-decoder of include/hmg_nn.h with the same parameter order
  (every layer's weights in order, then every layer's biases), forward and
  backward by the chain rule.

Pins (tests/test_nnref.py): scipy.ndimage.correlate in 'wrap' mode for the
convolution, the adjoint identity <conv(x), z> = <x, conv^T(z)>, and central
finite differences for the weight, bias and input gradients of a whole small
network.
"""
from __future__ import annotations

import numpy as np

TAPS = [((t % 3) - 1, ((t // 3) % 3) - 1, (t // 9) - 1) for t in range(27)]  # (dx, dy, dz)


def shift(x: np.ndarray, dx: int, dy: int, dz: int) -> np.ndarray:
    """out[..., z, y, x] = x[..., z + dz, y + dy, x + dx] with periodic wrap."""
    return np.roll(x, shift=(-dz, -dy, -dx), axis=(-3, -2, -1))


def conv3d(x, w, b=None):
    """x [B, Cin, D, H, W], w [Cout, Cin, 27], b [Cout] -> y [B, Cout, D, H, W]."""
    B, Cin = x.shape[:2]
    Cout = w.shape[0]
    y = np.zeros((B, Cout) + x.shape[2:])
    for t, (dx, dy, dz) in enumerate(TAPS):
        xs = shift(x, dx, dy, dz)
        y += np.einsum("oi,bizyx->bozyx", w[:, :, t], xs)
    if b is not None:
        y += b[None, :, None, None, None]
    return y


def conv3d_backward_data(dz, w):
    """Adjoint of conv3d in x: dx[b, i, v] = sum_{o, t} w[o, i, t] dz[b, o, v - d(t)]."""
    B = dz.shape[0]
    Cin = w.shape[1]
    dx = np.zeros((B, Cin) + dz.shape[2:])
    for t, (ddx, ddy, ddz) in enumerate(TAPS):
        dx += shift(np.einsum("oi,bozyx->bizyx", w[:, :, t], dz), -ddx, -ddy, -ddz)
    return dx


def conv3d_backward_weight(x, dz):
    """dw[o, i, t] = sum_{b, v} dz[b, o, v] x[b, i, v + d(t)];  db[o] = sum dz[b, o, v]."""
    Cout, Cin = dz.shape[1], x.shape[1]
    dw = np.zeros((Cout, Cin, 27))
    for t, (dx, dy, ddz) in enumerate(TAPS):
        dw[:, :, t] = np.einsum("bozyx,bizyx->oi", dz, shift(x, dx, dy, ddz))
    return dw, dz.sum(axis=(0, 2, 3, 4))


def pool2(x):
    B, C, D, H, W = x.shape
    return x.reshape(B, C, D // 2, 2, H // 2, 2, W // 2, 2).mean(axis=(3, 5, 7))


def pool2_backward(dy):
    return np.repeat(np.repeat(np.repeat(dy, 2, axis=2), 2, axis=3), 2, axis=4) / 8.0


def up2(x):
    return np.repeat(np.repeat(np.repeat(x, 2, axis=2), 2, axis=3), 2, axis=4)


def up2_backward(dy):
    B, C, D, H, W = dy.shape
    return dy.reshape(B, C, D // 2, 2, H // 2, 2, W // 2, 2).sum(axis=(3, 5, 7))


def round_bf16(a):
    """Round to the nearest bf16 (ties to even) and back to float64, by bit
    arithmetic on the float32 encoding (inputs are first rounded to float32)."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


class UNetRef:
    """The encoder-decoder of include/hmg_nn.h on a flat FP64 parameter vector.

    With ``operand_round`` (e.g. round_bf16) every convolution operand (input,
    weights, incoming gradient) is rounded the way matrix-core operands are,
    while sums stay in FP64."""

    def __init__(self, levels=4, base=8, cin=1, cout=18, operand_round=None):
        self.levels, self.base, self.cin, self.cout = levels, base, cin, cout
        self.R = operand_round if operand_round is not None else (lambda a: a)
        ch = lambda l: base << l
        convs = []
        for l in range(levels):
            convs.append((cin if l == 0 else ch(l - 1), ch(l), True))
            convs.append((ch(l), ch(l), True))
        for l in range(levels - 2, -1, -1):
            convs.append((ch(l + 1) + ch(l), ch(l), True))
            convs.append((ch(l), ch(l), True))
        convs.append((ch(0), cout, False))
        self.convs = convs
        off, self.woff = 0, []
        for ci, co, _ in convs:
            self.woff.append(off)
            off += co * ci * 27
        self.boff = []
        for ci, co, _ in convs:
            self.boff.append(off)
            off += co
        self.nparam = off

    def unpack(self, p, k):
        ci, co, _ = self.convs[k]
        w = p[self.woff[k]:self.woff[k] + co * ci * 27].reshape(co, ci, 27)
        return w, p[self.boff[k]:self.boff[k] + co]

    def forward(self, p, x):
        """Returns y and the cache needed by backward; cache[("pre", k)] holds
        the pre-activation of ReLU layer k."""
        L = self.levels
        cache = {"x": x}
        k = 0
        skips = []
        h = x
        for l in range(L):
            if l >= 1:
                h = pool2(skips[-1])
                cache[("pool", l)] = h
            w, b = self.unpack(p, k)
            cache[("pre", k)] = conv3d(self.R(h), self.R(w), b)
            a = np.maximum(cache[("pre", k)], 0.0)
            k += 1
            cache[("enc_in", l)] = h
            cache[("enc_a", l)] = a
            w, b = self.unpack(p, k)
            cache[("pre", k)] = conv3d(self.R(a), self.R(w), b)
            s = np.maximum(cache[("pre", k)], 0.0)
            k += 1
            cache[("skip", l)] = s
            skips.append(s)
        src = skips[-1]
        for l in range(L - 2, -1, -1):
            cat = np.concatenate([up2(src), skips[l]], axis=1)
            cache[("cat", l)] = cat
            w, b = self.unpack(p, k)
            cache[("pre", k)] = conv3d(self.R(cat), self.R(w), b)
            da = np.maximum(cache[("pre", k)], 0.0)
            k += 1
            cache[("dec_a", l)] = da
            w, b = self.unpack(p, k)
            cache[("pre", k)] = conv3d(self.R(da), self.R(w), b)
            db = np.maximum(cache[("pre", k)], 0.0)
            k += 1
            cache[("dec_b", l)] = db
            src = db
        cache["top"] = src
        w, b = self.unpack(p, k)
        y = conv3d(self.R(src), self.R(w), b)
        return y, cache

    def backward(self, p, cache, dy):
        """Gradient of <dy, y> with respect to the parameters (flat) and to x."""
        L = self.levels
        g = np.zeros_like(p)
        ch = lambda l: self.base << l

        def conv_bwd(k, xin, yout, dyout, relu, need_dx=True):
            w, _ = self.unpack(p, k)
            dz = dyout * (yout > 0) if relu else dyout
            dw, _ = conv3d_backward_weight(self.R(xin), self.R(dz))
            ci, co, _ = self.convs[k]
            g[self.woff[k]:self.woff[k] + co * ci * 27] += dw.ravel()
            g[self.boff[k]:self.boff[k] + co] += dz.sum(axis=(0, 2, 3, 4))
            return conv3d_backward_data(self.R(dz), self.R(w)) if need_dx else None

        k = len(self.convs) - 1
        d_src = conv_bwd(k, cache["top"], None, dy, False)
        k -= 1
        d_skip = [np.zeros_like(cache[("skip", l)]) for l in range(L)]
        for l in range(0, L - 1):
            kb, ka = k, k - 1
            k -= 2
            d_da = conv_bwd(kb, cache[("dec_a", l)], cache[("dec_b", l)], d_src, True)
            d_cat = conv_bwd(ka, cache[("cat", l)], cache[("dec_a", l)], d_da, True)
            d_skip[l] += d_cat[:, ch(l + 1):]
            d_src = up2_backward(d_cat[:, :ch(l + 1)])
        d_skip[L - 1] += d_src
        dx = None
        for l in range(L - 1, -1, -1):
            d_a = conv_bwd(2 * l + 1, cache[("enc_a", l)], cache[("skip", l)], d_skip[l], True)
            d_in = conv_bwd(2 * l, cache[("enc_in", l)], cache[("enc_a", l)], d_a, True)
            if l >= 1:
                d_skip[l - 1] += pool2_backward(d_in)
            else:
                dx = d_in
        return g, dx
