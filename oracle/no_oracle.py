"""FP64 CPU oracle of the warm-start network (numpy).

TEST INFRASTRUCTURE ONLY.  Only the test suite and the benchmark's CPU leg
may import this module; it shares no code with the GPU network library and
the GPU library never imports it.

The network maps six feature planes of an annulus problem (its parameters and
the radius, one value per node) to three planes, u_z / U, u_r / U and T, at
the same nodes.  It is a convolutional encoder-decoder with additive skips:

    e1 = relu(conv3x3(x))                 stride 1, H
    e2 = relu(conv3x3(e1, stride 2))      H / 2
    e3 = relu(conv3x3(e2, stride 2))      H / 4
    e4 = relu(conv3x3(e3, stride 2))      H / 8
    d1 = relu(conv3x3(up2(e4))) + e3      H / 4
    d2 = relu(conv3x3(up2(d1))) + e2      H / 2
    d3 = relu(conv3x3(up2(d2))) + e1      H
    y  = conv1x1(d3)

conv: y[o] = b[o] + sum_c sum_taps W[o, c, ky, kx] x_pad[c, s oy + ky, s ox + kx]
with zero padding (k - 1) / 2; up2 repeats every value over a 2 x 2 block
(nearest neighbour).  Loss: mean of (y - target)^2 over all outputs.
Optimiser: Adam (Kingma and Ba, 2015), bias-corrected moments.

Parameters are packed layer by layer: W[cout][cin][k][k] (C order), then
b[cout].  Arrays are (batch, channel, height, width).  Everything here is the
plain definition, written out with numpy in float64.
"""
from __future__ import annotations

import numpy as np


def layer_specs(widths):
    """(cin, cout, k, stride, upsample, relu, skip layer index or -1) per layer."""
    c1, c2, c3, c4 = widths
    return [
        (6, c1, 3, 1, False, True, -1),
        (c1, c2, 3, 2, False, True, -1),
        (c2, c3, 3, 2, False, True, -1),
        (c3, c4, 3, 2, False, True, -1),
        (c4, c3, 3, 1, True, True, 2),
        (c3, c2, 3, 1, True, True, 1),
        (c2, c1, 3, 1, True, True, 0),
        (c1, 3, 1, 1, False, False, -1),
    ]


def param_count(widths) -> int:
    return sum(co * ci * k * k + co for ci, co, k, _, _, _, _ in layer_specs(widths))


def unpack(params, widths):
    """Views (W, b) per layer into the flat parameter vector."""
    out, o = [], 0
    for ci, co, k, _, _, _, _ in layer_specs(widths):
        n = co * ci * k * k
        out.append((params[o:o + n].reshape(co, ci, k, k), params[o + n:o + n + co]))
        o += n + co
    return out


def upsample2(x):
    return np.repeat(np.repeat(x, 2, axis=2), 2, axis=3)


def upsample2_adjoint(g):
    b, c, h, w = g.shape
    return g.reshape(b, c, h // 2, 2, w // 2, 2).sum(axis=(3, 5))


def conv(x, W, b, stride):
    """Cross-correlation with zero padding (k - 1) / 2, then bias."""
    k = W.shape[2]
    p = (k - 1) // 2
    B, C, H, Wd = x.shape
    Ho, Wo = (H + 2 * p - k) // stride + 1, (Wd + 2 * p - k) // stride + 1
    xp = np.pad(x, ((0, 0), (0, 0), (p, p), (p, p)))
    y = np.zeros((B, W.shape[0], Ho, Wo))
    for ky in range(k):
        for kx in range(k):
            xs = xp[:, :, ky:ky + stride * (Ho - 1) + 1:stride, kx:kx + stride * (Wo - 1) + 1:stride]
            y += np.einsum("oc,bchw->bohw", W[:, :, ky, kx], xs)
    return y + b[None, :, None, None]


def conv_backward(x, W, dy, stride):
    """Gradients of conv with respect to x, W and b."""
    k = W.shape[2]
    p = (k - 1) // 2
    B, C, H, Wd = x.shape
    Ho, Wo = dy.shape[2], dy.shape[3]
    xp = np.pad(x, ((0, 0), (0, 0), (p, p), (p, p)))
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    for ky in range(k):
        for kx in range(k):
            sl = (slice(None), slice(None), slice(ky, ky + stride * (Ho - 1) + 1, stride),
                  slice(kx, kx + stride * (Wo - 1) + 1, stride))
            dW[:, :, ky, kx] = np.einsum("bohw,bchw->oc", dy, xp[sl])
            dxp[sl] += np.einsum("oc,bohw->bchw", W[:, :, ky, kx], dy)
    dx = dxp[:, :, p:p + H, p:p + Wd]
    return dx, dW, dy.sum(axis=(0, 2, 3))


def forward(params, widths, x):
    """Output y and the activations needed by the backward pass."""
    layers = unpack(np.asarray(params, dtype=np.float64), widths)
    acts = [np.asarray(x, dtype=np.float64)]
    cache = []
    for li, (ci, co, k, s, up, relu, skip) in enumerate(layer_specs(widths)):
        W, b = layers[li]
        xin = upsample2(acts[-1]) if up else acts[-1]
        z = conv(xin, W, b, s)
        a = np.maximum(z, 0.0) if relu else z
        if skip >= 0:
            a = a + acts[skip + 1]
        cache.append((xin, z))
        acts.append(a)
    return acts[-1], (acts, cache)


def loss_and_grads(params, widths, x, target):
    """Mean-square loss and its gradient with respect to the packed parameters."""
    params = np.asarray(params, dtype=np.float64)
    y, (acts, cache) = forward(params, widths, x)
    diff = y - target
    loss = float(np.mean(diff ** 2))
    layers = unpack(params, widths)
    specs = layer_specs(widths)
    grads = [None] * len(specs)
    dacts = [np.zeros_like(a) for a in acts]
    dacts[-1] = 2.0 * diff / diff.size
    for li in range(len(specs) - 1, -1, -1):
        ci, co, k, s, up, relu, skip = specs[li]
        W, _ = layers[li]
        xin, z = cache[li]
        da = dacts[li + 1]
        if skip >= 0:
            dacts[skip + 1] += da  # the skip adds the earlier activation unchanged
        dz = da * (z > 0.0) if relu else da
        dxin, dW, db = conv_backward(xin, W, dz, s)
        grads[li] = (dW, db)
        dacts[li] += upsample2_adjoint(dxin) if up else dxin
    flat = np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in grads])
    return loss, flat


def adam_step(params, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns new (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grads
    v = beta2 * v + (1.0 - beta2) * grads ** 2
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
