"""FP64 reference of the surrogate U-Net (forward and backward), for gradient checks.

Oracle / test infrastructure.  Periodic convolutions (kernel 3 per axis, or 1
for the head), 2x2(x2) periodic average pooling with ceil sizes (output j
covers inputs (2j + o) mod n), nearest upsampling cropped to the skip size,
channel concatenation [upsampled-path, skip], ReLU, mean-squared-error loss.

Architecture for L levels and base width c (c_l = c 2^l):
  encoder l < L-1 : conv3(. -> c_l) relu, conv3(c_l -> c_l) relu = skip_l, pool
  bottleneck      : conv3(. -> c_{L-1}) relu, conv3 relu
  decoder l       : upsample, conv3(c_{l+1} -> c_l) relu, concat [., skip_l],
                    conv3(2 c_l -> c_l) relu, conv3(c_l -> c_l) relu
  head            : conv1(c_0 -> cout)
Flat parameters: for every conv in that order, w[cout][cin][taps] then b[cout],
taps row-major over the (z,) y, x offsets -1, 0, 1.

Pinned by tests/test_oracle_unet.py (central finite differences in FP64).
"""
from __future__ import annotations

import itertools
import numpy as np


def layer_shapes(d, levels, base, cin, cout):
    """(cin, cout, ks) of every conv layer in parameter order."""
    out = []
    prev = cin
    for l in range(levels):
        c = base << l
        out.append((prev, c, 3))
        out.append((c, c, 3))
        prev = c
    for l in range(levels - 2, -1, -1):
        c, cu = base << l, base << (l + 1)
        out.append((cu, c, 3))
        out.append((2 * c, c, 3))
        out.append((c, c, 3))
    out.append((base, cout, 1))
    return out


def n_params(d, levels, base, cin, cout):
    return sum(co * ci * ks ** d + co for ci, co, ks in layer_shapes(d, levels, base, cin, cout))


def unpack(theta, d, levels, base, cin, cout):
    ws, off = [], 0
    for ci, co, ks in layer_shapes(d, levels, base, cin, cout):
        taps = ks ** d
        w = theta[off:off + co * ci * taps].reshape(co, ci, taps)
        off += co * ci * taps
        b = theta[off:off + co]
        off += co
        ws.append((w, b, ks))
    return ws


def _offsets(d, ks):
    r = ks // 2
    return list(itertools.product(*[range(-r, r + 1)] * d))


def conv(x, w, b, ks):
    """x (B, Cin, *S) -> (B, Cout, *S), periodic: out[q] = sum w[co, ci, t] x[ci, q + off_t] + b."""
    d = x.ndim - 2
    out = np.zeros((x.shape[0], w.shape[0]) + x.shape[2:])
    for t, off in enumerate(_offsets(d, ks)):
        xs = np.roll(x, shift=tuple(-o for o in off), axis=tuple(range(2, 2 + d)))
        out += np.einsum("oi,bi...->bo...", w[:, :, t], xs)
    return out + b.reshape((1, -1) + (1,) * d)


def conv_backward(x, w, ks, gy):
    """Gradients of conv w.r.t. x, w, b for upstream gradient gy."""
    d = x.ndim - 2
    gx = np.zeros_like(x)
    gw = np.zeros_like(w)
    for t, off in enumerate(_offsets(d, ks)):
        xs = np.roll(x, shift=tuple(-o for o in off), axis=tuple(range(2, 2 + d)))
        ax = [0] + list(range(2, 2 + d))
        gw[:, :, t] = np.tensordot(gy, xs, axes=(ax, ax))
        gxs = np.einsum("oi,bo...->bi...", w[:, :, t], gy)
        gx += np.roll(gxs, shift=tuple(off), axis=tuple(range(2, 2 + d)))
    gb = gy.sum(axis=tuple([0] + list(range(2, 2 + d))))
    return gx, gw, gb


def pool(x):
    d = x.ndim - 2
    S = x.shape[2:]
    So = tuple((n + 1) // 2 for n in S)
    out = np.zeros(x.shape[:2] + So)
    for o in itertools.product(*[(0, 1)] * d):
        idx = tuple(np.mod(2 * np.arange(m) + oo, n) for m, oo, n in zip(So, o, S))
        out += x[(slice(None), slice(None)) + np.ix_(*idx)]
    return out / 2 ** d


def pool_backward(gy, S):
    d = gy.ndim - 2
    So = gy.shape[2:]
    gx = np.zeros(gy.shape[:2] + tuple(S))
    for o in itertools.product(*[(0, 1)] * d):
        idx = tuple(np.mod(2 * np.arange(m) + oo, n) for m, oo, n in zip(So, o, S))
        np.add.at(gx, (slice(None), slice(None)) + np.ix_(*idx), gy / 2 ** d)
    return gx


def up(x, S):
    idx = tuple(np.arange(n) // 2 for n in S)
    return x[(slice(None), slice(None)) + np.ix_(*idx)]


def up_backward(gy, Si):
    d = gy.ndim - 2
    gx = np.zeros(gy.shape[:2] + tuple(Si))
    idx = tuple(np.arange(n) // 2 for n in gy.shape[2:])
    np.add.at(gx, (slice(None), slice(None)) + np.ix_(*idx), gy)
    return gx


def forward(theta, x, levels, base, cout, keep=False):
    d = x.ndim - 2
    ws = unpack(theta, d, levels, base, x.shape[1], cout)
    tape = []
    k = 0

    def cv(inp, relu=True):
        nonlocal k
        w, b, ks = ws[k]
        z = conv(inp, w, b, ks)
        y = np.maximum(z, 0.0) if relu else z
        tape.append((k, inp, y, relu))
        k += 1
        return y

    skips, cur = [], x
    for l in range(levels):
        a = cv(cur)
        s = cv(a)
        if l < levels - 1:
            skips.append(s)
            cur = pool(s)
        else:
            cur = s
    for l in range(levels - 2, -1, -1):
        u = up(cur, skips[l].shape[2:])
        a = cv(u)
        cat = np.concatenate([a, skips[l]], axis=1)
        b1 = cv(cat)
        cur = cv(b1)
    out = cv(cur, relu=False)
    return (out, tape, ws) if keep else out


def loss_and_grad(theta, x, target, levels, base):
    """MSE loss and its gradient w.r.t. theta (flat), by explicit backpropagation."""
    cout = target.shape[1]
    out, tape, ws = forward(theta, x, levels, base, cout, keep=True)
    n = out.size
    loss = float(np.sum((out - target) ** 2) / n)
    g_out = 2.0 * (out - target) / n
    return loss, backward(theta, x, tape, ws, g_out, levels)


def backward(theta, x, tape, ws, g_out, levels):
    d = x.ndim - 2
    grads = [None] * len(ws)

    def bcv(idx, gy):
        k, inp, y, relu = tape[idx]
        w, b, ks = ws[k]
        if relu:
            gy = gy * (y > 0)
        gx, gw, gb = conv_backward(inp, w, ks, gy)
        grads[k] = (gw, gb)
        return gx

    # tape order: encoder (2 per level), decoder (3 per level), head
    idx = len(tape) - 1
    g = bcv(idx, g_out)
    idx -= 1
    skip_grads = {}
    for l in range(0, levels - 1):
        # decoder levels were taped from l = L-2 down to 0; walk back from level 0 up
        g = bcv(idx, g)              # conv(c_l -> c_l)
        idx -= 1
        gcat = bcv(idx, g)           # conv(2 c_l -> c_l)
        idx -= 1
        c = gcat.shape[1] // 2
        skip_grads[l] = gcat[:, c:]
        gu = bcv(idx, gcat[:, :c])   # conv(c_{l+1} -> c_l) on the upsampled tensor
        idx -= 1
        Si = tape[2 * (l + 1) + 1][2].shape[2:]   # output size of level l+1
        g = up_backward(gu, Si)
    for l in range(levels - 1, -1, -1):
        if l < levels - 1:
            g = g + skip_grads[l]
        g = bcv(2 * l + 1, g)
        g = bcv(2 * l, g)
        if l > 0:
            g = pool_backward(g, tape[2 * (l - 1) + 1][2].shape[2:])
    flat = []
    for gw, gb in grads:
        flat.append(gw.reshape(-1))
        flat.append(gb)
    return np.concatenate(flat)
