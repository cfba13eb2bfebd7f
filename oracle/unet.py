"""FP64 reference of the learned continuation predictor (test infrastructure).

Used only by the tests, by smoke() and by the benchmark's CPU baseline; the
GPU path never imports it.

The predictor is a convolutional U-Net on the vertex grid (an extension
beyond the paper of the continuation in Sec. 4; the paper itself predicts
with pseudo-arclength).  This module states the network in plain numpy, in the
order the computation is defined, so that the GPU kernels can be checked
value by value:

  base start      psi_b: the secant step psi + r (psi - e^{i chi} psi_prev)
                  of the continuation (Sec. 4), or psi itself without history;
  input channels  x = (Re psi, Im psi, Re s, Im s, mu, 50 dmu) with the base
                  step's slope s = (psi_b - psi) / dmu, on an N x N vertex
                  grid (N = 2^(levels-1) m + 1);
  encoder level l two 3x3 convolutions (zero padding), each followed by
                  SiLU(z) = z / (1 + exp(-z)); channels base * 2^l; between
                  levels vertex subsampling (keep every other node);
  decoder         linear vertex interpolation to the finer grid, channel
                  concatenation [upsampled, skip], two 3x3 conv + SiLU;
  head            1x1 convolution to 2 channels o = (o_re, o_im);
  prediction      psi_pred = psi_b + dmu (o_re + i o_im): the network corrects
                  the base step (a zero network is the secant predictor).

Loss of one sample (a design choice of this extension: the paper defines no
network and no loss) (psi, psi_b, target) at (mu, dmu), the target already
phase-aligned to psi, with w = (t - psi_b) / dmu the correction to learn:
L = sum_i d_i |o_i - w_i|^2 / sum_i d_i (|w_i|^2 + EPS), i.e.
||D^(1/2)(psi_pred - t)||^2 relative to ||D^(1/2)(psi_b - t)||^2 (every
sample weighs about the same; just below 1 for a zero network), with an
absolute floor EPS (in slope^2 units) so that samples whose secant start is
already nearly exact cannot dominate.

Parameters: one flat vector; per layer the weights W[co, ky, kx, ci]
(row-major, ky/kx = 0..2 for offsets -1..1) followed by the bias b[co]; the
head stores W[co, ci] then b[co].  Adam as in Kingma & Ba (2015), bias-
corrected moments.
"""
import numpy as np


def layer_specs(levels, base, in_ch=6, out_ch=2):
    """(c_in, c_out, kernel) of every convolution in execution order."""
    specs = []
    ch = [base * 2 ** l for l in range(levels)]
    c = in_ch
    for l in range(levels):
        specs += [(c, ch[l], 3), (ch[l], ch[l], 3)]
        c = ch[l]
    for l in range(levels - 2, -1, -1):
        specs += [(c + ch[l], ch[l], 3), (ch[l], ch[l], 3)]
        c = ch[l]
    specs.append((c, out_ch, 1))
    return specs


def num_params(specs):
    return sum(co * k * k * ci + co for ci, co, k in specs)


def unpack(theta, specs):
    out, o = [], 0
    for ci, co, k in specs:
        nw = co * k * k * ci
        W = theta[o:o + nw].reshape(co, k, k, ci)
        o += nw
        b = theta[o:o + co]
        o += co
        out.append((W, b))
    return out


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def _mix(Wt, x):
    """sum_i Wt[o, i] x[i, h, w] (a channel mixing, as one matrix product)."""
    ci, H, Wd = x.shape
    return (Wt @ x.reshape(ci, H * Wd)).reshape(Wt.shape[0], H, Wd)


def _corr(a, b):
    """sum_{h,w} a[o, h, w] b[i, h, w] (as one matrix product)."""
    return a.reshape(a.shape[0], -1) @ b.reshape(b.shape[0], -1).T


def conv(x, W, b):
    """x (ci, H, W); W (co, k, k, ci); zero padding, same size."""
    co, k, _, ci = W.shape
    H, Wd = x.shape[1:]
    if k == 1:
        return _mix(W[:, 0, 0, :], x) + b[:, None, None]
    xp = np.zeros((ci, H + 2, Wd + 2))
    xp[:, 1:-1, 1:-1] = x
    out = np.zeros((co, H, Wd)) + b[:, None, None]
    for ky in range(3):
        for kx in range(3):
            out += _mix(W[:, ky, kx, :], xp[:, ky:ky + H, kx:kx + Wd])
    return out


def conv_backward(x, W, dout):
    """Gradients of conv(x, W, b) for the upstream gradient dout:
    returns (dx, dW, db)."""
    co, k, _, ci = W.shape
    H, Wd = x.shape[1:]
    db = dout.sum(axis=(1, 2))
    if k == 1:
        dW = _corr(dout, x)[:, None, None, :]
        dx = _mix(W[:, 0, 0, :].T, dout)
        return dx, dW, db
    xp = np.zeros((ci, H + 2, Wd + 2))
    xp[:, 1:-1, 1:-1] = x
    dW = np.zeros_like(W)
    dxp = np.zeros_like(xp)
    for ky in range(3):
        for kx in range(3):
            dW[:, ky, kx, :] = _corr(dout, xp[:, ky:ky + H, kx:kx + Wd])
            dxp[:, ky:ky + H, kx:kx + Wd] += _mix(W[:, ky, kx, :].T, dout)
    return dxp[:, 1:-1, 1:-1], dW, db


def down(x):
    return x[:, ::2, ::2].copy()


def down_backward(dy, shape):
    dx = np.zeros(shape)
    dx[:, ::2, ::2] = dy
    return dx


def up(x):
    """Linear interpolation from an n x n to a (2n-1) x (2n-1) vertex grid."""
    c, h, w = x.shape
    y = np.zeros((c, 2 * h - 1, 2 * w - 1))
    y[:, ::2, ::2] = x
    y[:, 1::2, ::2] = 0.5 * (x[:, :-1, :] + x[:, 1:, :])
    y[:, ::2, 1::2] = 0.5 * (x[:, :, :-1] + x[:, :, 1:])
    y[:, 1::2, 1::2] = 0.25 * (x[:, :-1, :-1] + x[:, 1:, :-1] + x[:, :-1, 1:] + x[:, 1:, 1:])
    return y


def up_backward(dy):
    c, H, Wd = dy.shape
    h, w = (H + 1) // 2, (Wd + 1) // 2
    dx = np.zeros((c, h, w))
    dx += dy[:, ::2, ::2]
    e = dy[:, 1::2, ::2]
    dx[:, :-1, :] += 0.5 * e
    dx[:, 1:, :] += 0.5 * e
    e = dy[:, ::2, 1::2]
    dx[:, :, :-1] += 0.5 * e
    dx[:, :, 1:] += 0.5 * e
    e = dy[:, 1::2, 1::2]
    dx[:, :-1, :-1] += 0.25 * e
    dx[:, 1:, :-1] += 0.25 * e
    dx[:, :-1, 1:] += 0.25 * e
    dx[:, 1:, 1:] += 0.25 * e
    return dx


def input_planes(psi, psi_b, mu, dmu, N):
    p = psi.reshape(N, N)
    sl = ((psi_b - psi) / dmu).reshape(N, N)
    return np.stack([p.real, p.imag, sl.real, sl.imag, np.full((N, N), mu), np.full((N, N), 50.0 * dmu)])


def forward(theta, specs, levels, x, keep=False):
    """Network output o (2, N, N) for the input planes x; with keep, also the
    intermediate values that backward needs."""
    P = unpack(theta, specs)
    enc, skips = [], []
    h = x
    for l in range(levels):
        if l > 0:
            h = down(h)
        a0 = h
        z0 = conv(a0, *P[2 * l])
        h1 = silu(z0)
        z1 = conv(h1, *P[2 * l + 1])
        h = silu(z1)
        enc.append((a0, z0, h1, z1))
        skips.append(h)
    dec = []
    li = 2 * levels
    for l in range(levels - 2, -1, -1):
        u = up(h)
        cat = np.concatenate([u, skips[l]], axis=0)
        z0 = conv(cat, *P[li])
        h1 = silu(z0)
        z1 = conv(h1, *P[li + 1])
        h = silu(z1)
        dec.append((l, li, cat, z0, h1, z1, u.shape[0]))
        li += 2
    o = conv(h, *P[li])
    if not keep:
        return o
    return o, {"enc": enc, "dec": dec, "head_in": h, "head": li}


def backward(theta, specs, levels, tape, do):
    """Flat gradient of the parameters for the upstream gradient do = dL/do."""
    P = unpack(theta, specs)
    grads = [None] * len(specs)
    li = tape["head"]
    dh, dW, db = conv_backward(tape["head_in"], P[li][0], do)
    grads[li] = (dW, db)
    dskip = [None] * levels
    for (l, li, cat, z0, h1, z1, cu) in reversed(tape["dec"]):
        dz1 = dh * silu_grad(z1)
        dh1, dW, db = conv_backward(h1, P[li + 1][0], dz1)
        grads[li + 1] = (dW, db)
        dz0 = dh1 * silu_grad(z0)
        dcat, dW, db = conv_backward(cat, P[li][0], dz0)
        grads[li] = (dW, db)
        dskip[l] = dcat[cu:]
        dh = up_backward(dcat[:cu])
    for l in range(levels - 1, -1, -1):
        a0, z0, h1, z1 = tape["enc"][l]
        if dskip[l] is not None and l < levels - 1:
            dh = dh + dskip[l]
        dz1 = dh * silu_grad(z1)
        dh1, dW, db = conv_backward(h1, P[2 * l + 1][0], dz1)
        grads[2 * l + 1] = (dW, db)
        dz0 = dh1 * silu_grad(z0)
        da0, dW, db = conv_backward(a0, P[2 * l][0], dz0)
        grads[2 * l] = (dW, db)
        if l > 0:
            dh = down_backward(da0, (a0.shape[0],) + tape["enc"][l - 1][3].shape[1:])
    return np.concatenate([np.concatenate([g[0].ravel(), g[1].ravel()]) for g in grads])


EPS = 1e-4


def loss_and_grad_output(o, psi, psi_b, target, dmu, vol, N):
    """Loss of one aligned sample and dL/do (2, N, N)."""
    want = (target - psi_b).reshape(N, N) / dmu
    r = o[0] + 1j * o[1] - want
    w = vol.reshape(N, N)
    sw = (w * (np.abs(want) ** 2 + EPS)).sum()
    L = float((w * np.abs(r) ** 2).sum() / sw)
    do = np.stack([2.0 * w * r.real / sw, 2.0 * w * r.imag / sw])
    return L, do


def predict(theta, specs, levels, psi, psi_b, mu, dmu, N):
    """psi_pred = psi_b + dmu (o_re + i o_im)."""
    o = forward(theta, specs, levels, input_planes(psi, psi_b, mu, dmu, N))
    return psi_b + dmu * (o[0] + 1j * o[1]).ravel()


def loss_and_grad(theta, specs, levels, psi, psi_b, mu, dmu, target, vol, N):
    """Loss of one sample and the flat parameter gradient."""
    o, tape = forward(theta, specs, levels, input_planes(psi, psi_b, mu, dmu, N), keep=True)
    L, do = loss_and_grad_output(o, psi, psi_b, target, dmu, vol, N)
    return L, backward(theta, specs, levels, tape, do)


def adam_step(theta, m, v, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step t >= 1), in place; returns theta."""
    m *= beta1
    m += (1.0 - beta1) * g
    v *= beta2
    v += (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    theta -= lr * mh / (np.sqrt(vh) + eps)
    return theta


def volumes(N, side):
    """Voronoi volumes d_i of the N x N vertex grid (Sec. 3): h^2 inside,
    halved on each boundary axis."""
    h = side / (N - 1)
    e = np.full(N, h)
    e[0] = e[-1] = h / 2
    return np.outer(e, e).ravel()
