"""Learned effective action: a small convolutional network added to the
linear effective model ("Formalism of SLDQMC": the "..." of Eq. 2, more-body
interactions beyond the pair couplings J).  FP64 reference of its forward
pass, gradient, Adam step and single-flip change.  Test infrastructure only.

Architecture (on the field viewed as [L][Ly][Lx], periodic in all three axes):
    a1[c]  = b1[c] + sum_{d in 3^3} W1[c][d] s[x + d - 1]            (8 channels)
    h1     = tanh(a1)
    a2[c]  = b2[c] + sum_{c', d} W2[c][c'][d] h1[c'][x + d - 1]      (8 channels)
    h2     = tanh(a2)
    S_net  = b3 + sum_c w3[c] sum_x h2[c][x]
A second convolution followed by a global sum would collapse to a single
convolution if it were linear, hence the tanh after both.  The learned action
is S_theta = S_lin + S_net; S_net is trained on the residual of the linear
fit with the mean squared error.

Parameter vector (1969 entries), in this order:
    W1 [8][3][3][3], b1 [8], W2 [8][8][3][3][3], b2 [8], w3 [8], b3
with the kernel offset (dt, dy, dx) in {0,1,2} meaning a displacement of
(dt-1, dy-1, dx-1) along (time, y, x).
"""
from __future__ import annotations

import numpy as np

C = 8
N_PARAMS = C * 27 + C + C * C * 27 + C + C + 1


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + C * 27].reshape(C, 3, 3, 3); o += C * 27
    b1 = p[o:o + C]; o += C
    W2 = p[o:o + C * C * 27].reshape(C, C, 3, 3, 3); o += C * C * 27
    b2 = p[o:o + C]; o += C
    w3 = p[o:o + C]; o += C
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, w3, [b3]])


def _shift(x, d):
    """y[..., t, y, x] = x[..., t + dt - 1, y + dy - 1, x + dx - 1] (periodic)."""
    dt, dy, dx = d
    return np.roll(x, shift=(1 - dt, 1 - dy, 1 - dx), axis=(-3, -2, -1))


OFFSETS = [(dt, dy, dx) for dt in range(3) for dy in range(3) for dx in range(3)]


def forward(params, model, s):
    """(S_net, cache) for one field s int8 [L][N]."""
    W1, b1, W2, b2, w3, b3 = unpack(params)
    x = np.asarray(s, dtype=np.float64).reshape(model.n_slices, model.ly, model.lx)
    a1 = np.zeros((C,) + x.shape)
    for d in OFFSETS:
        sx = _shift(x, d)
        for c in range(C):
            a1[c] += W1[c][d] * sx
    a1 += b1[:, None, None, None]
    h1 = np.tanh(a1)
    a2 = np.zeros_like(a1)
    for d in OFFSETS:
        sh = _shift(h1, d)
        for c in range(C):
            a2[c] += np.tensordot(W2[c, :, d[0], d[1], d[2]], sh, axes=1)
    a2 += b2[:, None, None, None]
    h2 = np.tanh(a2)
    pool = h2.sum(axis=(1, 2, 3))
    S = float(b3 + w3 @ pool)
    return S, (x, h1, h2, pool)


def gradient(params, model, s, g_S):
    """d(g_S * S_net)/d params for one field (g_S = dLoss/dS_net)."""
    W1, b1, W2, b2, w3, b3 = unpack(params)
    _, (x, h1, h2, pool) = forward(params, model, s)
    gw3 = g_S * pool
    gb3 = g_S
    dz2 = g_S * w3[:, None, None, None] * (1.0 - h2 * h2)
    gb2 = dz2.sum(axis=(1, 2, 3))
    gW2 = np.zeros_like(W2)
    dh1 = np.zeros_like(h1)
    for d in OFFSETS:
        sh = _shift(h1, d)
        gW2[:, :, d[0], d[1], d[2]] = np.einsum("ctyx,ktyx->ck", dz2, sh)
        # a2[c](x) uses h1[c'](x + d - 1): scatter dz2 back to x + d - 1
        back = np.roll(dz2, shift=(d[0] - 1, d[1] - 1, d[2] - 1), axis=(1, 2, 3))
        dh1 += np.einsum("ck,ctyx->ktyx", W2[:, :, d[0], d[1], d[2]], back)
    dz1 = dh1 * (1.0 - h1 * h1)
    gb1 = dz1.sum(axis=(1, 2, 3))
    gW1 = np.zeros_like(W1)
    for d in OFFSETS:
        sx = _shift(x, d)
        gW1[:, d[0], d[1], d[2]] = np.einsum("ctyx,tyx->c", dz1, sx)
    return pack(gW1, gb1, gW2, gb2, gw3, gb3)


def loss_and_gradient(params, model, fields, targets):
    """Mean squared error of S_net against targets over a batch, and its gradient."""
    n = len(fields)
    loss = 0.0
    grad = np.zeros(N_PARAMS)
    for s, y in zip(fields, targets):
        S, _ = forward(params, model, s)
        r = S - float(y)
        loss += r * r / n
        grad += gradient(params, model, s, 2.0 * r / n)
    return loss, grad


def adam(params, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015) with bias correction; t counts from 1."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def flip_delta(params, model, s, i, l):
    """S_net(s with s_{i,l} flipped) - S_net(s), by two forward passes."""
    s2 = np.array(s, copy=True)
    s2[l - 1, i] = -s2[l - 1, i]
    return forward(params, model, s2)[0] - forward(params, model, s)[0]
