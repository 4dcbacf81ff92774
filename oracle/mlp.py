"""FP64 oracle of the learned coarse-grained pair force -- TEST INFRASTRUCTURE ONLY.

The learned CG force replaces F^CG of Eq. (1) (Sec. 2.2: a force between centres
of mass) by a small network of the centre distance r:

    f(r) = s * taper(r) * [ W3 . silu(W2 silu(W1 x + b1) + b2) + b3 ],   x = r / rc,

positive = repulsive, acting along R_ab / r; taper(r) = 1 below rc - tw and a
cos^2 ramp to 0 at rc (the same squared-cosine shape as the resolution function
of Sec. 2.3); below r_min a cubic table is used instead (the table is the
fallback).  silu(z) = z / (1 + e^-z).

It is trained by force matching (multiscale coarse-graining, Izvekov & Voth 2005,
a published method not described in the paper): for frames of centres R_I and
mapped forces F^map_I (the sum of the atomistic non-bonded forces on molecule I;
bonds cancel inside the sum), the prediction F_I = sum_J f(r_IJ) (R_I - R_J)/r_IJ
and the loss chi2 = 1/(3 N_f N) sum_frames sum_I |F_I - F^map_I|^2.  For an
unordered pair {I, J} the loss gradient w.r.t. f(r_IJ) is
g_IJ = 2/(3 N_f N) (e_I - e_J) . R_hat_IJ with e = F - F^map.

Parameter layout (float64 vector, H = 64): W1[H], b1[H], W2[H*H] (row = output
unit), b2[H], W3[H], b3[1].  Written with plain NumPy matmuls, no fusion.

FP8 variant (``forward_fp8``): the second layer's inputs h1 and weights W2 rounded to
FP8 E4M3 (OCP format: 4 exponent bits, bias 7, 3 mantissa bits, largest finite 448,
subnormal step 2^-9, round to nearest even) after division by per-tensor scales
s_w = max|W2| / 448 and s_g = G / 448, with G = 1.01 max(0.2785, max_u |silu(b1_u)|,
max_u |silu(W1_u + b1_u)|) / ln 2 a bound on |h1| / ln 2 over x in [0, 1] (silu is
monotone above its minimum -0.27846); the product is scaled back by s_w s_g.
Pinned by central finite differences and closed-form special cases
(tests/test_oracle_mlp.py).
"""
from __future__ import annotations

import numpy as np


def unpack(params, H=64):
    p = np.asarray(params, dtype=np.float64)
    o = 0
    W1 = p[o:o + H]; o += H
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + H]; o += H
    b3 = p[o:o + 1]; o += 1
    assert o == p.size
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([W1, b1, W2.ravel(), b2, W3, np.atleast_1d(b3)])


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * sigmoid(z)


def silu_grad(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def e4m3_round(x):
    """Round to the nearest FP8 E4M3 (OCP) value, ties to even; |x| <= 448 is required."""
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    with np.errstate(divide="ignore"):
        e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    e = np.maximum(e, -6.0)                  # below 2^-6: subnormals, fixed step 2^-9
    step = 2.0 ** (e - 3)
    q = np.round(a / step) * step            # np.round rounds halves to even
    assert np.all(q <= 448.0), "value beyond the E4M3 range"
    return np.sign(x) * q


def fp8_scales(params, H=64):
    """(s_w, s_g) of the FP8 variant (see the module docstring)."""
    W1, b1, W2, b2, W3, b3 = unpack(params, H)
    g = max(0.2785, float(np.abs(silu(b1)).max()), float(np.abs(silu(W1 + b1)).max()))
    G = 1.01 * g / np.log(2.0)
    wmax = float(np.abs(W2).max())
    return (wmax / 448.0 if wmax > 0 else 1.0), G / 448.0


def forward_fp8(params, r, rc, scale, tw, H=64):
    """f(r) of the FP8 variant: h1 and W2 in E4M3 with per-tensor scales, the rest FP64."""
    W1, b1, W2, b2, W3, b3 = unpack(params, H)
    s_w, s_g = fp8_scales(params, H)
    x = np.asarray(r, dtype=np.float64) / rc
    h1 = silu(x[:, None] * W1[None, :] + b1[None, :])
    g = e4m3_round(h1 / np.log(2.0) / s_g)             # the scaled |h1| / ln 2, quantised
    Wq = e4m3_round(W2 / s_w)
    z2 = (g @ Wq.T) * (s_w * s_g) * np.log(2.0) + b2[None, :]
    y = silu(z2) @ W3 + b3[0]
    return scale * taper(r, rc, tw) * y


def taper(r, rc, tw):
    """1 below rc - tw, cos^2(pi/2 (r - (rc - tw))/tw) on the ramp, 0 at and beyond rc."""
    r = np.asarray(r, dtype=np.float64)
    u = (r - (rc - tw)) / tw
    out = np.cos(0.5 * np.pi * np.clip(u, 0.0, 1.0)) ** 2
    out = np.where(u <= 0.0, 1.0, out)
    return np.where(u >= 1.0, 0.0, out)


def network(params, r, rc, H=64):
    """y(r) of the bare network (before scale and taper) and the cache for backward."""
    W1, b1, W2, b2, W3, b3 = unpack(params, H)
    x = np.asarray(r, dtype=np.float64) / rc
    z1 = x[:, None] * W1[None, :] + b1[None, :]
    h1 = silu(z1)
    z2 = h1 @ W2.T + b2[None, :]
    h2 = silu(z2)
    y = h2 @ W3 + b3[0]
    return y, (x, z1, h1, z2, h2)


def forward(params, r, rc, scale, tw, H=64):
    """f(r) = scale * taper(r) * y(r) (no table fallback; callers pick r >= r_min)."""
    y, _ = network(params, r, rc, H)
    return scale * taper(r, rc, tw) * y


def backward(params, r, dLdf, rc, scale, tw, H=64):
    """Gradient of sum_p dLdf_p f(r_p) w.r.t. the parameters (analytic, float64 vector)."""
    W1, b1, W2, b2, W3, b3 = unpack(params, H)
    y, (x, z1, h1, z2, h2) = network(params, r, rc, H)
    dy = np.asarray(dLdf, dtype=np.float64) * scale * taper(r, rc, tw)   # dL/dy per pair
    gW3 = h2.T @ dy
    gb3 = np.array([dy.sum()])
    dz2 = (dy[:, None] * W3[None, :]) * silu_grad(z2)
    gW2 = dz2.T @ h1                      # (out, in)
    gb2 = dz2.sum(axis=0)
    dh1 = dz2 @ W2
    dz1 = dh1 * silu_grad(z1)
    gW1 = dz1.T @ x
    gb1 = dz1.sum(axis=0)
    return pack(gW1, gb1, gW2, gb2, gW3, gb3)


def pairs_within(com, box, rc):
    """Unordered centre pairs (I < J) with minimum-image distance < rc, brute force.
    Returns (I, J, r, rhat) with rhat = (R_I - R_J)/r."""
    com = np.asarray(com, dtype=np.float64)
    n = com.shape[1]
    box = np.asarray(box, dtype=np.float64)
    I, J = np.triu_indices(n, k=1)
    d = com[:, I] - com[:, J]
    d -= box[:, None] * np.round(d / box[:, None])
    r = np.sqrt((d * d).sum(axis=0))
    m = r < rc
    return I[m], J[m], r[m], d[:, m] / r[m][None, :]


def predicted_forces(params, com, box, rc, scale, tw, H=64, pairs=None, r_min=0.0, table=None):
    """F_I = sum_J f(r_IJ) R_hat_IJ on every centre (3, N)."""
    I, J, r, rhat = pairs if pairs is not None else pairs_within(com, box, rc)
    f = forward(params, r, rc, scale, tw, H)
    if table is not None:
        from oracle.tables import eval_table_fp64
        low = r < r_min
        if low.any():
            f = f.copy()
            f[low] = eval_table_fp64(table[0], table[1], table[2], r[low])
    n = com.shape[1]
    F = np.zeros((3, n))
    for d in range(3):
        np.add.at(F[d], I, f * rhat[d])
        np.add.at(F[d], J, -f * rhat[d])
    return F


def fm_loss_and_grad(params, frames, box, rc, scale, tw, H=64, r_min=0.0, table=None):
    """Force-matching loss and its gradient over frames = [(com (3,N), fmap (3,N)), ...].
    Pairs below r_min take the table's force (when a table is given) and carry no
    gradient."""
    n_f = len(frames)
    grad = np.zeros_like(np.asarray(params, dtype=np.float64))
    loss = 0.0
    for com, fmap in frames:
        n = com.shape[1]
        c = 1.0 / (3.0 * n_f * n)
        I, J, r, rhat = pairs_within(com, box, rc)
        F = predicted_forces(params, com, box, rc, scale, tw, H, pairs=(I, J, r, rhat), r_min=r_min, table=table)
        keep = r >= r_min
        I, J, r, rhat = I[keep], J[keep], r[keep], rhat[:, keep]
        e = F - fmap
        loss += c * float((e * e).sum())
        g = 2.0 * c * ((e[:, I] - e[:, J]) * rhat).sum(axis=0)
        grad += backward(params, r, g, rc, scale, tw, H)
    return loss, grad


def adam_step(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015), step counted from 1; returns new (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
