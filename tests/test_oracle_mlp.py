"""Pins of the FP64 oracle of the learned CG force (oracle/mlp.py) and of the C
oracle's network evaluation: finite differences, closed-form special cases,
library routines (scipy's periodic k-d tree) and invariants."""
import math

import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle
from oracle import mlp
from paper_1806_10841_amd import inputs

RC, TW, SCALE = 3.0, 0.5, 7.0


def _params(seed=0):
    return inputs.mlp_init(seed)


def test_silu_and_derivative():
    z = np.linspace(-8, 8, 41)
    assert np.allclose(mlp.silu(np.array([0.0, 50.0, -50.0])), [0.0, 50.0, 0.0], atol=1e-12)
    h = 1e-6
    fd = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.silu_grad(z))) < 1e-8


def test_taper_values():
    assert mlp.taper(np.array([RC - TW - 0.1, RC - TW]), RC, TW).tolist() == [1.0, 1.0]
    assert mlp.taper(np.array([RC, RC + 1]), RC, TW).tolist() == [0.0, 0.0]
    assert abs(mlp.taper(np.array([RC - TW / 2]), RC, TW)[0] - 0.5) < 1e-15


def test_closed_form_special_networks():
    p = _params(1)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p)
    # W2 = 0, b2 = 0: second hidden layer is silu(0) = 0, so f = scale * taper * b3
    q = mlp.pack(W1, b1, np.zeros_like(W2), np.zeros_like(b2), W3, np.array([0.37]))
    r = np.array([1.2, 2.0, 2.6, 2.9])
    np.testing.assert_allclose(mlp.forward(q, r, RC, SCALE, TW), SCALE * 0.37 * mlp.taper(r, RC, TW), rtol=1e-15)
    # b2 = 40 dominates: silu(40 + small) = 40 + small to 1e-16, so y = W3 . (W2 h1 + 40) + b3
    q = mlp.pack(W1, b1, 1e-3 * W2, np.full_like(b2, 40.0), W3, np.array([0.0]))
    x = r / RC
    h1 = (x[:, None] * W1 + b1) / (1 + np.exp(-(x[:, None] * W1 + b1)))
    y = (h1 @ (1e-3 * W2).T + 40.0) @ W3
    np.testing.assert_allclose(mlp.forward(q, r, RC, 1.0, TW) / mlp.taper(r, RC, TW).clip(1e-300), y, rtol=1e-12)


def test_backward_matches_finite_differences():
    p = _params(2)
    rng = np.random.default_rng(0)
    r = rng.uniform(1.4, 3.0, size=50)
    dldf = rng.normal(size=50)
    g = mlp.backward(p, r, dldf, RC, SCALE, TW)
    L = lambda q: float(dldf @ mlp.forward(q, r, RC, SCALE, TW))
    idx = np.concatenate([rng.choice(p.size, 40, replace=False), [p.size - 1, 0, 64, 128]])
    for i in idx:
        h = 1e-6 * max(1.0, abs(p[i]))
        e = np.zeros_like(p); e[i] = h
        fd = (L(p + e) - L(p - e)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def _cg_frame(n_side=6, seed=3):
    L = n_side * (1 / 0.1) ** (1 / 3)
    box = (L, L, L)
    rng = np.random.default_rng(seed)
    com = inputs.lattice_points((n_side,) * 3, box, rng, jitter=0.4)
    fmap = rng.normal(size=com.shape) * 5.0
    return com, fmap, box


def test_pairs_within_matches_kdtree():
    com, _, box = _cg_frame()
    I, J, r, rhat = mlp.pairs_within(com, box, RC)
    ref = np.array(sorted(cKDTree(com.T, boxsize=np.array(box)).query_pairs(RC)))
    np.testing.assert_array_equal(np.stack([I, J], axis=1), ref)
    assert np.allclose(np.linalg.norm(rhat, axis=0), 1.0)


def test_fm_gradient_matches_finite_differences():
    com, fmap, box = _cg_frame()
    frames = [(com, fmap), (com[:, ::-1].copy(), fmap[:, ::-1].copy())]
    p = _params(4)
    loss, g = mlp.fm_loss_and_grad(p, frames, box, RC, SCALE, TW)
    rng = np.random.default_rng(1)
    for i in np.concatenate([rng.choice(p.size, 25, replace=False), [p.size - 1]]):
        h = 1e-6 * max(1.0, abs(p[i]))
        e = np.zeros_like(p); e[i] = h
        lp, _ = mlp.fm_loss_and_grad(p + e, frames, box, RC, SCALE, TW)
        lm, _ = mlp.fm_loss_and_grad(p - e, frames, box, RC, SCALE, TW)
        fd = (lp - lm) / (2 * h)
        # central-difference rounding noise is ~eps * loss / h
        assert abs(fd - g[i]) <= 1e-6 * abs(g[i]) + 1e-9 * loss, (i, fd, g[i])


def test_fm_loss_of_zero_network():
    """f == 0: the loss is the mean squared mapped-force component."""
    com, fmap, box = _cg_frame()
    p = _params(5)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p)
    z = mlp.pack(W1, b1, W2, b2, np.zeros_like(W3), np.zeros(1))
    loss, g = mlp.fm_loss_and_grad(z, [(com, fmap)], box, RC, SCALE, TW)
    assert abs(loss - float((fmap ** 2).sum()) / (3 * com.shape[1])) < 1e-12 * loss


def test_predicted_forces_newton3():
    com, _, box = _cg_frame()
    F = mlp.predicted_forces(_params(6), com, box, RC, SCALE, TW)
    assert np.max(np.abs(F.sum(axis=1))) < 1e-12 * np.abs(F).sum()


def test_adam_first_step():
    rng = np.random.default_rng(2)
    p, g = rng.normal(size=10), rng.normal(size=10)
    q, m, v = mlp.adam_step(p, g, np.zeros(10), np.zeros(10), 1, 1e-3)
    np.testing.assert_allclose(q, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_c_oracle_network_matches_numpy():
    """The C oracle's FP64 network (used inside Eq. (1) forces) equals the NumPy one."""
    p = _params(7)
    wl = inputs.workload("small_cg").with_(cg_kind=inputs.CG_MLP, rc_cg=RC)
    m = oracle.Model(wl, mlp=(p, RC, SCALE, TW, 0.0))
    r = np.linspace(1.2, 3.2, 57)
    np.testing.assert_allclose(m.mlp_eval(r), mlp.forward(p, r, RC, SCALE, TW), rtol=1e-13, atol=1e-13)


def test_c_oracle_mlp_forces_are_pair_forces():
    """Eq. (1) in the w == 0 limit with the network as F^CG equals the NumPy prediction."""
    p = _params(8)
    wl = inputs.workload("small_cg").with_(cg_kind=inputs.CG_MLP, rc_cg=RC)
    x, _ = inputs.make_state(wl)
    f, amag, _, st = oracle.Model(wl, mlp=(p, RC, SCALE, TW, 0.0)).forces(x)
    assert st == 0
    Fn = mlp.predicted_forces(p, x, wl.box, RC, SCALE, TW)
    np.testing.assert_allclose(f, Fn, rtol=0, atol=1e-12 * np.abs(Fn).max())


# ---------------------------------------------------------------- FP8 E4M3 variant
def _e4m3_codes():
    """All finite non-negative E4M3 (OCP) values from the bit layout: exponent field e
    (bias 7), mantissa m; e = 0 is subnormal (m 2^-9); (e, m) = (15, 7) is NaN."""
    vals = []
    for e in range(16):
        for m in range(8):
            if e == 15 and m == 7:
                continue
            vals.append((m / 8.0) * 2.0 ** -6 if e == 0 else (1 + m / 8.0) * 2.0 ** (e - 7))
    return np.array(sorted(vals))


def test_e4m3_round_matches_enumeration():
    codes = _e4m3_codes()
    assert codes[-1] == 448.0 and codes[1] == 2.0 ** -9
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.uniform(-448, 448, 2000), rng.uniform(-0.05, 0.05, 2000),
                        (codes[1:] + codes[:-1]) / 2])          # exact ties
    got = mlp.e4m3_round(x)
    for xi, gi in zip(x, got):
        a = abs(xi)
        i = np.searchsorted(codes, a)
        lo, hi = codes[max(i - 1, 0)], codes[min(i, len(codes) - 1)]
        if a - lo < hi - a:
            ref = lo
        elif hi - a < a - lo:
            ref = hi
        else:   # tie: the code with an even mantissa (even index in the sorted list)
            ref = lo if np.searchsorted(codes, lo) % 2 == 0 else hi
        assert gi == np.copysign(ref, xi), (xi, gi, ref)


def test_e4m3_closed_form_values():
    x = [1.0, 1.0625, 1.1875, 0.1, 448.0, 2.0 ** -9, 7 * 2.0 ** -9, 2.0 ** -10, -2.5]
    ref = [1.0, 1.0, 1.25, 0.1015625, 448.0, 2.0 ** -9, 7 * 2.0 ** -9, 0.0, -2.5]
    assert mlp.e4m3_round(x).tolist() == ref


def test_forward_fp8_special_cases():
    p = _params(7)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p)
    r = np.linspace(0.5, 2.9, 50)
    # W2 = 0: layer 2 sees only its bias, so no quantisation error is possible
    q = mlp.pack(W1, b1, np.zeros_like(W2), b2, W3, b3)
    np.testing.assert_allclose(mlp.forward_fp8(q, r, RC, SCALE, TW), mlp.forward(q, r, RC, SCALE, TW),
                               rtol=1e-13, atol=1e-13)
    # in general within the E4M3 rounding of two factors (2^-4 each) through silu
    f8, f = mlp.forward_fp8(p, r, RC, SCALE, TW), mlp.forward(p, r, RC, SCALE, TW)
    assert np.linalg.norm(f8 - f) <= 0.25 * np.linalg.norm(f)
