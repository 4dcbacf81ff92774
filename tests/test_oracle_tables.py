"""Pins of the oracle's tabulated CG force (oracle/tables.py, the C oracle's table lookup),
of the learned force's table fallback below r_min, and of the FP8 variant's scales.

Each check compares against something other than the code under test: values of a
hand-built table worked out by hand, the analytic WCA force within the cubic Hermite
interpolation error bound h^4/384 max|f''''| (plus the FP32 rounding of the
coefficients), the analytic-WCA oracle forces (the CG limit, w = 0), and scales of
hand-built networks whose silu maxima are known closed-form numbers.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import mlp, tables
from paper_1806_10841_amd import inputs

SIG_CG, EPS_CG = 2.31, 1.0
RC_CG = SIG_CG * 2.0 ** (1.0 / 6.0)
LO, HI, NK = 1.5, 3.0, 2048


# ------------------------------------------------------------------ hand-built table
# three knots on [1, 3] (h = 1), interval 0: 1 + 2t + 3t^2 + 4t^3, interval 1: 5 + 6t + 7t^2 + 8t^3
HAND = np.array([[1, 2, 3, 4], [5, 6, 7, 8]], dtype=np.float32)
HAND_CASES = [
    # r, value worked out by hand, table-range flag
    (1.0, 1.0, 0),      # first knot: interval 0, t = 0
    (1.5, 3.25, 0),     # interval 0, t = 1/2: 1 + 1 + 0.75 + 0.5
    (2.0, 5.0, 0),      # the middle knot starts interval 1
    (2.5, 10.75, 0),    # interval 1, t = 1/2: 5 + 3 + 1.75 + 1
    (3.0, 26.0, 0),     # last knot: clamped to interval 1 (n - 2), t = 1
    (3.5, 56.75, 0),    # beyond the last knot: the last cubic continued, t = 3/2
    (0.5, 0.25, oracle.TABLE_RANGE),   # below the first knot: interval 0 at t = -1/2, flagged
]


@pytest.mark.parametrize("r,want,flag", HAND_CASES)
def test_table_eval_hand_built(r, want, flag):
    got, st = oracle.table_eval(HAND, 1.0, 3.0, [r])
    assert got[0] == want
    assert st == flag
    # the NumPy evaluation used by the host-side checks follows the same definition
    assert tables.eval_table_fp64(HAND, 1.0, 3.0, np.array([r]))[0] == want


def _wca_force(r, sig=SIG_CG, eps=EPS_CG, rc=RC_CG):
    """Analytic WCA force magnitude of the plain method's CG potential (repulsive > 0)."""
    s6 = (sig / r) ** 6
    return np.where(r < rc, 24.0 * eps * s6 * (2.0 * s6 - 1.0) / r, 0.0)


def _slope_at(r, sig=SIG_CG, eps=EPS_CG):
    s6 = (sig / r) ** 6
    return 24.0 * eps * s6 * (7.0 - 26.0 * s6) / (r * r)


def _wca_d4_bound(r, sig=SIG_CG, eps=EPS_CG):
    """Upper bound of the fourth derivative's magnitude on [r, inf) for
    f = 24 eps (2 sig^12 r^-13 - sig^6 r^-7): the fourth derivatives of r^-13 and r^-7 are
    43680 r^-17 and 5040 r^-11, both decreasing in r."""
    return 24.0 * eps * (2.0 * sig ** 12 * 43680.0 / r ** 17 + sig ** 6 * 5040.0 / r ** 11)


def _table_error_bound(coef, lo, hi, r, sig, eps, rc):
    """Bound on |table(r) - f_WCA(r)| for r < rc: the cubic Hermite error h^4/384 times the
    largest fourth derivative on r's interval plus the FP32 rounding of its coefficients
    (2^-24 |c_i|, t in [0, 1]); on the interval holding or ending at the cutoff (a kink, or
    a jump of a force cut without a shift), |f| plus h |f'| at its left knot."""
    n = coef.shape[0] + 1
    h = (hi - lo) / (n - 1)
    k = np.clip(np.floor((np.asarray(r) - lo) / h), 0, n - 2).astype(np.int64)
    rk = lo + h * k
    c = np.abs(coef.astype(np.float64)[k]).sum(axis=1)
    b = h ** 4 / 384.0 * _wca_d4_bound(rk, sig, eps) + 2.0 ** -24 * c * 1.0001
    kink = rk + h * (1.0 + 1e-9) >= rc
    jump = np.abs(_wca_force(rk, sig, eps, rc)) + h * np.abs(_slope_at(rk, sig, eps))
    return np.where(kink, jump + 2.0 ** -24 * c * 1.0001, b)


def test_hermite_wca_table_within_interpolation_bound():
    """The 2048-knot table both sides receive reproduces the analytic WCA force within the
    cubic Hermite error bound on every interval below the cutoff, plus the FP32 rounding of
    its coefficients; it is exactly zero beyond the interval holding the cutoff."""
    coef, lo, hi = tables.hermite_wca_table(SIG_CG, EPS_CG, RC_CG, LO, HI, NK)
    h = (hi - lo) / (NK - 1)
    knots = lo + h * np.arange(NK)
    k_cut = int(np.floor((RC_CG - lo) / h))          # the interval holding the cutoff (kink)
    tt = np.linspace(0.0, 1.0, 9)[:-1]
    worst = 0.0
    for k in range(NK - 1):
        r = knots[k] + h * tt
        got, st = oracle.table_eval(coef, lo, hi, r)
        assert st == 0
        want = _wca_force(r)
        if k <= k_cut:
            bound = _table_error_bound(coef, lo, hi, r, SIG_CG, EPS_CG, RC_CG)
            err = np.abs(got - want)
            assert np.all(err <= bound), (k, err.max(), bound.max())
            if k < k_cut:
                worst = max(worst, (err / bound).max())
        else:
            assert np.all(got == 0.0), k
    assert worst > 1e-2   # the bound is not vacuous at this knot spacing


def _cg_pair_bounds(wl, x, coef):
    """Per-site sum over CG-interacting pairs (r < rc_cg) of (1 - ww) times the table's
    error bound at the pair's distance, shared by mass fraction (equal masses)."""
    m = oracle.Model(wl)
    com, w, _, _ = m.weights(x)
    nbs = m.neighbours_of(com, np.arange(wl.n_mol), r_list=wl.rc_cg)
    box = np.asarray(wl.box)
    out = np.zeros(wl.n_mol)
    for a, nb in enumerate(nbs):
        if len(nb) == 0:
            continue
        d = com[:, nb] - com[:, a:a + 1]
        d -= box[:, None] * np.round(d / box[:, None])
        r = np.sqrt((d * d).sum(axis=0))
        b = _table_error_bound(coef, LO, HI, r, wl.sig_cg, wl.eps_cg, wl.rc_cg)
        out[a] = ((1.0 - w[a] * w[nb]) * b).sum() / wl.sites_per_mol
    return np.repeat(out, wl.sites_per_mol)


def test_cg_table_forces_equal_analytic_wca():
    """w = 0 everywhere (pure CG): Eq. (1) forces with the WCA table as F^CG equal the
    oracle's analytic-WCA forces within the table's error, summed over each site's pairs
    at their own distances; the CG potential of a table is not defined, so only forces
    are compared."""
    wl = inputs.workload("small_cg").with_(cg_kind=inputs.CG_WCA)
    x, _ = inputs.make_state(wl)
    table = tables.hermite_wca_table(wl.sig_cg, wl.eps_cg, wl.rc_cg, LO, HI, NK)
    f_tab, _, _, st = oracle.Model(wl.with_(cg_kind=inputs.CG_TABLE), table=table).forces(x)
    assert st == 0
    f_wca, _, _, st = oracle.Model(wl).forces(x)
    assert st == 0
    bound = _cg_pair_bounds(wl, x, table[0])
    d = np.abs(f_tab - f_wca).max(axis=0)
    assert np.all(d <= bound + 1e-13 * np.abs(f_wca).max(axis=0)), (d / bound).max()
    # and not trivially: for the typical site the bound is far below the force itself
    assert np.median(bound) < 1e-5 * np.median(np.abs(f_wca).max(axis=0))


def test_hybrid_table_forces_differ_only_in_cg_part():
    """With a hybrid layer, replacing the analytic CG force by its table changes each site's
    force by at most (1 - ww) times the table error per pair: the AT part is untouched, and
    a site whose pairs are all atomistic (ww = 1) would see no change at all."""
    wl = inputs.workload("small_slab").with_(pair_precision=64)
    x, _ = inputs.make_state(wl)
    table = tables.hermite_wca_table(wl.sig_cg, wl.eps_cg, wl.rc_cg, LO, HI, NK)
    f_tab, _, _, st = oracle.Model(wl.with_(cg_kind=inputs.CG_TABLE), table=table).forces(x)
    assert st == 0
    f_wca, _, _, _ = oracle.Model(wl).forces(x)
    bound = _cg_pair_bounds(wl, x, table[0])
    d = np.abs(f_tab - f_wca).max(axis=0)
    assert np.all(d <= bound + 1e-13 * np.abs(f_wca).max(axis=0)), (d / np.maximum(bound, 1e-300)).max()
    assert (d[bound == 0] == 0).all()
    # the bound is not vacuous: the changes reach a sizeable part of it somewhere
    assert (d / np.maximum(bound, 1e-300)).max() > 1e-3


# ------------------------------------------------------------------ learned force fallback
def test_mlp_eval_uses_table_below_r_min():
    """The learned CG force falls back to the table strictly below r_min (the reading
    of the fallback): equal bits to the table lookup there, the FP64 network at and above
    r_min, and the network everywhere when no table is installed."""
    p = inputs.mlp_init(5)
    rc, scale, tw, r_min = 3.0, 7.0, 0.5, 2.2
    wl = inputs.workload("small_cg").with_(cg_kind=inputs.CG_MLP)
    r_lo = np.array([1.5, 1.9, 2.0, 2.19999])
    r_hi = np.array([2.2, 2.5, 2.9])
    m = oracle.Model(wl, table=(HAND, 1.0, 3.0), mlp=(p, rc, scale, tw, r_min))
    got_lo = m.mlp_eval(r_lo)
    np.testing.assert_array_equal(got_lo, oracle.table_eval(HAND, 1.0, 3.0, r_lo)[0])
    got_hi = m.mlp_eval(r_hi)
    np.testing.assert_allclose(got_hi, mlp.forward(p, r_hi, rc, scale, tw), rtol=1e-13, atol=1e-13)
    # no table: the network below r_min as well
    m0 = oracle.Model(wl, mlp=(p, rc, scale, tw, r_min))
    np.testing.assert_allclose(m0.mlp_eval(r_lo), mlp.forward(p, r_lo, rc, scale, tw), rtol=1e-13, atol=1e-13)
    # the hand table's own values at two of the points (interval 0 and interval 1)
    assert got_lo[0] == 3.25 and got_lo[2] == 5.0


# ------------------------------------------------------------------ FP8 scales
SILU_2 = 1.7615941559557649     # 2 / (1 + e^-2)
SILU_3 = 2.8577223804673        # 3 / (1 + e^-3)
SILU_MIN = -0.27846454276107380  # the minimum of silu (at z = -1.27846)


def _hand_network(w1, b1, w2):
    H = 64
    W1, B1, W2 = np.zeros(H), np.zeros(H), np.zeros((H, H))
    for k, v in w1.items():
        W1[k] = v
    for k, v in b1.items():
        B1[k] = v
    for (i, j), v in w2.items():
        W2[i, j] = v
    return mlp.pack(W1, B1, W2, np.zeros(H), np.ones(H), np.zeros(1))


@pytest.mark.parametrize("w1,b1,g", [
    ({}, {5: 2.0}, SILU_2),              # largest |h1| at x = 0: silu(b1)
    ({7: 3.0}, {}, SILU_3),              # largest |h1| at x = 1: silu(W1 + b1)
    ({7: 3.0}, {5: 2.0}, SILU_3),        # both present: the larger
    ({}, {}, 0.2785),                    # all h1 small: the floor above |min silu|
    ({3: -1.0}, {3: -0.3}, 0.2785),      # a negative unit never exceeds the floor
])
def test_fp8_scales_hand_networks(w1, b1, g):
    """s_w = max|W2| / 448 and s_g = 1.01 G_h / (448 ln 2), G_h the largest |h1| over
    x in [0, 1] (silu is monotone above its minimum, so it is taken at x = 0 or 1, or is
    the floor 0.2785 >= |min silu|)."""
    p = _hand_network(w1, b1, {(1, 2): -3.5, (4, 0): 2.0})
    s_w, s_g = mlp.fp8_scales(p)
    assert s_w == 3.5 / 448.0
    assert abs(s_g - 1.01 * g / (448.0 * math.log(2.0))) <= 1e-15 * s_g
    assert 0.2785 > abs(SILU_MIN)
    # the scaled h1 / ln 2 of the network stays inside E4M3's range on a dense grid of x
    W1, B1 = mlp.unpack(p)[:2]
    xs = np.linspace(0.0, 1.0, 2001)
    h1 = mlp.silu(xs[:, None] * W1[None, :] + B1[None, :])
    assert np.abs(h1).max() / math.log(2.0) / s_g <= 448.0


def test_fp8_scale_of_zero_weights():
    p = _hand_network({}, {}, {})
    s_w, _ = mlp.fp8_scales(p)
    assert s_w == 1.0


def test_silu_constants():
    # the closed-form numbers above, from the definition silu(z) = z / (1 + e^-z)
    assert abs(SILU_2 - 2.0 / (1.0 + math.exp(-2.0))) < 1e-15
    assert abs(SILU_3 - 3.0 / (1.0 + math.exp(-3.0))) < 1e-13
    z = -1.2784645427610738
    assert abs(mlp.silu(np.array([z]))[0] - SILU_MIN) < 1e-15
    assert abs(mlp.silu_grad(np.array([z]))[0]) < 1e-12
