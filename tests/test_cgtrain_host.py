"""Host-side helpers of the learned-vs-tabulated comparison (no GPU): the force-matched
table fit recovers a known pair force from frames whose forces that pair force made
(the least-squares problem is then consistent, so lstsq must return it up to the
spline's resolution), tiling, and the pair-distance helper."""
import numpy as np

import oracle
from paper_1806_10841_amd import cgtrain


def _ftrue(r):
    return np.where(r < 3.0, 5.0 * np.exp(-2.0 * (r - 1.0)) * (3.0 - r) ** 2, 0.0)


def test_fit_table_recovers_pair_force():
    rng = np.random.default_rng(0)
    box = (12.0, 12.0, 12.0)
    coms, fms = [], []
    for _ in range(3):
        c = rng.uniform(0.0, 12.0, size=(3, 200))
        I, J, r, rh = cgtrain._pairs(c, box, 3.0)
        F = np.zeros((3, 200))
        for d in range(3):
            np.add.at(F[d], I, _ftrue(r) * rh[d])
            np.add.at(F[d], J, -_ftrue(r) * rh[d])
        coms.append(c)
        fms.append(F)
    coef, lo, hi = cgtrain.fit_table(np.array(coms), np.array(fms), box, r_fit_lo=0.3, r_lo=0.2)
    assert (lo, hi) == (0.2, 3.0) and coef.shape == (2047, 4)
    rr = np.linspace(0.6, 2.9, 50)
    v, st = oracle.table_eval(coef, lo, hi, rr)
    assert st == 0
    assert np.abs(v - _ftrue(rr)).max() <= 1e-3 * np.abs(_ftrue(rr)).max()
    # zero at the cutoff, and a wall (non-decreasing towards r -> r_lo) below the data
    v_end, _ = oracle.table_eval(coef, lo, hi, [2.99999])
    assert abs(v_end[0]) < 1e-3
    vl, _ = oracle.table_eval(coef, lo, hi, np.linspace(0.2, 0.3, 11))
    assert np.all(np.diff(vl) <= 1e-6)


def test_tile_frame_and_min_distance():
    rng = np.random.default_rng(1)
    box = (5.0, 6.0, 7.0)
    c = rng.uniform(0.0, 1.0, size=(3, 10)) * np.asarray(box)[:, None]
    t, box2 = cgtrain.tile_frame(c, box, (2, 2, 1))
    assert box2 == (10.0, 12.0, 7.0) and t.shape == (3, 40)
    np.testing.assert_array_equal(t[:, 10:20], c + np.array([[0.0], [6.0], [0.0]]))
    # brute-force minimum image distance
    d = c[:, :, None] - c[:, None, :]
    d -= np.asarray(box)[:, None, None] * np.round(d / np.asarray(box)[:, None, None])
    r = np.sqrt((d ** 2).sum(axis=0))[np.triu_indices(10, 1)]
    rmin = cgtrain.min_pair_distance(c[None], box, rc=3.0)
    assert abs(rmin - r[r < 3.0].min()) < 1e-12
