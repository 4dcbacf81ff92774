"""Host checks of the seeded input generators (no GPU): rigid bodies of 2 and 3 sites
keep unit bonds, sit on the lattice points they were placed at, and fill the workload's
site arrays."""
import itertools

import numpy as np
import pytest

from paper_1806_10841_amd import inputs


@pytest.mark.parametrize("spm", [2, 3])
def test_small_bodies_are_unit_edge_and_centred(spm):
    rng = np.random.default_rng(3)
    com = rng.uniform(0.0, 10.0, size=(3, 50))
    x = inputs.body_positions(com, spm, rng)
    assert x.shape == (3, 50 * spm)
    sites = x.T.reshape(50, spm, 3)
    for a, b in itertools.combinations(range(spm), 2):
        d = np.linalg.norm(sites[:, a] - sites[:, b], axis=1)
        np.testing.assert_allclose(d, 1.0, rtol=0, atol=1e-14)
    np.testing.assert_allclose(sites.mean(axis=1), com.T, rtol=0, atol=1e-13)


@pytest.mark.parametrize("name", ["small_dumbbell", "small_triangle"])
def test_shape_workloads_fill_their_arrays(name):
    wl = inputs.workload(name)
    x, v = inputs.make_state(wl)
    assert x.shape == v.shape == (3, wl.n_mol * wl.sites_per_mol)
    assert (x >= 0).all() and (x < np.asarray(wl.box)[:, None]).all()
    np.testing.assert_allclose(v.sum(axis=1), 0.0, atol=1e-10)     # equal masses: zero momentum
