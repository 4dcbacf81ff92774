"""Force bars shared by the GPU parity tests.

The oracle reports, per site, the term scale A_i: the sum of the magnitudes of the terms
each contribution to the site is made of before they cancel.  Bonds are computed in FP64
on both sides even when the pair arithmetic is FP32, and a tetrahedron's stiff harmonic
bonds make A_i large (3 K (r + b0) per site, about 2,400 at K = 400), so the FP32 bar is
taken against the non-bonded part of the scale, A_i^nb (the oracle's scale with the bonds
removed from the model), with the bonded rest held to FP64 rounding:

    |F_gpu,i - F_orc,i| <= tol A_i^nb + 1e-12 (A_i - A_i^nb).
"""
import numpy as np

import oracle


def nonbonded_model(wl, **kw):
    """The oracle model of the same workload without bonded terms (its A_i is A_i^nb)."""
    return oracle.Model(wl.with_(bond_kind=0), **kw)


def fp32_site_bar(amag, amag_nb, tol=1e-5):
    return tol * amag_nb + 1e-12 * np.maximum(amag - amag_nb, 0.0)


def assert_fp32_sites(fg, fo, amag, amag_nb, tol=1e-5, where="", axis=0):
    """Per-site FP32 bar (axis: the coordinate axis of fg/fo) and normwise tol."""
    err = np.abs(fg - fo).max(axis=axis)
    bar = fp32_site_bar(amag, amag_nb, tol)
    bad = err > bar
    ratio = (err / np.maximum(bar, 1e-300)).max()
    assert not bad.any(), f"{where}: {int(bad.sum())} sites over the FP32 bar, worst ratio {ratio:.3e}"
    if np.linalg.norm(fo) > 1e-12 * np.linalg.norm(amag):
        assert np.linalg.norm(fg - fo) <= tol * np.linalg.norm(fo), where
    return float(ratio)
