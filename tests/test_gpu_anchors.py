"""GPU parity of the self-adjusting AT region (Sec. 2.5: spheres around anchor molecules
whose union is the AT region) against the FP64 oracle, through the C ABI.

Bars: weights to 1e-15 absolute (the only new arithmetic is the nearest-anchor distance);
forces FP64 1e-12 and FP32 1e-5 of A_i; FP64 trajectories 1e-9 in position.  The
weights of the moving region are checked on the final state of a trajectory too.
"""
import numpy as np
import pytest

import oracle
from _bars import assert_fp32_sites, nonbonded_model
from paper_1806_10841_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SPH = inputs.REGION_SPHERES


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    return torch.device("cuda:0")


def _ctx(wl, anchors):
    from paper_1806_10841_amd import binding
    c = binding.Context(wl)
    c.set_anchors(anchors)
    return c


def _t(a, dev):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)


def _wl(name, **kw):
    base = dict(region=SPH, d_at=2.5, d_hy=2.0)
    if name == "c2":
        base = dict(region=SPH, d_at=4.0, d_hy=3.0)
    base.update(kw)
    return inputs.workload(name).with_(**base)


def _assert_close(fg, fo, amag, tol, where):
    err = np.abs(fg - fo).max(axis=0)
    ratio = (err / np.maximum(amag, 1e-300)).max()
    assert ratio <= tol, f"{where}: worst ratio {ratio:.3e}"
    assert np.linalg.norm(fg - fo) <= tol * np.linalg.norm(fo), where


@pytest.mark.parametrize("name,k", [("small_sphere", 1), ("small_sphere", 9), ("small_sphere", 1024),
                                    ("c1", 5), ("c2", 300)])
def test_weights(dev, name, k):
    wl = _wl(name)
    an = inputs.anchor_molecules(wl.n_mol, k, k)
    x, _ = inputs.make_state(wl)
    com_o, w_o, _, st = oracle.Model(wl, anchors=an).weights(x)
    assert st == 0 and ((w_o > 0) & (w_o < 1)).any()
    com, w = _ctx(wl, an).weights(_t(x, dev))
    np.testing.assert_array_equal(com.cpu().numpy(), com_o)
    assert np.abs(w.cpu().numpy() - w_o).max() <= 1e-15


@pytest.mark.parametrize("d_at,d_hy,clustered", [(6.0, 4.0, False), (9.0, 5.0, False), (2.5, 2.0, True)])
def test_forces_anchor_grid_shapes(dev, d_at, d_hy, clustered):
    """The step's nearest-anchor search bins the anchors in cells at least as wide as the
    hybrid shell's end: two cells per axis (reach 10 in a 25.8 box), a single cell (reach
    14), and 64 anchors packed around the box centre (the molecules nearest to it, as the
    atoms of one macromolecule would be), many to a cell.  FP64 forces against the oracle."""
    wl = _wl("small_sphere", d_at=d_at, d_hy=d_hy)
    x, _ = inputs.make_state(wl)
    if clustered:
        L = wl.box[0]
        p = x.T.reshape(wl.n_mol, wl.sites_per_mol, 3)
        d = p - p[:, :1]
        d -= L * np.round(d / L)
        com = p[:, 0] + d.mean(axis=1)
        off = _min_image(com - np.array(wl.center), L)
        an = np.sort(np.argsort((off ** 2).sum(axis=1))[:64]).astype(np.int32)
    else:
        an = inputs.anchor_molecules(wl.n_mol, 9, 2)
    fo, amag, _, st = oracle.Model(wl, anchors=an).forces(x)
    _, w_o, _, _ = oracle.Model(wl, anchors=an).weights(x)
    assert st == 0 and ((w_o > 0) & (w_o < 1)).any()
    f = _ctx(wl, an).forces(_t(x, dev))
    torch.cuda.synchronize()
    _assert_close(f.cpu().numpy(), fo, amag, 1e-12, f"d_at {d_at} clustered {clustered}")


@pytest.mark.parametrize("name,k,prec", [("small_sphere", 9, 64), ("c1", 5, 64), ("tiny_slab", 3, 64),
                                         ("small_sphere", 9, 32)])
def test_forces(dev, name, k, prec):
    wl = _wl(name, pair_precision=prec)
    if name == "tiny_slab":
        wl = wl.with_(d_at=1.0, d_hy=2.0)
    an = inputs.anchor_molecules(wl.n_mol, k, 2)
    x, _ = inputs.make_state(wl)
    fo, amag, eo, st = oracle.Model(wl, anchors=an).forces(x)
    assert st == 0
    f, e = _ctx(wl, an).forces(_t(x, dev), energy=True)
    torch.cuda.synchronize()
    tol = 1e-12 if prec == 64 else 1e-5
    if prec == 64:
        _assert_close(f.cpu().numpy(), fo, amag, tol, name)
    else:
        _, amag_nb, _, _ = nonbonded_model(wl, anchors=an).forces(x)
        assert_fp32_sites(f.cpu().numpy(), fo, amag, amag_nb, tol, name)
    np.testing.assert_allclose(e.cpu().numpy(), eo, rtol=tol, atol=tol * np.abs(eo).max())


def _min_image(d, L):
    return d - L * np.round(d / L)


@pytest.mark.parametrize("name,k,steps", [("c1", 5, 100), ("small_sphere", 9, 40)])
def test_integrate_fp64_matches_oracle_vv(dev, name, k, steps):
    """The region follows the anchors at every step (trajectory and the final weights)."""
    wl = _wl(name, pair_precision=64)
    an = inputs.anchor_molecules(wl.n_mol, k, 7)
    x, v = inputs.make_state(wl)
    m = oracle.Model(wl, anchors=an)
    xo, vo, fo, _, st = m.vv(x, v, wl.dt, steps)
    assert st == 0
    ctx = _ctx(wl, an)
    xt, vt = _t(x, dev), _t(v, dev)
    ft = torch.empty_like(xt)
    nreb = ctx.integrate(xt, vt, ft, wl.dt, steps)
    torch.cuda.synchronize()
    tol = 1e-9
    xg = xt.cpu().numpy()
    assert np.abs(_min_image(xg - xo, wl.box[0])).max() < tol
    assert np.abs(vt.cpu().numpy() - vo).max() < 100 * tol
    if name == "c1":
        assert nreb >= 1
    _, w_o, _, _ = m.weights(xg)
    _, w = ctx.weights(xt)
    assert np.abs(w.cpu().numpy() - w_o).max() <= 1e-15


def test_c2_full_size_sampled_and_momentum(dev):
    """64,000 tetrahedra, 64 anchors, FP32 pairs: sampled molecules of each resolution
    against the oracle; then 200 steps conserve momentum (force interpolation keeps
    Newton's third law with any weights)."""
    wl = _wl("c2")
    an = inputs.anchor_molecules(wl.n_mol, 64, 5)
    x, v = inputs.make_state(wl)
    m = oracle.Model(wl, anchors=an)
    _, w, _, _ = m.weights(x)
    rng = np.random.default_rng(6)
    sel = []
    for mask in (w == 1.0, (w > 0) & (w < 1), w == 0.0):
        idx = np.flatnonzero(mask)
        assert len(idx) > 0
        sel.append(rng.choice(idx, size=min(60, len(idx)), replace=False))
    sel = np.sort(np.concatenate(sel))
    fo, amag, st = m.forces_sampled(x, sel)
    assert st == 0
    ctx = _ctx(wl, an)
    xt, vt = _t(x, dev), _t(v, dev)
    f = ctx.forces(xt).cpu().numpy()
    fg = np.stack([f[:, 4 * a:4 * a + 4] for a in sel])
    _, amag_nb, _ = nonbonded_model(wl, anchors=an).forces_sampled(x, sel)
    assert_fp32_sites(fg, fo, amag, amag_nb, 1e-5, "anchors c2 sampled", axis=1)
    ft = torch.empty_like(xt)
    p0 = vt.sum(dim=1).cpu().numpy()
    nreb = ctx.integrate(xt, vt, ft, wl.dt, 200)
    torch.cuda.synchronize()
    assert nreb >= 1
    p1 = vt.sum(dim=1).cpu().numpy()
    assert np.abs(p1 - p0).max() < 1e-6 * np.abs(vt.cpu().numpy()).sum(axis=1).max() / 1e3


def test_errors(dev):
    from paper_1806_10841_amd import binding
    wl = _wl("small_sphere")
    x, _ = inputs.make_state(wl)
    xt = _t(x, dev)
    c = binding.Context(wl)
    with pytest.raises(binding.AdresError):
        c.forces(xt)                                   # no anchors yet
    with pytest.raises(binding.AdresError):
        c.weights(xt)
    for bad in (np.zeros(0, np.int32), np.array([wl.n_mol], np.int32), np.array([-1], np.int32),
                np.arange(1025, dtype=np.int32)):
        with pytest.raises(binding.AdresError):
            c.set_anchors(bad)
    c.set_anchors(np.array([3], np.int32))
    assert torch.isfinite(c.forces(xt)).all()
    c.set_tdforce(np.ones(4), 1.0, 3.0)                 # a correction field is allowed ...
    counts = torch.zeros(4, dtype=torch.int64, device=dev)
    c.density_profile(xt, counts)                       # ... and a profile ...
    with pytest.raises(binding.AdresError):            # ... but no closed-form bin volumes
        c.tdforce_update(counts, 1, 1.0)
    with pytest.raises(binding.AdresError):            # sampled volumes need the configuration
        c.region_volumes(None, 100, 1, counts)
    with pytest.raises(binding.AdresError):
        c.region_volumes(xt, 0, 1, counts)
    with pytest.raises(binding.AdresError):
        binding.Context(wl.with_(scheme=inputs.SCHEME_HAMILTONIAN))
    s = binding.Context(inputs.workload("small_sphere"))
    with pytest.raises(binding.AdresError):
        s.set_anchors(np.array([3], np.int32))


def test_respa_with_anchor_spheres_matches_oracle(dev):
    """RESPA (CG part on every second step) with the self-adjusting region: the weights
    follow the anchors on every inner step, against the oracle's RESPA."""
    wl = _wl("c1", pair_precision=64)
    an = inputs.anchor_molecules(wl.n_mol, 5, 7)
    x, v = inputs.make_state(wl)
    xo, vo, _, _, st = oracle.Model(wl, anchors=an).respa(x, v, wl.dt / 2, 2, 40)
    assert st == 0
    ctx = _ctx(wl, an)
    xt, vt = _t(x, dev), _t(v, dev)
    ft = torch.empty_like(xt)
    ctx.integrate_respa(xt, vt, ft, wl.dt / 2, 2, 40)
    torch.cuda.synchronize()
    assert np.abs(_min_image(xt.cpu().numpy() - xo, wl.box[0])).max() < 1e-9
    assert np.abs(vt.cpu().numpy() - vo).max() < 1e-7


@pytest.mark.parametrize("name,k,prec", [("small_sphere", 9, 64), ("c1", 5, 64), ("small_sphere", 9, 32)])
def test_forces_with_correction_around_anchors(dev, name, k, prec):
    """A correction field around the nearest anchor (Sec. 2.5 with Sec. 2.4): forces and
    the correction potential against the oracle."""
    wl = _wl(name, pair_precision=prec)
    an = inputs.anchor_molecules(wl.n_mol, k, 4)
    td = (np.linspace(0.8, -0.3, 16), 1.5, 5.0)
    x, _ = inputs.make_state(wl)
    fo, amag, eo, st = oracle.Model(wl, anchors=an, td=td).forces(x)
    assert st == 0 and eo[3] != 0.0
    c = _ctx(wl, an)
    c.set_tdforce(*td)
    f, e = c.forces(_t(x, dev), energy=True)
    torch.cuda.synchronize()
    tol = 1e-12 if prec == 64 else 1e-5
    if prec == 64:
        _assert_close(f.cpu().numpy(), fo, amag, tol, name)
    else:
        _, amag_nb, _, _ = nonbonded_model(wl, anchors=an, td=td).forces(x)
        assert_fp32_sites(f.cpu().numpy(), fo, amag, amag_nb, tol, name)
    np.testing.assert_allclose(e.cpu().numpy(), eo, rtol=tol, atol=tol * np.abs(eo).max())


def test_integrate_with_correction_around_anchors(dev):
    """The nearest-anchor offsets follow the anchors through steps and list rebuilds."""
    wl = _wl("c1", pair_precision=64)
    an = inputs.anchor_molecules(wl.n_mol, 5, 7)
    td = (np.linspace(0.8, -0.3, 16), 1.5, 5.0)
    x, v = inputs.make_state(wl)
    xo, vo, _, _, st = oracle.Model(wl, anchors=an, td=td).vv(x, v, wl.dt, 100)
    assert st == 0
    c = _ctx(wl, an)
    c.set_tdforce(*td)
    xt, vt = _t(x, dev), _t(v, dev)
    ft = torch.empty_like(xt)
    nreb = c.integrate(xt, vt, ft, wl.dt, 100)
    torch.cuda.synchronize()
    assert nreb >= 1
    assert np.abs(_min_image(xt.cpu().numpy() - xo, wl.box[0])).max() < 1e-9
    assert np.abs(vt.cpu().numpy() - vo).max() < 1e-7


def test_anchor_density_profile_and_sampled_volumes_match_oracle(dev):
    """Density profile by nearest-anchor distance and sampled bin volumes (same SplitMix64
    points on both sides): integer counts equal to the oracle's; a refinement with them."""
    wl = _wl("small_sphere")
    an = inputs.anchor_molecules(wl.n_mol, 9, 3)
    x, _ = inputs.make_state(wl)
    n, lo, hi = 20, 0.25, 8.0
    m = oracle.Model(wl, anchors=an)
    c = _ctx(wl, an)
    c.set_tdforce(np.linspace(0.5, -0.5, n), lo, hi)
    xt = _t(x, dev)
    counts = torch.zeros(n, dtype=torch.int64, device=dev)
    c.density_profile(xt, counts)
    vol = torch.zeros(n, dtype=torch.int64, device=dev)
    c.region_volumes(xt, 300_000, 99, vol)
    c.region_volumes(xt, 300_000, 100, vol)
    torch.cuda.synchronize()
    ref = m.density_profile(x, n, lo, hi)
    np.testing.assert_array_equal(counts.cpu().numpy(), ref)
    vref = m.region_volumes(x, 300_000, 99, n, lo, hi)
    vref = m.region_volumes(x, 300_000, 100, n, lo, hi, vref)
    np.testing.assert_array_equal(vol.cpu().numpy(), vref)
    c.tdforce_update_sampled(counts, 1, vol, 600_000, 0.3)
    F2 = m.tdforce_update(np.linspace(0.5, -0.5, n), lo, hi, ref, 1, 0.3, vol_counts=vref, n_vol_samples=600_000)
    np.testing.assert_allclose(c.get_tdforce(), F2, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("region", [inputs.REGION_SLAB_X, inputs.REGION_SPHERE])
def test_sampled_volumes_static_regions_match_oracle(dev, region):
    from paper_1806_10841_amd import binding
    wl = inputs.workload("small_sphere").with_(region=region)
    x, _ = inputs.make_state(wl)
    n, lo, hi = 16, 0.5, 8.5
    c = binding.Context(wl)
    c.set_tdforce(np.zeros(n), lo, hi)
    vol = torch.zeros(n, dtype=torch.int64, device=dev)
    c.region_volumes(None, 1_000_003, 7, vol)     # ragged: not a multiple of the workgroup
    torch.cuda.synchronize()
    np.testing.assert_array_equal(vol.cpu().numpy(), oracle.Model(wl).region_volumes(x, 1_000_003, 7, n, lo, hi))
