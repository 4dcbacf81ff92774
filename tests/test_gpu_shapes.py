"""GPU parity for molecules of two and three sites (dumbbells and triangles, unit bonds)
through the C ABI: the 2- and 3-site instantiations of every kernel (centres, reorder,
Eq. (1) forces with bonds, velocity Verlet, RESPA, Eq. (2)) against the FP64 oracle.

Bars, as for tetrahedra: centres and neighbour lists bit-exact; weights to 1e-15; FP64
forces and energies to 1e-12 and FP32-pair forces to 1e-5 of the per-site term scale A_i;
FP64 trajectories to 1e-9 in position.
"""
import numpy as np
import pytest

import oracle
from _bars import assert_fp32_sites, nonbonded_model
from paper_1806_10841_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SHAPES = ["small_dumbbell", "small_triangle"]


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    return torch.device("cuda:0")


def _ctx(wl):
    from paper_1806_10841_amd import binding
    return binding.Context(wl)


def _t(a, dev):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)


def _min_image(d, L):
    return d - L * np.round(d / L)


def _assert_close(fg, fo, amag, tol, where):
    err = np.abs(fg - fo).max(axis=0)
    ratio = err / np.maximum(amag, 1e-300)
    assert (ratio <= tol).all(), f"{where}: worst ratio {ratio.max():.3e}"
    assert np.linalg.norm(fg - fo) <= tol * np.linalg.norm(fo), where


@pytest.mark.parametrize("name", SHAPES)
def test_centres_weights_and_list(dev, name):
    wl = inputs.workload(name)
    x, _ = inputs.make_state(wl)
    m = oracle.Model(wl)
    com_o, w_o, _, st = m.weights(x)
    assert st == 0
    assert (w_o == 1).any() and (w_o == 0).any() and ((w_o > 0) & (w_o < 1)).any()
    ctx = _ctx(wl)
    com, w = ctx.weights(_t(x, dev))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(com.cpu().numpy(), com_o)
    assert np.abs(w.cpu().numpy() - w_o).max() <= 1e-15
    ref = m.pairs(com_o)
    n = ctx.build_verlet(_t(x, dev))
    assert n == len(ref)
    np.testing.assert_array_equal(ctx.get_pairs(), ref)


@pytest.mark.parametrize("name", SHAPES)
@pytest.mark.parametrize("scheme", [inputs.SCHEME_FORCE, inputs.SCHEME_HAMILTONIAN])
def test_forces_fp64(dev, name, scheme):
    wl = inputs.workload(name).with_(pair_precision=64, scheme=scheme)
    x, _ = inputs.make_state(wl)
    fo, amag, eo, st = oracle.Model(wl).forces(x)
    assert st == 0
    assert eo[0] > 0 and eo[1] > 0, "atom pairs and CG pairs both interact"
    f, e = _ctx(wl).forces(_t(x, dev), energy=True)
    torch.cuda.synchronize()
    _assert_close(f.cpu().numpy(), fo, amag, 1e-12, name)
    np.testing.assert_allclose(e.cpu().numpy(), eo, rtol=1e-12, atol=1e-12 * np.abs(eo).max())


@pytest.mark.parametrize("name", SHAPES)
def test_forces_fp32_pairs(dev, name):
    wl = inputs.workload(name).with_(pair_precision=32)
    x, _ = inputs.make_state(wl)
    fo, amag, eo, st = oracle.Model(wl).forces(x)
    _, amag_nb, _, _ = nonbonded_model(wl).forces(x)
    f, e = _ctx(wl).forces(_t(x, dev), energy=True)
    torch.cuda.synchronize()
    assert_fp32_sites(f.cpu().numpy(), fo, amag, amag_nb, 1e-5, name)
    np.testing.assert_allclose(e.cpu().numpy(), eo, rtol=1e-5, atol=1e-5 * np.abs(eo).max())


@pytest.mark.parametrize("name", SHAPES)
def test_integrate_fp64_matches_oracle(dev, name):
    """100 velocity-Verlet steps (state reordered on the device at every rebuild)."""
    wl = inputs.workload(name).with_(pair_precision=64)
    x, v = inputs.make_state(wl)
    xo, vo, fo, _, st = oracle.Model(wl).vv(x, v, wl.dt, 100)
    assert st == 0
    ctx = _ctx(wl)
    xt, vt = _t(x, dev), _t(v, dev)
    ft = torch.empty_like(xt)
    ctx.integrate(xt, vt, ft, wl.dt, 100)
    torch.cuda.synchronize()
    tol = 1e-9
    assert np.abs(_min_image(xt.cpu().numpy() - xo, wl.box[0])).max() < tol
    assert np.abs(vt.cpu().numpy() - vo).max() < 100 * tol
    assert np.abs(ft.cpu().numpy() - fo).max() < 1e4 * tol * max(1.0, np.abs(fo).max())


@pytest.mark.parametrize("name", SHAPES)
def test_respa_fp64_matches_oracle(dev, name):
    wl = inputs.workload(name).with_(pair_precision=64)
    x, v = inputs.make_state(wl)
    dt = wl.dt / 2
    xo, vo, fo, _, st = oracle.Model(wl).respa(x, v, dt, 3, 20)
    assert st == 0
    ctx = _ctx(wl)
    xt, vt = _t(x, dev), _t(v, dev)
    ft = torch.empty_like(xt)
    ctx.integrate_respa(xt, vt, ft, dt, 3, 20)
    torch.cuda.synchronize()
    tol = 1e-9
    assert np.abs(_min_image(xt.cpu().numpy() - xo, wl.box[0])).max() < tol
    assert np.abs(vt.cpu().numpy() - vo).max() < 100 * tol
