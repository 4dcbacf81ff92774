"""GPU edge cases through the C ABI: a sharp AT/CG interface (no hybrid layer, d_hy = 0,
where the weight is a step function) in both schemes against the FP64 oracle, and sizes
and parameters that set-up must refuse.

Bars: centres bit-exact and weights exactly 0 or 1 as the oracle's; FP64 forces to 1e-12
of A_i; FP64 trajectories to 1e-9 in position."""
import numpy as np
import pytest

import oracle
from paper_1806_10841_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


@pytest.mark.parametrize("scheme", [inputs.SCHEME_FORCE, inputs.SCHEME_HAMILTONIAN])
def test_sharp_interface(dev, scheme):
    wl = inputs.workload("c1").with_(d_hy=0.0, pair_precision=64, scheme=scheme)
    x, v = inputs.make_state(wl)
    m = oracle.Model(wl)
    com_o, w_o, _, st = m.weights(x)
    assert st == 0
    assert set(np.unique(w_o)) == {0.0, 1.0}
    ctx = _ctx(wl)
    com, w = ctx.weights(_t(x, dev))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(com.cpu().numpy(), com_o)
    np.testing.assert_array_equal(w.cpu().numpy(), w_o)
    fo, amag, eo, st = m.forces(x)
    assert st == 0
    f, e = ctx.forces(_t(x, dev), energy=True)
    torch.cuda.synchronize()
    err = np.abs(f.cpu().numpy() - fo).max(axis=0)
    assert (err <= 1e-12 * np.maximum(amag, 1e-300)).all()
    np.testing.assert_allclose(e.cpu().numpy(), eo, rtol=1e-12, atol=1e-12 * np.abs(eo).max())
    xo, vo, _, _, st = m.vv(x, v, wl.dt, 50)
    assert st == 0
    xt, vt = _t(x, dev), _t(v, dev)
    ft = torch.empty_like(xt)
    ctx.integrate(xt, vt, ft, wl.dt, 50)
    torch.cuda.synchronize()
    assert np.abs(_min_image(xt.cpu().numpy() - xo, wl.box[0])).max() < 1e-9
    assert np.abs(vt.cpu().numpy() - vo).max() < 1e-7


@pytest.mark.parametrize("change", [dict(n_mol=0), dict(sites_per_mol=5),
                                    dict(d_hy=-1.0), dict(d_at=-0.5), dict(region=7),
                                    dict(site_mass=(1.0, 1.0, 0.0, 1.0))])
def test_setup_refuses(dev, change):
    from paper_1806_10841_amd import binding
    with pytest.raises(binding.AdresError) as ei:
        _ctx(inputs.workload("tiny_slab").with_(**change))
    assert ei.value.status == -1
