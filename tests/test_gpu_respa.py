"""GPU parity of multiple time stepping (Sec. 2.6, RESPA) against the FP64 oracle, through
the C ABI: FP64 trajectories of both schemes (with a correction force) against the
oracle's RESPA, one inner step identical to velocity Verlet, the learned CG force on
the outer step, the conserved energy of Eq. (2), the Langevin temperature, and the
full-size headline geometry.

Bars: FP64 trajectories to 1e-9 in position after up to 100 inner steps, as for
velocity Verlet; one inner step per outer step bit-identical to adres_integrate.
"""
import numpy as np
import pytest

import oracle
from paper_1806_10841_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

HAM = inputs.SCHEME_HAMILTONIAN


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    return torch.device("cuda:0")


def _ctx(wl, td=None):
    from paper_1806_10841_amd import binding
    c = binding.Context(wl)
    if td is not None:
        c.set_tdforce(*td)
    return c


def _t(a, dev):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)


def _min_image(d, L):
    return d - L * np.round(d / L)


@pytest.mark.parametrize("name,scheme,td,n_inner,n_outer", [
    ("tiny_slab", 0, False, 2, 50),
    ("c1", 0, False, 4, 25),
    ("small_sphere", HAM, True, 3, 12),
    ("tiny_slab", HAM, True, 5, 20),
    ("small_kg", 0, False, 2, 25),
])
def test_respa_fp64_matches_oracle(dev, name, scheme, td, n_inner, n_outer):
    wl = inputs.workload(name).with_(pair_precision=64, scheme=scheme)
    tab = None
    if td:
        lo, hi = max(wl.d_at - 0.5, 0.0), wl.d_at + wl.d_hy + 0.5
        tab = (np.linspace(0.6, -0.4, 12), lo, hi)
    x, v = inputs.make_state(wl)
    dt = wl.dt / 2
    xo, vo, fo, _, st = oracle.Model(wl, td=tab).respa(x, v, dt, n_inner, n_outer)
    assert st == 0
    ctx = _ctx(wl, tab)
    xt, vt = _t(x, dev), _t(v, dev)
    ft = torch.empty_like(xt)
    nreb = ctx.integrate_respa(xt, vt, ft, dt, n_inner, n_outer)
    torch.cuda.synchronize()
    tol = 1e-9
    assert np.abs(_min_image(xt.cpu().numpy() - xo, wl.box[0])).max() < tol
    assert np.abs(vt.cpu().numpy() - vo).max() < 100 * tol
    assert np.abs(ft.cpu().numpy() - fo).max() < 1e4 * tol * max(1.0, np.abs(fo).max())
    if name == "c1":
        assert nreb >= 1, "the rebuild path was not exercised"


@pytest.mark.parametrize("name", ["c1", "small_slab", "c2"])
def test_single_inner_step_is_integrate(dev, name):
    wl = inputs.workload(name)
    x, v = inputs.make_state(wl)
    out = []
    for respa in (False, True):
        ctx = _ctx(wl)
        xt, vt = _t(x, dev), _t(v, dev)
        ft = torch.empty_like(xt)
        if respa:
            ctx.integrate_respa(xt, vt, ft, wl.dt, 1, 60)
        else:
            ctx.integrate(xt, vt, ft, wl.dt, 60)
        torch.cuda.synchronize()
        out.append((xt, vt, ft))
    for a, b in zip(*out):
        assert torch.equal(a, b)


def test_learned_cg_on_the_outer_step(dev):
    """All-CG sites with the network as the CG force: RESPA skips the network on inner
    steps; one inner step equals integrate; the pair forces still cancel (momentum)."""
    RC, TW = 3.0, 0.5
    p = inputs.mlp_init(12).astype(np.float32)
    wl = inputs.workload("small_cg").with_(cg_kind=inputs.CG_MLP, rc_cg=RC, pair_precision=32)
    x, v = inputs.make_state(wl)
    res = []
    for mode in ("vv", "respa1", "respa3"):
        ctx = _ctx(wl)
        ctx.mlp_set(p, RC, 1.0, TW, 0.0)
        xt, vt = _t(x, dev), _t(v, dev)
        ft = torch.empty_like(xt)
        p0 = vt.sum(dim=1).cpu().numpy()
        if mode == "vv":
            ctx.integrate(xt, vt, ft, 0.005, 60)
        elif mode == "respa1":
            ctx.integrate_respa(xt, vt, ft, 0.005, 1, 60)
        else:
            ctx.integrate_respa(xt, vt, ft, 0.005, 3, 20)
        torch.cuda.synchronize()
        assert torch.isfinite(xt).all()
        assert np.abs(vt.sum(dim=1).cpu().numpy() - p0).max() < 1e-9 * wl.n_mol
        res.append(xt.clone())
    assert torch.equal(res[0], res[1])
    assert not torch.equal(res[0], res[2])


def test_hamiltonian_respa_conserves_energy(dev):
    """Eq. (2) with RESPA (3 inner steps): the energy error of the GPU's own trajectory
    falls as dt^2."""
    wl = inputs.workload("tiny_slab").with_(pair_precision=64, scheme=HAM)
    x, v = inputs.make_state(wl)
    m = oracle.Model(wl)

    def trace(dt, n_outer):
        ctx = _ctx(wl)
        xt, vt = _t(x, dev), _t(v, dev)
        ft = torch.empty_like(xt)
        out = []
        for k in range(11):
            if k:
                ctx.integrate_respa(xt, vt, ft, dt, 3, n_outer)
            _, e = ctx.forces(xt, energy=True)
            out.append(e.sum().item() + m.kinetic(vt.cpu().numpy()))
        return np.array(out)

    t1, t2 = trace(0.002, 4), trace(0.001, 8)
    f1, f2 = np.abs(t1 - t1[0]).max(), np.abs(t2 - t2[0]).max()
    assert f1 < 5e-3 * abs(t1[0]) + 1e-2, (f1, t1[0])
    assert 2.5 < f1 / f2 < 6.0, (f1, f2)


def test_respa_langevin_temperature(dev):
    """gamma > 0 with RESPA: the thermostat acts on every inner step; the kinetic
    temperature relaxes to kT."""
    wl = inputs.workload("small_slab").with_(rho_max=1.0)
    x, v = inputs.make_state(wl)
    v = v * 1.25
    ctx = _ctx(wl)
    xt, vt = _t(x, dev), _t(v, dev)
    ft = torch.empty_like(xt)
    ctx.integrate_respa(xt, vt, ft, 0.004, 2, 800, gamma=2.0, kT=1.0, seed=42)
    temps = []
    for _ in range(10):
        ctx.integrate_respa(xt, vt, ft, 0.004, 2, 50, gamma=2.0, kT=1.0, seed=43)
        ke = 0.5 * (vt ** 2).sum().item()
        temps.append(2 * ke / (3 * x.shape[1]))
    assert abs(np.mean(temps) - 1.0) < 0.05, temps


def test_respa_c2_full_size(dev):
    """64,000 tetrahedra, FP32 pairs, CG part on a twice longer step: 100 outer steps,
    momentum conserved (both parts obey Newton's third law), lists rebuilt, no errors."""
    wl = inputs.workload("c2")
    x, v = inputs.make_state(wl)
    ctx = _ctx(wl)
    xt, vt = _t(x, dev), _t(v, dev)
    ft = torch.empty_like(xt)
    p0 = vt.sum(dim=1).cpu().numpy()
    nreb = ctx.integrate_respa(xt, vt, ft, wl.dt, 2, 100)
    torch.cuda.synchronize()
    p1 = vt.sum(dim=1).cpu().numpy()
    assert nreb >= 1
    assert np.abs(p1 - p0).max() < 1e-6 * np.abs(vt.cpu().numpy()).sum(axis=1).max() / 1e3
    assert torch.isfinite(xt).all() and torch.isfinite(vt).all()


def test_respa_argument_errors(dev):
    from paper_1806_10841_amd import binding
    wl = inputs.workload("tiny_slab")
    x, v = inputs.make_state(wl)
    ctx = _ctx(wl)
    xt, vt = _t(x, dev), _t(v, dev)
    ft = torch.empty_like(xt)
    for n_inner, n_outer in ((0, 5), (2, -1), (70000, 70000)):
        with pytest.raises(binding.AdresError):
            ctx.integrate_respa(xt, vt, ft, 0.005, n_inner, n_outer)
    ctx.integrate_respa(xt, vt, ft, 0.005, 3, 0)       # no steps: forces only
    torch.cuda.synchronize()
    fo, _, _, _ = oracle.Model(wl).forces(x)
    assert np.abs(ft.cpu().numpy() - fo).max() < 1e-10 * np.abs(fo).max()
