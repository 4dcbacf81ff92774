"""Parity at the full sizes of the paper-scale workloads, through the C ABI, in the
configuration the benchmark uses (one context per workload, FP32 pair arithmetic with FP64
sums and integration, the library's own launch shapes).

The oracle cannot afford every output at these sizes, so each test compares outputs it
computes one by one -- the neighbour sets of sampled molecules (bit-exact, brute force over
all molecules), the forces on sampled molecules (1e-5 of the oracle's term scale A_i for FP32
pairs; the BF16 bar 2^-7 normwise where the learned CG force is used) -- plus properties that
hold at any size: Newton's third law (net force at FP64 summation rounding), momentum
conservation under velocity Verlet, a finite state.

Workloads: C2 64,000 tetrahedra (x-slab); C3 200,000 Kremer-Grest beads (FENE + WCA);
C4 256,000 CG sites (learned CG force); C5 1,000,000 tetrahedra (sphere), tabulated or
learned CG force.
"""
import numpy as np
import pytest

import oracle
from _bars import assert_fp32_sites, nonbonded_model
from oracle import tables
from paper_1806_10841_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

BF16_NORM = 2.0 ** -7
RC_MLP, TW, SCALE = 3.0, 0.5, 8.0


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available()
    return torch.device("cuda:0")


def _ctx(wl):
    from paper_1806_10841_amd import binding
    return binding.Context(wl)


def _t(a, dev):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)


def _sample_by_class(w, per_class, seed):
    rng = np.random.default_rng(seed)
    out = []
    for mask in (w == 1.0, (w > 0) & (w < 1), w == 0.0):
        idx = np.flatnonzero(mask)
        if len(idx):
            out.append(rng.choice(idx, size=min(per_class, len(idx)), replace=False))
    return np.sort(np.concatenate(out))


def _check_sampled_neighbours(ctx, m, com_o, sel):
    """The library's pair set restricted to the sampled molecules equals the oracle's
    brute-force neighbour sets (bit-exact)."""
    pairs = ctx.get_pairs()
    near = np.isin(pairs[:, 0], sel) | np.isin(pairs[:, 1], sel)
    sub = pairs[near]
    for t, ref in zip(sel, m.neighbours_of(com_o, sel)):
        got = np.sort(np.concatenate([sub[sub[:, 0] == t, 1], sub[sub[:, 1] == t, 0]]))
        np.testing.assert_array_equal(got, ref)


def _sampled_forces(f, sel, spm):
    return np.stack([f[:, spm * a:spm * a + spm] for a in sel])        # (n_sel, 3, spm)


def _newton3(f):
    tot = np.abs(f.sum(axis=1))
    assert np.all(tot <= 1e-9 * np.abs(f).sum(axis=1)), tot


def test_c2_integrate_matches_oracle_vv(dev):
    """The benchmark's own path (adres_integrate: kick-drift, fused steps, closing kick) on
    the full 64,000-tetrahedron state for 3 steps against the oracle's velocity Verlet over
    all molecules.  Bar: each force evaluation is within 1e-5 A_i, so after n steps
    |dx| <= n^2 dt^2 1e-5 max A / m and |dv| <= 2 n dt 1e-5 max A / m."""
    wl = inputs.workload("c2")
    x, v = inputs.make_state(wl)
    m = oracle.Model(wl)
    n = 3
    xo, vo, fo, _, st = m.vv(x, v, wl.dt, n)
    assert st == 0
    _, amag, _, _ = m.forces(x)
    ctx = _ctx(wl)
    xt, vt = _t(x, dev), _t(v, dev)
    ft = torch.empty_like(xt)
    ctx.integrate(xt, vt, ft, wl.dt, n)
    a_max = amag.max()
    d = xt.cpu().numpy() - xo
    d -= wl.box[0] * np.round(d / wl.box[0])
    assert np.abs(d).max() <= n * n * wl.dt ** 2 * 1e-5 * a_max, np.abs(d).max()
    assert np.abs(vt.cpu().numpy() - vo).max() <= 2 * n * wl.dt * 1e-5 * a_max
    _newton3(ft.cpu().numpy())


@pytest.mark.parametrize("n", [61, 97])
def test_c2_forces_from_a_list_in_use(dev, n):
    """The closing forces F(x_n) of an n-step run come from the list of its last rebuild,
    after the molecules have moved up to their motion budgets since (more than r_skin/2 for
    compact molecules and for those of weight zero): sampled AT, HY and CG molecules and the
    molecules that moved furthest, within 1e-5 A_i of the oracle's forces at the same
    positions (the oracle builds no list)."""
    wl = inputs.workload("c2")
    x, v = inputs.make_state(wl)
    ctx = _ctx(wl)
    xt, vt = _t(x, dev), _t(v, dev)
    ft = torch.empty_like(xt)
    nreb = ctx.integrate(xt, vt, ft, wl.dt, n)
    torch.cuda.synchronize()
    assert nreb >= 2
    xn = xt.cpu().numpy()
    m = oracle.Model(wl)
    com_o, w_o, _, st = m.weights(xn)
    assert st == 0
    com_0, _, _, _ = m.weights(x)
    moved = com_o - com_0
    moved -= np.asarray(wl.box)[:, None] * np.round(moved / np.asarray(wl.box)[:, None])
    far = np.argsort(np.linalg.norm(moved, axis=0))[-60:]
    sel = np.unique(np.concatenate([_sample_by_class(w_o, 80, n), far]))
    fo, amag, st = m.forces_sampled(xn, sel)
    assert st == 0
    fg = _sampled_forces(ft.cpu().numpy(), sel, 4)
    _, amag_nb, _ = nonbonded_model(wl).forces_sampled(xn, sel)
    assert_fp32_sites(fg, fo, amag, amag_nb, 1e-5, f"c2 after {n} steps", axis=1)


def test_c3_kremer_grest_full_size(dev):
    """200,000 beads in FENE chains of 200: sampled neighbour sets bit-exact, sampled forces
    (WCA + FENE) within 1e-5 A_i, Newton's third law; 20 NVE steps conserve momentum and a
    Langevin run (gamma 0.5, T 1) stays finite without a FENE error."""
    wl = inputs.workload("c3")
    x, v = inputs.make_state(wl)
    m = oracle.Model(wl)
    com_o, _, _, st = m.weights(x)
    assert st == 0
    sel = np.sort(np.random.default_rng(3).choice(wl.n_mol, 300, replace=False))
    fo, amag, st = m.forces_sampled(x, sel)
    assert st == 0
    ctx = _ctx(wl)
    xt = _t(x, dev)
    f = ctx.forces(xt).cpu().numpy()
    _check_sampled_neighbours(ctx, m, com_o, sel)
    fg = _sampled_forces(f, sel, 1)
    _, amag_nb, _ = nonbonded_model(wl).forces_sampled(x, sel)
    assert_fp32_sites(fg, fo, amag, amag_nb, 1e-5, "c3 sampled", axis=1)
    _newton3(f)
    vt = _t(v, dev)
    ft = torch.empty_like(xt)
    p0 = vt.sum(dim=1).cpu().numpy()
    ctx.integrate(xt, vt, ft, wl.dt, 20)
    p1 = vt.sum(dim=1).cpu().numpy()
    assert np.abs(p1 - p0).max() <= 1e-9 * np.abs(vt.cpu().numpy()).sum(axis=1).max()
    ctx.integrate(xt, vt, ft, wl.dt, 50, gamma=wl.gamma, kT=wl.kT, seed=9)
    assert torch.isfinite(xt).all() and torch.isfinite(vt).all()


def test_c4_learned_cg_full_size(dev):
    """256,000 CG sites with the learned CG force (BF16 matrix cores): sampled neighbour sets
    bit-exact, sampled forces within 2^-7 of the FP64 network normwise, Newton's third law
    exact per pair; 20 steps conserve momentum."""
    wl = inputs.workload("c4")
    x, v = inputs.make_state(wl)
    p = inputs.mlp_init(44).astype(np.float32)
    m = oracle.Model(wl, mlp=(p.astype(np.float64), RC_MLP, SCALE, TW, 0.0))
    com_o, _, _, _ = m.weights(x)
    sel = np.sort(np.random.default_rng(4).choice(wl.n_mol, 300, replace=False))
    fo, _, st = m.forces_sampled(x, sel)
    assert st == 0
    ctx = _ctx(wl)
    ctx.mlp_set(p, RC_MLP, SCALE, TW, 0.0)
    xt = _t(x, dev)
    f = ctx.forces(xt).cpu().numpy()
    _check_sampled_neighbours(ctx, m, com_o, sel)
    fg = _sampled_forces(f, sel, 1)
    assert np.linalg.norm(fg - fo) <= BF16_NORM * np.linalg.norm(fo)
    _newton3(f)
    vt = _t(v, dev)
    ft = torch.empty_like(xt)
    p0 = vt.sum(dim=1).cpu().numpy()
    ctx.integrate(xt, vt, ft, wl.dt, 20)
    p1 = vt.sum(dim=1).cpu().numpy()
    assert np.abs(p1 - p0).max() <= 1e-9 * np.abs(vt.cpu().numpy()).sum(axis=1).max()
    assert torch.isfinite(xt).all()


def _c5_table(wl):
    """The plain CG force (WCA between centres, cut at its minimum) as a 2048-knot table."""
    return tables.hermite_wca_table(wl.sig_cg, wl.eps_cg, wl.sig_cg * 2 ** (1 / 6), 1.5, 3.0, 2048)


def test_c5_sphere_table_full_size(dev):
    """1,000,000 tetrahedra (4M atoms), spherical atomistic region r 12 + hybrid shell 5,
    tabulated CG force: sampled AT, HY and CG molecules (neighbour sets bit-exact, forces
    within 1e-5 A_i), Newton's third law; 5 steps conserve momentum."""
    wl = inputs.workload("c5")
    x, v = inputs.make_state(wl)
    table = _c5_table(wl)
    m = oracle.Model(wl, table=table)
    com_o, w_o, _, st = m.weights(x)
    assert st == 0
    sel = _sample_by_class(w_o, 100, 5)
    fo, amag, st = m.forces_sampled(x, sel)
    assert st == 0
    ctx = _ctx(wl)
    ctx.set_cg_table(*table)
    xt = _t(x, dev)
    f = ctx.forces(xt).cpu().numpy()
    _check_sampled_neighbours(ctx, m, com_o, sel)
    fg = _sampled_forces(f, sel, 4)
    _, amag_nb, _ = nonbonded_model(wl, table=table).forces_sampled(x, sel)
    assert_fp32_sites(fg, fo, amag, amag_nb, 1e-5, "c5 sampled", axis=1)
    _newton3(f)
    vt = _t(v, dev)
    ft = torch.empty_like(xt)
    p0 = vt.sum(dim=1).cpu().numpy()
    ctx.integrate(xt, vt, ft, wl.dt, 5)
    p1 = vt.sum(dim=1).cpu().numpy()
    assert np.abs(p1 - p0).max() <= 1e-9 * np.abs(vt.cpu().numpy()).sum(axis=1).max()
    assert torch.isfinite(xt).all()


@pytest.mark.parametrize("kind,bar", [(inputs.CG_MLP, BF16_NORM), (inputs.CG_MLP_FP8, 2.0 ** -2)])
def test_c5_sphere_learned_cg_full_size(dev, kind, bar):
    """The same 1,000,000-tetrahedron sphere with the learned CG force between centres (the
    table as fallback below r_min), BF16 or FP8 matrix cores: sampled AT, HY and CG
    molecules against the FP64 network within the BF16 bar (2^-7) or the FP8 bar (2^-2)."""
    wl = inputs.workload("c5").with_(cg_kind=kind, rc_cg=RC_MLP)
    x, _ = inputs.make_state(wl)
    table = _c5_table(wl)
    p = inputs.mlp_init(45).astype(np.float32)
    r_min = 1.6
    m = oracle.Model(wl.with_(cg_kind=inputs.CG_MLP), table=table, mlp=(p.astype(np.float64), RC_MLP, SCALE, TW, r_min))
    _, w_o, _, _ = m.weights(x)
    sel = _sample_by_class(w_o, 100, 6)
    fo, _, st = m.forces_sampled(x, sel)
    assert st == 0
    ctx = _ctx(wl)
    ctx.set_cg_table(*table)
    ctx.mlp_set(p, RC_MLP, SCALE, TW, r_min)
    f = ctx.forces(_t(x, dev)).cpu().numpy()
    fg = _sampled_forces(f, sel, 4)
    assert np.linalg.norm(fg - fo) <= bar * np.linalg.norm(fo)
    _newton3(f)
