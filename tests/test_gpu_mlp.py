"""GPU parity of the learned CG force against the FP64 oracle (oracle/mlp.py and the C
oracle's Eq. (1) with the network as F^CG).

Bar: layer 2 runs in BF16 with FP32 accumulation, so outputs agree with the FP64
oracle to 2^-7 normwise (the BF16 unit roundoff is 2^-8; inputs h1 and W2 are both
rounded), and every single value to 2^-6 of the output scale.
"""
import numpy as np
import pytest

import oracle
from oracle import mlp as omlp
from oracle import tables
from paper_1806_10841_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

RC, TW, SCALE = 3.0, 0.5, 12.0
BF16_NORM = 2.0 ** -7


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available()
    return torch.device("cuda:0")


def _ctx(wl):
    from paper_1806_10841_amd import binding
    return binding.Context(wl)


@pytest.mark.parametrize("seed,n", [(0, 1), (1, 31), (2, 1000), (3, 100003)])
def test_mlp_eval_matches_oracle(dev, seed, n):
    """Tiles of 32 pairs with a ragged tail; r spans the taper and the cutoff."""
    p = inputs.mlp_init(seed)
    r = inputs.random_pair_distances(n, 1.0, 3.2, seed)
    ctx = _ctx(inputs.workload("small_cg").with_(cg_kind=inputs.CG_MLP, rc_cg=RC))
    ctx.mlp_set(p.astype(np.float32), RC, SCALE, TW, 0.0)
    f = ctx.mlp_eval(torch.tensor(r, device=dev)).cpu().numpy().astype(np.float64)
    # the device holds FP32 weights: compare against the FP64 network of those weights
    ref = omlp.forward(p.astype(np.float32).astype(np.float64), r, RC, SCALE, TW)
    scale = max(np.abs(ref).max(), 1e-30)
    assert np.linalg.norm(f - ref) <= BF16_NORM * np.linalg.norm(ref) + 1e-30
    assert np.abs(f - ref).max() <= 2.0 ** -6 * scale
    assert np.all(f[r >= RC] == 0.0)


def test_mlp_table_fallback(dev):
    p = inputs.mlp_init(5)
    coef, lo, hi = tables.hermite_wca_table(2.31, 1.0, 2.31 * 2 ** (1 / 6), 0.9, 3.0, 2048)
    r = np.linspace(0.95, 3.1, 997)
    wl = inputs.workload("small_cg").with_(cg_kind=inputs.CG_MLP, rc_cg=RC)
    ctx = _ctx(wl)
    ctx.set_cg_table(coef, lo, hi)
    ctx.mlp_set(p.astype(np.float32), RC, SCALE, TW, 1.6)
    f = ctx.mlp_eval(torch.tensor(r, device=dev)).cpu().numpy().astype(np.float64)
    low = r < 1.6
    ref_low = tables.eval_table_fp64(coef, lo, hi, r[low])
    np.testing.assert_allclose(f[low], ref_low, rtol=1e-5, atol=1e-5 * np.abs(ref_low).max())
    ref_hi = omlp.forward(p.astype(np.float32).astype(np.float64), r[~low], RC, SCALE, TW)
    assert np.linalg.norm(f[~low] - ref_hi) <= BF16_NORM * np.linalg.norm(ref_hi)


@pytest.mark.parametrize("name", ["small_cg", "small_slab"])
def test_forces_with_learned_cg(dev, name):
    """Eq. (1) with the network as F^CG (pure CG sites, and hybrid tetrahedra)."""
    p = inputs.mlp_init(11).astype(np.float32).astype(np.float64)
    wl = inputs.workload(name).with_(cg_kind=inputs.CG_MLP, rc_cg=RC, pair_precision=32)
    x, _ = inputs.make_state(wl)
    fo, amag, _, st = oracle.Model(wl, mlp=(p, RC, SCALE, TW, 0.0)).forces(x)
    assert st == 0
    ctx = _ctx(wl)
    ctx.mlp_set(p.astype(np.float32), RC, SCALE, TW, 0.0)
    f = ctx.forces(torch.tensor(x, device=dev)).cpu().numpy()
    assert np.linalg.norm(f - fo) <= BF16_NORM * np.linalg.norm(fo)
    # Newton's third law holds exactly per pair (one network value per unordered pair)
    assert np.all(np.abs(f.sum(axis=1)) <= 1e-9 * np.abs(f).sum(axis=1))


def test_integrate_with_learned_cg(dev):
    p = inputs.mlp_init(12).astype(np.float32)
    wl = inputs.workload("small_cg").with_(cg_kind=inputs.CG_MLP, rc_cg=RC, pair_precision=32)
    x, v = inputs.make_state(wl)
    ctx = _ctx(wl)
    ctx.mlp_set(p, RC, 1.0, TW, 0.0)
    xt, vt = torch.tensor(x, device=dev), torch.tensor(v, device=dev)
    ft = torch.empty_like(xt)
    p0 = vt.sum(dim=1).cpu().numpy()
    ctx.integrate(xt, vt, ft, 0.005, 200)
    assert torch.isfinite(xt).all()
    assert np.abs(vt.sum(dim=1).cpu().numpy() - p0).max() < 1e-9 * wl.n_mol
