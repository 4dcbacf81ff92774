"""GPU parity of the learned CG force against the FP64 oracle (oracle/mlp.py and the C
oracle's Eq. (1) with the network as F^CG).

Bar: layer 2 runs in BF16 with FP32 accumulation.  Rounding h1 and W2 to BF16
(unit roundoff 2^-9 each) perturbs z2_n by at most 2^-8 sum_k |W2_nk h1_k|, silu is
1.1-Lipschitz, so each output obeys |df| <= 2^-7 s taper(r) S(r) with the term scale
S = |b3| + sum_n |W3_n| (|h2_n| + sum_k |W2_nk h1_k|) (margin 2 included); over many
pairs the errors also stay below 2^-7 normwise.
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


def _term_scale(p, r):
    """S(r) = |b3| + sum_n |W3_n| (|h2_n| + sum_k |W2_nk h1_k|) from the FP64 network."""
    W1, b1, W2, b2, W3, b3 = omlp.unpack(p)
    _, (x, z1, h1, z2, h2) = omlp.network(p, r, RC)
    inner = np.abs(h1) @ np.abs(W2).T
    return abs(b3[0]) + (np.abs(h2) + inner) @ np.abs(W3)


@pytest.mark.parametrize("seed,n", [(0, 1), (1, 31), (2, 1000), (3, 100003)])
def test_mlp_eval_matches_oracle(dev, seed, n):
    """Tiles of 32 pairs with a ragged tail; r spans the taper and the cutoff."""
    p = inputs.mlp_init(seed)
    r = inputs.random_pair_distances(n, 1.0, 3.2, seed)
    ctx = _ctx(inputs.workload("small_cg").with_(cg_kind=inputs.CG_MLP, rc_cg=RC))
    ctx.mlp_set(p.astype(np.float32), RC, SCALE, TW, 0.0)
    f = ctx.mlp_eval(torch.tensor(r, device=dev)).cpu().numpy().astype(np.float64)
    # the device holds FP32 weights: compare against the FP64 network of those weights
    p64 = p.astype(np.float32).astype(np.float64)
    ref = omlp.forward(p64, r, RC, SCALE, TW)
    bound = 2.0 ** -7 * SCALE * omlp.taper(r, RC, TW) * _term_scale(p64, r)
    assert np.all(np.abs(f - ref) <= bound + 1e-30), np.max(np.abs(f - ref) / np.maximum(bound, 1e-300))
    if n >= 100:
        assert np.linalg.norm(f - ref) <= BF16_NORM * np.linalg.norm(ref)
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


def _cg_frames(n_frames, n_side=12, seed=21):
    """Frames of CG centres (jittered lattice at the workload density) with mapped forces
    drawn from a smooth pair force plus noise (the gradient test needs no physics)."""
    L = n_side * (1 / 0.1) ** (1 / 3)
    box = (L, L, L)
    rng = np.random.default_rng(seed)
    coms, fmaps = [], []
    for _ in range(n_frames):
        com = inputs.wrap_into_box(inputs.lattice_points((n_side,) * 3, box, rng, jitter=0.5), box)
        coms.append(com)
        fmaps.append(rng.normal(size=com.shape) * 3.0)
    return np.stack(coms), np.stack(fmaps), box


def _cg_workload(n, box):
    return inputs.workload("small_cg").with_(n_mol=n, box=box, center=tuple(b / 2 for b in box),
                                             cg_kind=inputs.CG_MLP, rc_cg=RC, pair_precision=32)


def test_fm_gradient_matches_oracle(dev):
    """Loss and gradient of force matching (2 frames of 1728 sites) against the FP64 oracle.
    Bar: 2^-6 normwise for the whole gradient and per parameter block (BF16 rounding of h1,
    W2 and dz2, each 2^-9 relative, through sums with moderate cancellation)."""
    coms, fmaps, box = _cg_frames(2)
    n = coms.shape[2]
    p32 = inputs.mlp_init(31).astype(np.float32)
    p = p32.astype(np.float64)
    frames = [(coms[k], fmaps[k]) for k in range(2)]
    loss_o, g_o = omlp.fm_loss_and_grad(p, frames, box, RC, SCALE, TW)
    ctx = _ctx(_cg_workload(n, box))
    ctx.mlp_set(p32, RC, SCALE, TW, 0.0)
    loss, g = ctx.mlp_fm_grad(torch.tensor(coms, device=dev), torch.tensor(fmaps, device=dev))
    assert abs(loss - loss_o) <= 2.0 ** -7 * loss_o
    assert np.linalg.norm(g - g_o) <= 2.0 ** -6 * np.linalg.norm(g_o)
    H = 64
    blocks = {"W1": slice(0, H), "b1": slice(H, 2 * H), "W2": slice(2 * H, 2 * H + H * H),
              "b2": slice(2 * H + H * H, 3 * H + H * H), "W3": slice(3 * H + H * H, 4 * H + H * H)}
    for name, sl in blocks.items():
        assert np.linalg.norm(g[sl] - g_o[sl]) <= 2.0 ** -6 * np.linalg.norm(g_o[sl]) + 1e-12, name
    assert abs(g[-1] - g_o[-1]) <= 2.0 ** -6 * abs(g_o[-1]) + 2.0 ** -6 * np.abs(g_o).max() * 1e-2
    # deterministic: a second evaluation gives the same bits
    loss2, g2 = ctx.mlp_fm_grad(torch.tensor(coms, device=dev), torch.tensor(fmaps, device=dev))
    assert loss2 == loss and np.array_equal(g2, g)


def test_adam_step_matches_oracle(dev):
    """One Adam step on the device equals the oracle's Adam applied to the device gradient."""
    coms, fmaps, box = _cg_frames(1, seed=22)
    n = coms.shape[2]
    p32 = inputs.mlp_init(32).astype(np.float32)
    ctx = _ctx(_cg_workload(n, box))
    ctx.mlp_set(p32, RC, SCALE, TW, 0.0)
    tc, tf = torch.tensor(coms, device=dev), torch.tensor(fmaps, device=dev)
    _, g = ctx.mlp_fm_grad(tc, tf)
    ctx.mlp_train_step(tc, tf, 1e-3)
    q = ctx.mlp_get().astype(np.float64)
    ref, _, _ = omlp.adam_step(p32.astype(np.float64), g, np.zeros_like(g), np.zeros_like(g), 1, 1e-3)
    assert np.abs(q - ref).max() <= 1e-6


def test_training_reduces_loss(dev):
    coms, fmaps, box = _cg_frames(2, seed=23)
    n = coms.shape[2]
    # mapped forces that a pair force can represent: the CG WCA force of the frames
    fm = np.stack([omlp.predicted_forces(inputs.mlp_init(40), c, box, RC, SCALE, TW) for c in coms])
    ctx = _ctx(_cg_workload(n, box))
    ctx.mlp_set(inputs.mlp_init(41).astype(np.float32), RC, SCALE, TW, 0.0)
    tc, tf = torch.tensor(coms, device=dev), torch.tensor(fm, device=dev)
    losses = [ctx.mlp_train_step(tc, tf, 3e-3) for _ in range(60)]
    assert losses[-1] < 0.2 * losses[0], (losses[0], losses[-1])


# ---------------------------------------------------------------- FP8 E4M3 variant
def _fp8_workload(name="small_cg"):
    return inputs.workload(name).with_(cg_kind=inputs.CG_MLP_FP8, rc_cg=RC, pair_precision=32)


def test_mlp_fp8_eval_matches_oracle(dev):
    """The FP8 variant against (a) the oracle's definition of it (h1 and W2 rounded to E4M3
    with the same per-tensor scales, everything else FP64): equal up to FP32 arithmetic and
    rare rounding-boundary flips, 2^-8 normwise; (b) the FP64 network: the E4M3 rounding of
    two factors (2^-4 each) through silu, 2^-2 normwise, its RMSE printed."""
    p32 = inputs.mlp_init(13).astype(np.float32)
    p = p32.astype(np.float64)
    r = inputs.random_pair_distances(100003, 0.5, RC, 3)
    ctx = _ctx(_fp8_workload())
    ctx.mlp_set(p32, RC, SCALE, TW, 0.0)
    f = ctx.mlp_eval(torch.tensor(r, device=dev)).cpu().numpy().astype(np.float64)
    ref8 = omlp.forward_fp8(p, r, RC, SCALE, TW)
    ref = omlp.forward(p, r, RC, SCALE, TW)
    print(f"FP8 vs FP64 network: relative RMSE {np.linalg.norm(f - ref) / np.linalg.norm(ref):.4f}")
    assert np.linalg.norm(f - ref8) <= 2.0 ** -8 * np.linalg.norm(ref8)
    assert np.linalg.norm(f - ref) <= 2.0 ** -2 * np.linalg.norm(ref)


@pytest.mark.parametrize("name", ["small_cg", "small_slab"])
def test_forces_with_learned_cg_fp8(dev, name):
    """Eq. (1) with the FP8 network as F^CG against the oracle's FP64 network: 2^-2 normwise
    (the FP8 bar); Newton's third law exact per pair."""
    p = inputs.mlp_init(11).astype(np.float32).astype(np.float64)
    wl = _fp8_workload(name)
    x, _ = inputs.make_state(wl)
    fo, _, _, st = oracle.Model(wl.with_(cg_kind=inputs.CG_MLP), mlp=(p, RC, SCALE, TW, 0.0)).forces(x)
    assert st == 0
    ctx = _ctx(wl)
    ctx.mlp_set(p.astype(np.float32), RC, SCALE, TW, 0.0)
    f = ctx.forces(torch.tensor(x, device=dev)).cpu().numpy()
    assert np.linalg.norm(f - fo) <= 2.0 ** -2 * np.linalg.norm(fo)
    assert np.all(np.abs(f.sum(axis=1)) <= 1e-9 * np.abs(f).sum(axis=1))


def test_fp8_kind_is_not_trained(dev):
    from paper_1806_10841_amd import binding
    coms, fmaps, box = _cg_frames(1, seed=24)
    wl = _cg_workload(coms.shape[2], box).with_(cg_kind=inputs.CG_MLP_FP8)
    ctx = _ctx(wl)
    ctx.mlp_set(inputs.mlp_init(3).astype(np.float32), RC, SCALE, TW, 0.0)
    with pytest.raises(binding.AdresError):
        ctx.mlp_train_step(torch.tensor(coms, device=dev), torch.tensor(fmaps, device=dev), 1e-3)
