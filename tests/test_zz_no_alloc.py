"""The allocation-free force entry point (adres_forces_noalloc) through the C ABI: the same
forces and energies as adres_forces on the same inputs, on two calls in a row, the second
with a smaller system (its static scratch keeps the first call's partials, which must not
leak into the second), and its refusals."""
import numpy as np
import pytest

from paper_1806_10841_amd import binding, inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _run(name, seed):
    wl = inputs.workload(name)
    x, _ = inputs.make_state(wl, seed=seed)
    xt = torch.tensor(x, device="cuda")
    ref = binding.Context(wl)
    f_ref, e_ref = ref.forces(xt, energy=True)
    ctx = binding.Context(wl)
    ctx.build_verlet(xt)           # sizes the lists (the entry point does not grow them)
    f = torch.empty_like(xt)
    e = torch.full((4,), np.nan, dtype=torch.float64, device="cuda")
    ctx.forces_noalloc(xt, f, e)
    torch.cuda.synchronize()
    assert torch.equal(f, f_ref), name
    assert torch.equal(e, e_ref), name
    ref.close()
    ctx.close()


def test_noalloc_matches_forces_twice_second_smaller():
    assert torch.cuda.is_available()
    _run("c2", 1)          # 1,000 workgroup partials
    _run("tiny_slab", 2)   # then a single workgroup: stale partials of the first call stay unused


def test_noalloc_twice_on_one_context_and_without_energy():
    wl = inputs.workload("small_slab")
    ctx = binding.Context(wl)
    ref = binding.Context(wl)
    for seed in (3, 4):
        x, _ = inputs.make_state(wl, seed=seed)
        xt = torch.tensor(x, device="cuda")
        f_ref, e_ref = ref.forces(xt, energy=True)
        f = torch.empty_like(xt)
        e = torch.empty(4, dtype=torch.float64, device="cuda")
        ctx.forces_noalloc(xt, f, e)
        f2 = torch.empty_like(xt)
        ctx.forces_noalloc(xt, f2)
        torch.cuda.synchronize()
        assert torch.equal(f, f_ref) and torch.equal(e, e_ref) and torch.equal(f2, f_ref)


def test_noalloc_refuses_more_molecules_than_its_scratch():
    # 1,000,000 molecules need 15,625 workgroup partials, more than the 8,192 slots:
    # refused before anything runs
    wl = inputs.workload("c5")
    ctx = binding.Context(wl)
    x = torch.zeros((3, wl.n_mol * wl.sites_per_mol), dtype=torch.float64, device="cuda")
    f = torch.empty_like(x)
    with pytest.raises(binding.AdresError) as ei:
        ctx.forces_noalloc(x, f)
    assert ei.value.status == -5 and "524288" in str(ei.value)
    ctx.close()
