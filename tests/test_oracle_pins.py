"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types the oracle's formulas: they check special values, closed
forms, invariants, finite-difference gradients of independently computed
energies, library routines (scipy's periodic k-d tree, NumPy matrix powers) and
brute force, so that a dropped term, a wrong sign or index or a transposed
operand in the oracle fails at least one of them.
"""
import math

import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle
from paper_1806_10841_amd import inputs

EPS = np.finfo(np.float64).eps


def _wl(**kw):
    """A small custom workload (no bonds unless asked)."""
    base = dict(name="pin", n_mol=2, sites_per_mol=1, box=(20.0, 20.0, 20.0), site_mass=(1.0,),
                region=inputs.REGION_ALL_AT, center=(10.0, 10.0, 10.0), d_at=2.0, d_hy=3.0,
                bond_kind=inputs.BOND_NONE, rho_max=0.0)
    base.update(kw)
    return inputs.Workload(**base)


def _soa(points):
    return np.ascontiguousarray(np.asarray(points, dtype=np.float64).T)


# ---------------------------------------------------------------- resolution function
class TestWeightFunction:
    """Sec. 2.2: lambda = 1 in AT, 0 in CG, smooth in HY; Sec. 2.3: squared cosine."""

    @pytest.mark.parametrize("d_at,d_hy", [(4.0, 3.0), (10.0, 5.0), (12.0, 5.0), (0.5, 0.25)])
    def test_special_values(self, d_at, d_hy):
        w = lambda d: oracle.weight_of_distance(d, d_at, d_hy)
        assert w(0.0) == 1.0 and w(d_at) == 1.0
        assert w(d_at + d_hy) == 0.0 and w(d_at + 2 * d_hy) == 0.0
        # the midpoint of a squared-cosine ramp is exactly one half (up to cos rounding)
        assert abs(w(d_at + 0.5 * d_hy) - 0.5) < 4 * EPS
        # quarter points: cos^2(pi/8) and cos^2(3 pi/8) sum to one
        assert abs(w(d_at + 0.25 * d_hy) + w(d_at + 0.75 * d_hy) - 1.0) < 8 * EPS

    def test_monotone_and_c1(self):
        d_at, d_hy = 4.0, 3.0
        d = np.linspace(d_at - 0.5, d_at + d_hy + 0.5, 4001)
        w = np.array([oracle.weight_of_distance(q, d_at, d_hy) for q in d])
        assert np.all(np.diff(w) <= 0.0)
        # slope at the midpoint of cos^2 over a ramp of width d_hy is -pi / (2 d_hy)
        h = 1e-6
        mid = d_at + d_hy / 2
        slope = (oracle.weight_of_distance(mid + h, d_at, d_hy)
                 - oracle.weight_of_distance(mid - h, d_at, d_hy)) / (2 * h)
        assert abs(slope + math.pi / (2 * d_hy)) < 1e-8
        # C1 at both ends: one-sided slopes vanish (w = 1 - O(h^2), O(h^2))
        for end, val in ((d_at, 1.0), (d_at + d_hy, 0.0)):
            for hh in (1e-3, 1e-4):
                inside = end + hh if val == 1.0 else end - hh
                assert abs(oracle.weight_of_distance(inside, d_at, d_hy) - val) < 3 * hh * hh

    def test_step_function_limit(self):
        # d_hy -> 0 gives a sharp interface
        assert oracle.weight_of_distance(1.0 - 1e-12, 1.0, 0.0) == 1.0
        assert oracle.weight_of_distance(1.0 + 1e-12, 1.0, 0.0) == 0.0

    def test_slab_and_sphere_through_com(self):
        """Weights of single-site molecules at chosen positions, periodic slab and sphere."""
        L = 20.0
        xs = np.array([10.0, 12.0, 13.5, 15.0, 0.2, 19.9, 6.5, 8.0])
        pts = np.stack([xs, np.full_like(xs, 3.0), np.full_like(xs, 17.0)], axis=1)
        wl = _wl(n_mol=len(xs), region=inputs.REGION_SLAB_X)
        com, w, rho, st = oracle.Model(wl).weights(_soa(pts))
        assert st == 0
        np.testing.assert_array_equal(com[0], xs)
        # |x - 10| = 0, 2, 3.5, 5, 9.8 (through the boundary), 9.9, 3.5, 2
        assert w[0] == 1.0 and w[1] == 1.0 and w[7] == 1.0
        assert w[3] == 0.0 and w[4] == 0.0 and w[5] == 0.0
        assert abs(w[2] - 0.5) < 4 * EPS and abs(w[6] - 0.5) < 4 * EPS
        # sphere: same distances placed radially along a diagonal
        u = np.array([1.0, 2.0, 2.0]) / 3.0
        dist = np.array([0.0, 2.0, 3.5, 5.0 + 1e-9, 6.0])   # 5 itself is rounding-sensitive
        pts = np.array([10.0, 10.0, 10.0]) + dist[:, None] * u[None, :]
        wl = _wl(n_mol=len(dist), region=inputs.REGION_SPHERE)
        _, w, _, _ = oracle.Model(wl).weights(_soa(pts))
        assert w[0] == 1.0 and w[1] == 1.0 and w[3] == 0.0 and w[4] == 0.0
        assert abs(w[2] - 0.5) < 1e-14


# ---------------------------------------------------------------- centre of mass
class TestCentreOfMass:
    def test_straddling_molecule(self):
        """A 4-site molecule split by the periodic boundary; unequal masses."""
        L = 10.0
        pts = [[9.8, 5.0, 5.0], [0.4, 5.0, 5.0], [9.6, 5.5, 5.0], [0.2, 4.5, 5.0]]
        masses = (1.0, 2.0, 3.0, 2.0)
        wl = _wl(n_mol=1, sites_per_mol=4, box=(L, L, L), site_mass=masses, rho_max=2.0)
        com, _, rho, st = oracle.Model(wl).weights(_soa(pts))
        unwrapped = np.array([9.8, 10.4, 9.6, 10.2])
        exp_x = np.mod((unwrapped * np.array(masses)).sum() / 8.0, L)
        assert abs(com[0, 0] - exp_x) < 1e-13
        assert abs(com[1, 0] - (5.0 + 1.0 * 3 * 0.5 / 8 - 0.5 * 2 / 8)) < 1e-13
        assert abs(com[2, 0] - 5.0) < 1e-13

    def test_translation_invariance(self):
        wl = inputs.workload("small_slab")
        x, _ = inputs.make_state(wl)
        m = oracle.Model(wl)
        com0, _, _, _ = m.weights(x)
        shift = np.array([3.7, -11.2, 40.1])
        x1 = inputs.wrap_into_box(x + shift[:, None], wl.box)
        com1, _, _, _ = m.weights(x1)
        for d in range(3):
            L = wl.box[d]
            diff = np.mod(com1[d] - com0[d] - shift[d] + L / 2, L) - L / 2
            assert np.max(np.abs(diff)) < 1e-12

    def test_stretch_flag(self):
        wl = _wl(n_mol=1, sites_per_mol=2, site_mass=(1.0, 1.0), rho_max=0.8)
        # two unit masses 1.7 apart: each site is 0.85 > 0.8 from the centre of mass
        _, _, rho, st = oracle.Model(wl).weights(_soa([[5, 5, 5], [6.7, 5, 5]]))
        assert st & oracle.STRETCH and abs(rho[0] - 0.85) < 1e-14
        _, _, rho, st = oracle.Model(wl).weights(_soa([[5, 5, 5], [6.5, 5, 5]]))
        assert st == 0 and abs(rho[0] - 0.75) < 1e-14


# ---------------------------------------------------------------- pair potentials
def _two_body(r, **kw):
    """Force on particle 0 (x component) and total energies for two particles on the x axis."""
    wl = _wl(**kw)
    x = _soa([[5.0, 5.0, 5.0], [5.0 + r, 5.0, 5.0]])
    f, amag, e, st = oracle.Model(wl).forces(x)
    return f, e, st


class TestPairTerms:
    def test_wca_closed_form(self):
        f, e, st = _two_body(1.0)
        assert st == 0
        assert abs(f[0, 0] + 24.0) < 1e-12 and abs(f[0, 1] - 24.0) < 1e-12   # 24 eps / sigma, repulsive
        assert abs(e[0] - 1.0) < 1e-12                                         # U(sigma) = eps
        rc = 2 ** (1 / 6)
        f, e, _ = _two_body(rc * (1 - 1e-9))
        assert abs(f[0, 0]) < 1e-6 and abs(e[0]) < 1e-12                      # zero at the cutoff
        f, e, _ = _two_body(rc * (1 + 1e-12))
        assert f[0, 0] == 0.0 and e[0] == 0.0

    @pytest.mark.parametrize("kw", [dict(), dict(eps_at=2.0, sig_at=1.3, rc_at=1.3 * 2 ** (1 / 6))])
    def test_wca_force_is_minus_gradient(self, kw):
        for r in (0.92, 1.0, 1.05, 1.1):
            r = r * kw.get("sig_at", 1.0)
            h = 1e-6
            _, ep, _ = _two_body(r + h, **kw)
            _, em, _ = _two_body(r - h, **kw)
            f, _, _ = _two_body(r, **kw)
            # particle 1 sits at +r: F_1 = -dU/dr
            assert abs(f[0, 1] - (-(ep[0] - em[0]) / (2 * h))) < 1e-6 * max(1, abs(f[0, 1]))

    def test_fene_closed_form(self):
        kw = dict(bond_kind=inputs.BOND_FENE, k_bond=30.0, r0_bond=1.5, chain_len=2)
        f, e, st = _two_body(1.0, **kw)
        # FENE at r = 1, R0 = 1.5: 30 * 1 / (1 - 1/2.25) = 54 (attractive); WCA at sigma: 24
        assert abs(f[0, 1] - (-54.0 + 24.0)) < 1e-11
        assert abs(e[2] - (-0.5 * 30 * 2.25 * math.log(1 - 1 / 2.25))) < 1e-12
        for r in (0.9, 1.2, 1.4):
            h = 1e-6
            _, ep, _ = _two_body(r + h, **kw)
            _, em, _ = _two_body(r - h, **kw)
            f, _, _ = _two_body(r, **kw)
            assert abs(f[0, 1] + ((ep.sum() - em.sum()) / (2 * h))) < 1e-5 * max(1, abs(f[0, 1]))
        _, _, st = _two_body(1.5, **kw)
        assert st & oracle.FENE
        # beads of different chains are not bonded
        f, e, _ = _two_body(1.3, bond_kind=inputs.BOND_FENE, k_bond=30.0, r0_bond=1.5, chain_len=1)
        assert f[0, 0] == 0.0 and e[2] == 0.0

    def test_harmonic_bond(self):
        wl = _wl(n_mol=1, sites_per_mol=2, site_mass=(1.0, 1.0), bond_kind=inputs.BOND_HARMONIC,
                 k_bond=400.0, r0_bond=1.0, rho_max=5.0)
        for r in (0.9, 1.0, 1.13):
            x = _soa([[5.0, 5.0, 5.0], [5.0 + r, 5.0, 5.0]])
            f, _, e, _ = oracle.Model(wl).forces(x)
            assert abs(f[0, 1] - (-400.0 * (r - 1.0))) < 1e-10
            assert abs(e[2] - 200.0 * (r - 1.0) ** 2) < 1e-10


# ---------------------------------------------------------------- pair list
class TestPairList:
    @pytest.mark.parametrize("name", ["small_slab", "tiny_slab", "small_cg"])
    def test_matches_periodic_kdtree(self, name):
        wl = inputs.workload(name)
        x, _ = inputs.make_state(wl, seed=123)
        m = oracle.Model(wl)
        com, _, _, _ = m.weights(x)
        rl = m.r_list()
        mine = m.pairs(com)
        pts = com.T.copy()
        tree = cKDTree(pts, boxsize=np.asarray(wl.box))
        ref = np.array(sorted(tree.query_pairs(rl, output_type="set")), dtype=np.int64)
        assert len(mine) == len(ref) and len(ref) > 0
        np.testing.assert_array_equal(mine, ref)
        # lexicographic, a < b
        assert np.all(mine[:, 0] < mine[:, 1])
        key = mine[:, 0].astype(np.int64) * wl.n_mol + mine[:, 1]
        assert np.all(np.diff(key) > 0)

    def test_neighbours_of_matches_pair_set(self):
        """The per-molecule brute force (NumPy) gives the same sets as the C pair list."""
        wl = inputs.workload("small_slab")
        x, _ = inputs.make_state(wl, seed=5)
        m = oracle.Model(wl)
        com, _, _, _ = m.weights(x)
        pairs = m.pairs(com)
        sel = np.array([0, 7, 123, 500, 999])
        for t, nb in zip(sel, m.neighbours_of(com, sel)):
            ref = np.sort(np.concatenate([pairs[pairs[:, 0] == t, 1], pairs[pairs[:, 1] == t, 0]]))
            np.testing.assert_array_equal(nb, ref)

    def test_list_radius(self):
        m = oracle.Model(inputs.workload("c2"))
        assert abs(m.r_list() - (max(2.31 * 2 ** (1 / 6), 2 ** (1 / 6) + 1.6) + 0.3)) < 1e-15
        m = oracle.Model(inputs.workload("c3"))   # (single beads, skin 0.5)
        assert abs(m.r_list() - (2 ** (1 / 6) + 0.5)) < 1e-15
        m = oracle.Model(inputs.workload("c4"))
        assert abs(m.r_list() - 3.3) < 1e-15


# ---------------------------------------------------------------- Eq. (1) and its limits
def _energy_grad_check(wl, x, n_check=12, h=1e-6, seed=0, td=None):
    """Central finite differences of the oracle's total potential vs its forces."""
    m = oracle.Model(wl, td=td)
    f, amag, e, st = m.forces(x)
    assert st == 0
    rng = np.random.default_rng(seed)
    ns = x.shape[1]
    for _ in range(n_check):
        q, s = rng.integers(3), rng.integers(ns)
        xp, xm = x.copy(), x.copy()
        xp[q, s] += h
        xm[q, s] -= h
        ep = m.forces(xp)[2].sum()
        em = m.forces(xm)[2].sum()
        fd = -(ep - em) / (2 * h)
        assert abs(f[q, s] - fd) < 2e-5 * max(1.0, amag[s]), (q, s, f[q, s], fd)


class TestLimitsAndEq1:
    def test_all_at_limit_is_gradient(self):
        wl = inputs.workload("tiny_slab").with_(region=inputs.REGION_ALL_AT)
        x, _ = inputs.make_state(wl)
        _energy_grad_check(wl, x)

    def test_all_cg_limit_is_gradient_with_mass_fractions(self):
        # unequal masses: the CG force reaches each site with its mass fraction, which is
        # exactly -dU_CG(R)/dx_i = -(m_i / M) dU/dR
        wl = inputs.workload("tiny_slab").with_(region=inputs.REGION_ALL_CG, site_mass=(1.0, 2.0, 3.0, 4.0))
        x, _ = inputs.make_state(wl)
        _energy_grad_check(wl, x)

    def test_all_cg_net_force_is_com_force(self):
        """Sum over a molecule's sites = WCA(sigma_cg) between centres of mass."""
        wl = _wl(n_mol=2, sites_per_mol=4, site_mass=(1.0, 1.0, 1.0, 1.0), region=inputs.REGION_ALL_CG,
                 rho_max=0.8)
        rng = np.random.default_rng(3)
        body = inputs.tetra_positions(np.array([[6.0, 8.0], [6.0, 6.3], [6.0, 6.9]]), rng)
        f, _, e, st = oracle.Model(wl).forces(body)
        R0 = body[:, :4].mean(axis=1)
        R1 = body[:, 4:].mean(axis=1)
        D = R0 - R1
        r = np.linalg.norm(D)
        s6 = (2.31 / r) ** 6
        fmag = 24 * s6 * (2 * s6 - 1) / r
        assert r < 2.31 * 2 ** (1 / 6) and fmag > 1.0
        np.testing.assert_allclose(f[:, :4].sum(axis=1), fmag * D / r, rtol=1e-12, atol=1e-12)
        # no torque about the centre of mass from the CG part
        torque = np.cross((body[:, :4] - R0[:, None]).T, f[:, :4].T).sum(axis=0)
        assert np.max(np.abs(torque)) < 1e-12
        assert abs(e[1] - (4 * s6 * (s6 - 1) + 1)) < 1e-12

    def test_interpolation_is_affine_in_ww(self):
        """Eq. (1): two molecules moved together through the hybrid slab; at each position
        F = ww F_AT + (1 - ww) F_CG with F_AT, F_CG the two limits."""
        L = 24.0
        rng = np.random.default_rng(5)
        body = inputs.tetra_positions(np.array([[0.0, 0.0], [0.0, 1.9], [0.0, 0.4]]), rng)
        kw = dict(n_mol=2, sites_per_mol=4, site_mass=(1.0, 1.0, 1.0, 1.0), box=(L, L, L),
                  center=(12.0, 12.0, 12.0), d_at=2.0, d_hy=3.0, rho_max=0.8)
        seen = set()
        for xc in np.linspace(12.0, 18.5, 27):
            x = body + np.array([[xc], [10.0], [10.0]])
            x = inputs.wrap_into_box(x, (L, L, L))
            fm, _, _, _ = oracle.Model(_wl(region=inputs.REGION_SLAB_X, **kw)).forces(x)
            fa, _, _, _ = oracle.Model(_wl(region=inputs.REGION_ALL_AT, **kw)).forces(x)
            fc, _, _, _ = oracle.Model(_wl(region=inputs.REGION_ALL_CG, **kw)).forces(x)
            _, w, _, _ = oracle.Model(_wl(region=inputs.REGION_SLAB_X, **kw)).weights(x)
            ww = w[0] * w[1]
            seen.add("at" if ww == 1 else "cg" if ww == 0 else "hy")
            np.testing.assert_allclose(fm, ww * fa + (1 - ww) * fc, rtol=0, atol=1e-12 * np.abs(fa).max())
        assert seen == {"at", "cg", "hy"}

    def test_newton_third_law_hybrid(self):
        """Sec. 2.3: force interpolation keeps Newton's third law exactly."""
        wl = inputs.workload("small_slab")
        x, _ = inputs.make_state(wl)
        f, amag, e, st = oracle.Model(wl).forces(x)
        assert st == 0
        assert np.all(np.abs(f.sum(axis=1)) < 64 * EPS * amag.sum())

    def test_amag_bounds_force(self):
        wl = inputs.workload("tiny_slab")
        x, _ = inputs.make_state(wl)
        f, amag, _, _ = oracle.Model(wl).forces(x)
        assert np.all(np.linalg.norm(f, axis=0) <= amag * (1 + 1e-12))

    def test_sampled_equals_full(self):
        wl = inputs.workload("small_slab")
        x, _ = inputs.make_state(wl)
        m = oracle.Model(wl)
        f, amag, _, _ = m.forces(x)
        sel = np.array([0, 17, 500, 999])
        fs, am, _ = m.forces_sampled(x, sel)
        for k, a in enumerate(sel):
            np.testing.assert_array_equal(fs[k], f[:, 4 * a:4 * a + 4])
            np.testing.assert_array_equal(am[k], amag[4 * a:4 * a + 4])


# ---------------------------------------------------------------- velocity Verlet
class TestVelocityVerlet:
    def test_harmonic_discrete_map(self):
        """One bond, motion along its axis: VV is the linear map [[1-a/2, dt],[-w2 dt (1-a/4), 1-a/2]]
        on (q, u) = (r - b0, dr/dt), a = w2 dt^2, w2 = 2K/m (reduced mass m/2)."""
        K, m, dt, n = 400.0, 1.0, 0.01, 250
        wl = _wl(n_mol=1, sites_per_mol=2, site_mass=(m, m), bond_kind=inputs.BOND_HARMONIC,
                 k_bond=K, r0_bond=1.0, rho_max=5.0)
        q0, u0 = 0.07, -0.3
        x = _soa([[5.0, 5.0, 5.0], [6.0 + q0, 5.0, 5.0]])
        v = _soa([[-u0 / 2, 0, 0], [u0 / 2, 0, 0]])
        xo, vo, _, _, st = oracle.Model(wl).vv(x, v, dt, n)
        w2 = 2 * K / m
        a = w2 * dt * dt
        Mx = np.array([[1 - a / 2, dt], [-w2 * dt * (1 - a / 4), 1 - a / 2]])
        q, u = np.linalg.matrix_power(Mx, n) @ np.array([q0, u0])
        assert abs((xo[0, 1] - xo[0, 0] - 1.0) - q) < 1e-11
        assert abs((vo[0, 1] - vo[0, 0]) - u) < 1e-10
        # centre of mass does not move
        assert abs(xo[0].mean() - (5.5 + q0 / 2)) < 1e-12

    def _nve_fluct(self, wl, dt, n):
        x, v = inputs.make_state(wl)
        _, _, _, e, st = oracle.Model(wl).vv(x, v, dt, n)
        tot = e.sum(axis=1)
        return tot, st

    @pytest.mark.parametrize("region", [inputs.REGION_ALL_AT, inputs.REGION_ALL_CG])
    def test_nve_limits_dt2(self, region):
        """Conservative limits (w == 1, w == 0) conserve energy to O(dt^2) under VV."""
        wl = inputs.workload("tiny_slab").with_(region=region)
        t1, st = self._nve_fluct(wl, 0.002, 100)
        t2, _ = self._nve_fluct(wl, 0.001, 200)
        assert st == 0
        f1 = np.max(np.abs(t1 - t1[0]))
        f2 = np.max(np.abs(t2 - t2[0]))
        assert f1 < 5e-3 * abs(t1[0]) + 1e-2
        assert 2.5 < f1 / f2 < 6.0, (f1, f2)

    def test_nve_kg_chain(self):
        wl = inputs.workload("small_kg").with_(n_mol=1000, chain_len=50,
                                               box=((1000 / 0.85) ** (1 / 3),) * 3)
        t1, st = self._nve_fluct(wl, 0.002, 50)
        assert st == 0
        assert np.max(np.abs(t1 - t1[0])) < 1e-3 * abs(t1[0])

    def test_reversibility(self):
        wl = inputs.workload("tiny_slab")
        x, v = inputs.make_state(wl)
        m = oracle.Model(wl)
        x1, v1, _, _, _ = m.vv(x, v, 0.005, 40)
        x2, v2, _, _, _ = m.vv(x1, -v1, 0.005, 40)
        d = np.mod(x2 - x + 0.5 * wl.box[0], wl.box[0]) - 0.5 * wl.box[0]
        assert np.max(np.abs(d)) < 1e-9
        assert np.max(np.abs(v2 + v)) < 1e-8

    def test_momentum_conserved_hybrid(self):
        wl = inputs.workload("small_slab")
        x, v = inputs.make_state(wl)
        _, v1, _, e, st = oracle.Model(wl).vv(x, v, 0.005, 20)
        assert st == 0
        assert np.max(np.abs(v1.sum(axis=1) - v.sum(axis=1))) < 1e-10


# ---------------------------------------------------------------- golden closed forms
def _golden(kind):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.txt")
    rows = []
    with open(path) as f:
        for line in f:
            parts = line.split()
            if parts and parts[0] == kind:
                rows.append([float(v) for v in parts[1:]])
    assert rows, kind
    return rows


def test_golden_weights():
    for d_at, d_hy, d, w in _golden("weight"):
        assert abs(oracle.weight_of_distance(d, d_at, d_hy) - w) <= 1e-15, (d_at, d_hy, d)


def test_weight_without_hybrid_layer_is_a_step():
    # d_hy = 0: exactly 1 up to and including d_at, exactly 0 beyond (no cosine evaluated)
    for d_at in (0.0, 1.5, 4.0):
        for d, w in ((0.0, 1.0), (d_at, 1.0), (np.nextafter(d_at, np.inf), 0.0), (d_at + 3.0, 0.0)):
            assert oracle.weight_of_distance(d, d_at, 0.0) == w, (d_at, d)


def test_golden_wca():
    from oracle import tables
    for sig, eps, r, f in _golden("wca"):
        got, _ = tables.wca_force(np.array([r]), sig, eps, sig * 2 ** (1 / 6) * (1 + 1e-12))
        assert abs(got[0] - f) <= 1e-12 * max(1.0, abs(f)), (sig, eps, r, got[0])


def test_golden_tetra_rho():
    (edge, rho), = _golden("tetra_rho")
    wl = inputs.workload("c1").with_(n_mol=1, box=(10.0, 10.0, 10.0), center=(5.0, 5.0, 5.0))
    a = edge / (2.0 * math.sqrt(2.0))
    verts = np.array([[a, a, a], [a, -a, -a], [-a, a, -a], [-a, -a, a]]) + 5.0
    _, _, rh, st = oracle.Model(wl).weights(np.ascontiguousarray(verts.T))
    assert st == 0 and abs(rh[0] - rho) <= 1e-15


# ---------------------------------------------------------------- Eq. (2): H-AdResS
class TestHamiltonianScheme:
    """Potential energy interpolation (Eq. (2)): the forces are minus the gradient of the
    interpolated potential, drift term included, so central differences of the oracle's
    own energy pin them in the hybrid case; in the w == 1 and w == 0 limits the scheme is
    force interpolation; and velocity Verlet conserves its energy to O(dt^2) even with a
    hybrid layer, which force interpolation cannot (Sec. 2.3)."""

    @pytest.mark.parametrize("name", ["tiny_slab", "small_sphere"])
    def test_forces_are_minus_gradient(self, name):
        wl = inputs.workload(name).with_(scheme=inputs.SCHEME_HAMILTONIAN)
        if name == "small_sphere":
            wl = wl.with_(n_mol=216, box=((216 / 0.1) ** (1 / 3),) * 3, d_at=2.0, d_hy=3.0,
                          center=(((216 / 0.1) ** (1 / 3)) / 2,) * 3)
        x, _ = inputs.make_state(wl, seed=11)
        _, w, _, _ = oracle.Model(wl).weights(x)
        assert ((w > 0) & (w < 1)).any()
        _energy_grad_check(wl, x, n_check=16)

    @pytest.mark.parametrize("region", [inputs.REGION_ALL_AT, inputs.REGION_ALL_CG])
    def test_limits_equal_force_interpolation(self, region):
        wl = inputs.workload("tiny_slab").with_(region=region)
        x, _ = inputs.make_state(wl, seed=4)
        f1, a1, e1, _ = oracle.Model(wl).forces(x)
        f2, a2, e2, _ = oracle.Model(wl.with_(scheme=inputs.SCHEME_HAMILTONIAN)).forces(x)
        np.testing.assert_array_equal(f1, f2)
        np.testing.assert_allclose(e1, e2, rtol=1e-14)

    def test_drift_breaks_newton3_only_in_hybrid_layer(self):
        wl = inputs.workload("tiny_slab").with_(scheme=inputs.SCHEME_HAMILTONIAN)
        x, _ = inputs.make_state(wl)
        m = oracle.Model(wl)
        f, amag, _, _ = m.forces(x)
        _, w, _, _ = m.weights(x)
        hy = (w > 0) & (w < 1)
        assert hy.any()
        net = np.abs(f.sum(axis=1)).max()
        assert net > 1e3 * EPS * amag.sum()

    def test_nve_conserves_energy_with_hybrid_layer(self):
        wl = inputs.workload("tiny_slab").with_(scheme=inputs.SCHEME_HAMILTONIAN)
        x, v = inputs.make_state(wl)
        m = oracle.Model(wl)
        _, _, _, e1, st = m.vv(x, v, 0.002, 100)
        _, _, _, e2, _ = m.vv(x, v, 0.001, 200)
        assert st == 0
        t1, t2 = e1.sum(axis=1), e2.sum(axis=1)
        f1, f2 = np.max(np.abs(t1 - t1[0])), np.max(np.abs(t2 - t2[0]))
        assert f1 < 5e-3 * abs(t1[0]) + 1e-2
        assert 2.5 < f1 / f2 < 6.0, (f1, f2)


# ---------------------------------------------------------------- correction force (Sec. 2.4)
class TestCorrectionForce:
    """The correction (thermodynamic) force along the resolution coordinate: closed forms of
    its piecewise-linear table and of the potential, the direction (slab sign, sphere
    unit offset), the mass-fraction split, forces = -grad of the energy including its
    potential, the density histogram against NumPy's, and the refinement step on density
    profiles whose slopes are known exactly."""

    LO, HI, N = 2.0, 6.0, 8          # bin centres 2.25, 2.75, ..., 5.75; h = 0.5

    def _single(self, region, R, td, masses=(1.0,)):
        wl = _wl(n_mol=1, sites_per_mol=len(masses), site_mass=masses, region=region,
                 rho_max=0.8 if len(masses) > 1 else 0.0)
        if len(masses) == 1:
            x = _soa([R])
        else:
            rng = np.random.default_rng(5)
            x = inputs.tetra_positions(np.asarray(R, dtype=np.float64).reshape(3, 1), rng)
        return oracle.Model(wl, td=td), x

    def test_linear_table_closed_form_slab(self):
        a, b = 0.7, -0.3
        h = (self.HI - self.LO) / self.N
        cent = self.LO + (np.arange(self.N) + 0.5) * h
        F = a + b * cent
        d0, dn = cent[0], cent[-1]
        for d in [0.5, 1.99, 2.0, 2.1, 2.25, 3.1, 4.0, 5.6, 5.75, 5.9, 6.0, 7.5]:
            for side in (1.0, -1.0):
                m, x = self._single(inputs.REGION_SLAB_X, (10.0 + side * d, 10.0, 10.0), (F, self.LO, self.HI))
                f, amag, e, st = m.forces(x)
                assert st == 0
                if d < self.LO or d >= self.HI:
                    val = 0.0
                elif d <= d0:
                    val = F[0]
                elif d >= dn:
                    val = F[-1]
                else:
                    val = a + b * d
                np.testing.assert_allclose(f[:, 0], [side * val, 0.0, 0.0], atol=1e-14)
                # potential: -(F_0 (d_0 - lo) + integral of a + b s from d_0, F_n-1 beyond d_n-1)
                top = min(max(d, self.LO), self.HI)
                U = 0.0
                U -= F[0] * (min(top, d0) - self.LO)
                if top > d0:
                    t = min(top, dn)
                    U -= a * (t - d0) + 0.5 * b * (t * t - d0 * d0)
                if top > dn:
                    U -= F[-1] * (top - dn)
                assert abs(e[3] - U) < 1e-13, (d, e[3], U)

    def test_sphere_direction_and_mass_fractions(self):
        F = np.linspace(1.0, 2.0, self.N)
        masses = (1.0, 2.0, 3.0, 4.0)
        rng = np.random.default_rng(2)
        for _ in range(5):
            u = rng.normal(size=3); u /= np.linalg.norm(u)
            d = rng.uniform(self.LO + 0.1, self.HI - 0.1)
            R = np.array([10.0, 10.0, 10.0]) + d * u
            m, x = self._single(inputs.REGION_SPHERE, R, (F, self.LO, self.HI), masses)
            com, _, _, _ = m.weights(x)
            q = com[:, 0] - 10.0
            dd = np.linalg.norm(q)
            f, _, _, st = m.forces(x)
            assert st == 0
            # single molecule: no pair or bond forces, only the correction
            h = (self.HI - self.LO) / self.N
            val = np.interp(dd, self.LO + (np.arange(self.N) + 0.5) * h, F)
            for i, mi in enumerate(masses):
                np.testing.assert_allclose(f[:, i], (mi / 10.0) * val * q / dd, rtol=1e-12, atol=1e-14)

    @pytest.mark.parametrize("scheme", [inputs.SCHEME_FORCE, inputs.SCHEME_HAMILTONIAN])
    def test_forces_are_minus_gradient_with_correction(self, scheme):
        # a hybrid slab in the all-AT limit of the pair forces is conservative (FI has no
        # energy otherwise); with the Hamiltonian scheme the hybrid layer is kept
        wl = inputs.workload("tiny_slab").with_(scheme=scheme)
        if scheme == inputs.SCHEME_FORCE:
            wl = wl.with_(d_at=50.0)
        rng = np.random.default_rng(8)
        F = rng.normal(size=12)
        x, _ = inputs.make_state(wl, seed=11)
        _energy_grad_check(wl, x, n_check=16, td=(F, 0.3, 3.9))

    def test_zero_table_is_no_correction(self):
        wl = inputs.workload("tiny_slab")
        x, _ = inputs.make_state(wl)
        f0, _, e0, _ = oracle.Model(wl).forces(x)
        f1, _, e1, _ = oracle.Model(wl, td=(np.zeros(5), 0.5, 3.0)).forces(x)
        np.testing.assert_array_equal(f0, f1)
        assert e1[3] == 0.0

    @pytest.mark.parametrize("name", ["small_slab", "small_sphere"])
    def test_density_histogram_equals_numpy(self, name):
        wl = inputs.workload(name)
        x, _ = inputs.make_state(wl)
        m = oracle.Model(wl)
        com, _, _, _ = m.weights(x)
        c = np.asarray(wl.center)[:, None]
        L = np.asarray(wl.box)[:, None]
        q = com - c
        q = q - L * np.round(q / L)
        d = np.abs(q[0]) if wl.region == inputs.REGION_SLAB_X else np.sqrt((q * q).sum(axis=0))
        lo, hi, nb = 1.0, 0.5 * wl.box[0] - 0.5, 37
        counts = m.density_profile(x, nb, lo, hi)
        ref, _ = np.histogram(d, bins=nb, range=(lo, hi))
        np.testing.assert_array_equal(counts, ref)
        # accumulates
        counts2 = m.density_profile(x, nb, lo, hi, counts.copy())
        np.testing.assert_array_equal(counts2, 2 * ref)

    def test_update_on_linear_slab_profile(self):
        wl = inputs.workload("small_slab")
        m = oracle.Model(wl)
        n, lo, hi, frames, c = 9, 1.0, 10.0, 7, 0.25
        h = (hi - lo) / n
        alpha, beta = 40, 3
        counts = alpha + beta * np.arange(n)
        F = np.linspace(-1.0, 1.0, n)
        V = 2.0 * h * wl.box[1] * wl.box[2]
        got = m.tdforce_update(F, lo, hi, counts, frames, c)
        np.testing.assert_allclose(got, F - c * beta / (frames * V * h), rtol=0, atol=1e-14)

    def test_update_on_uniform_sphere_profile(self):
        # counts proportional to the shell volumes ((k+1)^3 - k^3 for lo = 0): a flat
        # density, so the update leaves the force unchanged up to rounding
        wl = inputs.workload("small_sphere")
        m = oracle.Model(wl)
        n, lo, hi, frames, c = 10, 0.0, 5.0, 3, 2.0
        k = np.arange(n)
        counts = 6 * (3 * k * k + 3 * k + 1)
        F = np.linspace(0.5, -0.5, n)
        h = (hi - lo) / n
        rho = 6 / (frames * (4.0 / 3.0) * np.pi * h ** 3)
        got = m.tdforce_update(F, lo, hi, counts, frames, c)
        assert np.abs(got - F).max() <= 1e-12 * c * rho / h
        # and a density rising by one shell volume's worth per bin moves it by a known slope
        counts2 = (6 + k) * (3 * k * k + 3 * k + 1)
        got2 = m.tdforce_update(F, lo, hi, counts2, frames, c)
        drho = 1 / (frames * (4.0 / 3.0) * np.pi * h ** 3)      # rho_k = (6 + k) drho
        np.testing.assert_allclose(got2, F - c * drho / h, rtol=1e-12)


# ---------------------------------------------------------------- multiple time stepping (Sec. 2.6)
class TestRespa:
    """RESPA with the CG part on the outer step: the two parts add up to the full force,
    each part vanishes where its model is absent, one inner step per outer step is
    velocity Verlet, the integrator is time-reversible, and with the Hamiltonian scheme
    it conserves energy to O(dt^2)."""

    @pytest.mark.parametrize("name,scheme,td", [("tiny_slab", 0, False), ("small_sphere", 1, True),
                                                ("tiny_slab", 1, True)])
    def test_parts_add_up(self, name, scheme, td):
        wl = inputs.workload(name).with_(scheme=scheme)
        if name == "small_sphere":
            wl = wl.with_(n_mol=216, box=((216 / 0.1) ** (1 / 3),) * 3, d_at=2.0, d_hy=3.0,
                          center=(((216 / 0.1) ** (1 / 3)) / 2,) * 3)
        tab = (np.linspace(0.5, -0.5, 9), 0.5, 3.5) if td else None
        x, _ = inputs.make_state(wl, seed=3)
        m = oracle.Model(wl, td=tab)
        f, amag, e, _ = m.forces(x)
        ff, _, _, _ = m.forces_part(x, 1)
        fs, _, _, _ = m.forces_part(x, 2)
        assert np.abs(ff).max() > 0 and np.abs(fs).max() > 0
        assert np.all(np.abs(ff + fs - f) <= 8 * EPS * amag)

    def test_each_part_vanishes_without_its_model(self):
        wl = inputs.workload("tiny_slab").with_(region=inputs.REGION_ALL_AT)
        x, _ = inputs.make_state(wl)
        fs, _, _, _ = oracle.Model(wl).forces_part(x, 2)
        assert np.all(fs == 0.0)
        wl = inputs.workload("tiny_slab").with_(region=inputs.REGION_ALL_CG, bond_kind=inputs.BOND_NONE)
        ff, _, _, _ = oracle.Model(wl).forces_part(x, 1)
        assert np.all(ff == 0.0)

    def test_single_inner_step_is_velocity_verlet(self):
        wl = inputs.workload("tiny_slab")
        x, v = inputs.make_state(wl)
        m = oracle.Model(wl)
        x1, v1, f1, _, _ = m.vv(x, v, wl.dt, 20)
        x2, v2, f2, _, _ = m.respa(x, v, wl.dt, 1, 20)
        np.testing.assert_allclose(x2, x1, atol=1e-11)
        np.testing.assert_allclose(v2, v1, atol=1e-9)
        np.testing.assert_allclose(f2, f1, atol=1e-7 * np.abs(f1).max())
        # and a longer outer step is a different integrator
        x3, _, _, _, _ = m.respa(x, v, wl.dt / 2, 2, 20)
        x4, _, _, _, _ = m.vv(x, v, wl.dt / 2, 40)
        assert np.abs(x3 - x4).max() > 1e-9

    def test_time_reversible(self):
        wl = inputs.workload("tiny_slab").with_(scheme=inputs.SCHEME_HAMILTONIAN)
        x, v = inputs.make_state(wl)
        m = oracle.Model(wl)
        x1, v1, _, _, st = m.respa(x, v, 0.002, 3, 15)
        assert st == 0
        x2, v2, _, _, _ = m.respa(x1, -v1, 0.002, 3, 15)
        d = x2 - x
        d -= np.asarray(wl.box)[:, None] * np.round(d / np.asarray(wl.box)[:, None])
        assert np.abs(d).max() < 1e-9
        assert np.abs(v2 + v).max() < 1e-8

    def test_hamiltonian_energy_error_is_dt2(self):
        wl = inputs.workload("tiny_slab").with_(scheme=inputs.SCHEME_HAMILTONIAN)
        x, v = inputs.make_state(wl)
        m = oracle.Model(wl)
        _, _, _, e1, st = m.respa(x, v, 0.002, 2, 50)
        _, _, _, e2, _ = m.respa(x, v, 0.001, 2, 100)
        assert st == 0
        t1, t2 = e1.sum(axis=1), e2.sum(axis=1)
        f1, f2 = np.abs(t1 - t1[0]).max(), np.abs(t2 - t2[0]).max()
        assert f1 < 5e-3 * abs(t1[0]) + 1e-2
        assert 2.5 < f1 / f2 < 6.0, (f1, f2)


# ---------------------------------------------------------------- self-adjusting regions (Sec. 2.5)
class TestAnchorSpheres:
    """The AT region as the union of spheres around anchor molecules: one anchor is exactly
    a static sphere centred at its centre of mass, several anchors give the largest of the
    single-sphere weights, anchors are atomistic, and the region follows the anchors."""

    def _wl(self):
        return inputs.workload("small_sphere").with_(region=inputs.REGION_SPHERES, d_at=2.5, d_hy=2.0)

    def test_one_anchor_is_a_static_sphere(self):
        wl = self._wl()
        x, _ = inputs.make_state(wl)
        an = np.array([417], dtype=np.int32)
        m = oracle.Model(wl, anchors=an)
        com, w, _, st = m.weights(x)
        assert st == 0
        ws = wl.with_(region=inputs.REGION_SPHERE, center=tuple(com[:, 417]))
        com2, w2, _, _ = oracle.Model(ws).weights(x)
        np.testing.assert_array_equal(w, w2)
        assert ((w > 0) & (w < 1)).any() and (w == 1).sum() > 1
        f1, _, e1, _ = m.forces(x)
        f2, _, e2, _ = oracle.Model(ws).forces(x)
        np.testing.assert_array_equal(f1, f2)

    def test_several_anchors_take_the_largest_weight(self):
        wl = self._wl()
        x, _ = inputs.make_state(wl)
        an = inputs.anchor_molecules(wl.n_mol, 9, 3)
        com, w, _, _ = oracle.Model(wl, anchors=an).weights(x)
        single = []
        for a in an:
            ws = wl.with_(region=inputs.REGION_SPHERE, center=tuple(com[:, a]))
            single.append(oracle.Model(ws).weights(x)[1])
        np.testing.assert_array_equal(w, np.max(single, axis=0))
        assert np.all(w[an] == 1.0)

    def test_region_follows_the_anchor(self):
        wl = self._wl()
        x, _ = inputs.make_state(wl)
        an = np.array([100], dtype=np.int32)
        m = oracle.Model(wl, anchors=an)
        _, w0, _, _ = m.weights(x)
        x2 = x.copy()
        x2[:, 400:404] += np.array([[3.0], [-2.0], [1.0]])      # move anchor 100 (sites 400..403)
        x2 = inputs.wrap_into_box(x2, wl.box)
        com2, w2, _, _ = m.weights(x2)
        ws = wl.with_(region=inputs.REGION_SPHERE, center=tuple(com2[:, 100]))
        np.testing.assert_array_equal(w2, oracle.Model(ws).weights(x2)[1])
        assert not np.array_equal(w0, w2)

    def test_newton3_with_anchor_spheres(self):
        wl = self._wl()
        x, _ = inputs.make_state(wl)
        an = inputs.anchor_molecules(wl.n_mol, 5, 1)
        f, amag, _, st = oracle.Model(wl, anchors=an).forces(x)
        assert st == 0
        assert np.all(np.abs(f.sum(axis=1)) <= 64 * EPS * amag.sum())

    def test_one_anchor_with_correction_is_a_static_sphere(self):
        wl = self._wl()
        x, _ = inputs.make_state(wl)
        an = np.array([417], dtype=np.int32)
        td = (np.linspace(1.0, -0.5, 10), 1.0, 5.5)
        m = oracle.Model(wl, anchors=an, td=td)
        com, _, _, _ = m.weights(x)
        ws = wl.with_(region=inputs.REGION_SPHERE, center=tuple(com[:, 417]))
        f1, _, e1, _ = m.forces(x)
        f2, _, e2, _ = oracle.Model(ws, td=td).forces(x)
        np.testing.assert_array_equal(f1, f2)
        np.testing.assert_array_equal(e1, e2)
        assert e1[3] != 0.0

    def test_correction_points_away_from_the_nearest_anchor(self):
        # three single-site molecules far apart: anchors 0 and 1, molecule 2 nearer to 1
        wl = _wl(n_mol=3, region=inputs.REGION_SPHERES, d_at=1.0, d_hy=1.0, box=(30.0, 30.0, 30.0),
                 center=(15.0, 15.0, 15.0))
        x = _soa([[5.0, 5.0, 5.0], [20.0, 20.0, 20.0], [22.0, 21.5, 21.5]])   # beyond every pair cutoff
        F = np.linspace(2.0, 3.0, 8)
        lo, hi = 0.5, 4.5
        f, _, e, st = oracle.Model(wl, anchors=np.array([0, 1], np.int32), td=(F, lo, hi)).forces(x)
        assert st == 0
        q = x[:, 2] - x[:, 1]
        d = np.linalg.norm(q)
        h = (hi - lo) / len(F)
        val = np.interp(d, lo + (np.arange(len(F)) + 0.5) * h, F)
        np.testing.assert_allclose(f[:, 2], val * q / d, rtol=1e-12)
        np.testing.assert_array_equal(f[:, :2], 0.0)    # anchors: d = 0, no reaction

    def test_correction_is_minus_gradient_for_non_anchor_sites(self):
        # w == 1 everywhere (anchor spheres larger than the box): pair forces are
        # conservative, the correction is the gradient of U_corr for every non-anchor site
        wl = inputs.workload("tiny_slab").with_(region=inputs.REGION_SPHERES, d_at=20.0, d_hy=1.0)
        x, _ = inputs.make_state(wl, seed=3)
        an = np.array([5, 40], dtype=np.int32)
        td = (np.random.default_rng(2).normal(size=12), 0.2, 4.0)
        m = oracle.Model(wl, anchors=an, td=td)
        f, amag, e, st = m.forces(x)
        assert st == 0 and e[3] != 0.0
        rng = np.random.default_rng(0)
        sites = [s for s in range(x.shape[1]) if s // 4 not in an]
        for _ in range(16):
            qd, s = rng.integers(3), int(rng.choice(sites))
            xp, xm = x.copy(), x.copy()
            xp[qd, s] += 1e-6
            xm[qd, s] -= 1e-6
            fd = -(m.forces(xp)[2].sum() - m.forces(xm)[2].sum()) / 2e-6
            assert abs(f[qd, s] - fd) < 2e-5 * max(1.0, amag[s]), (qd, s, f[qd, s], fd)


# ---------------------------------------------------------------- sampled bin volumes (Sec. 2.4 + 2.5)
class TestSampledVolumes:
    """Bin volumes by uniform sampling (SplitMix64 points) for regions without closed-form
    bins: they reproduce the exact slab and sphere volumes within binomial error, the
    anchor-sphere density profile is NumPy's histogram of nearest-anchor distances, and a
    refinement with sampled volumes has the closed form of a known profile."""

    @pytest.mark.parametrize("region", [inputs.REGION_SLAB_X, inputs.REGION_SPHERE, inputs.REGION_SPHERES])
    def test_volumes_match_closed_forms(self, region):
        wl = inputs.workload("small_sphere").with_(region=region)
        x, _ = inputs.make_state(wl)
        an = None
        if region == inputs.REGION_SPHERES:
            an = np.array([100], np.int32)       # one anchor: its shells are spheres
        m = oracle.Model(wl, anchors=an)
        n, lo, hi, N = 12, 0.5, 6.5, 400_000
        vc = m.region_volumes(x, N, 12345, n, lo, hi)
        h = (hi - lo) / n
        r = lo + np.arange(n + 1) * h
        L = np.asarray(wl.box)
        if region == inputs.REGION_SLAB_X:
            V = np.full(n, 2 * h * L[1] * L[2])
        else:
            V = 4.0 / 3.0 * np.pi * (r[1:] ** 3 - r[:-1] ** 3)
        p = V / L.prod()
        assert np.all(np.abs(vc - N * p) <= 5 * np.sqrt(N * p * (1 - p)) + 1), (vc, N * p)
        # same seed, same points; another seed, other points
        np.testing.assert_array_equal(vc, m.region_volumes(x, N, 12345, n, lo, hi))
        assert not np.array_equal(vc, m.region_volumes(x, N, 54321, n, lo, hi))

    def test_anchor_density_profile_is_histogram_of_nearest_distance(self):
        wl = inputs.workload("small_sphere").with_(region=inputs.REGION_SPHERES, d_at=2.5, d_hy=2.0)
        x, _ = inputs.make_state(wl)
        an = inputs.anchor_molecules(wl.n_mol, 7, 2)
        m = oracle.Model(wl, anchors=an)
        com, _, _, _ = m.weights(x)
        L = np.asarray(wl.box)[:, None, None]
        q = com[:, :, None] - com[:, an][:, None, :]
        q = q - L * np.round(q / L)
        d = np.sqrt((q * q).sum(axis=0)).min(axis=1)
        n, lo, hi = 20, 0.25, 8.0
        ref, _ = np.histogram(d, bins=n, range=(lo, hi))
        np.testing.assert_array_equal(m.density_profile(x, n, lo, hi), ref)

    def test_update_with_uniform_sampled_volumes(self):
        wl = inputs.workload("small_slab")
        m = oracle.Model(wl)
        n, lo, hi, frames, c = 9, 1.0, 10.0, 7, 0.25
        h = (hi - lo) / n
        counts = 40 + 3 * np.arange(n)
        vol = np.full(n, 1000, dtype=np.int64)
        V = 1000 / 1_000_000 * np.prod(wl.box)
        F = np.linspace(-1.0, 1.0, n)
        got = m.tdforce_update(F, lo, hi, counts, frames, c, vol_counts=vol, n_vol_samples=1_000_000)
        np.testing.assert_allclose(got, F - c * 3 / (frames * V * h), rtol=0, atol=1e-12)
