"""FP64 CPU oracle of the AdResS hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does, and this
package never imports the product: the two meet only in the seeded input
generators (``paper_1806_10841_amd.inputs``), which the *callers* use to make the
arrays handed to both sides.

``adres_oracle.c`` holds the definitions (centre of mass, resolution weight,
brute-force pair set, Eq. (1) forces summed over all molecules, bonded terms,
velocity Verlet); this module compiles it with gcc (``-O2 -ffp-contract=off
-fopenmp``) and wraps it with ctypes.  ``mlp.py`` is the FP64 NumPy oracle of
the learned CG force (forward, analytic backward, force-matching loss) and
``tables.py`` builds and evaluates cubic force tables.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "adres_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

STRETCH, FENE, TABLE_RANGE, NONFINITE = 1, 2, 4, 8
MAX_SITES = 8


def build(force: bool = True) -> str:
    """Compile the C oracle into oracle/liboracle.so (gcc, FP64, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [
        ("n_mol", C.c_int32), ("spm", C.c_int32),
        ("box", C.c_double * 3),
        ("mass", C.c_double * MAX_SITES),
        ("region", C.c_int32),
        ("center", C.c_double * 3), ("d_at", C.c_double), ("d_hy", C.c_double),
        ("eps_at", C.c_double), ("sig_at", C.c_double), ("rc_at", C.c_double),
        ("eps_cg", C.c_double), ("sig_cg", C.c_double), ("rc_cg", C.c_double),
        ("cg_kind", C.c_int32), ("bond_kind", C.c_int32),
        ("k_bond", C.c_double), ("r0_bond", C.c_double),
        ("chain_len", C.c_int32),
        ("rho_max", C.c_double),
        ("tab", C.POINTER(C.c_float)), ("tab_n", C.c_int32),
        ("tab_lo", C.c_double), ("tab_hi", C.c_double),
        ("mlp", C.POINTER(C.c_double)), ("mlp_hidden", C.c_int32),
        ("mlp_rc", C.c_double), ("mlp_scale", C.c_double), ("mlp_taper", C.c_double),
        ("mlp_rmin", C.c_double),
        ("scheme", C.c_int32),
        ("td", C.POINTER(C.c_double)), ("td_n", C.c_int32),
        ("td_lo", C.c_double), ("td_hi", C.c_double),
        ("anchors", C.POINTER(C.c_int32)), ("n_anchors", C.c_int32),
    ]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            L = C.CDLL(_LIB)
            P = C.POINTER(Params)
            dp = C.POINTER(C.c_double)
            L.orc_weights.argtypes = [P, dp, dp, dp, dp]
            L.orc_weights.restype = C.c_int
            L.orc_pairs.argtypes = [P, dp, C.c_double, C.POINTER(C.c_int32), C.c_int64]
            L.orc_pairs.restype = C.c_int64
            L.orc_forces.argtypes = [P, dp, dp, dp, dp]
            L.orc_forces.restype = C.c_int
            L.orc_forces_sampled.argtypes = [P, dp, C.POINTER(C.c_int64), C.c_int64, dp, dp]
            L.orc_forces_sampled.restype = C.c_int
            L.orc_vv.argtypes = [P, dp, dp, dp, C.c_double, C.c_int32, dp]
            L.orc_vv.restype = C.c_int
            L.orc_kinetic.argtypes = [P, dp]
            L.orc_kinetic.restype = C.c_double
            L.orc_weight_of_distance.argtypes = [C.c_double, C.c_double, C.c_double]
            L.orc_weight_of_distance.restype = C.c_double
            L.orc_table_eval.argtypes = [C.POINTER(C.c_float), C.c_int, C.c_double, C.c_double,
                                         C.c_double, C.POINTER(C.c_int)]
            L.orc_table_eval.restype = C.c_double
            L.orc_mlp_eval.argtypes = [P, C.c_double, C.POINTER(C.c_int)]
            L.orc_mlp_eval.restype = C.c_double
            L.orc_forces_part.argtypes = [P, dp, dp, dp, dp, C.c_int]
            L.orc_forces_part.restype = C.c_int
            L.orc_respa.argtypes = [P, dp, dp, dp, C.c_double, C.c_int32, C.c_int32, dp]
            L.orc_respa.restype = C.c_int
            L.orc_density_profile.argtypes = [P, dp, C.c_int32, C.c_double, C.c_double,
                                              C.POINTER(C.c_int64)]
            L.orc_density_profile.restype = C.c_int
            L.orc_tdforce_update.argtypes = [P, dp, C.c_int32, C.c_double, C.c_double,
                                             C.POINTER(C.c_int64), C.c_int64, C.c_double,
                                             C.POINTER(C.c_int64), C.c_int64]
            L.orc_tdforce_update.restype = None
            L.orc_region_volumes.argtypes = [P, dp, C.c_int64, C.c_uint64, C.c_int32, C.c_double, C.c_double,
                                             C.POINTER(C.c_int64)]
            L.orc_region_volumes.restype = C.c_int
            L.orc_num_threads.restype = C.c_int
            L.orc_set_num_threads.argtypes = [C.c_int]
            L.orc_set_num_threads.restype = None
            _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Model:
    """A workload's parameters marshalled for the C oracle, plus optional CG table/MLP.

    ``wl`` is any object with the attributes of ``inputs.Workload``.  ``table`` is
    (coef float32 [(n-1), 4], r_lo, r_hi); ``mlp`` is (params float64, rc, scale,
    taper_width, r_min); ``td`` is the correction force (values float64 [n] at the bin
    centres, lo, hi); ``anchors`` the anchor molecules of a self-adjusting region."""

    def __init__(self, wl, table=None, mlp=None, hidden=64, td=None, anchors=None):
        self.wl = wl
        p = Params()
        p.n_mol, p.spm = wl.n_mol, wl.sites_per_mol
        p.box = (C.c_double * 3)(*wl.box)
        m = list(wl.site_mass) + [0.0] * (MAX_SITES - len(wl.site_mass))
        p.mass = (C.c_double * MAX_SITES)(*m)
        p.region = wl.region
        p.center = (C.c_double * 3)(*wl.center)
        p.d_at, p.d_hy = wl.d_at, wl.d_hy
        p.eps_at, p.sig_at, p.rc_at = wl.eps_at, wl.sig_at, wl.rc_at
        p.eps_cg, p.sig_cg, p.rc_cg = wl.eps_cg, wl.sig_cg, wl.rc_cg
        p.cg_kind = wl.cg_kind
        p.bond_kind = wl.bond_kind
        p.k_bond, p.r0_bond = wl.k_bond, wl.r0_bond
        p.chain_len = max(int(wl.chain_len), 1)
        p.rho_max = wl.rho_max
        p.scheme = getattr(wl, "scheme", 0)
        self._keep = []
        if table is not None:
            coef, lo, hi = table
            coef = np.ascontiguousarray(coef, dtype=np.float32)
            self._keep.append(coef)
            p.tab = coef.ctypes.data_as(C.POINTER(C.c_float))
            p.tab_n = coef.shape[0] + 1
            p.tab_lo, p.tab_hi = lo, hi
        if mlp is not None:
            prm, rc, scale, taper, rmin = mlp
            prm = np.ascontiguousarray(prm, dtype=np.float64)
            self._keep.append(prm)
            p.mlp = _dp(prm)
            p.mlp_hidden = hidden
            p.mlp_rc, p.mlp_scale, p.mlp_taper, p.mlp_rmin = rc, scale, taper, rmin
        if td is not None:
            F, lo, hi = td
            F = np.ascontiguousarray(F, dtype=np.float64)
            self._keep.append(F)
            p.td = _dp(F)
            p.td_n = len(F)
            p.td_lo, p.td_hi = lo, hi
        if anchors is not None:
            an = np.ascontiguousarray(anchors, dtype=np.int32)
            self._keep.append(an)
            p.anchors = an.ctypes.data_as(C.POINTER(C.c_int32))
            p.n_anchors = len(an)
        self.p = p
        self.n_sites = wl.n_mol * wl.sites_per_mol

    # -- definitions ---------------------------------------------------------
    def r_list(self):
        """Molecule-pair list radius: r_mol + skin, r_mol the largest centre-of-mass
        distance at which two molecules can still interact (CG cutoff, or the atom
        cutoff plus twice the largest site-to-centre distance)."""
        wl = self.wl
        r_mol = 0.0
        if wl.region != 0:
            r_mol = max(r_mol, wl.rc_cg)
        if wl.region != 3:
            r_mol = max(r_mol, wl.rc_at + 2.0 * wl.rho_max)
        return r_mol + wl.r_skin

    def weights(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        n = self.wl.n_mol
        com = np.empty((3, n)); w = np.empty(n); rho = np.empty(n)
        st = lib().orc_weights(C.byref(self.p), _dp(x), _dp(com), _dp(w), _dp(rho))
        return com, w, rho, st

    def pairs(self, com, r_list=None):
        com = np.ascontiguousarray(com, dtype=np.float64)
        rl = self.r_list() if r_list is None else r_list
        rl2 = rl * rl
        n = lib().orc_pairs(C.byref(self.p), _dp(com), rl2, None, 0)
        out = np.empty((max(n, 1), 2), dtype=np.int32)
        lib().orc_pairs(C.byref(self.p), _dp(com), rl2,
                        out.ctypes.data_as(C.POINTER(C.c_int32)), n)
        return out[:n]

    def neighbours_of(self, com, sel, r_list=None):
        """Molecules within the list radius of each selected molecule, by brute force over
        all molecules (NumPy, same arithmetic as the C pair test: minimum image by one
        conditional shift, r2 = (dx*dx + dy*dy) + dz*dz < r_list^2).  Returns a list of
        sorted index arrays, one per selected molecule."""
        com = np.asarray(com, dtype=np.float64)
        rl = self.r_list() if r_list is None else r_list
        rl2 = rl * rl
        out = []
        for t in np.asarray(sel, dtype=np.int64):
            d2 = None
            for k in range(3):
                L = self.wl.box[k]
                h = 0.5 * L
                d = com[k] - com[k, t]
                d = np.where(d > h, d - L, np.where(d < -h, d + L, d))
                d2 = d * d if d2 is None else d2 + d * d
            nb = np.flatnonzero(d2 < rl2)
            out.append(nb[nb != t])
        return out

    def forces(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        f = np.empty_like(x); amag = np.empty(self.n_sites); e = np.zeros(4)
        st = lib().orc_forces(C.byref(self.p), _dp(x), _dp(f), _dp(amag), _dp(e))
        return f, amag, e, st

    def forces_part(self, x, part):
        """Forces of one part of the multiple-time-step split: 0 all, 1 fast (atomistic pair
        part, -V^AT grad w, bonds), 2 slow (CG pair part, +V^CG grad w, correction)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        f = np.empty_like(x); amag = np.empty(self.n_sites); e = np.zeros(4)
        st = lib().orc_forces_part(C.byref(self.p), _dp(x), _dp(f), _dp(amag), _dp(e), part)
        return f, amag, e, st

    def respa(self, x, v, dt, n_inner, n_outer):
        """RESPA with inner step dt; returns (x, v, f_total, energies[(n_outer+1), 5], status)."""
        x = np.array(x, dtype=np.float64, copy=True)
        v = np.array(v, dtype=np.float64, copy=True)
        f = np.empty_like(x)
        e = np.zeros((n_outer + 1, 5))
        st = lib().orc_respa(C.byref(self.p), _dp(x), _dp(v), _dp(f), dt, n_inner, n_outer, _dp(e))
        return x, v, f, e, st

    def forces_sampled(self, x, sel):
        """Forces on the sites of molecules ``sel``: returns f (n_sel, 3, spm), amag (n_sel, spm)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        sel = np.ascontiguousarray(sel, dtype=np.int64)
        spm = self.wl.sites_per_mol
        f = np.empty((len(sel), 3, spm)); amag = np.empty((len(sel), spm))
        st = lib().orc_forces_sampled(C.byref(self.p), _dp(x), sel.ctypes.data_as(C.POINTER(C.c_int64)),
                                      len(sel), _dp(f), _dp(amag))
        return f, amag, st

    def vv(self, x, v, dt, n_steps):
        """Velocity Verlet; returns (x, v, f, energies[(n_steps+1), 5], status), the energy
        columns U_AT, U_CG, U_bond, U_corr, kinetic."""
        x = np.array(x, dtype=np.float64, copy=True)
        v = np.array(v, dtype=np.float64, copy=True)
        f = np.empty_like(x)
        e = np.zeros((n_steps + 1, 5))
        st = lib().orc_vv(C.byref(self.p), _dp(x), _dp(v), _dp(f), dt, n_steps, _dp(e))
        return x, v, f, e, st

    def density_profile(self, x, n_bins, lo, hi, counts=None):
        """Adds the molecules' centre-of-mass distance histogram over [lo, hi) (n_bins equal
        bins) to ``counts`` (int64, a new zero array if None) and returns it."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        if counts is None:
            counts = np.zeros(n_bins, dtype=np.int64)
        st = lib().orc_density_profile(C.byref(self.p), _dp(x), n_bins, lo, hi,
                                       counts.ctypes.data_as(C.POINTER(C.c_int64)))
        assert st == 0, st
        return counts

    def tdforce_update(self, F, lo, hi, counts, n_frames, prefactor, vol_counts=None, n_vol_samples=0):
        """One refinement step of the correction force values F (returns a new array);
        with vol_counts the bin volumes are the sampled ones (region_volumes)."""
        F = np.array(F, dtype=np.float64, copy=True)
        counts = np.ascontiguousarray(counts, dtype=np.int64)
        vp = None
        if vol_counts is not None:
            vol_counts = np.ascontiguousarray(vol_counts, dtype=np.int64)
            vp = vol_counts.ctypes.data_as(C.POINTER(C.c_int64))
        lib().orc_tdforce_update(C.byref(self.p), _dp(F), len(F), lo, hi,
                                 counts.ctypes.data_as(C.POINTER(C.c_int64)), n_frames, prefactor,
                                 vp, int(n_vol_samples))
        return F

    def region_volumes(self, x, n_samples, seed, n_bins, lo, hi, counts=None):
        """Adds the resolution-distance histogram of n_samples uniform points (SplitMix64
        keyed by seed) to counts (int64, new zeros if None) and returns it."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        if counts is None:
            counts = np.zeros(n_bins, dtype=np.int64)
        st = lib().orc_region_volumes(C.byref(self.p), _dp(x), int(n_samples), int(seed) & (2**64 - 1),
                                      n_bins, lo, hi, counts.ctypes.data_as(C.POINTER(C.c_int64)))
        assert st == 0, st
        return counts

    def kinetic(self, v):
        v = np.ascontiguousarray(v, dtype=np.float64)
        return lib().orc_kinetic(C.byref(self.p), _dp(v))

    def mlp_eval(self, r):
        st = C.c_int(0)
        return np.array([lib().orc_mlp_eval(C.byref(self.p), float(q), C.byref(st)) for q in np.ravel(r)])


def weight_of_distance(d, d_at, d_hy):
    return lib().orc_weight_of_distance(float(d), float(d_at), float(d_hy))


def table_eval(coef, lo, hi, r):
    coef = np.ascontiguousarray(coef, dtype=np.float32)
    st = C.c_int(0)
    fp = coef.ctypes.data_as(C.POINTER(C.c_float))
    out = np.array([lib().orc_table_eval(fp, coef.shape[0] + 1, lo, hi, float(q), C.byref(st))
                    for q in np.ravel(r)])
    return out, st.value


def num_threads():
    return lib().orc_num_threads()


def set_num_threads(n):
    """OpenMP threads of later oracle calls (timing)."""
    lib().orc_set_num_threads(int(n))
