"""ctypes binding of libadres.so (the C ABI declared in include/adres.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  PyTorch provides device memory (``data_ptr``) and the stream
(``torch.cuda.current_stream().cuda_stream``).  There is no fallback: if the
library is not built, or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libadres.so")
MAX_SITES = 4

STATUS = {
    0: "ADRES_OK", -1: "ADRES_E_ARG", -2: "ADRES_E_NOMEM", -3: "ADRES_E_HIP", -4: "ADRES_E_BOX",
    -5: "ADRES_E_CAPACITY", -6: "ADRES_E_STRETCH", -7: "ADRES_E_NONFINITE", -8: "ADRES_E_FENE",
    -9: "ADRES_E_TABLE_RANGE", -10: "ADRES_E_STATE",
}


class AdresError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [
        ("n_mol", C.c_int32), ("sites_per_mol", C.c_int32),
        ("box", C.c_double * 3),
        ("site_mass", C.c_double * MAX_SITES),
        ("region", C.c_int32),
        ("center", C.c_double * 3), ("d_at", C.c_double), ("d_hy", C.c_double),
        ("eps_at", C.c_double), ("sig_at", C.c_double), ("rc_at", C.c_double),
        ("eps_cg", C.c_double), ("sig_cg", C.c_double), ("rc_cg", C.c_double),
        ("cg_kind", C.c_int32), ("bond_kind", C.c_int32),
        ("k_bond", C.c_double), ("r0_bond", C.c_double),
        ("chain_len", C.c_int32),
        ("r_skin", C.c_double), ("rho_max", C.c_double),
        ("pair_precision", C.c_int32),
        ("scheme", C.c_int32),
    ]


_lib = None

_SIGS = {
    "adres_create": ([C.POINTER(Params), C.c_void_p, C.POINTER(C.c_void_p)], C.c_int),
    "adres_destroy": ([C.c_void_p], None),
    "adres_weights": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "adres_build_cells": ([C.c_void_p, C.c_void_p], C.c_int),
    "adres_build_verlet": ([C.c_void_p, C.c_void_p, C.POINTER(C.c_int64)], C.c_int),
    "adres_forces": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "adres_forces_noalloc": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "adres_integrate": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int32,
                         C.c_double, C.c_double, C.c_uint64, C.POINTER(C.c_int32)], C.c_int),
    "adres_integrate_respa": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int32, C.c_int32,
                               C.c_double, C.c_double, C.c_uint64, C.POINTER(C.c_int32)], C.c_int),
    "adres_get_pairs": ([C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(C.c_int64)], C.c_int),
    "adres_get_cells": ([C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_int32)], C.c_int),
    "adres_set_cg_table": ([C.c_void_p, C.c_void_p, C.c_int32, C.c_double, C.c_double], C.c_int),
    "adres_set_tdforce": ([C.c_void_p, C.c_void_p, C.c_int32, C.c_double, C.c_double], C.c_int),
    "adres_set_anchors": ([C.c_void_p, C.c_void_p, C.c_int32], C.c_int),
    "adres_get_tdforce": ([C.c_void_p, C.c_void_p, C.c_int32], C.c_int),
    "adres_density_profile": ([C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "adres_tdforce_update": ([C.c_void_p, C.c_void_p, C.c_int64, C.c_double], C.c_int),
    "adres_region_volumes": ([C.c_void_p, C.c_void_p, C.c_int64, C.c_uint64, C.c_void_p], C.c_int),
    "adres_tdforce_update_sampled": ([C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_double],
                                     C.c_int),
    "adres_mlp_set": ([C.c_void_p, C.c_void_p, C.c_int32, C.c_double, C.c_double, C.c_double, C.c_double], C.c_int),
    "adres_mlp_get": ([C.c_void_p, C.c_void_p, C.c_int32], C.c_int),
    "adres_mlp_eval": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64], C.c_int),
    "adres_map_cg": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "adres_mlp_fm_grad": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p], C.c_int),
    "adres_mlp_train_step": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_double, C.c_void_p], C.c_int),
    "adres_kernel_timing": ([C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)], C.c_int),
    "adres_last_error": ([C.c_void_p], C.c_char_p),
}


def load_library(path: str = LIB_PATH):
    """Load libadres.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build() "
                               "(hipcc, gfx950); there is no CPU fallback")
        lib = C.CDLL(path)
        for name, (args, res) in _SIGS.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def params_from(wl) -> Params:
    """Marshal a workload description (attributes of inputs.Workload) into adres_params."""
    p = Params()
    p.n_mol, p.sites_per_mol = wl.n_mol, wl.sites_per_mol
    p.box = (C.c_double * 3)(*wl.box)
    m = list(wl.site_mass) + [0.0] * (MAX_SITES - len(wl.site_mass))
    p.site_mass = (C.c_double * MAX_SITES)(*m)
    p.region = wl.region
    p.center = (C.c_double * 3)(*wl.center)
    p.d_at, p.d_hy = wl.d_at, wl.d_hy
    p.eps_at, p.sig_at, p.rc_at = wl.eps_at, wl.sig_at, wl.rc_at
    p.eps_cg, p.sig_cg, p.rc_cg = wl.eps_cg, wl.sig_cg, wl.rc_cg
    p.cg_kind, p.bond_kind = wl.cg_kind, wl.bond_kind
    p.k_bond, p.r0_bond = wl.k_bond, wl.r0_bond
    p.chain_len = wl.chain_len
    p.r_skin, p.rho_max = wl.r_skin, wl.rho_max
    p.pair_precision = wl.pair_precision
    p.scheme = getattr(wl, "scheme", 0)
    return p


def _ptr(t, dtype=None, shape=None, min_numel=None, name="tensor"):
    """Device pointer of a contiguous torch tensor on the GPU, after checking its dtype
    (a torch dtype) and its exact shape (None entries match any extent) or its least
    element count: a wrong dtype or extent would make the kernels read or write outside
    the allocation, so a mismatch raises instead."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name}: expected a CUDA (HIP) torch tensor")
    check_tensor(t, dtype, shape, min_numel, name)
    return C.c_void_p(t.data_ptr())


def check_tensor(t, dtype=None, shape=None, min_numel=None, name="tensor"):
    """The layout checks of _ptr (contiguity, dtype, shape, element count), on any device."""
    if not t.is_contiguous():
        raise ValueError(f"{name}: tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if shape is not None:
        if t.dim() != len(shape) or any(s is not None and s != q for s, q in zip(shape, t.shape)):
            raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
    if min_numel is not None and t.numel() < min_numel:
        raise ValueError(f"{name}: needs at least {min_numel} elements, got {t.numel()}")


def _f64():
    import torch
    return torch.float64


def _i64():
    import torch
    return torch.int64


class Context:
    """One AdResS system on the current GPU (wraps an adres_ctx)."""

    def __init__(self, wl, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libadres needs a GPU (no CPU fallback)")
        self.lib = load_library()
        self.wl = wl
        self.params = params_from(wl)
        self.stream = torch.cuda.current_stream() if stream is None else stream
        h = C.c_void_p()
        st = self.lib.adres_create(C.byref(self.params), C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if st != 0:
            raise AdresError(st, "adres_create rejected the parameters")
        self.h = h
        self.n_sites = wl.n_mol * wl.sites_per_mol
        self._td_n = 0

    def close(self):
        if getattr(self, "h", None):
            self.lib.adres_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, what):
        if st != 0:
            msg = self.lib.adres_last_error(self.h).decode()
            raise AdresError(st, f"{what}: {msg}")

    # -- argument checks ---------------------------------------------------------
    def _x(self, t, name="x"):
        """A site array: float64 (3, n_sites)."""
        return _ptr(t, _f64(), (3, self.n_sites), name=name)

    def _counts(self, t, name="counts"):
        """A histogram over the installed correction table's bins: int64, 1-D."""
        return _ptr(t, _i64(), (None,), min_numel=max(self._td_n, 1), name=name)

    def _frames(self, com, fmap):
        """Frames of centres and mapped forces: float64 (n_frames, 3, n_mol) each."""
        shape = (com.shape[0] if com.dim() == 3 else -1, 3, self.wl.n_mol)
        return _ptr(com, _f64(), shape, name="com"), _ptr(fmap, _f64(), shape, name="f_map")

    # -- entry points ----------------------------------------------------------
    def weights(self, x):
        import torch
        com = torch.empty((3, self.wl.n_mol), dtype=torch.float64, device=x.device)
        w = torch.empty(self.wl.n_mol, dtype=torch.float64, device=x.device)
        self._check(self.lib.adres_weights(self.h, self._x(x), _ptr(com), _ptr(w)), "adres_weights")
        return com, w

    def build_cells(self, x):
        self._check(self.lib.adres_build_cells(self.h, self._x(x)), "adres_build_cells")

    def build_verlet(self, x):
        n = C.c_int64()
        self._check(self.lib.adres_build_verlet(self.h, self._x(x), C.byref(n)), "adres_build_verlet")
        return n.value

    def forces(self, x, f=None, energy=False):
        import torch
        if f is None:
            f = torch.empty_like(x)
        e = torch.zeros(4, dtype=torch.float64, device=x.device) if energy else None
        self._check(self.lib.adres_forces(self.h, self._x(x), self._x(f, "f"), _ptr(e, _f64(), (4,), name="energy")),
                    "adres_forces")
        return (f, e) if energy else f

    def forces_noalloc(self, x, f, energy=None):
        """adres_forces_noalloc into caller-provided f (and energy [4]); allocates nothing."""
        self._check(self.lib.adres_forces_noalloc(self.h, self._x(x), self._x(f, "f"),
                                                  _ptr(energy, _f64(), (4,), name="energy")),
                    "adres_forces_noalloc")
        return f

    def integrate_respa(self, x, v, f, dt, n_inner, n_outer, gamma=0.0, kT=1.0, seed=0):
        nreb = C.c_int32()
        st = self.lib.adres_integrate_respa(self.h, self._x(x), self._x(v, "v"), self._x(f, "f"), dt, n_inner,
                                            n_outer, gamma, kT, seed, C.byref(nreb))
        self._check(st, "adres_integrate_respa")
        return nreb.value

    def integrate(self, x, v, f, dt, n_steps, gamma=0.0, kT=1.0, seed=0):
        nreb = C.c_int32()
        st = self.lib.adres_integrate(self.h, self._x(x), self._x(v, "v"), self._x(f, "f"), dt, n_steps, gamma,
                                      kT, seed, C.byref(nreb))
        self._check(st, "adres_integrate")
        return nreb.value

    def get_pairs(self):
        n = C.c_int64()
        self._check(self.lib.adres_get_pairs(self.h, None, 0, C.byref(n)), "adres_get_pairs")
        out = np.empty((max(n.value, 1), 2), dtype=np.int32)
        self._check(self.lib.adres_get_pairs(self.h, out.ctypes.data_as(C.c_void_p), n.value, C.byref(n)),
                    "adres_get_pairs")
        return out[: n.value]

    def get_cells(self):
        nc = C.c_int32()
        self._check(self.lib.adres_get_cells(self.h, None, None, C.byref(nc)), "adres_get_cells")
        start = np.empty(nc.value + 1, dtype=np.int32)
        perm = np.empty(self.wl.n_mol, dtype=np.int32)
        self._check(self.lib.adres_get_cells(self.h, start.ctypes.data_as(C.c_void_p),
                                             perm.ctypes.data_as(C.c_void_p), C.byref(nc)), "adres_get_cells")
        return start, perm

    def set_cg_table(self, coef, r_lo, r_hi):
        coef = np.ascontiguousarray(coef, dtype=np.float32)
        assert coef.ndim == 2 and coef.shape[1] == 4
        self._check(self.lib.adres_set_cg_table(self.h, coef.ctypes.data_as(C.c_void_p), coef.shape[0] + 1,
                                                r_lo, r_hi), "adres_set_cg_table")

    def set_tdforce(self, table, d_lo, d_hi):
        """Install the correction force values (float64, at the bin centres of [d_lo, d_hi))."""
        table = np.ascontiguousarray(table, dtype=np.float64)
        self._check(self.lib.adres_set_tdforce(self.h, table.ctypes.data_as(C.c_void_p), table.size,
                                               d_lo, d_hi), "adres_set_tdforce")
        self._td_n = int(table.size)

    def set_anchors(self, mols):
        """Anchor molecules (caller indices) of a self-adjusting AT region."""
        mols = np.ascontiguousarray(mols, dtype=np.int32)
        self._check(self.lib.adres_set_anchors(self.h, mols.ctypes.data_as(C.c_void_p), mols.size),
                    "adres_set_anchors")

    def get_tdforce(self):
        out = np.empty(max(self._td_n, 1), dtype=np.float64)
        self._check(self.lib.adres_get_tdforce(self.h, out.ctypes.data_as(C.c_void_p), out.size),
                    "adres_get_tdforce")
        return out

    def density_profile(self, x, counts):
        """Add the centre-of-mass distance histogram of x to counts (int64 device tensor)."""
        self._check(self.lib.adres_density_profile(self.h, self._x(x), self._counts(counts)),
                    "adres_density_profile")

    def tdforce_update(self, counts, n_frames, prefactor):
        self._check(self.lib.adres_tdforce_update(self.h, self._counts(counts), int(n_frames), float(prefactor)),
                    "adres_tdforce_update")

    def region_volumes(self, x, n_samples, seed, vol_counts):
        """Add the bins of n_samples uniform points to vol_counts (int64 device tensor)."""
        xp = self._x(x) if x is not None else None
        self._check(self.lib.adres_region_volumes(self.h, xp, int(n_samples), int(seed) & (2**64 - 1),
                                                  self._counts(vol_counts, "vol_counts")), "adres_region_volumes")

    def tdforce_update_sampled(self, counts, n_frames, vol_counts, n_vol_samples, prefactor):
        self._check(self.lib.adres_tdforce_update_sampled(self.h, self._counts(counts), int(n_frames),
                                                          self._counts(vol_counts, "vol_counts"),
                                                          int(n_vol_samples), float(prefactor)),
                    "adres_tdforce_update_sampled")

    def mlp_set(self, params, rc, scale, taper_width, r_min=0.0):
        params = np.ascontiguousarray(params, dtype=np.float32)
        self._check(self.lib.adres_mlp_set(self.h, params.ctypes.data_as(C.c_void_p), params.size, rc, scale,
                                           taper_width, r_min), "adres_mlp_set")

    def mlp_get(self):
        out = np.empty(4353, dtype=np.float32)
        self._check(self.lib.adres_mlp_get(self.h, out.ctypes.data_as(C.c_void_p), out.size), "adres_mlp_get")
        return out

    def mlp_eval(self, r):
        import torch
        rp = _ptr(r, torch.float64, (None,), name="r")
        f = torch.empty(r.shape[0], dtype=torch.float32, device=r.device)
        self._check(self.lib.adres_mlp_eval(self.h, rp, _ptr(f), r.shape[0]), "adres_mlp_eval")
        return f

    def map_cg(self, x):
        """Eq. (1) forces at x, then per molecule (centre of mass, summed force)."""
        import torch
        f = torch.empty_like(x)
        com = torch.empty((3, self.wl.n_mol), dtype=torch.float64, device=x.device)
        fmap = torch.empty_like(com)
        self._check(self.lib.adres_map_cg(self.h, self._x(x), _ptr(f), _ptr(com), _ptr(fmap)), "adres_map_cg")
        return com, fmap

    def mlp_fm_grad(self, com, fmap):
        """com, fmap: device float64 tensors (n_frames, 3, n_mol)."""
        g = np.empty(4353, dtype=np.float64)
        loss = C.c_double()
        com_p, fmap_p = self._frames(com, fmap)
        self._check(self.lib.adres_mlp_fm_grad(self.h, com_p, fmap_p, com.shape[0],
                                               g.ctypes.data_as(C.c_void_p), C.byref(loss)), "adres_mlp_fm_grad")
        return loss.value, g

    def mlp_train_step(self, com, fmap, lr):
        loss = C.c_double()
        com_p, fmap_p = self._frames(com, fmap)
        self._check(self.lib.adres_mlp_train_step(self.h, com_p, fmap_p, com.shape[0], lr, C.byref(loss)),
                    "adres_mlp_train_step")
        return loss.value

    def kernel_timing(self, enable=True, every=1):
        """enable: False/0 off, True/1 force kernel, 2 the network's pair pre-pass; every:
        record every every-th launch.  Returns (ms, launches) recorded since the last call."""
        ms = C.c_double()
        n = C.c_int64()
        mode = int(enable) if not isinstance(enable, bool) else (1 if enable else 0)
        self._check(self.lib.adres_kernel_timing(self.h, mode, every, C.byref(ms), C.byref(n)),
                    "adres_kernel_timing")
        return ms.value, n.value
