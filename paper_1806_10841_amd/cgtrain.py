"""Learned vs tabulated CG force: data, fits and errors.

* ``generate_frames``: centres of mass and mapped forces (summed atomistic forces
  per molecule) from an all-atomistic (w == 1) Langevin run of tetrahedra, both
  produced on the GPU by the library (``adres_integrate``, ``adres_map_cg``).
* ``train_mlp``: force matching of the network on the GPU (``adres_mlp_train_step``,
  BF16 matrix cores, Adam).
* ``fit_table``: the tabulated alternative -- linear least squares for a cubic
  B-spline force on the same frames (NumPy ``lstsq``; host-side setup, not the hot
  path), resampled to a cubic table of the library's format.
* ``rmse_on_device``: force RMSE of a CG model against mapped forces, with the
  model's forces computed by the library.
"""
from __future__ import annotations

import math

import numpy as np

from . import binding, inputs


def tetra_workload(n_side, region=inputs.REGION_ALL_AT):
    """Tetrahedra on an n_side^3 lattice at molecular density 0.1."""
    L = n_side * (1 / 0.1) ** (1.0 / 3.0)
    base = inputs.workload("c2")
    return base.with_(name=f"tetra{n_side}", n_mol=n_side ** 3, box=(L, L, L), center=(L / 2, L / 2, L / 2),
                      region=region, pair_precision=32)


def cg_workload(n, box, cg_kind, rc=3.0):
    """1-site CG sites of total mass 4 (one per tetrahedron), all coarse-grained."""
    return inputs.workload("small_cg").with_(
        n_mol=n, box=tuple(box), center=tuple(b / 2 for b in box), site_mass=(4.0,), cg_kind=cg_kind,
        rc_cg=rc, pair_precision=32)


def generate_frames(n_side, n_frames, stride=20, warmup=400, seed=7, gamma=1.0, kT=1.0):
    """Frames (n_frames, 3, n_mol) of centres and mapped forces from a w == 1 run."""
    import torch
    wl = tetra_workload(n_side)
    x, v = inputs.make_state(wl, seed=seed)
    ctx = binding.Context(wl)
    dev = torch.device("cuda")
    xt, vt = torch.tensor(x, device=dev), torch.tensor(v, device=dev)
    ft = torch.empty_like(xt)
    ctx.integrate(xt, vt, ft, wl.dt, warmup, gamma=gamma, kT=kT, seed=seed)
    coms, fmaps = [], []
    for k in range(n_frames):
        ctx.integrate(xt, vt, ft, wl.dt, stride, gamma=gamma, kT=kT, seed=seed + 1 + k)
        com, fm = ctx.map_cg(xt)
        coms.append(com.clone())
        fmaps.append(fm.clone())
    ctx.close()
    return torch.stack(coms), torch.stack(fmaps), wl.box


def force_scale(fmaps):
    """RMS of the mapped force components (the network's output scale)."""
    return float(fmaps.double().pow(2).mean().sqrt())


def train_mlp(com, fmap, box, steps=300, lr=2e-3, batch=4, rc=3.0, tw=0.5, seed=0, r_min=0.0, table=None):
    """Force matching on the GPU; returns (params float32, loss history)."""
    n = com.shape[2]
    ctx = binding.Context(cg_workload(n, box, inputs.CG_MLP, rc))
    if table is not None:
        ctx.set_cg_table(*table)
    scale = force_scale(fmap)
    ctx.mlp_set(inputs.mlp_init(seed).astype(np.float32), rc, scale, tw, r_min)
    rng = np.random.default_rng(seed)
    hist = []
    nf = com.shape[0]
    for it in range(steps):
        idx = rng.choice(nf, size=min(batch, nf), replace=False)
        hist.append(ctx.mlp_train_step(com[idx].contiguous(), fmap[idx].contiguous(), lr))
    params = ctx.mlp_get()
    ctx.close()
    return params, scale, hist


def _pairs(com, box, rc):
    from scipy.spatial import cKDTree
    box = np.asarray(box, dtype=np.float64)
    pts = np.mod(com.T, box)
    pts[pts >= box] -= box[pts >= box]
    pr = cKDTree(pts, boxsize=box).query_pairs(rc, output_type="ndarray")
    d = com[:, pr[:, 0]] - com[:, pr[:, 1]]
    d -= box[:, None] * np.round(d / box[:, None])
    r = np.sqrt((d * d).sum(axis=0))
    return pr[:, 0], pr[:, 1], r, d / r


def _bspline_basis(r, lo, hi, n_basis):
    """Uniform cubic B-spline basis on [lo, hi] (n_basis functions), values at r."""
    h = (hi - lo) / (n_basis - 3)
    u = (r - lo) / h
    out = np.zeros((len(r), n_basis))
    for k in range(n_basis):
        t = u - (k - 3)   # support [k-3, k+1) in units of h
        b = np.zeros_like(t)
        m = (t >= 0) & (t < 1); b[m] = t[m] ** 3 / 6
        m = (t >= 1) & (t < 2); tt = t[m] - 1; b[m] = (-3 * tt ** 3 + 3 * tt ** 2 + 3 * tt + 1) / 6
        m = (t >= 2) & (t < 3); tt = t[m] - 2; b[m] = (3 * tt ** 3 - 6 * tt ** 2 + 4) / 6
        m = (t >= 3) & (t < 4); tt = t[m] - 3; b[m] = (1 - tt) ** 3 / 6
        out[:, k] = b
    return out


def fit_table(com, fmap, box, r_lo=1.5, rc=3.0, n_basis=40, n_knots=2048):
    """Force-matched cubic table: least squares for f(r) = sum_k c_k B_k(r) such that
    sum_J f(r_IJ) R_hat_IJ ~ F^map_I over all frames; returns (coef [(n-1),4] float32,
    r_lo, r_hi) evaluating f on [r_lo, rc] (zero at rc)."""
    com = np.asarray(com, dtype=np.float64)
    fmap = np.asarray(fmap, dtype=np.float64)
    rows, rhs = [], []
    for k in range(com.shape[0]):
        I, J, r, rh = _pairs(com[k], box, rc)
        rr = np.clip(r, r_lo, rc)
        B = _bspline_basis(rr, r_lo, rc, n_basis)      # (pairs, n_basis)
        n = com.shape[2]
        A = np.zeros((3 * n, n_basis))
        for d in range(3):
            np.add.at(A, d * n + I, B * rh[d][:, None])
            np.add.at(A, d * n + J, -B * rh[d][:, None])
        rows.append(A)
        rhs.append(fmap[k].reshape(-1))
    A = np.concatenate(rows)
    b = np.concatenate(rhs)
    c, *_ = np.linalg.lstsq(A, b, rcond=None)
    # resample to a cubic table (Hermite from values and derivatives by central differences)
    rk = np.linspace(r_lo, rc, n_knots)
    h = rk[1] - rk[0]
    f = _bspline_basis(rk, r_lo, rc, n_basis) @ c
    eps = 1e-4 * h
    df = (_bspline_basis(np.clip(rk + eps, r_lo, rc), r_lo, rc, n_basis) @ c
          - _bspline_basis(np.clip(rk - eps, r_lo, rc), r_lo, rc, n_basis) @ c) / (
        np.clip(rk + eps, r_lo, rc) - np.clip(rk - eps, r_lo, rc))
    f[-1] = 0.0
    f0, f1 = f[:-1], f[1:]
    d0, d1 = h * df[:-1], h * df[1:]
    coef = np.stack([f0, d0, 3 * (f1 - f0) - 2 * d0 - d1, 2 * (f0 - f1) + d0 + d1], axis=1)
    return coef.astype(np.float32), float(r_lo), float(rc)


def wca_table(sig=2.31, eps=1.0, r_lo=1.0, r_hi=3.0, n_knots=2048):
    """The plain method's CG force (WCA between centres) as a cubic table."""
    rc = sig * 2 ** (1 / 6)
    rk = np.linspace(r_lo, r_hi, n_knots)
    h = rk[1] - rk[0]
    s6 = (sig / rk) ** 6
    inside = rk < rc
    f = np.where(inside, 24 * eps * s6 * (2 * s6 - 1) / rk, 0.0)
    df = np.where(inside, 24 * eps * s6 * (7 - 26 * s6) / rk ** 2, 0.0)
    f0, f1 = f[:-1], f[1:]
    d0, d1 = h * df[:-1], h * df[1:]
    coef = np.stack([f0, d0, 3 * (f1 - f0) - 2 * d0 - d1, 2 * (f0 - f1) + d0 + d1], axis=1)
    return coef.astype(np.float32), float(r_lo), float(r_hi)


def rmse_on_device(com, fmap, box, cg_kind, table=None, mlp=None, rc=3.0):
    """RMSE (per force component) of a CG model's forces against mapped forces, with the
    model evaluated by the library on the CG sites of each frame."""
    import torch
    n = com.shape[2]
    ctx = binding.Context(cg_workload(n, box, cg_kind, rc))
    if table is not None:
        ctx.set_cg_table(*table)
    if mlp is not None:
        params, scale, tw, r_min = mlp
        ctx.mlp_set(params, rc, scale, tw, r_min)
    se, cnt = 0.0, 0
    for k in range(com.shape[0]):
        f = ctx.forces(com[k].contiguous())
        se += float((f - fmap[k]).pow(2).sum())
        cnt += f.numel()
    ctx.close()
    return math.sqrt(se / cnt)
