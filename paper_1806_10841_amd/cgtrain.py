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
    pts = np.where(pts >= box, pts - box, pts)
    pr = cKDTree(pts, boxsize=box).query_pairs(rc, output_type="ndarray")
    d = com[:, pr[:, 0]] - com[:, pr[:, 1]]
    d -= box[:, None] * np.round(d / box[:, None])
    r = np.sqrt((d * d).sum(axis=0))
    return pr[:, 0], pr[:, 1], r, d / r


def min_pair_distance(com, box, rc=3.0, quantile=0.0):
    """Smallest (or the given quantile of) centre-pair distance below rc over frames."""
    rs = np.concatenate([_pairs(np.asarray(c, dtype=np.float64), box, rc)[2] for c in com])
    return float(np.quantile(rs, quantile)) if quantile > 0 else float(rs.min())


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


def hermite_from_values(f, df, h):
    """Cubic coefficients [(n-1), 4] of the Hermite interpolant of knot values and slopes."""
    f0, f1 = f[:-1], f[1:]
    d0, d1 = h * df[:-1], h * df[1:]
    return np.stack([f0, d0, 3 * (f1 - f0) - 2 * d0 - d1, 2 * (f0 - f1) + d0 + d1], axis=1)


def fit_table(com, fmap, box, r_fit_lo, r_lo=0.5, rc=3.0, n_basis=40, n_knots=2048):
    """Force-matched cubic table (the tabulated CG force of the comparison).

    Linear least squares (NumPy ``lstsq``) for f(r) = sum_k c_k B_k(r) on [r_fit_lo, rc]
    such that sum_J f(r_IJ) R_hat_IJ ~ F^map_I over all frames (pairs closer than
    r_fit_lo are rare and enter at r_fit_lo).  Below r_fit_lo the force continues
    linearly with the slope at r_fit_lo when that slope is repulsive (else flat), so
    the table stays a wall where there is no data.  Returns (coef [(n_knots-1), 4]
    float32, r_lo, rc) with f(rc) = 0."""
    com = np.asarray(com, dtype=np.float64)
    fmap = np.asarray(fmap, dtype=np.float64)
    rows, rhs = [], []
    for k in range(com.shape[0]):
        I, J, r, rh = _pairs(com[k], box, rc)
        B = _bspline_basis(np.clip(r, r_fit_lo, rc), r_fit_lo, rc, n_basis)
        n = com.shape[2]
        A = np.empty((3 * n, n_basis))
        for d in range(3):
            for q in range(n_basis):
                w = B[:, q] * rh[d]
                A[d * n:(d + 1) * n, q] = (np.bincount(I, weights=w, minlength=n)
                                           - np.bincount(J, weights=w, minlength=n))
        rows.append(A)
        rhs.append(fmap[k].reshape(-1))
    c, *_ = np.linalg.lstsq(np.concatenate(rows), np.concatenate(rhs), rcond=None)

    def spline(x):
        return _bspline_basis(x, r_fit_lo, rc, n_basis) @ c

    rk = np.linspace(r_lo, rc, n_knots)
    h = rk[1] - rk[0]
    inside = rk >= r_fit_lo
    ri = rk[inside]
    eps = 1e-5
    f = np.empty_like(rk)
    df = np.empty_like(rk)
    f[inside] = spline(ri)
    up = np.minimum(ri + eps, rc)
    dn = np.maximum(ri - eps, r_fit_lo)
    df[inside] = (spline(up) - spline(dn)) / (up - dn)
    f0 = float(spline(np.array([r_fit_lo]))[0])
    s0 = float((spline(np.array([r_fit_lo + eps])) - spline(np.array([r_fit_lo])))[0] / eps)
    slope = min(s0, 0.0)
    f[~inside] = f0 + slope * (rk[~inside] - r_fit_lo)
    df[~inside] = slope
    f[-1] = 0.0
    return hermite_from_values(f, df, h).astype(np.float32), float(r_lo), float(rc)


def tile_frame(com, box, reps):
    """Copies of a centre frame (3, n) on a reps[0] x reps[1] x reps[2] grid of boxes."""
    com = np.asarray(com, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    out = []
    for a in range(reps[0]):
        for b in range(reps[1]):
            for c in range(reps[2]):
                out.append(com + (np.array([a, b, c]) * box)[:, None])
    return np.concatenate(out, axis=1), tuple(float(x) for x in box * np.asarray(reps))


def wca_table(sig=2.31, eps=1.0, r_lo=0.5, r_hi=3.0, n_knots=2048):
    """The plain method's CG force (WCA between centres) as a cubic table."""
    rc = sig * 2 ** (1 / 6)
    rk = np.linspace(r_lo, r_hi, n_knots)
    h = rk[1] - rk[0]
    s6 = (sig / rk) ** 6
    inside = rk < rc
    f = np.where(inside, 24 * eps * s6 * (2 * s6 - 1) / rk, 0.0)
    df = np.where(inside, 24 * eps * s6 * (7 - 26 * s6) / rk ** 2, 0.0)
    return hermite_from_values(f, df, h).astype(np.float32), float(r_lo), float(r_hi)


def rmse_on_device(com, fmap, box, cg_kind, table=None, mlp=None, rc=3.0):
    """RMSE (per force component) of a CG model's forces against mapped forces, with the
    model evaluated by the library on the CG sites of each frame.  cg_kind WCA is the
    plain method's CG force (sigma 2.31, cut at its minimum)."""
    import torch
    n = com.shape[2]
    if cg_kind == inputs.CG_WCA:
        rc = 2.31 * 2 ** (1 / 6)
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
