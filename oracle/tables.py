"""Cubic force tables for the CG part -- TEST INFRASTRUCTURE ONLY.

A table holds, per interval k of n equally spaced knots on [r_lo, r_hi], the
coefficients {c0, c1, c2, c3} of p_k(t) = ((c3 t + c2) t + c1) t + c0 in the local
coordinate t = (r - r_lo)/h - k.  Tables built here are inputs handed to both the
oracle and the library (like network weights); they are built from closed forms
in FP64 and rounded once to FP32.
"""
from __future__ import annotations

import numpy as np


def wca_force(r, sig, eps, rc):
    """WCA force magnitude f(r) = -dU/dr (positive = repulsive) and df/dr, zero at r >= rc."""
    r = np.asarray(r, dtype=np.float64)
    s6 = (sig / r) ** 6
    f = 24.0 * eps * s6 * (2.0 * s6 - 1.0) / r
    df = 24.0 * eps * s6 * (7.0 - 26.0 * s6) / (r * r)
    inside = r < rc
    return np.where(inside, f, 0.0), np.where(inside, df, 0.0)


def hermite_coefficients(f, df, h):
    """Cubic Hermite interpolant through (f, f') at consecutive knots: [(n-1), 4] FP64."""
    f0, f1 = f[:-1], f[1:]
    d0, d1 = h * df[:-1], h * df[1:]
    c0 = f0
    c1 = d0
    c2 = 3.0 * (f1 - f0) - 2.0 * d0 - d1
    c3 = 2.0 * (f0 - f1) + d0 + d1
    return np.stack([c0, c1, c2, c3], axis=1)


def hermite_wca_table(sig, eps, rc, r_lo, r_hi, n_knots):
    """2048-knot-style table of the CG WCA force; returns (coef float32 [(n-1),4], r_lo, r_hi)."""
    r = np.linspace(r_lo, r_hi, n_knots)
    h = (r_hi - r_lo) / (n_knots - 1)
    f, df = wca_force(r, sig, eps, rc)
    return hermite_coefficients(f, df, h).astype(np.float32), float(r_lo), float(r_hi)


def eval_table_fp64(coef, r_lo, r_hi, r):
    """Vectorised FP64 evaluation of a table (same definition as the C oracle)."""
    coef = np.asarray(coef, dtype=np.float64)
    n = coef.shape[0] + 1
    h = (r_hi - r_lo) / (n - 1)
    u = (np.asarray(r, dtype=np.float64) - r_lo) / h
    k = np.clip(np.floor(u), 0, n - 2)
    t = u - k
    c = coef[k.astype(np.int64)]
    return ((c[:, 3] * t + c[:, 2]) * t + c[:, 1]) * t + c[:, 0]
