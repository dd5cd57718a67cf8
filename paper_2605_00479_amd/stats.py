"""Ensemble statistics used to judge reduced-precision runs against FP64
(Kimpson, Flegg & Flegg, Sec. 4 opening: two-sample Kolmogorov-Smirnov test,
Wasserstein-1 distance, sample mean and variance of the end-time ensemble).

Plain numpy host code: it evaluates results, it is not part of the simulation.
"""
from __future__ import annotations

import math

import numpy as np


def ks_sf(lam: float) -> float:
    """Survival function of the Kolmogorov distribution,
    Q(lam) = 2 sum_{k>=1} (-1)^(k-1) exp(-2 k^2 lam^2); for small lam the
    equivalent theta-function form 1 - sqrt(2 pi)/lam sum exp(-(2k-1)^2 pi^2/(8 lam^2))."""
    if lam <= 0.0:
        return 1.0
    if lam < 1.0:
        s = 0.0
        for k in range(1, 20):
            s += math.exp(-((2 * k - 1) ** 2) * math.pi ** 2 / (8.0 * lam * lam))
        return max(0.0, min(1.0, 1.0 - math.sqrt(2.0 * math.pi) / lam * s))
    s = 0.0
    for k in range(1, 101):
        term = math.exp(-2.0 * k * k * lam * lam)
        s += term if k % 2 == 1 else -term
        if term < 1e-300:
            break
    return max(0.0, min(1.0, 2.0 * s))


def _ecdf_pair(a, b):
    a = np.sort(np.asarray(a, dtype=np.float64).ravel())
    b = np.sort(np.asarray(b, dtype=np.float64).ravel())
    grid = np.unique(np.concatenate([a, b]))
    fa = np.searchsorted(a, grid, side="right") / a.size
    fb = np.searchsorted(b, grid, side="right") / b.size
    return grid, fa, fb


def ks_2samp(a, b):
    """Two-sample KS: D = sup |F_a - F_b| over the pooled support and its
    asymptotic p-value with n_eff = n m / (n + m)."""
    na, nb = np.size(a), np.size(b)
    if na == 0 or nb == 0:
        return float("nan"), float("nan")
    _, fa, fb = _ecdf_pair(a, b)
    d = float(np.max(np.abs(fa - fb)))
    en = na * nb / (na + nb)
    return d, ks_sf(d * math.sqrt(en))


def wasserstein1(a, b) -> float:
    """W1 = integral |F_a - F_b| dx between the two empirical laws."""
    if np.size(a) == 0 or np.size(b) == 0:
        return float("nan")
    grid, fa, fb = _ecdf_pair(a, b)
    if grid.size < 2:
        return 0.0
    return float(np.sum(np.abs(fa - fb)[:-1] * np.diff(grid)))


def moments(x):
    x = np.asarray(x, dtype=np.float64).ravel()
    mean = float(x.mean()) if x.size else float("nan")
    var = float(x.var(ddof=1)) if x.size > 1 else float("nan")
    fano = var / mean if mean else float("nan")
    return mean, var, fano


def compare(ref, x) -> dict:
    """KS (D, p), W1 and mean / variance / Fano relative errors of x against ref."""
    d, p = ks_2samp(ref, x)
    m0, v0, f0 = moments(ref)
    m1, v1, f1 = moments(x)

    def rel(a, b):
        return abs(a - b) / abs(b) if b else float("nan")

    return {"ks_D": d, "ks_p": p, "w1": wasserstein1(ref, x), "mean": m1, "var": v1, "fano": f1,
            "mean_ref": m0, "var_ref": v0, "fano_ref": f0, "mean_rel_err": rel(m1, m0),
            "var_rel_err": rel(v1, v0), "fano_rel_err": rel(f1, f0)}
