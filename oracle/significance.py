"""Significance of IG^k_max, written plainly in binary64 (oracle side).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: only the tests may import it.  It shares
no code with the library; the chi-square distribution comes from scipy.stats (a library
primitive), everything else is written out from its definition.

Section "Theory", the paragraphs after equation IGmax: for an irrelevant variable and one
k-tuple, 2 IG follows a chi-square distribution; IG^k_max is the largest of many such values
and follows an extreme value distribution with one free parameter, the number of independent
tests, fitted to the irrelevant variables; p-values follow, IG_lim is the value whose p-value is
the significance level, and the p-values of many variables are adjusted by Holm or by
Benjamini-Hochberg(-Yekutieli) (section "Canonical package usage": ComputePValue, p.adjust).

Readings (shared with the library's documentation, since the fit itself is specified only in a
companion paper): df = (c-1) c^(k-1) with c = divisions + 1; Pr(IG_max <= x) = F(2x)^n_eff;
n_eff by maximum likelihood over the selected variables with IG > 0.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import stats


def chi2_df(k: int, divisions: int) -> int:
    """Cells of the (decision x tuple) table less its margin constraints, binary decision."""
    c = divisions + 1
    return (c - 1) * c ** (k - 1)


def log_cdf_max1(ig: float, df: int) -> float:
    """ln Pr(one tuple's IG <= ig) = ln F_chi2(2 ig; df)."""
    if ig <= 0:
        return -math.inf
    return float(stats.chi2.logcdf(2.0 * ig, df))


def fit_n_eff(ig, k: int, divisions: int, fit_mask=None) -> float:
    """Maximum likelihood n_eff: the log-likelihood of the maxima x_v is
    sum_v [ln n + (n - 1) ln F(2 x_v) + ln f(2 x_v) + ln 2]; its derivative in n vanishes at
    n = -m / sum_v ln F(2 x_v)."""
    df = chi2_df(k, divisions)
    total, m = 0.0, 0
    for v, x in enumerate(np.asarray(ig, dtype=np.float64)):
        if fit_mask is not None and not fit_mask[v]:
            continue
        if x <= 0:
            continue
        total += log_cdf_max1(float(x), df)
        m += 1
    if m == 0 or not total < 0:
        raise ValueError("no usable variable in the fit")
    return -m / total


def pvalues(ig, k: int, divisions: int, fit_mask=None, n_eff: float | None = None):
    """p_v = 1 - F(2 x_v)^n_eff, evaluated as -expm1(n_eff ln F); 1 for x_v <= 0."""
    df = chi2_df(k, divisions)
    if n_eff is None:
        n_eff = fit_n_eff(ig, k, divisions, fit_mask)
    out = []
    for x in np.asarray(ig, dtype=np.float64):
        if x <= 0:
            out.append(1.0)
        else:
            out.append(-math.expm1(n_eff * log_cdf_max1(float(x), df)))
    return np.array(out), n_eff


def ig_lim(k: int, divisions: int, n_eff: float, alpha: float) -> float:
    """The x with 1 - F(2x)^n_eff = alpha: F(2x) = (1 - alpha)^(1 / n_eff), i.e. the chi-square
    tail at 2x is 1 - (1 - alpha)^(1 / n_eff) (formed with expm1/log1p, then inverted as a tail)."""
    df = chi2_df(k, divisions)
    tail = -math.expm1(math.log1p(-alpha) / n_eff)
    return float(stats.chi2.isf(tail, df)) / 2.0


def p_adjust(p, method: str):
    """R's p.adjust definitions, with plain loops over the sorted p-values."""
    p = np.asarray(p, dtype=np.float64)
    n = len(p)
    order = sorted(range(n), key=lambda v: (p[v], v))
    out = np.empty(n)
    if method == "none":
        return p.copy()
    if method == "holm":
        running = 0.0
        for rank, v in enumerate(order):            # rank 0 = smallest p
            running = max(running, min(1.0, (n - rank) * p[v]))
            out[v] = running
        return out
    if method in ("BH", "BY"):
        scale = sum(1.0 / j for j in range(1, n + 1)) if method == "BY" else 1.0
        running = 1.0
        for rank in range(n - 1, -1, -1):
            v = order[rank]
            running = min(running, min(1.0, scale * n / (rank + 1) * p[v]))
            out[v] = running
        return out
    raise ValueError(method)
