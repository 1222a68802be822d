"""End-to-end feature selection: the canonical usage of section "Canonical package usage".

seed -> contrast variables -> IG^k_max of every variable -> fit of the IG_max distribution ->
p-values -> adjusted p-values (contrast variables left out) -> relevant variables (adjusted
p-value below the level), each step a call of libmdfs (mdfs_add_contrast, mdfs_max_ig,
mdfs_pvalues, mdfs_p_adjust, mdfs_ig_lim).  Host orchestration only.

Readings where the paper is silent:
* n_contrast defaults to max(n_var, 30): at least 30 variables for the fit, and as many
  contrast variables as originals;
* range defaults to 0 for one discretisation and 0.5 otherwise;
* the one-dimensional "raw" mode (k = 1, one discretisation: plain chi-square) uses a single
  test per variable (n_eff = 1); every other case uses the fitted law F(2x)^n_eff (the "lin" and
  "exp" modes of the paper are heuristics it does not specify);
* without contrast variables n_eff is fitted on all variables, then again without those whose
  adjusted p-value falls below the level, until that set no longer changes (at most 10 fits).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import mdfs


@dataclasses.dataclass
class MdfsResult:
    statistic: np.ndarray          # IG^k_max of the original variables (float32 -> float64)
    p_value: np.ndarray
    adjusted_p_value: np.ndarray
    relevant_variables: np.ndarray  # indices, by increasing p-value
    n_eff: float                   # fitted (or fixed) number of independent tests
    ig_lim: float                  # IG_max whose unadjusted p-value is the level
    contrast_indices: np.ndarray   # source variable of each contrast variable
    argmax: np.ndarray             # [n_var][k-1] partner tuple (indices >= n_var are contrast variables)
    argmax_disc: np.ndarray


def mdfs_run(data: torch.Tensor, y: torch.Tensor, k: int = 1, divisions: int = 1, n_disc: int = 1,
             range_: float | None = None, pseudocount: float = 0.25, seed: int = 0, n_contrast: int | None = None,
             p_adjust_method: str = "holm", level: float = 0.05, engine: str = "auto") -> MdfsResult:
    n_var = data.shape[0]
    if n_contrast is None:
        n_contrast = max(n_var, 30)
    if range_ is None:
        range_ = 0.0 if n_disc == 1 else 0.5
    if n_contrast > 0:
        data_c, src = mdfs.mdfs_add_contrast(data, n_contrast, seed)
    else:
        data_c, src = data, np.zeros(0, dtype=np.int32)
    ig, am, ad = mdfs.mdfs_max_ig(data_c, y, k, divisions, n_disc, pseudocount, range_, seed, engine=engine)
    ig = ig.cpu().numpy().astype(np.float64)
    am, ad = am.cpu().numpy(), ad.cpu().numpy()

    if k == 1 and n_disc == 1:
        p_all, n_eff = mdfs.mdfs_pvalues(ig, k, divisions, n_eff=1.0)
    elif n_contrast > 0:
        mask = np.zeros(len(ig), dtype=bool)
        mask[n_var:] = True
        p_all, n_eff = mdfs.mdfs_pvalues(ig, k, divisions, fit_mask=mask)
    else:
        keep = np.ones(n_var, dtype=bool)
        for _ in range(10):
            p_all, n_eff = mdfs.mdfs_pvalues(ig, k, divisions, fit_mask=keep)
            new_keep = mdfs.mdfs_p_adjust(p_all, p_adjust_method) >= level
            if np.array_equal(new_keep, keep) or not new_keep.any():
                break
            keep = new_keep
    p = p_all[:n_var]
    adj = mdfs.mdfs_p_adjust(p, p_adjust_method)
    rel = np.flatnonzero(adj < level)
    rel = rel[np.argsort(p[rel], kind="stable")]
    return MdfsResult(statistic=ig[:n_var], p_value=p, adjusted_p_value=adj, relevant_variables=rel, n_eff=n_eff,
                      ig_lim=mdfs.mdfs_ig_lim(k, divisions, n_eff, level), contrast_indices=src,
                      argmax=am[:n_var], argmax_disc=ad[:n_var])
