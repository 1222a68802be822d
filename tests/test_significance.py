"""The library's significance layer (host-side binary64 entry points) against the oracle.

mdfs_pvalues / mdfs_ig_lim / mdfs_p_adjust / mdfs_chi2_df run on the host and need no GPU; the
oracle side (oracle/significance.py) is pinned in test_oracle_pins.py.
"""
import math

import numpy as np
import pytest

from oracle import significance as sig
from paper_1811_00631_amd import mdfs


def rel_close(a, b, rtol):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return np.all(np.abs(a - b) <= rtol * np.maximum(np.abs(a), np.abs(b)))


@pytest.mark.parametrize("k,d", [(1, 1), (1, 2), (2, 1), (2, 2), (2, 4), (3, 2), (3, 4)])
def test_df(k, d):
    assert mdfs.mdfs_chi2_df(k, d) == sig.chi2_df(k, d)


@pytest.mark.parametrize("k,d", [(1, 2), (2, 2), (3, 2), (2, 4), (2, 1)])
def test_pvalues_fit_and_tails(k, d):
    g = np.random.default_rng(100 * k + d)
    df = sig.chi2_df(k, d)
    # maxima of 50 null values, a few strong signals (p-values down to 1e-200) and values <= 0
    ig = (g.chisquare(df, size=(300, 50)) / 2).max(axis=1)
    ig[:5] = [60.0, 150.0, 400.0, 0.0, -0.25]
    mask = np.ones(300, dtype=bool)
    mask[:3] = False                    # the planted signals are not used in the fit
    p, ne = mdfs.mdfs_pvalues(ig, k, d, fit_mask=mask)
    pr, ner = sig.pvalues(ig, k, d, fit_mask=mask)
    assert math.isclose(ne, ner, rel_tol=1e-11)
    assert rel_close(p, pr, 1e-9), np.max(np.abs(p - pr) / np.maximum(p, pr))
    assert p[3] == 1.0 and p[4] == 1.0 and 0 < p[2] < 1e-150
    # a fixed n_eff is used as given
    p1, ne1 = mdfs.mdfs_pvalues(ig, k, d, n_eff=7.25)
    pr1, _ = sig.pvalues(ig, k, d, n_eff=7.25)
    assert ne1 == 7.25 and rel_close(p1, pr1, 1e-9)


@pytest.mark.parametrize("k,d,ne,alpha", [(1, 2, 1.0, 0.05), (2, 2, 37.5, 0.05), (3, 2, 1e4, 1e-6),
                                          (2, 4, 3.0, 0.5), (2, 1, 2e6, 1e-12)])
def test_ig_lim(k, d, ne, alpha):
    x = mdfs.mdfs_ig_lim(k, d, ne, alpha)
    assert math.isclose(x, sig.ig_lim(k, d, ne, alpha), rel_tol=1e-9)
    p, _ = mdfs.mdfs_pvalues(np.array([x]), k, d, n_eff=ne)
    assert math.isclose(p[0], alpha, rel_tol=1e-8)


@pytest.mark.parametrize("method", ["none", "holm", "BH", "BY"])
def test_p_adjust(method):
    g = np.random.default_rng(3)
    for p in (np.round(g.uniform(size=500), 3), g.uniform(size=1) * 0.3, np.array([0.0, 1.0, 0.5, 0.5]),
              10.0 ** -g.uniform(0, 30, size=64)):
        assert rel_close(mdfs.mdfs_p_adjust(p, method), sig.p_adjust(p, method), 1e-14)


def test_errors():
    with pytest.raises(mdfs.MdfsError) as e:
        mdfs.mdfs_pvalues(np.array([1.0, np.nan]), 2, 2)
    assert e.value.code == -1
    with pytest.raises(mdfs.MdfsError) as e:
        mdfs.mdfs_pvalues(np.array([0.0, -1.0]), 2, 2)     # nothing usable for the fit
    assert e.value.code == -1
    with pytest.raises(mdfs.MdfsError) as e:
        mdfs.mdfs_pvalues(np.array([1.0]), 9, 2)
    assert e.value.code == -3
    with pytest.raises(mdfs.MdfsError) as e:
        mdfs.mdfs_chi2_df(2, 0)
    assert e.value.code == -4
    for a in (0.0, 1.0, float("nan")):
        with pytest.raises(mdfs.MdfsError):
            mdfs.mdfs_ig_lim(2, 2, 10.0, a)
    with pytest.raises(mdfs.MdfsError):
        mdfs.mdfs_ig_lim(2, 2, 0.0, 0.05)
    with pytest.raises(mdfs.MdfsError):
        mdfs.mdfs_p_adjust(np.array([0.5, 1.5]), "holm")
    with pytest.raises(KeyError):
        mdfs.mdfs_p_adjust(np.array([0.5]), "bonferroni")
