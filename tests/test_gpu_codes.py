"""mdfs_max_ig_codes: the sweep from caller-supplied codes."""
import itertools

import numpy as np
import pytest
import torch

import oracle
from paper_1811_00631_amd import mdfs, workloads

DEV = "cuda:0"
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("k,div,engine", [(2, 2, "mfma_fp4"), (2, 2, "mfma"), (2, 1, "auto"), (2, 4, "auto"),
                                          (3, 2, "mfma_fp4"), (3, 2, "bitset"), (3, 4, "bitset"), (1, 2, "auto")])
def test_codes_of_the_discretisation_give_identical_results(k, div, engine):
    # the oracle's codes of the library's own discretisation: every output bit-identical
    w = workloads.xor_small(seed=41, n_obj=700, n_var=45 if k == 3 else 130, divisions=div, n_disc=3)
    print(f"codes k={k} div={div} {engine}", flush=True)
    codes = oracle.discretize(w.data, div, 3, 0.5, 13, disc_offset=2)
    X, y = torch.from_numpy(w.data).to(DEV), torch.from_numpy(w.y).to(DEV)
    a = mdfs.mdfs_max_ig(X, y, k, div, 3, 0.25, 0.5, 13, disc_offset=2, engine=engine)
    b = mdfs.mdfs_max_ig_codes(torch.from_numpy(codes).to(DEV), y, k, div, 0.25, disc_offset=2, engine=engine)
    for u, v in zip(a, b):
        assert torch.equal(u, v)


def test_arbitrary_codes_match_the_oracle():
    # codes that no discretisation produces: skewed bins, one bin empty in one variable, a
    # constant variable; IG from the oracle's tables, tie rule of the library
    g = np.random.default_rng(77)
    n_obj, n_var, R, div = 300, 24, 2, 2
    codes = g.choice(3, size=(R, n_var, n_obj), p=[0.6, 0.3, 0.1]).astype(np.uint8)
    codes[:, 3] = np.minimum(codes[:, 3], 1)
    codes[:, 5] = 2
    y = (g.uniform(size=n_obj) < 0.4).astype(np.uint8)
    codes[:, 7] = ((y + codes[:, 8]) % 3).astype(np.uint8)     # a strong dependency
    b0, b1 = oracle.betas(y, 0.25)
    best = np.full(n_var, -np.inf)
    arg = np.zeros(n_var, dtype=np.int64)
    argd = np.zeros(n_var, dtype=np.int64)
    cands = [[] for _ in range(n_var)]
    for r in range(R):
        for i, j in itertools.combinations(range(n_var), 2):
            for member, other in ((0, j), (1, i)):
                v = (i, j)[member]
                ig = oracle.ig_member(codes[r], y, div + 1, [i, j], member, b0, b1)
                cands[v].append((ig, r, other))
    # the tie rule over the final maximum: candidates within tau = 1e-9 max(1, |max|) of it are
    # tied; the smallest discretisation wins, then the smallest partner
    for v in range(n_var):
        best[v] = max(c[0] for c in cands[v])
        tau = 1e-9 * max(1.0, abs(best[v]))
        argd[v], arg[v], _ = min((r, other, ig) for ig, r, other in cands[v] if ig >= best[v] - tau)
    print("arbitrary codes", flush=True)
    ig, am, ad = mdfs.mdfs_max_ig_codes(torch.from_numpy(codes).to(DEV), torch.from_numpy(y).to(DEV), 2, div, 0.25)
    ig = ig.cpu().numpy().astype(np.float64)
    err = np.abs(ig - best) / np.maximum(np.abs(best), 1.0)    # per element
    assert err.max() <= 1e-4
    assert np.array_equal(am.cpu().numpy()[:, 0], arg)
    assert np.array_equal(ad.cpu().numpy(), argd)
    assert ig[7] == ig.max() and am.cpu().numpy()[7, 0] == 8


def test_codes_out_of_range_rejected():
    codes = torch.zeros((1, 4, 50), dtype=torch.uint8, device=DEV)
    codes[0, 2, 17] = 3
    y = torch.zeros(50, dtype=torch.uint8, device=DEV)
    y[::2] = 1
    with pytest.raises(mdfs.MdfsError) as e:
        mdfs.mdfs_max_ig_codes(codes, y, 2, 2)
    assert e.value.code == -1 and "codes" in str(e.value)
    # a valid call on the same workspace afterwards succeeds (the flag is per call)
    codes[0, 2, 17] = 2
    mdfs.mdfs_max_ig_codes(codes, y, 2, 2)
