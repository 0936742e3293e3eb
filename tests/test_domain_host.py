"""The library's host classification of the active domain (Sec. 4.2, 4.3) against the oracle, on the
same block weights (no GPU needed): W, D_supp, D_soln and D_xsoln equal exactly."""
import numpy as np
import pytest

import paper_1601_00035_amd as nslgf
from oracle import blocks


@pytest.mark.parametrize("shape,n_xb", [((4, 5, 6), 1), ((7, 3, 9), 2), ((1, 1, 1), 0), ((8, 8, 8), 3)])
def test_classify_matches_oracle(shape, n_xb):
    rng = np.random.default_rng(sum(shape) + n_xb)
    mu = rng.exponential(1.0, shape) ** 3
    nu = rng.exponential(1.0, shape) ** 3
    mu[rng.random(shape) < 0.3] = 0.0
    for eps_supp, eps_soln in ((1e-2, 1e-2), (0.05, 0.2), (0.5, 0.01)):
        ref = blocks.classify(mu, nu, eps_supp, eps_soln, n_xb)
        got = nslgf.classify_blocks(mu, nu, eps_supp, eps_soln, n_xb)
        assert np.array_equal(got[0], ref[0])
        for g, r in zip(got[1:], ref[1:]):
            assert np.array_equal(g, r)


def test_classify_zero_weights_and_errors():
    z = np.zeros((2, 3, 4))
    W, supp, soln, xsoln = nslgf.classify_blocks(z, z, 0.0, 0.0, 1)
    assert not W.any() and not supp.any() and not xsoln.any()
    with pytest.raises(nslgf.NslgfError):
        nslgf.classify_blocks(-np.ones((2, 2, 2)), z[:2, :2, :2], 0.1, 0.1, 1)
    with pytest.raises(nslgf.NslgfError):
        nslgf.classify_blocks(z, z, np.nan, 0.1, 1)
    with pytest.raises(nslgf.NslgfError):
        nslgf.classify_blocks(z, z, 0.1, 0.1, -1)
