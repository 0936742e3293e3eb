"""The library's host evaluation of the refresh cadence (Sec. 4.4, Appendix D) against the oracle:
the truncation error d_alpha(k) and q_max (no GPU needed)."""
import math

import pytest

import paper_1601_00035_amd as nslgf
from oracle import refresh


@pytest.mark.parametrize("alpha", [1e-4, 0.013, 0.5, 3.0, 40.0, 250.0])
def test_trunc_error_matches_oracle(alpha):
    for k in (1, 2, 5, 17, 30):
        ref = refresh.trunc_error(alpha, k)
        got = nslgf.if_trunc_error(alpha, k)
        if ref < 1e-290:
            assert got < 1e-280
            continue
        assert abs(got - ref) <= 1e-12 * ref, (alpha, k, got, ref)
    assert nslgf.if_trunc_error(0.0, 4) == 0.0


CASES = [(0.05, 4, 0.7, 1e-8), (0.05, 4, 0.7, 1e-5), (0.0267, 16, 1.3, 1e-10), (0.0267, 16, 1.3, 1e-6),
         (0.3, 2, 0.2, 1e-4), (0.01, 8, 2.0, 1e-12), (0.05, 0, 0.7, 1e-12), (0.05, 3, 0.0, 1e-9),
         (0.002, 3, 0.5, 0.3)]


@pytest.mark.parametrize("beta,n_buf,umax,eps", CASES)
def test_refresh_interval_matches_oracle(beta, n_buf, umax, eps):
    cap = 5000
    ref = refresh.refresh_interval(beta, n_buf, umax, eps, q_cap=cap)
    if 0 < ref < cap:
        # the case is not decided by rounding: both neighbours of the boundary are clear of eps
        assert refresh.estimate(beta, ref, n_buf, umax) < eps * (1 - 1e-9)
        assert refresh.estimate(beta, ref + 1, n_buf, umax) > eps * (1 + 1e-9)
    assert nslgf.refresh_interval(beta, n_buf, umax, eps, cap) == ref


def test_host_errors():
    for args in ((-0.1, 3), (math.nan, 3), (0.1, 0)):
        with pytest.raises(nslgf.NslgfError):
            nslgf.if_trunc_error(*args)
    for args in ((-1.0, 2, 1.0, 1e-6), (0.1, -1, 1.0, 1e-6), (0.1, 2, -1.0, 1e-6), (0.1, 2, 1.0, 0.0),
                 (0.1, 2, 1.0, math.inf)):
        with pytest.raises(nslgf.NslgfError):
            nslgf.refresh_interval(*args)
    with pytest.raises(nslgf.NslgfError):
        nslgf.refresh_interval(0.1, 2, 1.0, 1e-6, 0)
