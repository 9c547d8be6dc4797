"""The library's host-side Chebyshev coefficient generator against the oracle's
(independent implementations of the same definition; no GPU needed)."""
import numpy as np
import pytest

from oracle import sign


@pytest.mark.parametrize("lam_lo,lam_max,n", [(0.186, 6.27, 200), (0.5, 6.5, 13), (0.9, 6.4, 57), (0.06 * 6.0, 6.0, 13)])
def test_coefficients_match_oracle(lam_lo, lam_max, n):
    from paper_1106_4964_amd import ovl

    s = ovl.Sign(lam_lo, lam_max, n=n)
    want = sign.chebyshev_coefficients((lam_lo / lam_max) ** 2, n)
    got = s.coeffs()
    assert s.n == n
    assert abs(s.eps - (lam_lo / lam_max) ** 2) < 1e-16
    assert np.max(np.abs(got - want)) < 1e-13 * np.max(np.abs(want))
    d_or = sign.measure_delta(want, s.eps)
    # both sum ~n rounding errors into 1 - sqrt(x) P(x): absolute agreement ~1e-14
    assert abs(s.delta - d_or) <= 1e-12 + 1e-9 * d_or


@pytest.mark.parametrize("sq,delta", [(0.0689, 1e-10), (0.1, 1e-8), (0.05, 1e-6)])
def test_order_choice_matches_oracle(sq, delta):
    from paper_1106_4964_amd import ovl

    s = ovl.Sign(sq, 1.0, delta=delta)
    assert s.n == sign.choose_order(sq * sq, delta)
    assert s.delta <= delta


def test_bad_sign_arguments():
    from paper_1106_4964_amd import ovl

    for args in [(1.0, 0.5), (0.0, 1.0), (-1.0, 2.0)]:
        with pytest.raises(ovl.OvlError):
            ovl.Sign(*args, n=10)
    with pytest.raises(ovl.OvlError):
        ovl.Sign(0.1, 1.0, delta=0.0, n=0)
