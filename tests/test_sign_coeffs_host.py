"""The library's host-side sign coefficients (the optimal polynomial of eq. 4
by its own Remez exchange) against the oracle's (an independent
implementation of the same definition; no GPU needed)."""
import numpy as np
import pytest

from oracle import sign


# (lam_lo, lam_max, n): optimal polynomials from delta ~ 0.1 (Fig. 2's case)
# down to ~5e-11 (the 24^3 x 64 workload's order), and one at the level of
# rounding (sqrt(eps) = 0.3, n = 120), where both keep the interpolant
@pytest.mark.parametrize("lam_lo,lam_max,n", [(0.186, 6.27, 200), (0.5, 6.5, 13), (0.9, 6.4, 57), (0.06 * 6.0, 6.0, 13),
                                              (0.0865, 1.0, 126), (0.3, 1.0, 120)])
def test_coefficients_match_oracle(lam_lo, lam_max, n):
    from paper_1106_4964_amd import ovl

    s = ovl.Sign(lam_lo, lam_max, n=n)
    eps = (lam_lo / lam_max) ** 2
    want = sign.minimax_coefficients(eps, n)
    got = s.coeffs()
    assert s.n == n
    assert abs(s.eps - eps) < 1e-16
    # the optimum is unique; the two exchanges stop within rounding of it
    assert np.max(np.abs(got - want)) < 1e-12 * np.max(np.abs(want))
    d_or = sign.measure_delta(want, s.eps)
    # both sum ~n rounding errors into 1 - sqrt(x) P(x): absolute agreement ~1e-14
    assert abs(s.delta - d_or) <= 1e-12 + 1e-9 * d_or
    # never worse than the interpolant of the same order (to rounding)
    assert s.delta <= sign.measure_delta(sign.chebyshev_coefficients(eps, n), eps) + 1e-12


# (0.1, 1e-8): the optimal polynomial, n = 84; (0.026, 1e-10): just above
# the exchange's order limit of 400, where both keep the interpolant
@pytest.mark.parametrize("sq,delta", [(0.1, 1e-8), (0.026, 1e-10)])
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
