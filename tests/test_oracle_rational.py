"""Pins for the oracle's rational sign function (eq. 4, 5, 12): optimality
of the Zolotarev coefficients (equioscillation), the multi-shift CG and the
double-pass evaluation against dense linear algebra, and the sign itself
against the exact sign of a dense H_w."""
import math

import numpy as np
import pytest

import synth_inputs as si
from oracle import dense, rational as ra, sign
from oracle.lattice import Lattice


def _extrema(r, npts=400_001):
    """Signed peak of the relative error on each interval between its sign
    changes, in order."""
    y = ra._grid(r.eps, 1.0, npts)
    e = 1.0 - np.sqrt(y) * ra.rational_eval(r, y)
    cuts = np.nonzero(np.sign(e[1:]) != np.sign(e[:-1]))[0] + 1
    return np.array([seg[np.argmax(np.abs(seg))] for seg in np.split(e, cuts)])


@pytest.mark.parametrize("n,lo", [(4, 0.05), (6, 0.05), (9, 0.02), (5, 0.2)])
def test_zolotarev_error_equioscillates(n, lo):
    """The best type-(n-1, n) relative approximation has an error curve
    that alternates 2n + 1 times with equal magnitude (Chebyshev's
    alternation theorem): a wrong index, modulus or scale in the closed form
    breaks either the count or the equal ripple."""
    r = ra.make_rational(lo, 1.0, n)
    ext = _extrema(r)
    assert len(ext) == 2 * n + 1
    assert np.all(np.sign(ext[1:]) == -np.sign(ext[:-1]))
    mag = np.abs(ext)
    assert mag.max() / mag.min() - 1.0 < 1e-5
    assert abs(ra.measure_delta(r) - mag.max()) < 1e-3 * mag.max()


def test_rational_converges_faster_than_the_polynomial():
    """At eps = 5e-3 the rational function of 12 terms is more accurate than
    the optimal polynomial of order 150; delta falls with n."""
    lo = math.sqrt(5e-3)
    deltas = [ra.measure_delta(ra.make_rational(lo, 1.0, n)) for n in (4, 8, 12)]
    assert deltas[0] > deltas[1] > deltas[2]
    poly_delta = sign.measure_delta(sign.minimax_coefficients(5e-3, 150), 5e-3, 100_000)
    assert deltas[2] < poly_delta


def test_partial_fractions_equal_product_form():
    r = ra.make_rational(0.1, 2.0, 7)
    d0, num, den = ra.zolotarev_product(r.eps, 7)
    y = np.array([r.eps, 0.01, 0.1, 0.37, 1.0])
    bb = 1.0 / r.eps
    want = math.sqrt(bb) * d0 * ra._prod(bb * y, num, den)
    assert np.max(np.abs(ra.rational_eval(r, y) / want - 1.0)) < 1e-12


@pytest.fixture(scope="module")
def hpd():
    rng = np.random.default_rng(0)
    M = rng.standard_normal((60, 60)) + 1j * rng.standard_normal((60, 60))
    A = M @ M.conj().T / 60
    A = A / np.linalg.eigvalsh(A).max()
    b = rng.standard_normal(60) + 1j * rng.standard_normal(60)
    return A, b


def test_multishift_cg_solves_every_shift(hpd):
    A, b = hpd
    shifts = [0.003, 0.05, 0.3, 2.0]
    xs, its = ra.multishift_cg(lambda v: A @ v, b, shifts, tol=1e-13)
    for i, s in enumerate(shifts):
        want = np.linalg.solve(A + s * np.eye(len(b)), b)
        assert np.linalg.norm(xs[i] - want) <= 1e-11 * np.linalg.norm(want)


def test_double_pass_and_multishift_equal_dense_rational(hpd):
    A, b = hpd
    w, V = np.linalg.eigh(A)
    r = ra.make_rational(math.sqrt(w.min()) * 0.99, 1.0, 10)
    want = V @ (ra.rational_eval(r, w) * (V.conj().T @ b))
    got, k = ra.double_pass(lambda v: A @ v, b, r, tol=1e-13)
    assert np.linalg.norm(got - want) <= 1e-10 * np.linalg.norm(want)
    xs, _ = ra.multishift_cg(lambda v: A @ v, b, r.c, tol=1e-13)
    assert np.linalg.norm(np.tensordot(r.b, xs, axes=1) - want) <= 1e-10 * np.linalg.norm(want)


@pytest.mark.parametrize("method", ["multishift", "double"])
def test_rational_sign_equals_exact_sign(method):
    """Q P(Q^2) psi with the rational P (and with the 6 lowest modes of H_w
    projected exactly, eq. 7) against the exact sign of the dense H_w on
    2^4: the error stays within the measured delta of P."""
    dims = (2, 2, 2, 2)
    lat = Lattice(dims)
    U = si.gauge_field(dims, 0.3, 1)
    H = dense.dense_hw(lat, U, 1.5)
    E = dense.exact_sign(H)
    lo, hi = dense.spectrum_bounds(H)
    psi = si.gaussian_spinor(dims, 3)
    want = (E @ psi.reshape(-1)).reshape(psi.shape)
    r = ra.make_rational(lo, hi * 1.0001, 12)
    out = ra.sign_apply_rational(lat, U, psi, 1.5, r, method=method, tol=1e-13)
    assert np.linalg.norm(out - want) <= 1.2 * ra.measure_delta(r) * np.linalg.norm(psi) + 1e-12
    V, lam = dense.lowmodes(lat, H, 6)
    r6 = ra.make_rational(abs(lam[-1]), hi * 1.0001, 8)
    out = ra.sign_apply_rational(lat, U, psi, 1.5, r6, V=V, lam=lam, method=method, tol=1e-13)
    assert np.linalg.norm(out - want) <= 1.2 * ra.measure_delta(r6) * np.linalg.norm(psi) + 1e-12
