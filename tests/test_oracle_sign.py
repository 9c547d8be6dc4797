"""Pins for the polynomial sign, projection and overlap operator (eq. 3-8, 11)."""
import math

import numpy as np
import pytest

import synth_inputs as si
from conftest import read_golden
from oracle import dense, dirac, sign
from oracle.lattice import Lattice

ANCH = read_golden("paper_anchors.txt")


# -- coefficient generator ----------------------------------------------------
@pytest.mark.parametrize("eps", [0.0, 0.01, 0.3])
def test_coefficients_exact_for_low_degree_polynomials(eps):
    """Interpolation of degree >= 2 reproduces x and x^2 exactly; their
    Chebyshev expansions in y follow from x = ((1-eps) y + 1 + eps)/2."""
    a, b = (1 - eps) / 2, (1 + eps) / 2
    c1 = sign.chebyshev_coefficients(eps, 5, f=lambda x: x)
    assert np.allclose(c1, [b, a, 0, 0, 0, 0], atol=1e-15)
    c2 = sign.chebyshev_coefficients(eps, 6, f=lambda x: x * x)
    # x^2 = a^2 y^2 + 2ab y + b^2,  y^2 = (T0 + T2)/2
    want = [a * a / 2 + b * b, 2 * a * b, a * a / 2, 0, 0, 0, 0]
    assert np.allclose(c2, want, atol=1e-15)


def test_interpolant_matches_function_at_nodes():
    eps, n = 0.004, 40
    c = sign.chebyshev_coefficients(eps, n)
    theta = math.pi * (np.arange(n + 1) + 0.5) / (n + 1)
    x = sign.x_of_y(np.cos(theta), eps)
    assert np.max(np.abs(sign.chebyshev_eval(c, np.cos(theta)) - x ** -0.5)) < 1e-12


def test_chebyshev_eval_agrees_with_numpy_chebval():
    rng = np.random.default_rng(0)
    c = rng.standard_normal(30)
    y = np.linspace(-1, 1, 101)
    assert np.max(np.abs(sign.chebyshev_eval(c, y) - np.polynomial.chebyshev.chebval(y, c))) < 1e-12


def test_fig2_anchor_optimal_polynomial():
    """Fig. 2: the optimal order-13 polynomial at sqrt(eps) ~ 0.06 has
    delta = 0.1 (to the caption's one digit and its "~").  The Chebyshev
    interpolant of the same order misses it by far (~0.18)."""
    n = int(ANCH["fig2_n"])
    eps = float(ANCH["fig2_sqrt_eps"]) ** 2
    d = sign.measure_delta(sign.minimax_coefficients(eps, n), eps)
    d_interp = sign.measure_delta(sign.chebyshev_coefficients(eps, n), eps)
    assert 0.9 * float(ANCH["fig2_delta"]) <= d <= 1.15 * float(ANCH["fig2_delta"])
    assert d_interp > 1.5 * d


def _alternation(e, tol):
    """Length of the longest sign-alternating sequence of grid points where
    |e| is within a factor (1 - tol) of max |e|."""
    top = np.max(np.abs(e))
    idx = np.flatnonzero(np.abs(e) >= (1.0 - tol) * top)
    count, last = 0, 0.0
    for i in idx:
        sgn = np.sign(e[i])
        if sgn != last:
            count += 1
            last = sgn
    return count


@pytest.mark.parametrize("sq,n", [(0.06, 13), (0.1, 30), (0.0689, 60), (0.2, 8)])
def test_optimal_polynomial_equioscillates(sq, n):
    """Chebyshev's alternation theorem characterises the optimal P of eq. (4)
    (weight sqrt(x) on the error of x^{-1/2}): |e| reaches its maximum with
    alternating sign at n + 2 points at least, and no other polynomial of
    order n does.  The interpolant does not (its error is larger near
    x = eps), and neither would an unweighted (absolute-error) optimum."""
    eps = sq * sq
    x = sign.delta_grid(eps, 400_000)
    x.sort()
    e = sign.relative_error(sign.minimax_coefficients(eps, n), eps, x)
    assert _alternation(e, 1e-6) >= n + 2
    e_interp = sign.relative_error(sign.chebyshev_coefficients(eps, n), eps, x)
    assert _alternation(e_interp, 1e-6) < n + 2
    # an absolute-error optimum levels |x^{-1/2} - P| instead: its relative error is not level
    c_abs = np.polynomial.chebyshev.chebfit(sign.y_of_x(x, eps), x ** -0.5, n)
    assert _alternation(sign.relative_error(c_abs, eps, x), 1e-6) < n + 2


@pytest.mark.parametrize("n", [40, 80, 120])
def test_delta_follows_order_law(n):
    """eq. (11) with A = 0.41, b = 2.1 (fitted to optimal polynomials): the
    optimal delta follows it to 25%; the interpolant sits ~1.8x above."""
    A, b = float(ANCH["order_law_A"]), float(ANCH["order_law_b"])
    sq = 0.0689
    d = sign.measure_delta(sign.minimax_coefficients(sq * sq, n), sq * sq)
    law = A * math.exp(-b * n * sq)
    assert law / 1.25 <= d <= 1.25 * law
    d_interp = sign.measure_delta(sign.chebyshev_coefficients(sq * sq, n), sq * sq)
    assert d_interp > 1.5 * d


def test_rounding_level_keeps_interpolant():
    """Where the interpolant's delta is already at FP64 rounding the exchange
    has nothing to level: the interpolant is returned unchanged."""
    eps = 0.3 ** 2
    c = sign.minimax_coefficients(eps, 120)
    assert sign.measure_delta(c, eps) <= sign.ROUNDING_DELTA
    assert np.array_equal(c, sign.chebyshev_coefficients(eps, 120))


def test_choose_order_is_minimal():
    eps, target = 0.0689 ** 2, 1e-8
    n = sign.choose_order(eps, target)
    assert sign.measure_delta(sign.minimax_coefficients(eps, n), eps) <= target
    assert sign.measure_delta(sign.minimax_coefficients(eps, n - 1), eps) > target
    # the optimal polynomials follow eq. (11): its order is within a few per cent
    assert abs(n - sign.order_law_n(eps, target)) <= 0.05 * n
    assert n < sign.interpolant_order(eps, target)


# -- dense references at 2^4 ----------------------------------------------------
@pytest.fixture(scope="module")
def small():
    lat = Lattice((2, 2, 2, 2))
    U = si.gauge_field(lat.dims, 0.3, seed=1)
    H = dense.dense_hw(lat, U, 1.5)
    lo, hi = dense.spectrum_bounds(H)
    return lat, U, H, lo, hi


def test_clenshaw_equals_spectral_polynomial(small):
    lat, U, H, lo, hi = small
    s = sign.make_sign(lo, hi, 30)
    psi = si.gaussian_spinor(lat.dims, 101)
    got = sign.clenshaw_p(lat, U, psi, 1.5, s)
    w, v = np.linalg.eigh(H)
    p = sign.chebyshev_eval(s.coeffs, sign.y_of_x((w / hi) ** 2, s.eps))
    want = (v * p) @ (v.conj().T @ psi.reshape(-1))
    assert np.max(np.abs(got.reshape(-1) - want)) < 1e-12 * np.max(np.abs(want))


def test_dw_count_is_2n_plus_1(small):
    lat, U, H, lo, hi = small
    s = sign.make_sign(lo, hi, 17)
    cnt = sign.Counter()
    sign.sign_apply(lat, U, si.gaussian_spinor(lat.dims, 1), 1.5, s, counter=cnt)
    assert cnt.dw == 2 * 17 + 1


@pytest.mark.parametrize("n", [40, 200])
def test_sign_within_delta_of_exact(small, n):
    """|x P(x^2) - sign x| <= delta on the spectrum, so ||(eps_P - sign H)psi|| <= delta ||psi||."""
    lat, U, H, lo, hi = small
    s = sign.make_sign(lo, hi, n)
    delta = sign.measure_delta(s.coeffs, s.eps)
    psi = si.gaussian_spinor(lat.dims, 102)
    got = sign.sign_apply(lat, U, psi, 1.5, s).reshape(-1)
    want = dense.exact_sign(H) @ psi.reshape(-1)
    err = np.linalg.norm(got - want) / np.linalg.norm(psi)
    assert err <= delta * 1.01 + 1e-14


def test_projection_exact_on_low_modes(small):
    lat, U, H, lo, hi = small
    V, lam = dense.lowmodes(lat, H, 6)
    s = sign.make_sign(abs(lam[-1]), hi, 60)
    for i in range(6):
        got = sign.sign_apply(lat, U, V[i], 1.5, s, V, lam)
        assert np.max(np.abs(got - np.sign(lam[i]) * V[i])) < 1e-13
    psi = si.gaussian_spinor(lat.dims, 103)
    delta = sign.measure_delta(s.coeffs, s.eps)
    got = sign.sign_apply(lat, U, psi, 1.5, s, V, lam).reshape(-1)
    want = dense.exact_sign(H) @ psi.reshape(-1)
    assert np.linalg.norm(got - want) <= delta * np.linalg.norm(psi) * 1.01 + 1e-13


def test_sign_squares_to_one_and_ginsparg_wilson(small):
    lat, U, H, lo, hi = small
    s = sign.make_sign(lo, hi, 200)
    delta = sign.measure_delta(s.coeffs, s.eps)
    psi = si.gaussian_spinor(lat.dims, 104)
    e1 = sign.sign_apply(lat, U, psi, 1.5, s)
    e2 = sign.sign_apply(lat, U, e1, 1.5, s)
    assert np.linalg.norm(e2 - psi) <= 3 * delta * np.linalg.norm(psi) + 1e-12
    # GW: gamma5 D + D gamma5 = D gamma5 D
    D = lambda v: sign.massless_overlap(lat, U, v, 1.5, s)  # noqa: E731
    g5 = dirac.gamma5
    lhs = g5(D(psi)) + D(g5(psi))
    rhs = D(g5(D(psi)))
    assert np.linalg.norm(lhs - rhs) <= 20 * delta * np.linalg.norm(psi) + 1e-12


def test_exact_overlap_spectrum_on_circle(small):
    lat, U, H, lo, hi = small
    Dm = np.eye(H.shape[0]) + dense.dense_gamma5(lat) @ dense.exact_sign(H)
    d = np.linalg.eigvals(Dm)
    assert np.max(np.abs(np.abs(d - 1) - 1)) < 1e-12


def test_massive_overlap_normal_identity(small):
    """D(m)^dag D(m) = m^2 + (rho^2 - m^2/4)(D + D^dag) holds to O(delta)."""
    lat, U, H, lo, hi = small
    rho, m = 1.5, 0.05
    s = sign.make_sign(lo, hi, 200)
    delta = sign.measure_delta(s.coeffs, s.eps)
    psi = si.gaussian_spinor(lat.dims, 105)
    Dm = lambda v, dag=False: sign.overlap_apply(lat, U, v, rho, m, s, dagger=dag)  # noqa: E731
    lhs = Dm(Dm(psi), dag=True)
    D = sign.massless_overlap(lat, U, psi, rho, s)
    Ddag = psi + sign.sign_apply(lat, U, dirac.gamma5(psi), rho, s)
    rhs = m * m * psi + (rho * rho - m * m / 4) * (D + Ddag)
    # exact when sign^2 = 1; the polynomial breaks it by O(delta), weighted by rho^2
    assert np.linalg.norm(lhs - rhs) < 4 * rho * rho * delta * np.linalg.norm(psi)
    # dagger is the adjoint
    phi = si.gaussian_spinor(lat.dims, 106)
    a = np.vdot(phi, Dm(psi))
    b = np.vdot(Dm(phi, dag=True), psi)
    assert abs(a - b) < 1e-12 * abs(a)


@pytest.mark.parametrize("chir", [1, -1])
def test_chiral_sector_operator(small, chir):
    """On a vector of chirality s (gamma5 v = s v), with the exact sign,
    D(m) D(m)^dag v = (2 rho^2 + m^2/2) v + 2 s (rho^2 - m^2/4) P_s sign(H_w) v
    with P_s = (1 + s gamma5)/2 (eq. 3 and 8), and D D^dag keeps the sector."""
    lat, U, H, lo, hi = small
    rho, m = 1.5, 0.03
    n = H.shape[0]
    G5 = dense.dense_gamma5(lat)
    E = dense.exact_sign(H)
    Dm = (rho + m / 2) * np.eye(n) + (rho - m / 2) * G5 @ E
    Ps = 0.5 * (np.eye(n) + chir * G5)
    v = Ps @ si.gaussian_spinor(lat.dims, 107).reshape(-1)
    assert np.linalg.norm(G5 @ v - chir * v) < 1e-14 * np.linalg.norm(v)
    lhs = Dm @ (Dm.conj().T @ v)
    rhs = (2 * rho * rho + m * m / 2) * v + 2 * chir * (rho * rho - m * m / 4) * (Ps @ (E @ v))
    assert np.linalg.norm(lhs - rhs) < 1e-12 * np.linalg.norm(lhs)
    assert np.linalg.norm(lhs - Ps @ lhs) < 1e-12 * np.linalg.norm(lhs)


@pytest.mark.parametrize("m", [0.01, 0.05, 0.3])
def test_mass_shift_structure(small, m):
    """With the exact sign, D(m) D(m)^dag = (rho^2 - m^2/4) (K + sigma(m))
    with the mass-independent K = gamma5 sign + sign gamma5 and
    sigma(m) = (2 rho^2 + m^2/2) / (rho^2 - m^2/4) (eq. 3 and 8): every mass
    is a shift of one operator, so one Krylov space serves them all."""
    lat, U, H, lo, hi = small
    rho = 1.5
    n = H.shape[0]
    G5 = dense.dense_gamma5(lat)
    E = dense.exact_sign(H)
    Dm = (rho + m / 2) * np.eye(n) + (rho - m / 2) * G5 @ E
    K = G5 @ E + E @ G5
    sigma = (2 * rho * rho + m * m / 2) / (rho * rho - m * m / 4)
    lhs = Dm @ Dm.conj().T
    rhs = (rho * rho - m * m / 4) * (K + sigma * np.eye(n))
    assert np.max(np.abs(lhs - rhs)) < 1e-12 * np.max(np.abs(lhs))
    # K + sigma is positive: K's spectrum lies in [-2, 2] and sigma > 2
    assert np.max(np.linalg.eigvalsh(K)) <= 2 + 1e-12 and sigma > 2


def test_free_field_overlap_closed_form():
    """U = 1: D(p) = 1 + (M(p) + i gamma.sin p)/omega(p), M = -rho + sum(1-cos p)."""
    lat = Lattice((4, 4, 2, 2))
    U = si.unit_gauge_field(lat.dims)
    s = sign.make_sign(0.5, 6.5, 120)
    delta = sign.measure_delta(s.coeffs, s.eps)
    rng = np.random.default_rng(3)
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    for k in [(0, 0, 0, 0), (1, 0, 1, 0), (2, 3, 1, 1)]:
        p = [2 * np.pi * k[mu] / lat.dims[mu] for mu in range(4)]
        ph = np.array([np.exp(1j * sum(p[mu] * c for mu, c in enumerate(lat.coords(i)))) for i in range(lat.N)])
        psi = ph[:, None, None] * u[None]
        M = -1.5 + sum(1 - np.cos(q) for q in p)
        sp = [np.sin(q) for q in p]
        om = math.sqrt(M * M + sum(x * x for x in sp))
        Dp = np.eye(4) + (M * np.eye(4) + 1j * sum(dirac.GAMMA[mu] * sp[mu] for mu in range(4))) / om
        want = np.matmul(Dp, psi)
        got = sign.massless_overlap(lat, U, psi, 1.5, s)
        assert np.linalg.norm(got - want) <= 2 * delta * np.linalg.norm(psi) + 1e-12
        if k == (0, 0, 0, 0):
            assert np.linalg.norm(got) <= 2 * delta * np.linalg.norm(psi) + 1e-12  # zero mode


def test_free_field_has_12_zero_modes():
    lat = Lattice((2, 2, 2, 2))
    H = dense.dense_hw(lat, si.unit_gauge_field(lat.dims), 1.5)
    D = np.eye(H.shape[0]) + dense.dense_gamma5(lat) @ dense.exact_sign(H)
    assert int(np.sum(np.abs(np.linalg.eigvals(D)) < 1e-10)) == 12


def test_overlap_gauge_covariance():
    lat = Lattice((2, 2, 2, 4))
    U = si.gauge_field(lat.dims, 0.3, seed=6)
    g = si.gauge_transform(lat.dims, seed=10)
    Ug = dirac.gauge_rotate(lat, U, g)
    H = dense.dense_hw(lat, U, 1.5)
    lo, hi = dense.spectrum_bounds(H)
    V, lam = dense.lowmodes(lat, H, 4)
    Vg = np.stack([dirac.colour_rotate(lat, v, g) for v in V])
    s = sign.make_sign(abs(lam[-1]), hi, 50)
    psi = si.gaussian_spinor(lat.dims, 7)
    lhs = sign.overlap_apply(lat, Ug, dirac.colour_rotate(lat, psi, g), 1.5, 0.01, s, Vg, lam)
    rhs = dirac.colour_rotate(lat, sign.overlap_apply(lat, U, psi, 1.5, 0.01, s, V, lam), g)
    assert np.max(np.abs(lhs - rhs)) < 1e-12


@pytest.mark.slow
def test_dense_sign_4444_with_projection():
    """4^4 (3072 x 3072): projected polynomial sign vs the exact sign."""
    lat = Lattice((4, 4, 4, 4))
    U = si.gauge_field(lat.dims, 0.3, seed=1)
    H = dense.dense_hw(lat, U, 1.5)
    V, lam = dense.lowmodes(lat, H, 20)
    hi = dense.spectrum_bounds(H)[1]
    s = sign.make_sign(abs(lam[-1]), hi, 100)
    delta = sign.measure_delta(s.coeffs, s.eps)
    psi = si.gaussian_spinor(lat.dims, 101)
    got = sign.sign_apply(lat, U, psi, 1.5, s, V, lam).reshape(-1)
    want = dense.exact_sign(H) @ psi.reshape(-1)
    assert np.linalg.norm(got - want) <= 1.01 * delta * np.linalg.norm(psi) + 1e-12


# -- eq. (8): the mass term of D(m), pinned without overlap_apply's own algebra --
def _free_field_plane_waves(lat, seed):
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    for k in [(0, 0, 0, 0), (1, 0, 1, 0), (2, 3, 1, 1), (3, 1, 0, 1)]:
        p = [2 * np.pi * k[mu] / lat.dims[mu] for mu in range(4)]
        ph = np.array([np.exp(1j * sum(p[mu] * c for mu, c in enumerate(lat.coords(i)))) for i in range(lat.N)])
        M = -1.5 + sum(1 - np.cos(q) for q in p)
        sp = [np.sin(q) for q in p]
        om = math.sqrt(M * M + sum(x * x for x in sp))
        Dp = np.eye(4) + (M * np.eye(4) + 1j * sum(dirac.GAMMA[mu] * sp[mu] for mu in range(4))) / om
        yield k, ph[:, None, None] * u[None], Dp


def _eq8_free_field_error(apply_dm, m, dagger):
    """max over plane waves of ||D(m) psi - want|| / ||psi|| with
    want = [rho D(p) + m (1 - D(p)/2)] psi (eq. 8), D(p) the closed form of
    the massless overlap at U = 1 (D(p)^dag for the adjoint)."""
    lat = Lattice((4, 4, 2, 2))
    rho = 1.5
    worst = 0.0
    for _, psi, Dp in _free_field_plane_waves(lat, 5):
        Dx = Dp.conj().T if dagger else Dp
        want = np.matmul(rho * Dx + m * (np.eye(4) - 0.5 * Dx), psi)
        got = apply_dm(lat, si.unit_gauge_field(lat.dims), psi, rho, m, dagger)
        worst = max(worst, np.linalg.norm(got - want) / np.linalg.norm(psi))
    return worst


_FREE_SIGN = sign.make_sign(0.5, 6.5, 120)


def _oracle_dm(lat, U, psi, rho, m, dagger):
    return sign.overlap_apply(lat, U, psi, rho, m, _FREE_SIGN, dagger=dagger)


@pytest.mark.parametrize("dagger", [False, True])
@pytest.mark.parametrize("m", [0.01, 0.05, 0.3])
def test_massive_overlap_free_field_closed_form(m, dagger):
    """eq. (8) D(m) = rho D + m (1 - D/2) and its adjoint against the
    momentum-space closed form of D at U = 1 (not through massless_overlap),
    to the sign error (rho - m/2) delta."""
    delta = sign.measure_delta(_FREE_SIGN.coeffs, _FREE_SIGN.eps)
    assert _eq8_free_field_error(_oracle_dm, m, dagger) <= 2 * 1.5 * delta + 1e-12


@pytest.mark.parametrize("dagger", [False, True])
def test_eq8_pin_catches_swapped_mass_term(dagger):
    """The pin above fails for D(-m), i.e. rho +- m/2 swapped: at p = 0 the
    massless D vanishes, so the two differ by 2 m ||psi||."""
    def swapped(lat, U, psi, rho, m, dag):
        return sign.overlap_apply(lat, U, psi, rho, -m, _FREE_SIGN, dagger=dag)

    delta = sign.measure_delta(_FREE_SIGN.coeffs, _FREE_SIGN.eps)
    for m in (0.01, 0.05):
        assert _eq8_free_field_error(swapped, m, dagger) > 1.9 * m
        assert _eq8_free_field_error(swapped, m, dagger) > 1e3 * (2 * 1.5 * delta + 1e-12)


@pytest.mark.parametrize("m", [0.01, 0.05, 0.3])
def test_massive_overlap_is_rho_d_plus_mass_term(small, m):
    """eq. (8) on an interacting 2^4 field: the dense D(m) and D(m)^dag built
    column by column from overlap_apply equal rho D + m (1 - D/2) and its
    conjugate transpose, with D the dense massless overlap (eq. 3) on the
    same polynomial."""
    lat, U, H, lo, hi = small
    rho = 1.5
    s = sign.make_sign(lo, hi, 30)
    D = dense.dense_operator(lat, lambda v: sign.massless_overlap(lat, U, v, rho, s))
    Dm = dense.dense_operator(lat, lambda v: sign.overlap_apply(lat, U, v, rho, m, s))
    Dmd = dense.dense_operator(lat, lambda v: sign.overlap_apply(lat, U, v, rho, m, s, dagger=True))
    one = np.eye(D.shape[0])
    want = rho * D + m * (one - 0.5 * D)
    assert np.max(np.abs(Dm - want)) < 1e-12 * np.max(np.abs(want))
    assert np.max(np.abs(Dmd - want.conj().T)) < 1e-12 * np.max(np.abs(want))
