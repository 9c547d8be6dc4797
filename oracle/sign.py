"""Polynomial sign function, low-mode projection and the overlap operator.

Oracle (test infrastructure).  Follows arXiv:1106.4964:

* eq. (4): P(x) approximates x^{-1/2} on [eps, 1]; its quality is
  delta = max_{x in [eps,1]} |1 - sqrt(x) P(x)|.
* eq. (5): sign(H_w) ~ Q P(Q^2) with Q = H_w / ||H_w||.
* Sec. V: P is expanded in Chebyshev polynomials and P(Q^2) psi is evaluated
  by a Clenshaw recursion (five vectors).
* eq. (11): the empirical order law delta = A exp(-b n sqrt(eps)) with
  A = 0.41, b = 2.1, used here only as the starting guess for n (the
  optimal polynomials below follow it to a few per cent).
* eq. (6)-(7): with the l eigenpairs (lambda_i, eta_i) of H_w closest to
  zero, psi = psi_l + psi_h, psi_l = sum_i (eta_i^dagger psi) eta_i, and
  sign(H_w) psi = sum_i sign(lambda_i) (eta_i^dagger psi) eta_i + Q P(Q^2) psi_h.
* eq. (3): D = 1 + gamma5 sign(H_w);  eq. (8): D(m) = rho D + m (1 - D/2).

Readings:
* eq. (4) asks for the P of order n that minimises delta (the optimal
  polynomial; Fig. 2 prints delta = 0.1 at n = 13, sqrt(eps) ~ 0.06).  The
  paper cites a "robust numerical method" for it without describing it;
  here it is the Remez exchange for the weighted minimax problem
  min_P max_x |1 - sqrt(x) P(x)|: P is held as Chebyshev coefficients in
  the variable y = (2x - 1 - eps)/(1 - eps) (c_0 carrying the usual 1/2),
  started from the Chebyshev interpolant of x^{-1/2} at the n+1
  Chebyshev-Gauss nodes, and the exchange levels the error on n+2 points
  until it alternates with equal size there and nowhere exceeds it.  When
  the interpolant's delta is already at the level of FP64 rounding
  (<= 1e-12) the extrema are noise and the interpolant is kept; so it is
  above order 400 (where the exchange's dense system gets large and the
  two differ by a few per cent in order).  n is the
  order of P in x = Q^2, so one sign apply costs 2n+1 applications of D_w.
* ||H_w|| is an upper bound lam_max on |spectrum(H_w)|, supplied as data.
* With low modes, sqrt(eps) = |lambda_l| / lam_max (Sec. V).
* The projection is applied once, to the input.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import dirac
from .lattice import Lattice

ORDER_LAW_A = 0.41
ORDER_LAW_B = 2.1


# ---------------------------------------------------------------------------
# Chebyshev approximation of x^{-1/2} on [eps, 1]
# ---------------------------------------------------------------------------
def x_of_y(y, eps):
    """Map y in [-1,1] to x in [eps,1]; inverse of y = (2x-1-eps)/(1-eps)."""
    return 0.5 * ((1.0 - eps) * np.asarray(y) + 1.0 + eps)


def y_of_x(x, eps):
    return (2.0 * np.asarray(x) - 1.0 - eps) / (1.0 - eps)


def chebyshev_coefficients(eps: float, n: int, f=None) -> np.ndarray:
    """c_0..c_n of the degree-n Chebyshev interpolant of f on [eps,1].

    c_k = 2/(n+1) sum_j f(x(cos theta_j)) cos(k theta_j),
    theta_j = pi (j + 1/2)/(n+1), j = 0..n, and c_0 is halved.
    f defaults to x^{-1/2}.
    """
    if f is None:
        f = lambda x: 1.0 / np.sqrt(x)  # noqa: E731
    j = np.arange(n + 1)
    theta = math.pi * (j + 0.5) / (n + 1)
    fx = f(x_of_y(np.cos(theta), eps))
    c = np.array([2.0 / (n + 1) * np.sum(fx * np.cos(k * theta)) for k in range(n + 1)])
    c[0] *= 0.5
    return c


def chebyshev_eval(c: np.ndarray, y) -> np.ndarray:
    """sum_k c_k T_k(y) for scalar/array y, by the three-term recurrence of T_k."""
    y = np.asarray(y, dtype=np.float64)
    t_prev = np.ones_like(y)
    total = c[0] * t_prev
    if len(c) == 1:
        return total
    t_cur = y.copy()
    total = total + c[1] * t_cur
    for k in range(2, len(c)):
        t_prev, t_cur = t_cur, 2.0 * y * t_cur - t_prev
        total = total + c[k] * t_cur
    return total


def delta_grid(eps: float, npts: int = 400_000) -> np.ndarray:
    """x points on [eps,1]: half uniform in x, half Chebyshev-clustered in y."""
    half = npts // 2
    xu = np.linspace(eps, 1.0, half)
    theta = np.linspace(0.0, math.pi, npts - half)
    xc = x_of_y(np.cos(theta), eps)
    return np.concatenate([xu, xc])


def measure_delta(c: np.ndarray, eps: float, npts: int = 400_000) -> float:
    """delta = max |1 - sqrt(x) P(x)| over the grid (eq. 4)."""
    x = delta_grid(eps, npts)
    p = chebyshev_eval(c, y_of_x(x, eps))
    return float(np.max(np.abs(1.0 - np.sqrt(x) * p)))


def order_law_n(eps: float, delta: float) -> int:
    """n from eq. (11): delta = A exp(-b n sqrt(eps)), rounded up."""
    return max(1, int(math.ceil(math.log(ORDER_LAW_A / delta) / (ORDER_LAW_B * math.sqrt(eps)))))


def interpolant_order(eps: float, delta: float, npts: int = 400_000, n_max: int = 20000) -> int:
    """Smallest n whose interpolant reaches measured delta <= target.

    Starts from the order law, brackets by doubling the step, then bisects
    (the measured delta decreases with n).
    """
    ok = lambda n: measure_delta(chebyshev_coefficients(eps, n), eps, npts) <= delta  # noqa: E731
    n = order_law_n(eps, delta)
    if ok(n):
        hi = n
        step = 1
        lo = n - step
        while lo >= 1 and ok(lo):
            hi = lo
            step *= 2
            lo = hi - step
        lo = max(lo, 0)
    else:
        lo = n
        step = 1
        hi = n + step
        while not ok(hi):
            lo = hi
            step *= 2
            hi = lo + step
            if hi > n_max:
                raise ValueError("order above n_max")
    # invariant: ok(hi), not ok(lo) (or lo == 0)
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if ok(mid):
            hi = mid
        else:
            lo = mid
    return hi


# ---------------------------------------------------------------------------
# The optimal polynomial of eq. (4): Remez exchange
# ---------------------------------------------------------------------------
ROUNDING_DELTA = 1e-12  # below this the interpolant is kept (see Readings)
MINIMAX_MAX_ORDER = 400  # above this too (the dense (n+2)^2 exchange system)


def relative_error(c: np.ndarray, eps: float, x) -> np.ndarray:
    """e(x) = 1 - sqrt(x) P(x), P = sum_k c_k T_k(y(x))  (the quantity of eq. 4)."""
    x = np.asarray(x, dtype=np.float64)
    return 1.0 - np.sqrt(x) * chebyshev_eval(c, y_of_x(x, eps))


def _zero_in(c, eps, a, b, steps=60):
    """A zero of e in each [a_i, b_i], where e(a_i) and e(b_i) differ in sign (bisection)."""
    a = np.array(a, dtype=np.float64)
    b = np.array(b, dtype=np.float64)
    ea = relative_error(c, eps, a)
    for _ in range(steps):
        m = 0.5 * (a + b)
        em = relative_error(c, eps, m)
        left = np.sign(em) != np.sign(ea)  # the zero lies in [a, m]
        b = np.where(left, m, b)
        a = np.where(left, a, m)
        ea = np.where(left, ea, em)
    return 0.5 * (a + b)


def _peak_in(c, eps, a, b, steps=80):
    """The point of largest |e| in each [a_i, b_i] (golden-section search on
    |e|, which has one peak between consecutive zeros; the interval ends are
    candidates too, for the peaks at x = eps and x = 1)."""
    a = np.array(a, dtype=np.float64)
    b = np.array(b, dtype=np.float64)
    lo, hi = a.copy(), b.copy()
    g = (math.sqrt(5.0) - 1.0) / 2.0
    for _ in range(steps):
        x1 = hi - g * (hi - lo)
        x2 = lo + g * (hi - lo)
        f1 = np.abs(relative_error(c, eps, x1))
        f2 = np.abs(relative_error(c, eps, x2))
        keep_left = f1 > f2
        hi = np.where(keep_left, x2, hi)
        lo = np.where(keep_left, lo, x1)
    cand = np.stack([a, 0.5 * (lo + hi), b])
    f = np.abs(relative_error(c, eps, cand))
    return cand[np.argmax(f, axis=0), np.arange(cand.shape[1])]


_MINIMAX_CACHE: dict = {}


def minimax_coefficients(eps: float, n: int, maxit: int = 60) -> np.ndarray:
    """c_0..c_n of the order-n P that minimises delta of eq. (4) on [eps, 1]
    (computed once per (eps, n, maxit); a copy is returned)."""
    key = (float(eps), int(n), int(maxit))
    if key not in _MINIMAX_CACHE:
        _MINIMAX_CACHE[key] = _remez(float(eps), int(n), int(maxit))
    return _MINIMAX_CACHE[key].copy()


def _remez(eps: float, n: int, maxit: int) -> np.ndarray:
    """c_0..c_n of the order-n P that minimises delta of eq. (4) on [eps, 1].

    Remez exchange.  Given n+2 points r_0 < ... < r_{n+1}, the linear system
    sum_k c_k T_k(y(r_i)) + (-1)^i E / sqrt(r_i) = 1 / sqrt(r_i) makes
    e(r_i) = (-1)^i E; e then has a zero between consecutive r_i, and the
    new points are the peaks of |e| between consecutive zeros (and the ends).
    The levelled |E| rises and max|e| falls to the common optimum; the loop
    stops when they agree to 1e-10, or when the gap stops shrinking because
    e is at the level of rounding."""
    c0 = chebyshev_coefficients(eps, n)
    if measure_delta(c0, eps) <= ROUNDING_DELTA or n > MINIMAX_MAX_ORDER:
        return c0
    # start: the interpolant's error vanishes at the nodes, so it has one
    # peak in each of the n+2 gaps between eps, the nodes and 1
    theta = math.pi * (np.arange(n + 1) + 0.5) / (n + 1)
    nodes = np.sort(x_of_y(np.cos(theta), eps))
    edges = np.concatenate([[eps], nodes, [1.0]])
    ref = _peak_in(c0, eps, edges[:-1], edges[1:])
    c = c0
    best_gap = math.inf
    stall = 0
    for _ in range(maxit):
        A = np.empty((n + 2, n + 2))
        A[:, : n + 1] = np.polynomial.chebyshev.chebvander(y_of_x(ref, eps), n)
        A[:, n + 1] = (-1.0) ** np.arange(n + 2) / np.sqrt(ref)
        sol = np.linalg.solve(A, 1.0 / np.sqrt(ref))
        c, E = sol[: n + 1], abs(sol[n + 1])
        zeros = _zero_in(c, eps, ref[:-1], ref[1:])
        edges = np.concatenate([[eps], zeros, [1.0]])
        ref = _peak_in(c, eps, edges[:-1], edges[1:])
        gap = np.max(np.abs(relative_error(c, eps, ref))) / E - 1.0
        if gap < 1e-10:
            break
        if gap < 0.999 * best_gap:
            best_gap, stall = gap, 0
        else:
            stall += 1
            if stall >= 3:
                break
    return c if measure_delta(c, eps) < measure_delta(c0, eps) else c0


def choose_order(eps: float, delta: float, npts: int = 400_000, n_max: int = 20000) -> int:
    """Smallest n whose optimal polynomial reaches measured delta <= target.

    The optimal delta is below the interpolant's at every n and falls with
    n, so the search starts at the interpolant's order and steps down."""
    n = interpolant_order(eps, delta, npts, n_max)
    while n > 1 and measure_delta(minimax_coefficients(eps, n - 1), eps, npts) <= delta:
        n -= 1
    return n


@dataclass
class SignApprox:
    """Descriptor of the polynomial sign: Q = H_w/lam_max, x = Q^2 in [eps,1]."""

    lam_max: float
    eps: float
    coeffs: np.ndarray  # c_0..c_n (c_0 already halved)

    @property
    def n(self) -> int:
        return len(self.coeffs) - 1


def make_sign(lam_lo: float, lam_max: float, n: int) -> SignApprox:
    """The optimal order-n polynomial for eps = (lam_lo / lam_max)^2 (eq. 4-5)."""
    eps = (lam_lo / lam_max) ** 2
    return SignApprox(lam_max=lam_max, eps=eps, coeffs=minimax_coefficients(eps, n))


# ---------------------------------------------------------------------------
# Operators
# ---------------------------------------------------------------------------
class Counter:
    """Counts applications of D_w made by the functions below."""

    def __init__(self):
        self.dw = 0


def _hw(lat, U, v, rho, counter):
    if counter is not None:
        counter.dw += 1
    return dirac.hw_apply(lat, U, v, rho)


def apply_Y(lat, U, v, rho, s: SignApprox, counter=None):
    """Y v = (2 Q^2 - 1 - eps)/(1 - eps) v with Q = H_w/lam_max."""
    q2v = _hw(lat, U, _hw(lat, U, v, rho, counter), rho, counter) / s.lam_max**2
    return (2.0 * q2v - (1.0 + s.eps) * v) / (1.0 - s.eps)


def clenshaw_p(lat, U, psi, rho, s: SignApprox, counter=None):
    """P(Q^2) psi by Clenshaw: b_k = c_k psi + 2 Y b_{k+1} - b_{k+2}, k = n..1,
    then P psi = c_0 psi + Y b_1 - b_2 (b_{n+1} = b_{n+2} = 0)."""
    c = s.coeffs
    n = s.n
    b1 = np.zeros_like(psi)  # b_{k+1}
    b2 = np.zeros_like(psi)  # b_{k+2}
    for k in range(n, 0, -1):
        if k == n:
            bk = c[k] * psi
        else:
            bk = c[k] * psi + 2.0 * apply_Y(lat, U, b1, rho, s, counter) - b2
        b2, b1 = b1, bk
    if n == 0:
        return c[0] * psi
    return c[0] * psi + apply_Y(lat, U, b1, rho, s, counter) - b2


def project_low(V: np.ndarray, psi: np.ndarray):
    """c_i = eta_i^dagger psi; returns (c, psi_h = psi - sum_i c_i eta_i)."""
    if V is None or len(V) == 0:
        return np.zeros(0, dtype=np.complex128), psi.copy()
    Vf = V.reshape(len(V), -1)
    c = Vf.conj() @ psi.reshape(-1)
    psi_h = psi - (c @ Vf).reshape(psi.shape)
    return c, psi_h


def sign_apply(lat, U, psi, rho, s: SignApprox, V=None, lam=None, counter=None):
    """sign(H_w) psi by eq. (7): exact on the low modes, Q P(Q^2) on psi_h."""
    psi = np.asarray(psi).reshape(lat.N, 4, 3)
    c, psi_h = project_low(V, psi)
    out = _hw(lat, U, clenshaw_p(lat, U, psi_h, rho, s, counter), rho, counter) / s.lam_max
    if len(c):
        low = (np.sign(lam) * c) @ V.reshape(len(V), -1)
        out = out + low.reshape(psi.shape)
    return out


def overlap_apply(lat, U, psi, rho, m, s: SignApprox, V=None, lam=None, dagger=False, counter=None):
    """D(m) psi = (rho + m/2) psi + (rho - m/2) gamma5 sign(H_w) psi   (eq. 3, 8);
    D(m)^dagger psi = (rho + m/2) psi + (rho - m/2) sign(H_w) gamma5 psi."""
    psi = np.asarray(psi).reshape(lat.N, 4, 3)
    if dagger:
        e = sign_apply(lat, U, dirac.gamma5(psi), rho, s, V, lam, counter)
    else:
        e = dirac.gamma5(sign_apply(lat, U, psi, rho, s, V, lam, counter))
    return (rho + 0.5 * m) * psi + (rho - 0.5 * m) * e


def massless_overlap(lat, U, psi, rho, s: SignApprox, V=None, lam=None):
    """D psi = psi + gamma5 sign(H_w) psi (eq. 3)."""
    psi = np.asarray(psi).reshape(lat.N, 4, 3)
    return psi + dirac.gamma5(sign_apply(lat, U, psi, rho, s, V, lam))
