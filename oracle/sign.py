"""Polynomial sign function, low-mode projection and the overlap operator.

Oracle (test infrastructure).  Follows arXiv:1106.4964:

* eq. (4): P(x) approximates x^{-1/2} on [eps, 1]; its quality is
  delta = max_{x in [eps,1]} |1 - sqrt(x) P(x)|.
* eq. (5): sign(H_w) ~ Q P(Q^2) with Q = H_w / ||H_w||.
* Sec. V: P is expanded in Chebyshev polynomials and P(Q^2) psi is evaluated
  by a Clenshaw recursion (five vectors).
* eq. (11): the empirical order law delta = A exp(-b n sqrt(eps)) with
  A = 0.41, b = 2.1, used here only as the starting guess for n.
* eq. (6)-(7): with the l eigenpairs (lambda_i, eta_i) of H_w closest to
  zero, psi = psi_l + psi_h, psi_l = sum_i (eta_i^dagger psi) eta_i, and
  sign(H_w) psi = sum_i sign(lambda_i) (eta_i^dagger psi) eta_i + Q P(Q^2) psi_h.
* eq. (3): D = 1 + gamma5 sign(H_w);  eq. (8): D(m) = rho D + m (1 - D/2).

Readings:
* The paper cites a "robust numerical method" for the coefficients without
  describing it.  Here P is the Chebyshev interpolant of x^{-1/2} at the n+1
  Chebyshev-Gauss nodes of the variable y = (2x - 1 - eps)/(1 - eps); c_0
  carries the usual factor 1/2.  n is the order of P in x = Q^2, so one sign
  apply costs 2n+1 applications of D_w.
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


def choose_order(eps: float, delta: float, npts: int = 400_000, n_max: int = 20000) -> int:
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
    eps = (lam_lo / lam_max) ** 2
    return SignApprox(lam_max=lam_max, eps=eps, coeffs=chebyshev_coefficients(eps, n))


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
