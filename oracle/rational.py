"""Rational sign function: Zolotarev coefficients, multi-shift CG, and the
single-pass and double-pass evaluations of P(Q^2) psi (oracle).

Test infrastructure.  Follows arXiv:1106.4964:

* eq. (4): P(x) approximates x^{-1/2} on [eps, 1] with quality
  delta = max |1 - sqrt(x) P(x)|; here P is the optimal rational function of
  type (n-1, n), whose coefficients are known in closed form (Zolotarev).
* eq. (5): sign(H_w) ~ Q P(Q^2), Q = H_w / ||H_w||.
* eq. (12): P(Q^2) psi = sum_i b_i (Q^2 + c_i)^{-1} psi, the shifted
  systems solved together by a multi-shift CG (single pass, 2n + 3 vectors).
* Sec. V, the double-pass variant: a first Lanczos pass on Q^2 gives the
  tridiagonal T_k and the second pass regenerates the Lanczos vectors and
  sums P(T_k) e_1 along them, so the work does not depend on n and only a
  few vectors are kept, at twice the applications of Q^2.
* eq. (6)-(7): the low modes of H_w are projected exactly as for the
  polynomial.

Readings (the paper cites these methods without restating them):
* Zolotarev's optimal approximation of x^{-1/2} on [1, b], b = 1/eps, in
  product form: d0 prod_{l<n} (x + c_{2l}) / prod_{l<=n} (x + c_{2l-1}),
  c_l = sn^2(l K'/(2n); k') / (1 - sn^2(l K'/(2n); k')), l = 1..2n-1, with
  k' = sqrt(1 - 1/b) and K' the complete elliptic integral of modulus k';
  d0 makes the relative error equioscillate: 2 / (max + min) of
  sqrt(x) prod(...) over the interval.  Rescaled to y = x / b in [eps, 1]
  and written as partial fractions sum_i b_i / (y + c_i).
* Multi-shift CG (Jegerlehner): one Krylov space of A = Q^2 (Hermitian,
  positive) serves every shifted system A + c_i; the shifted iterates follow
  from the base recurrence through the zeta_i polynomials.  The base system
  is the smallest shift (the worst conditioned); a shifted system stops
  updating once its own residual zeta_i r meets the tolerance.
* Double pass: Lanczos with the plain FP64 three-term recurrence (no
  re-orthogonalisation) until the estimated truncation error of
  y = P(T_k) e_1 - the coupling beta_k |y_k| to the next vector, summed as a
  geometric series with the observed decay of |y_k| - is below tol |y_1|,
  then the same recurrence again.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy.special import ellipj, ellipk

from . import sign as poly


@dataclass
class RationalSign:
    """P(y) = sum_i b_i / (y + c_i) on [eps, 1], y = Q^2 = (H_w / lam_max)^2."""

    lam_max: float
    eps: float
    b: np.ndarray
    c: np.ndarray

    @property
    def n(self) -> int:
        return len(self.c)


def zolotarev_product(eps: float, n: int):
    """(d0, numerator roots c_2l, denominator roots c_{2l-1}) of the optimal
    type-(n-1, n) approximation of x^{-1/2} on [1, 1/eps] (x unscaled)."""
    bb = 1.0 / eps
    mp = 1.0 - 1.0 / bb  # k'^2, the parameter scipy's elliptic functions take
    Kp = ellipk(mp)
    sn = np.array([ellipj(l * Kp / (2 * n), mp)[0] for l in range(1, 2 * n)])
    cl = sn**2 / (1.0 - sn**2)  # c_1 .. c_{2n-1}
    num = cl[1::2]  # c_2, c_4, ..., c_{2n-2}
    den = cl[0::2]  # c_1, c_3, ..., c_{2n-1}
    x = _grid(1.0, bb)
    f = np.sqrt(x) * _prod(x, num, den)
    d0 = 2.0 / (f.max() + f.min())
    return d0, num, den


def _prod(x, num, den):
    x = np.asarray(x, dtype=np.float64)
    out = np.ones_like(x)
    for r in num:
        out = out * (x + r)
    for r in den:
        out = out / (x + r)
    return out


def _grid(lo: float, hi: float, npts: int = 200_001) -> np.ndarray:
    """Points of [lo, hi], uniform in log x (the relative error of the
    approximation oscillates on a logarithmic scale)."""
    return np.exp(np.linspace(math.log(lo), math.log(hi), npts))


def make_rational(lam_lo: float, lam_max: float, n: int) -> RationalSign:
    """Partial fractions of the Zolotarev approximation for
    eps = (lam_lo / lam_max)^2, in the variable y = Q^2."""
    eps = (lam_lo / lam_max) ** 2
    d0, num, den = zolotarev_product(eps, n)
    bb = 1.0 / eps
    # residue of prod(x + num) / prod(x + den) at x = -den_l
    a = np.empty(n)
    for l in range(n):
        p = -den[l]
        a[l] = np.prod(num + p) / np.prod(np.delete(den, l) + p)
    # 1/sqrt(y) = sqrt(b) / sqrt(b y) ~ sqrt(b) d0 sum_l a_l / (b y + den_l)
    return RationalSign(lam_max=lam_max, eps=eps, b=d0 * a / math.sqrt(bb), c=den / bb)


def rational_eval(r: RationalSign, y) -> np.ndarray:
    y = np.asarray(y, dtype=np.float64)
    return sum(bi / (y + ci) for bi, ci in zip(r.b, r.c))


def measure_delta(r: RationalSign, npts: int = 200_001) -> float:
    """delta = max |1 - sqrt(y) P(y)| over [eps, 1] (eq. 4)."""
    y = _grid(r.eps, 1.0, npts)
    return float(np.max(np.abs(1.0 - np.sqrt(y) * rational_eval(r, y))))


# ---------------------------------------------------------------------------
# Krylov evaluations of P(A) psi for a Hermitian positive A (here A = Q^2)
# ---------------------------------------------------------------------------
def multishift_cg(apply_A, psi, shifts, tol: float = 1e-12, maxiter: int = 10000):
    """x_i = (A + shifts_i)^{-1} psi for every i from one CG run.

    CG runs on the base system A + s0, s0 = min(shifts); the system with
    sigma_i = shifts_i - s0 has residuals collinear to the base ones,
    r^i_k = zeta^i_k r_k, and its own step lengths alpha^i_k and directions
    p^i_k follow from the base scalars.  Returns (x [n, ...], iterations)."""
    psi = np.asarray(psi).astype(np.complex128)
    shifts = np.asarray(shifts, dtype=np.float64)
    s0 = shifts.min()
    sig = shifts - s0
    n = len(shifts)
    x = np.zeros((n,) + psi.shape, dtype=np.complex128)
    ps = np.array([psi] * n)  # shifted directions
    p = psi.copy()  # base direction
    r = psi.copy()
    rr = np.vdot(r, r).real
    bn = math.sqrt(rr)
    zeta_prev = np.ones(n)
    zeta = np.ones(n)
    alpha_prev, beta_prev = 1.0, 0.0
    active = np.ones(n, dtype=bool)
    its = 0
    while its < maxiter and active.any():
        q = apply_A(p) + s0 * p
        alpha = rr / np.vdot(p, q).real
        # converged shifts keep their zeta (their recurrence is not used)
        den = alpha * beta_prev * (zeta_prev - zeta) + zeta_prev * alpha_prev * (1.0 + sig * alpha)
        zeta_next = np.where(active, zeta * zeta_prev * alpha_prev / np.where(active, den, 1.0), zeta)
        alpha_s = alpha * zeta_next / zeta
        for i in range(n):
            if active[i]:
                x[i] += alpha_s[i] * ps[i]
        r = r - alpha * q
        rr_new = np.vdot(r, r).real
        beta = rr_new / rr
        p = r + beta * p
        beta_s = beta * (zeta_next / zeta) ** 2
        for i in range(n):
            if active[i]:
                ps[i] = zeta_next[i] * r + beta_s[i] * ps[i]
                if abs(zeta_next[i]) * math.sqrt(rr_new) <= tol * bn:
                    active[i] = False
        zeta_prev, zeta = zeta, zeta_next
        alpha_prev, beta_prev = alpha, beta
        rr = rr_new
        its += 1
    return x, its


def tridiag_rational_e1(alphas, betas, r: RationalSign) -> np.ndarray:
    """y = P(T) e_1 = sum_i b_i (T + c_i)^{-1} e_1 for the k x k tridiagonal T
    with diagonal alphas and off-diagonal betas[:k-1]."""
    k = len(alphas)
    T = np.diag(alphas) + np.diag(betas[: k - 1], 1) + np.diag(betas[: k - 1], -1)
    e1 = np.zeros(k)
    e1[0] = 1.0
    return sum(bi * np.linalg.solve(T + ci * np.eye(k), e1) for bi, ci in zip(r.b, r.c))


def _tail(beta, y):
    """Estimated size of everything the truncation at k drops: the coupling
    beta_k |y_k| to the next Lanczos vector, summed as a geometric series
    with the observed decay q = |y_k / y_{k-1}| of the coefficients."""
    q = abs(y[-1]) / max(abs(y[-2]), 1e-300)
    return beta * abs(y[-1]) / max(1.0 - q, 1e-3)


def double_pass(apply_A, psi, r: RationalSign, tol: float = 1e-12, kmax: int = 5000):
    """P(A) psi ~ ||psi|| V_k P(T_k) e_1 in two passes.  Pass 1 runs the
    Lanczos recurrence from v_1 = psi / ||psi|| and stops at the first k
    where the estimated tail (`_tail`) is below tol |(P(T_k) e_1)_1| (or the
    Krylov space is exhausted); pass 2 reruns the same recurrence to
    regenerate v_1..v_k and sums y_j v_j.  Returns (out, k)."""
    psi = np.asarray(psi).astype(np.complex128)
    nrm = np.linalg.norm(psi)
    # pass 1: T_k only
    v = psi / nrm
    v_prev = np.zeros_like(v)
    alphas, betas = [], []
    beta = 0.0
    y = None
    for _ in range(kmax):
        w = apply_A(v) - beta * v_prev
        a = np.vdot(v, w).real
        w = w - a * v
        beta = np.linalg.norm(w)
        alphas.append(a)
        betas.append(beta)
        y = tridiag_rational_e1(np.array(alphas), np.array(betas), r)
        if beta == 0.0 or (len(y) >= 2 and _tail(beta, y) <= tol * abs(y[0])):
            break
        v_prev, v = v, w / beta
    k = len(alphas)
    # pass 2: the same recurrence, accumulating y_j v_j
    v = psi / nrm
    v_prev = np.zeros_like(v)
    out = y[0] * v
    for j in range(1, k):
        w = apply_A(v) - (betas[j - 2] if j >= 2 else 0.0) * v_prev
        w = w - alphas[j - 1] * v
        v_prev, v = v, w / betas[j - 1]
        out = out + y[j] * v
    return nrm * out, k


def sign_apply_rational(lat, U, psi, rho, r: RationalSign, V=None, lam=None, method: str = "multishift",
                        tol: float = 1e-12):
    """sign(H_w) psi with the rational P (eq. 5, 7, 12): the low modes
    exactly, Q P(Q^2) on the rest by multi-shift CG or double pass."""
    psi = np.asarray(psi).reshape(lat.N, 4, 3)
    c, psi_h = poly.project_low(V, psi)

    def apply_A(v):  # Q^2 v
        return poly._hw(lat, U, poly._hw(lat, U, v, rho, None), rho, None) / r.lam_max**2

    if method == "multishift":
        xs, _ = multishift_cg(apply_A, psi_h, r.c, tol=tol)
        pq = np.tensordot(r.b, xs, axes=1)
    else:
        pq, _ = double_pass(apply_A, psi_h, r, tol=tol)
    out = poly._hw(lat, U, pq, rho, None) / r.lam_max
    if len(c):
        out = out + ((np.sign(lam) * c) @ V.reshape(len(V), -1)).reshape(psi.shape)
    return out
