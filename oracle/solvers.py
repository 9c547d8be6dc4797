"""Spectral bounds and Krylov solvers for the oracle (test infrastructure).

* lanczos_bound: the normalisation ||H_w|| of eq. (5) must be an upper bound
  on |spectrum(H_w)| or Q^2 leaves [eps,1] and the Chebyshev series
  diverges.  The paper does not say how it is obtained; here: plain FP64
  Lanczos on H_w with full reorthogonalisation; for the two extreme Ritz
  values theta (which approach the spectrum's ends from inside) the bound is
  |theta| + |beta_k s_k|, the Ritz residual norm, s_k being the last
  component of the Ritz vector.
* cgne: the paper computes propagators with CG on the overlap operator
  (Sec. II, Sec. V) without fixing the normal-equation form.  The reading
  used here is CG on A = D(m) D(m)^dagger with x = D(m)^dagger y (Craig's
  method), so the recursively updated residual is b - D(m) x; after it
  reaches tol the true residual is recomputed in FP64 and the solve restarts
  from the current x until the true residual is <= tol (defect correction).
* fgcr: flexible GCR with a right preconditioner M (restart length k), used
  with the learned preconditioner; falls back to cgne on stagnation or NaN.
"""
from __future__ import annotations

import numpy as np


def vdot(a, b) -> complex:
    return complex(np.vdot(np.asarray(a).reshape(-1), np.asarray(b).reshape(-1)))


def norm(a) -> float:
    return float(np.linalg.norm(np.asarray(a).reshape(-1)))


def lanczos_bound(apply_h, v0: np.ndarray, steps: int = 60):
    """Returns (bound, theta_min, theta_max); bound = max over the two extreme
    Ritz pairs of |theta| + ||H y - theta y||."""
    shape = v0.shape
    q = v0.reshape(-1) / norm(v0)
    Q = [q]
    alphas, betas = [], []
    beta = 0.0
    q_prev = np.zeros_like(q)
    for j in range(steps):
        w = np.asarray(apply_h(Q[-1].reshape(shape))).reshape(-1)
        a = np.vdot(Q[-1], w).real
        w = w - a * Q[-1] - beta * q_prev
        for qq in Q:  # full reorthogonalisation
            w = w - np.vdot(qq, w) * qq
        alphas.append(a)
        beta = np.linalg.norm(w)
        betas.append(beta)
        if beta < 1e-14:
            break
        q_prev = Q[-1]
        Q.append(w / beta)
    k = len(alphas)
    T = np.diag(alphas) + np.diag(betas[: k - 1], 1) + np.diag(betas[: k - 1], -1)
    theta, s = np.linalg.eigh(T)
    res = np.abs(betas[k - 1] * s[k - 1, :])  # Ritz residual norms
    bound = max(abs(theta[0]) + res[0], abs(theta[-1]) + res[-1])
    return float(bound), float(theta[0]), float(theta[-1])


def cgne(apply_d, apply_ddag, b, tol=1e-10, maxiter=10000, x0=None, inner_tol=None, history=None):
    """Solve D x = b by CG on D D^dagger; stop on FP64 true residual <= tol.

    Returns (x, stats) with stats = dict(iterations, restarts, true_residual).
    """
    b = np.asarray(b)
    bn = norm(b)
    x = np.zeros_like(b) if x0 is None else np.array(x0, copy=True)
    inner_tol = tol if inner_tol is None else inner_tol
    its = 0
    restarts = 0
    while True:
        r = b - apply_d(x)
        true_res = norm(r) / bn
        if history is not None:
            history.append(("true", its, true_res))
        if true_res <= tol or its >= maxiter:
            return x, dict(iterations=its, restarts=restarts, true_residual=true_res)
        rr = vdot(r, r).real
        p = apply_ddag(r)
        target = (inner_tol * bn) ** 2
        while its < maxiter:
            pp = vdot(p, p).real
            if not np.isfinite(pp) or pp <= 0:
                raise FloatingPointError("CG breakdown: p^dagger p = %r" % pp)
            alpha = rr / pp
            x = x + alpha * p
            r = r - alpha * apply_d(p)
            rr_new = vdot(r, r).real
            its += 1
            if history is not None:
                history.append(("iter", its, np.sqrt(rr_new) / bn))
            if rr_new <= target:
                break
            beta = rr_new / rr
            rr = rr_new
            p = apply_ddag(r) + beta * p
        restarts += 1


def fgcr(apply_a, precond, b, tol=1e-10, restart=16, maxiter=2000, x0=None,
         fallback=None, stagnation=0.9):
    """Right-preconditioned flexible GCR: z = M r, w = A z, orthogonalise w.

    If the residual falls by less than `stagnation` over one restart cycle,
    or becomes non-finite, `fallback(b, x)` finishes the solve.
    Returns (x, stats) with stats = dict(iterations, true_residual, fallback_used).
    """
    b = np.asarray(b)
    bn = norm(b)
    x = np.zeros_like(b) if x0 is None else np.array(x0, copy=True)
    its = 0
    r = b - apply_a(x)
    res = norm(r) / bn
    while its < maxiter:
        res_start = res
        Z, W = [], []
        for _ in range(restart):
            z = precond(r)
            w = apply_a(z)
            for zi, wi in zip(Z, W):
                beta = vdot(wi, w)
                w = w - beta * wi
                z = z - beta * zi
            nw = norm(w)
            if not np.isfinite(nw) or nw == 0.0:
                break
            w = w / nw
            z = z / nw
            alpha = vdot(w, r)
            x = x + alpha * z
            r = r - alpha * w
            Z.append(z)
            W.append(w)
            its += 1
            res = norm(r) / bn
            if res <= tol or its >= maxiter:
                break
        r = b - apply_a(x)  # true residual at every restart
        res = norm(r) / bn
        if res <= tol:
            return x, dict(iterations=its, true_residual=res, fallback_used=False)
        if not np.isfinite(res) or res > stagnation * res_start:
            if fallback is None:
                break
            x_start = x if np.all(np.isfinite(x)) else np.zeros_like(b)
            x2, st = fallback(b, x_start)
            return x2, dict(iterations=its + st["iterations"], true_residual=st["true_residual"],
                            fallback_used=True)
    return x, dict(iterations=its, true_residual=res, fallback_used=False)
