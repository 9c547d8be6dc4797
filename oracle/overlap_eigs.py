"""Overlap eigenpairs from one chiral sector, and deflation of D(m) (oracle).

Test infrastructure.  Follows arXiv:1106.4964:

* Sec. V: the low eigenvectors of the overlap operator are computed as
  eigenvectors of gamma5 D in one chiral sector, whose vectors have definite
  chirality and need only half the storage (two of the four spins in the
  chiral basis).
* eq. (3): D = 1 + gamma5 eps, eps = sign(H_w) Hermitian with eps^2 = 1, so
  gamma5 D = gamma5 + eps is Hermitian and D is normal; its eigenvalues lie on
  the circle |d - 1| = 1.
* eq. (9): with the l' eigenpairs D xi_i = d_i xi_i closest to zero,
  D(m)^{-1} psi = sum_i xi_i^dag psi / (rho d_i + m (1 - d_i / 2)) xi_i
                  + D(m)^{-1} psi_h,
  psi_h = psi - sum_i (xi_i^dag psi) xi_i, and the second term is solved by CG
  at the reduced condition number ||D|| / |d_l'|.

Reading (the paper names the sector method but not the step from sector
eigenvectors to eigenvectors of D): with P_s = (1 + s gamma5)/2, the
restriction of gamma5 D to sector s is s P_s + P_s eps P_s, which has the
eigenvectors of K_s = s P_s eps P_s.  For an eigenvector v of K_s in the
sector (eigenvalue k, |k| <= 1) the vector P_{-s} eps v has norm
sn = sqrt(1 - k^2); with u = P_{-s} eps v / sn the plane span(v, u) is
invariant under D, which acts on it (columns D v, D u) as
[[1 + k, s sn], [-s sn, 1 + k]], so
    xi_+- = (v +- i u) / sqrt(2),   d_+- = 1 + k +- i s sn.
|k| = 1 gives one real eigenvalue (d = 0 for k = -1, d = 2 for k = +1) with
xi = v of definite chirality.  Small |d| means k close to -1: the wanted
modes are the lowest eigenvalues of K_s in either sector.  Each pair of D
shows up once in each sector, so one sector gives all of them except the
real modes of the other chirality.

The sector operator is passed in as `apply_eps` (a callable v -> eps v), so
the same code runs on the exact sign (dense eigendecomposition) and on the
polynomial approximation.  All arithmetic is complex128.
"""
from __future__ import annotations

import numpy as np

from . import solvers


def chiral_project(psi: np.ndarray, s: int) -> np.ndarray:
    """P_s psi, P_s = (1 + s gamma5)/2 with gamma5 = diag(1, 1, -1, -1)."""
    out = np.zeros_like(psi)
    if s > 0:
        out[..., 0:2, :] = psi[..., 0:2, :]
    else:
        out[..., 2:4, :] = psi[..., 2:4, :]
    return out


def sector_matrix(apply_eps, N: int, s: int) -> np.ndarray:
    """Dense matrix of K_s = s P_s eps P_s on the 6N-dimensional sector s
    (columns are the sector's unit vectors: site, the two spins of
    chirality s, colour, in that order)."""
    spins = (0, 1) if s > 0 else (2, 3)
    dim = 6 * N
    M = np.empty((dim, dim), dtype=np.complex128)
    e = np.zeros((N, 4, 3), dtype=np.complex128)
    for j in range(dim):
        site, rest = divmod(j, 6)
        sp, col = divmod(rest, 3)
        e[site, spins[sp], col] = 1.0
        y = apply_eps(e)
        M[:, j] = s * y[:, spins, :].reshape(-1)
        e[site, spins[sp], col] = 0.0
    return M


def sector_lowest(apply_eps, N: int, s: int, count: int):
    """The `count` lowest eigenpairs (k, v) of K_s, v as [count, N, 4, 3]."""
    M = sector_matrix(apply_eps, N, s)
    M = 0.5 * (M + M.conj().T)
    w, X = np.linalg.eigh(M)
    spins = (0, 1) if s > 0 else (2, 3)
    V = np.zeros((count, N, 4, 3), dtype=np.complex128)
    for k in range(count):
        V[k][:, spins, :] = X[:, k].reshape(N, 2, 3)
    return w[:count].copy(), V


def sector_lowest_dense(E: np.ndarray, N: int, s: int, count: int):
    """sector_lowest for a dense eps (matrix E on [N, 4, 3] fields flattened in
    C order): K_s is s times the submatrix of E on the sector's components."""
    spins = (0, 1) if s > 0 else (2, 3)
    idx = np.array([12 * site + 3 * sp + c for site in range(N) for sp in spins for c in range(3)])
    M = s * E[np.ix_(idx, idx)]
    w, X = np.linalg.eigh(0.5 * (M + M.conj().T))
    V = np.zeros((count, N * 12), dtype=np.complex128)
    V[:, idx] = X[:, :count].T
    return w[:count].copy(), V.reshape(count, N, 4, 3)


def overlap_pairs(apply_eps, k: np.ndarray, V: np.ndarray, s: int, real_tol: float = 1e-9):
    """Eigenpairs (d, xi) of D = 1 + gamma5 eps from sector eigenpairs (k, v)
    of K_s.  Returns (d [n], Xi [n, N, 4, 3]) ordered by (|d|, arg d); a
    sector eigenpair gives two eigenpairs of D, a real mode (|k| = 1 to
    real_tol) one."""
    ds, xis = [], []
    for ki, v in zip(k, V):
        ki = float(np.clip(ki, -1.0, 1.0))
        # sn = ||P_{-s} eps v|| = sqrt(1 - k^2), taken from the vector itself:
        # the square root of 1 - k^2 loses digits when d is nearly real
        w = chiral_project(apply_eps(v), -s)
        sn = float(np.linalg.norm(w.reshape(-1)))
        if sn <= real_tol:
            ds.append(complex(1.0 + ki, 0.0))
            xis.append(v)
            continue
        u = w / sn
        for sg in (+1, -1):
            ds.append(complex(1.0 + ki, sg * s * sn))
            xis.append((v + sg * 1j * u) / np.sqrt(2.0))
    ds = np.array(ds)
    order = np.lexsort((np.angle(ds), np.abs(ds)))
    return ds[order], np.stack(xis)[order]


def mass_eigenvalue(d, rho: float, m: float):
    """Eigenvalue of D(m) = rho D + m (1 - D/2) on an eigenvector of D (eq. 8)."""
    return rho * d + m * (1.0 - 0.5 * d)


def deflated_solve(apply_d, apply_ddag, b, d, Xi, rho: float, m: float, tol: float = 1e-10, maxiter: int = 10000,
                   max_cycles: int = 20):
    """eq. (9) inside an FP64 defect-correction loop.  Each cycle takes the
    true residual r = b - D(m) x, adds the low part
    sum_i xi_i (xi_i^dag r) / (rho d_i + m (1 - d_i/2)) to x, and solves
    D(m) e = r_h (r minus its components along the xi_i) by CGNE for the
    high part; the cycle repeats because the xi_i are eigenvectors only to
    their own accuracy.  Returns (x, stats)."""
    b = np.asarray(b)
    bn = np.linalg.norm(b)
    Xf = Xi.reshape(len(Xi), -1)
    lam = mass_eigenvalue(d, rho, m)
    x = np.zeros_like(b)
    its = 0
    for cycle in range(max_cycles + 1):
        r = b - apply_d(x)
        res = np.linalg.norm(r) / bn
        if res <= tol or cycle == max_cycles or its >= maxiter:
            return x, dict(iterations=its, true_residual=res, cycles=cycle)
        coef = Xf.conj() @ r.reshape(-1)
        x = x + ((coef / lam) @ Xf).reshape(b.shape)
        r_h = r - (coef @ Xf).reshape(b.shape)
        rn = np.linalg.norm(r_h)
        e, st = solvers.cgne(apply_d, apply_ddag, r_h, tol=0.5 * tol * bn / max(rn, 1e-300), maxiter=maxiter - its)
        its += st["iterations"]
        x = x + e
