"""Wilson-Dirac operator and H_w for the oracle (test infrastructure).

Follows Sec. II of arXiv:1106.4964:
  eq. (1)  D_w(m;U) = (m + 4) 1 - 1/2 sum_{mu=+-1..+-4} T_mu(U)        (a = 1)
  eq. (2)  (T_{+mu} psi)_n = U_mu(n) (1 - gamma_mu) psi_{n+mu}
           (T_{-mu} psi)_n = U_mu(n-mu)^dagger (1 + gamma_mu) psi_{n-mu}
  gamma5-hermiticity  D_w^dagger = gamma5 D_w gamma5, so H_w = gamma5 D_w is
  Hermitian.

Readings (the paper is silent or ambiguous):
* The paper writes the spin projector to the right of a 4x3 "matrix"
  psi; here it acts from the left on the spin index (equivalent
  representation, every invariant unchanged).
* Chiral gamma basis (the paper states its basis is chiral, Sec. V):
  gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] (k = 1,2,3),
  gamma_4 = [[0, 1], [1, 0]],  gamma5 = gamma1 gamma2 gamma3 gamma4
          = diag(1, 1, -1, -1).
* H_w is built from D_w at mass -rho (rho = 1.5), the kernel of D(m) in
  eq. (8); boundaries are periodic in all directions.

Fields are complex128 in the canonical lexicographic layout
psi[N][4 spin][3 colour], U[N][4 mu][3][3]; internally they are viewed as
[Lt,Lz,Ly,Lx,...] arrays so the hop in direction mu is a roll of axis 3-mu.
"""
from __future__ import annotations

import numpy as np

from .lattice import Lattice

SIGMA = np.array(
    [[[0, 1], [1, 0]], [[0, -1j], [1j, 0]], [[1, 0], [0, -1]]], dtype=np.complex128
)


def gamma_matrices() -> np.ndarray:
    """gamma_1..gamma_4 of the chiral basis, shape [4,4,4] (index mu = 0..3)."""
    g = np.zeros((4, 4, 4), dtype=np.complex128)
    for k in range(3):
        g[k][0:2, 2:4] = -1j * SIGMA[k]
        g[k][2:4, 0:2] = 1j * SIGMA[k]
    g[3][0:2, 2:4] = np.eye(2)
    g[3][2:4, 0:2] = np.eye(2)
    return g


GAMMA = gamma_matrices()
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
ID4 = np.eye(4, dtype=np.complex128)


def _axis(mu: int) -> int:
    # array axes are (t, z, y, x, ...): direction mu=0 (x) is axis 3
    return 3 - mu


def _as_lattice(lat: Lattice, psi: np.ndarray, U: np.ndarray):
    p = np.asarray(psi).reshape(lat.shape + (4, 3))
    u = np.asarray(U).reshape(lat.shape + (4, 3, 3))
    return p, u


def spin_mul(gamma: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """(gamma psi)[..., s, a] = sum_t gamma[s, t] psi[..., t, a]."""
    return np.matmul(gamma, psi)


def colour_mul(u: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """(U psi)[..., s, a] = sum_b U[..., a, b] psi[..., s, b]."""
    return np.matmul(psi, np.swapaxes(u, -1, -2))


def colour_mul_dag(u: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """(U^dagger psi)[..., s, a] = sum_b conj(U[..., b, a]) psi[..., s, b]."""
    return np.matmul(psi, u.conj())


def transport(lat: Lattice, U: np.ndarray, psi: np.ndarray, d: int) -> np.ndarray:
    """Parallel transport without spin projector, in direction d (0..7).

    d < 4  (+mu):  (T psi)(n) = U_mu(n) psi(n + mu)
    d >= 4 (-mu):  (T psi)(n) = U_mu(n - mu)^dagger psi(n - mu)
    Returns a lexicographic [N,4,3] field.
    """
    p, u = _as_lattice(lat, psi, U)
    mu = d % 4
    ax = _axis(mu)
    if d < 4:
        out = colour_mul(u[..., mu, :, :], np.roll(p, -1, axis=ax))
    else:
        out = colour_mul_dag(np.roll(u[..., mu, :, :], 1, axis=ax), np.roll(p, 1, axis=ax))
    return out.reshape(lat.N, 4, 3)


def hopping(lat: Lattice, U: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """sum over the 8 directions of T_mu psi (eq. 2), spin projectors included."""
    out = np.zeros((lat.N, 4, 3), dtype=np.complex128)
    for mu in range(4):
        out += spin_mul(ID4 - GAMMA[mu], transport(lat, U, psi, mu))
        out += spin_mul(ID4 + GAMMA[mu], transport(lat, U, psi, mu + 4))
    return out


def wilson_dslash(lat: Lattice, U: np.ndarray, psi: np.ndarray, m: float) -> np.ndarray:
    """D_w(m) psi on the whole lattice (eq. 1)."""
    psi = np.asarray(psi).reshape(lat.N, 4, 3)
    return (m + 4.0) * psi - 0.5 * hopping(lat, U, psi)


def wilson_dslash_parity(lat: Lattice, U, psi, m: float, parity: int) -> np.ndarray:
    """The sites of one parity (0 even, 1 odd) of D_w(m) psi; other sites zero."""
    full = wilson_dslash(lat, U, psi, m)
    mask = np.array([lat.parity(*lat.coords(i)) == parity for i in range(lat.N)])
    full[~mask] = 0
    return full


def gamma5(psi: np.ndarray) -> np.ndarray:
    return spin_mul(GAMMA5, np.asarray(psi))


def hw_apply(lat: Lattice, U: np.ndarray, psi: np.ndarray, rho: float) -> np.ndarray:
    """H_w psi = gamma5 D_w(-rho) psi."""
    return gamma5(wilson_dslash(lat, U, psi, -rho))


def gauge_rotate(lat: Lattice, U: np.ndarray, g: np.ndarray) -> np.ndarray:
    """U_mu(n) -> g(n) U_mu(n) g(n+mu)^dagger (test helper for covariance)."""
    u = np.asarray(U).reshape(lat.shape + (4, 3, 3))
    gg = np.asarray(g).reshape(lat.shape + (3, 3))
    out = np.empty_like(u)
    for mu in range(4):
        g_fwd = np.roll(gg, -1, axis=_axis(mu))
        out[..., mu, :, :] = gg @ u[..., mu, :, :] @ np.swapaxes(g_fwd.conj(), -1, -2)
    return out.reshape(lat.N, 4, 3, 3)


def colour_rotate(lat: Lattice, psi: np.ndarray, g: np.ndarray) -> np.ndarray:
    """psi(n) -> g(n) psi(n) on the colour index."""
    return colour_mul(np.asarray(g).reshape(lat.N, 3, 3), np.asarray(psi).reshape(lat.N, 4, 3))
