"""Seeded synthetic inputs shared by the CPU oracle and the GPU library.

This module only draws random numbers and shapes them into lattice fields.
It contains none of the overlap method's arithmetic (no Dirac operator, no
sign function, no solver), so the oracle and the GPU path can both take
their inputs from here without sharing any of the code they check.

Canonical host layouts (complex128, sites in lexicographic order with x
fastest: lex = x + Lx*(y + Ly*(z + Lz*t))):
  gauge field   [N][4 mu][3][3]   U_mu(x) lives on the link x -> x+mu
  spinor field  [N][4 spin][3 colour]

The link distribution follows the synthetic recipe of near-unit SU(3)
fields: U = exp(i*c*H) with H a traceless Hermitian 3x3 matrix
H = sum_a h_a * lambda_a / sqrt(2), h_a ~ N(0,1) and lambda_a the eight
Gell-Mann matrices.  The exponential is taken through the eigendecomposition
of H, so U is unitary with det U = 1 to rounding.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "volume",
    "gell_mann",
    "gauge_field",
    "unit_gauge_field",
    "gauge_transform",
    "gaussian_spinor",
    "point_source",
    "point_sources",
    "orthonormal_spinors",
]


def volume(dims) -> int:
    lx, ly, lz, lt = (int(d) for d in dims)
    return lx * ly * lz * lt


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape [8,3,3], complex128."""
    g = np.zeros((8, 3, 3), dtype=np.complex128)
    g[0][0, 1] = g[0][1, 0] = 1
    g[1][0, 1] = -1j
    g[1][1, 0] = 1j
    g[2][0, 0] = 1
    g[2][1, 1] = -1
    g[3][0, 2] = g[3][2, 0] = 1
    g[4][0, 2] = -1j
    g[4][2, 0] = 1j
    g[5][1, 2] = g[5][2, 1] = 1
    g[6][1, 2] = -1j
    g[6][2, 1] = 1j
    g[7][0, 0] = g[7][1, 1] = 1 / np.sqrt(3)
    g[7][2, 2] = -2 / np.sqrt(3)
    return g


def _expi_hermitian(h: np.ndarray, c: float) -> np.ndarray:
    """exp(i*c*H) for a batch of Hermitian 3x3 matrices via eigh."""
    w, v = np.linalg.eigh(h)
    phase = np.exp(1j * c * w)
    return np.einsum("...ik,...k,...jk->...ij", v, phase, v.conj(), optimize=True)


def _random_su3(rng: np.random.Generator, count: int, c: float) -> np.ndarray:
    coef = rng.standard_normal((count, 8))
    h = np.tensordot(coef, gell_mann(), axes=(1, 0)) / np.sqrt(2.0)
    return _expi_hermitian(h, c)


def gauge_field(dims, c: float, seed: int) -> np.ndarray:
    """Near-unit SU(3) links U = exp(i c H), shape [N,4,3,3] complex128."""
    n = volume(dims)
    rng = np.random.default_rng(seed)
    u = _random_su3(rng, n * 4, c)
    return np.ascontiguousarray(u.reshape(n, 4, 3, 3))


def unit_gauge_field(dims) -> np.ndarray:
    """Free field: every link is the 3x3 identity."""
    n = volume(dims)
    u = np.zeros((n, 4, 3, 3), dtype=np.complex128)
    u[:, :, 0, 0] = u[:, :, 1, 1] = u[:, :, 2, 2] = 1
    return u


def gauge_transform(dims, seed: int, c: float = 2.0) -> np.ndarray:
    """One random SU(3) matrix per site, shape [N,3,3] (far from unity)."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(_random_su3(rng, volume(dims), c))


def gaussian_spinor(dims, seed: int) -> np.ndarray:
    """Every real component N(0,1); shape [N,4,3] complex128."""
    n = volume(dims)
    rng = np.random.default_rng(seed)
    r = rng.standard_normal((n, 4, 3, 2))
    return np.ascontiguousarray(r[..., 0] + 1j * r[..., 1])


def point_source(dims, spin: int, colour: int, site=(0, 0, 0, 0)) -> np.ndarray:
    """Unit source delta_{x,site} delta_{alpha,spin} delta_{a,colour}."""
    lx, ly, lz, _ = (int(d) for d in dims)
    x, y, z, t = site
    lex = x + lx * (y + ly * (z + lz * t))
    b = np.zeros((volume(dims), 4, 3), dtype=np.complex128)
    b[lex, spin, colour] = 1.0
    return b


def point_sources(dims, site=(0, 0, 0, 0)) -> np.ndarray:
    """The 12 spin x colour point sources, shape [12,N,4,3]; index = 3*spin+colour."""
    return np.stack([point_source(dims, s, c, site) for s in range(4) for c in range(3)])


def orthonormal_spinors(dims, count: int, seed: int) -> np.ndarray:
    """`count` random orthonormal spinor fields, shape [count,N,4,3] (QR of Gaussians)."""
    n = volume(dims)
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n * 12, count)) + 1j * rng.standard_normal((n * 12, count))
    q, _ = np.linalg.qr(g)
    return np.ascontiguousarray(q.T.reshape(count, n, 4, 3))
