"""Dense-matrix references on tiny lattices (test infrastructure).

For 2^4 (192 x 192) and 4^4 (3072 x 3072) lattices the operators of
arXiv:1106.4964 Sec. II are small enough to write out as dense matrices:
H_w = gamma5 D_w(-rho) is built column by column from the oracle's apply,
and the exact matrix sign function is V sign(Lambda) V^dagger from its
eigendecomposition (the object that eq. (5) approximates).  sign(0) is
taken as +1; the synthetic fields have a spectral gap so it never occurs.

A field [N,4,3] flattens in C order: index = 12*site + 3*spin + colour.
"""
from __future__ import annotations

import numpy as np

from . import dirac
from .lattice import Lattice


def dense_operator(lat: Lattice, apply) -> np.ndarray:
    """Matrix of a linear map on [N,4,3] fields, built from unit vectors."""
    dim = 12 * lat.N
    mat = np.empty((dim, dim), dtype=np.complex128)
    e = np.zeros(dim, dtype=np.complex128)
    for j in range(dim):
        e[j] = 1.0
        mat[:, j] = np.asarray(apply(e.reshape(lat.N, 4, 3))).reshape(-1)
        e[j] = 0.0
    return mat


def dense_hw(lat: Lattice, U, rho: float) -> np.ndarray:
    return dense_operator(lat, lambda v: dirac.hw_apply(lat, U, v, rho))


def dense_gamma5(lat: Lattice) -> np.ndarray:
    return np.kron(np.eye(lat.N), np.kron(dirac.GAMMA5, np.eye(3)))


def eig_sorted_by_magnitude(H: np.ndarray):
    """Eigenpairs of a Hermitian matrix ordered by (|lambda|, lambda, index)."""
    w, v = np.linalg.eigh(H)
    order = np.lexsort((np.arange(len(w)), w, np.abs(w)))
    return w[order], v[:, order]


def exact_sign(H: np.ndarray) -> np.ndarray:
    w, v = np.linalg.eigh(H)
    s = np.where(w >= 0, 1.0, -1.0)
    return (v * s) @ v.conj().T


def lowmodes(lat: Lattice, H: np.ndarray, ell: int):
    """The ell eigenpairs of H with smallest |lambda|: (V [ell,N,4,3], lam [ell])."""
    w, v = eig_sorted_by_magnitude(H)
    V = np.ascontiguousarray(v[:, :ell].T).reshape(ell, lat.N, 4, 3)
    return V, w[:ell].copy()


def spectrum_bounds(H: np.ndarray):
    """(min |lambda|, max |lambda|) of a Hermitian matrix."""
    w = np.linalg.eigvalsh(H)
    return float(np.min(np.abs(w))), float(np.max(np.abs(w)))
