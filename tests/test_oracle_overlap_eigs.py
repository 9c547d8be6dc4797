"""Pins for the oracle's overlap eigenpairs (one chiral sector, Sec. V) and
the deflated solve of eq. (9), against dense eigendecompositions, the
free-field closed form and dense LU solves."""
import math

import numpy as np
import pytest

import synth_inputs as si
from oracle import dense, dirac, overlap_eigs as oe, sign, solvers
from oracle.lattice import Lattice

RHO = 1.5


def _dense_setup(dims, U):
    lat = Lattice(dims)
    H = dense.dense_hw(lat, U, RHO)
    E = dense.exact_sign(H)
    G5 = dense.dense_gamma5(lat)
    D = np.eye(H.shape[0]) + G5 @ E
    apply_eps = lambda v: (E @ v.reshape(-1)).reshape(v.shape)  # noqa: E731
    return lat, H, E, D, apply_eps


@pytest.fixture(scope="module")
def small():
    dims = (2, 2, 2, 2)
    return _dense_setup(dims, si.gauge_field(dims, 0.3, seed=1))


def _all_pairs(lat, apply_eps):
    """Every eigenpair of D: all of sector +1 and the real modes of sector -1."""
    kp, Vp = oe.sector_lowest(apply_eps, lat.N, +1, 6 * lat.N)
    dp, Xp = oe.overlap_pairs(apply_eps, kp, Vp, +1)
    km, Vm = oe.sector_lowest(apply_eps, lat.N, -1, 6 * lat.N)
    real = np.abs(np.abs(km) - 1.0) < 1e-9
    dm, Xm = oe.overlap_pairs(apply_eps, km[real], Vm[real], -1) if real.any() else (np.zeros(0), None)
    d = np.concatenate([dp, dm])
    X = np.concatenate([Xp, Xm]) if Xm is not None else Xp
    return d, X


def _sorted(d):
    return d[np.lexsort((np.round(d.imag, 9), np.round(d.real, 9)))]


def test_sector_eigenpairs_are_eigenpairs_of_d(small):
    lat, H, E, D, apply_eps = small
    d, X = _all_pairs(lat, apply_eps)
    assert len(d) == D.shape[0]
    # the spectrum matches a general eigensolver on the dense D
    ref = np.linalg.eigvals(D)
    assert np.max(np.abs(_sorted(d) - _sorted(ref))) < 1e-10
    # each vector is an eigenvector, the set is orthonormal, d is on the GW
    # circle.  u = P eps v / sqrt(1 - k^2) divides by |Im d|, and nearly real
    # pairs come from nearly degenerate k, so they are checked at 1e-9 and the
    # others (|Im d| >= 0.05, the modes deflation uses) at rounding level.
    Xf = X.reshape(len(X), -1)
    tight = np.abs(d.imag) >= 0.05
    for di, xi, ti in zip(d, Xf, tight):
        assert np.linalg.norm(D @ xi - di * xi) < (1e-12 if ti else 1e-9)
    G = Xf.conj() @ Xf.T - np.eye(len(d))
    assert np.max(np.abs(G)) < 1e-9
    assert np.max(np.abs(G[np.ix_(tight, tight)])) < 1e-12
    assert np.max(np.abs(np.abs(d - 1.0) - 1.0)) < 1e-12


def test_one_sector_gives_the_lowest_pairs_ordered(small):
    lat, H, E, D, apply_eps = small
    k, V = oe.sector_lowest(apply_eps, lat.N, +1, 8)
    d, X = oe.overlap_pairs(apply_eps, k, V, +1)
    # the lowest sector eigenvalues give the smallest |d| of the whole spectrum
    # (apart from real modes of the other chirality, checked for absence)
    ref = np.sort(np.abs(np.linalg.eigvals(D)))
    assert np.all(np.diff(np.abs(d)) >= -1e-12)
    km, _ = oe.sector_lowest(apply_eps, lat.N, -1, 6 * lat.N)
    assert not np.any(np.abs(km + 1.0) < 1e-9)  # no zero modes of chirality -1
    assert np.max(np.abs(np.abs(d) - ref[: len(d)])) < 1e-10


@pytest.mark.parametrize("sct", [1, -1])
def test_dense_slice_equals_sector_operator(small, sct):
    lat, H, E, D, apply_eps = small
    k1, V1 = oe.sector_lowest(apply_eps, lat.N, sct, 10)
    k2, V2 = oe.sector_lowest_dense(E, lat.N, sct, 10)
    assert np.max(np.abs(k1 - k2)) < 1e-13
    # same invariant subspaces: projector difference
    P1 = V1.reshape(10, -1).T @ V1.reshape(10, -1).conj()
    P2 = V2.reshape(10, -1).T @ V2.reshape(10, -1).conj()
    assert np.max(np.abs(P1 - P2)) < 1e-10


def test_free_field_closed_form():
    """U = 1: D(p) = 1 + (M(p) + i gamma.sin p)/omega(p) has the eigenvalues
    1 + (M +- i |sin p|)/omega, each twice per colour (eq. 3 at U = 1)."""
    dims = (4, 2, 2, 2)
    lat, H, E, D, apply_eps = _dense_setup(dims, si.unit_gauge_field(dims))
    d, X = _all_pairs(lat, apply_eps)
    want = []
    for k in np.ndindex(*dims):
        p = [2 * math.pi * k[mu] / dims[mu] for mu in range(4)]
        M = -RHO + sum(1 - math.cos(q) for q in p)
        sn = math.sqrt(sum(math.sin(q) ** 2 for q in p))
        om = math.sqrt(M * M + sn * sn)
        for sg in (+1, -1):
            want += [1 + (M + sg * 1j * sn) / om] * 6
    assert np.max(np.abs(_sorted(d) - _sorted(np.array(want)))) < 1e-10


@pytest.mark.parametrize("m", [0.01, 0.05])
def test_eq9_full_basis_equals_dense_solve(small, m):
    """eq. (9) with every eigenpair: sum_i xi_i (xi_i^dag b) / (rho d_i + m (1 - d_i/2))
    is D(m)^{-1} b, D(m) = rho D + m (1 - D/2) solved by LU."""
    lat, H, E, D, apply_eps = small
    d, X = _all_pairs(lat, apply_eps)
    Dm = RHO * D + m * (np.eye(D.shape[0]) - 0.5 * D)
    b = si.gaussian_spinor(lat.dims, 11).reshape(-1)
    Xf = X.reshape(len(X), -1)
    x = ((Xf.conj() @ b) / oe.mass_eigenvalue(d, RHO, m)) @ Xf
    want = np.linalg.solve(Dm, b)
    assert np.linalg.norm(x - want) < 1e-11 * np.linalg.norm(want)


def test_deflated_cg_converges_in_fewer_iterations():
    """eq. (9) with the 16 smallest pairs on a 4x4x2x2 field (eigenvectors of
    the exact sign, the operator with the polynomial sign, so the pairs are
    approximate): the deflated defect-correction solve reaches the same FP64
    true residual 1e-10 with fewer CG iterations than plain CGNE."""
    dims = (4, 4, 2, 2)
    U = si.gauge_field(dims, 0.3, seed=3)
    lat, H, E, D, apply_eps = _dense_setup(dims, U)
    lo, hi = dense.spectrum_bounds(H)
    s = sign.make_sign(lo, hi * 1.0001, 150)
    m = 0.01
    Dm = lambda v: sign.overlap_apply(lat, U, v, RHO, m, s)  # noqa: E731
    Dmd = lambda v: sign.overlap_apply(lat, U, v, RHO, m, s, dagger=True)  # noqa: E731
    k, V = oe.sector_lowest(apply_eps, lat.N, +1, 8)
    d, X = oe.overlap_pairs(apply_eps, k, V, +1)
    b = si.point_source(dims, 0, 0)
    x0, st0 = solvers.cgne(Dm, Dmd, b, tol=1e-10)
    x1, st1 = oe.deflated_solve(Dm, Dmd, b, d, X, RHO, m, tol=1e-10)
    assert st0["true_residual"] <= 1e-10 and st1["true_residual"] <= 1e-10
    assert np.linalg.norm(x1 - x0) <= 1e-8 * np.linalg.norm(x0)
    assert st1["iterations"] < 0.8 * st0["iterations"], (st0, st1)
