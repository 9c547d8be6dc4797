"""Pins for the oracle's Lanczos bound, CG (CGNE) and FGCR."""
import numpy as np
import pytest

import synth_inputs as si
from oracle import dense, dirac, ptc, sign, solvers
from oracle.lattice import Lattice


@pytest.fixture(scope="module")
def setup():
    lat = Lattice((2, 2, 2, 2))
    U = si.gauge_field(lat.dims, 0.3, seed=2)
    H = dense.dense_hw(lat, U, 1.5)
    lo, hi = dense.spectrum_bounds(H)
    s = sign.make_sign(lo, hi, 60)
    return lat, U, H, lo, hi, s


def test_lanczos_bound_is_upper_bound(setup):
    lat, U, H, lo, hi, s = setup
    v0 = si.gaussian_spinor(lat.dims, 1)
    bound, tmin, tmax = solvers.lanczos_bound(lambda v: dirac.hw_apply(lat, U, v, 1.5), v0, 40)
    assert bound >= hi
    assert bound <= 1.1 * hi


def test_lanczos_bound_4444():
    lat = Lattice((4, 4, 4, 4))
    U = si.gauge_field(lat.dims, 0.25, seed=3)
    v0 = si.gaussian_spinor(lat.dims, 2)
    bound, _, _ = solvers.lanczos_bound(lambda v: dirac.hw_apply(lat, U, v, 1.5), v0, 60)
    # free-field value 6.5 is the scale; the bound must sit just above max|lambda|
    H = dense.dense_hw(Lattice((2, 2, 2, 2)), si.unit_gauge_field((2, 2, 2, 2)), 1.5)
    assert 6.0 < bound < 7.5


@pytest.mark.parametrize("m", [0.01, 0.05])
def test_cgne_matches_dense_lu(setup, m):
    lat, U, H, lo, hi, s = setup
    rho = 1.5
    Dm = lambda v: sign.overlap_apply(lat, U, v, rho, m, s)  # noqa: E731
    Dmd = lambda v: sign.overlap_apply(lat, U, v, rho, m, s, dagger=True)  # noqa: E731
    b = si.point_source(lat.dims, 1, 2)
    x, st = solvers.cgne(Dm, Dmd, b, tol=1e-10)
    assert st["true_residual"] <= 1e-10
    assert np.linalg.norm(b - Dm(x)) / np.linalg.norm(b) <= 1e-10
    # dense matrix of the same (polynomial) operator, solved by LU
    M = dense.dense_operator(lat, Dm)
    xd = np.linalg.solve(M, b.reshape(-1))
    kappa = np.linalg.cond(M)
    assert np.linalg.norm(x.reshape(-1) - xd) <= 2 * kappa * 1e-10 * np.linalg.norm(xd)


def test_cgne_maxiter_reports_unconverged(setup):
    lat, U, H, lo, hi, s = setup
    Dm = lambda v: sign.overlap_apply(lat, U, v, 1.5, 0.01, s)  # noqa: E731
    Dmd = lambda v: sign.overlap_apply(lat, U, v, 1.5, 0.01, s, dagger=True)  # noqa: E731
    b = si.gaussian_spinor(lat.dims, 4)
    x, st = solvers.cgne(Dm, Dmd, b, tol=1e-10, maxiter=3)
    assert st["iterations"] == 3 and st["true_residual"] > 1e-10


def test_cgne_resume_from_partial_solution(setup):
    lat, U, H, lo, hi, s = setup
    Dm = lambda v: sign.overlap_apply(lat, U, v, 1.5, 0.05, s)  # noqa: E731
    Dmd = lambda v: sign.overlap_apply(lat, U, v, 1.5, 0.05, s, dagger=True)  # noqa: E731
    b = si.gaussian_spinor(lat.dims, 5)
    x1, _ = solvers.cgne(Dm, Dmd, b, tol=1e-10, maxiter=20)
    x2, st = solvers.cgne(Dm, Dmd, b, tol=1e-10, x0=x1)
    assert st["true_residual"] <= 1e-10


def test_fgcr_identity_and_exact_preconditioner(setup):
    lat, U, H, lo, hi, s = setup
    Dm = lambda v: sign.overlap_apply(lat, U, v, 1.5, 0.01, s)  # noqa: E731
    b = si.gaussian_spinor(lat.dims, 6)
    # M = 1 and no restart within the 192-dimensional space: plain (full) GCR
    x, st = solvers.fgcr(Dm, lambda r: r, b, tol=1e-10, restart=192, maxiter=500)
    assert st["true_residual"] <= 1e-10 and not st["fallback_used"]
    Minv = np.linalg.inv(dense.dense_operator(lat, Dm))
    exact = lambda r: (Minv @ r.reshape(-1)).reshape(r.shape)  # noqa: E731
    x, st = solvers.fgcr(Dm, exact, b, tol=1e-10)
    assert st["iterations"] <= 2 and st["true_residual"] <= 1e-10


def test_fgcr_nan_preconditioner_falls_back(setup):
    lat, U, H, lo, hi, s = setup
    Dm = lambda v: sign.overlap_apply(lat, U, v, 1.5, 0.01, s)  # noqa: E731
    Dmd = lambda v: sign.overlap_apply(lat, U, v, 1.5, 0.01, s, dagger=True)  # noqa: E731
    b = si.gaussian_spinor(lat.dims, 7)
    bad = lambda r: np.full_like(r, np.nan)  # noqa: E731
    fb = lambda bb, x0: solvers.cgne(Dm, Dmd, bb, tol=1e-10, x0=x0)  # noqa: E731
    x, st = solvers.fgcr(Dm, bad, b, tol=1e-10, fallback=fb)
    assert st["fallback_used"] and st["true_residual"] <= 1e-10
