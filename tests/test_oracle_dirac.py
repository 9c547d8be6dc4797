"""Pins for the oracle's gamma algebra and Wilson operator (Sec. II, eq. 1-2)."""
import itertools

import numpy as np
import pytest

import synth_inputs as si
from oracle import dirac
from oracle.lattice import Lattice

G = dirac.GAMMA
G5 = dirac.GAMMA5


def test_clifford_and_hermiticity():
    for mu, nu in itertools.product(range(4), range(4)):
        anti = G[mu] @ G[nu] + G[nu] @ G[mu]
        assert np.array_equal(anti, 2.0 * (mu == nu) * np.eye(4))
    for mu in range(4):
        assert np.array_equal(G[mu], G[mu].conj().T)
        vals = set(np.round(G[mu].ravel(), 12).tolist())
        assert vals <= {0, 1, -1, 1j, -1j}


def test_gamma5_is_chiral_diag():
    assert np.array_equal(G5, np.diag([1, 1, -1, -1]).astype(complex))
    for mu in range(4):
        assert np.array_equal(G5 @ G[mu], -G[mu] @ G5)


def _plane_wave(lat, k, u):
    p = [2 * np.pi * k[mu] / lat.dims[mu] for mu in range(4)]
    phase = np.empty(lat.N, dtype=complex)
    for lex in range(lat.N):
        c = lat.coords(lex)
        phase[lex] = np.exp(1j * sum(p[mu] * c[mu] for mu in range(4)))
    return p, phase[:, None, None] * u[None, :, :]


@pytest.mark.parametrize("m", [-1.5, 0.0, 0.1])
@pytest.mark.parametrize("k", [(0, 0, 0, 0), (1, 0, 0, 0), (0, 1, 2, 0), (1, 1, 1, 3), (2, 3, 1, 1)])
def test_free_field_momentum_closed_form(m, k):
    """U = 1: D_w(e^{ipx} u) = [m + sum(1-cos p) + i sum gamma_mu sin p_mu] e^{ipx} u."""
    lat = Lattice((4, 6, 4, 8))
    U = si.unit_gauge_field(lat.dims)
    rng = np.random.default_rng(7)
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    p, psi = _plane_wave(lat, k, u)
    got = dirac.wilson_dslash(lat, U, psi, m)
    Mp = (m + sum(1 - np.cos(q) for q in p)) * np.eye(4) + 1j * sum(G[mu] * np.sin(p[mu]) for mu in range(4))
    want = np.matmul(Mp, psi)
    assert np.max(np.abs(got - want)) < 1e-14 * 10


def test_free_hw_spectrum_bounds():
    """Free H_w(-1.5) has |lambda| = sqrt(M(p)^2 + sum sin^2 p) in [0.5, 6.5]."""
    from oracle import dense
    lat = Lattice((2, 2, 2, 2))
    H = dense.dense_hw(lat, si.unit_gauge_field(lat.dims), 1.5)
    lo, hi = dense.spectrum_bounds(H)
    assert abs(lo - 0.5) < 1e-13 and abs(hi - 6.5) < 1e-13


def test_gamma5_hermiticity():
    lat = Lattice((4, 4, 2, 6))
    U = si.gauge_field(lat.dims, 0.3, seed=3)
    phi = si.gaussian_spinor(lat.dims, 11)
    psi = si.gaussian_spinor(lat.dims, 12)
    lhs = np.vdot(phi, dirac.hw_apply(lat, U, psi, 1.5))
    rhs = np.vdot(dirac.hw_apply(lat, U, phi, 1.5), psi)
    assert abs(lhs - rhs) <= 1e-14 * abs(lhs) * 10


def test_dense_hw_exactly_hermitian_2444():
    from oracle import dense
    lat = Lattice((2, 2, 2, 2))
    H = dense.dense_hw(lat, si.gauge_field(lat.dims, 0.3, seed=1), 1.5)
    assert np.max(np.abs(H - H.conj().T)) < 1e-15


def test_gauge_covariance():
    lat = Lattice((4, 2, 4, 4))
    U = si.gauge_field(lat.dims, 0.3, seed=5)
    g = si.gauge_transform(lat.dims, seed=9)
    psi = si.gaussian_spinor(lat.dims, 13)
    Ug = dirac.gauge_rotate(lat, U, g)
    lhs = dirac.wilson_dslash(lat, Ug, dirac.colour_rotate(lat, psi, g), 0.1)
    rhs = dirac.colour_rotate(lat, dirac.wilson_dslash(lat, U, psi, 0.1), g)
    assert np.max(np.abs(lhs - rhs)) < 1e-13


def test_mass_term_and_linearity():
    lat = Lattice((2, 4, 2, 4))
    U = si.gauge_field(lat.dims, 0.3, seed=2)
    a = si.gaussian_spinor(lat.dims, 1)
    b = si.gaussian_spinor(lat.dims, 2)
    d = dirac.wilson_dslash(lat, U, a, 0.7) - dirac.wilson_dslash(lat, U, a, -0.2)
    assert np.max(np.abs(d - 0.9 * a)) < 1e-13
    lin = dirac.wilson_dslash(lat, U, a + 2j * b, 0.1)
    assert np.max(np.abs(lin - dirac.wilson_dslash(lat, U, a, 0.1) - 2j * dirac.wilson_dslash(lat, U, b, 0.1))) < 1e-13


def test_single_link_brute_force():
    """One non-trivial link: only the two sites it joins see it (eq. 2 by hand)."""
    lat = Lattice((2, 2, 2, 2))
    U = si.unit_gauge_field(lat.dims)
    V = si.gauge_transform(lat.dims, seed=4)[0]
    s = lat.lex(0, 0, 0, 0)
    mu = 2  # z
    U[s, mu] = V
    psi = si.gaussian_spinor(lat.dims, 5)
    out = dirac.wilson_dslash(lat, U, psi, 0.0)
    free = dirac.wilson_dslash(lat, si.unit_gauge_field(lat.dims), psi, 0.0)
    nb = lat.lex(0, 0, 1, 0)  # L=2: +z and -z neighbours coincide
    P_minus = np.eye(4) - G[mu]
    P_plus = np.eye(4) + G[mu]
    # at s the +z term carries V, the -z term (from the link at (0,0,1,0)) is unit
    want_s = free[s] - 0.5 * (P_minus @ psi[nb] @ V.T) + 0.5 * (P_minus @ psi[nb])
    # at nb the -z term is U_z(s)^dag psi(s)
    want_nb = free[nb] - 0.5 * (P_plus @ psi[s] @ V.conj()) + 0.5 * (P_plus @ psi[s])
    assert np.max(np.abs(out[s] - want_s)) < 1e-14
    assert np.max(np.abs(out[nb] - want_nb)) < 1e-14
    others = [i for i in range(lat.N) if i not in (s, nb)]
    assert np.max(np.abs(out[others] - free[others])) < 1e-14


def test_parity_restriction():
    lat = Lattice((4, 2, 2, 2))
    U = si.gauge_field(lat.dims, 0.3, seed=8)
    psi = si.gaussian_spinor(lat.dims, 3)
    full = dirac.wilson_dslash(lat, U, psi, 0.2)
    ev = dirac.wilson_dslash_parity(lat, U, psi, 0.2, 0)
    od = dirac.wilson_dslash_parity(lat, U, psi, 0.2, 1)
    assert np.array_equal(ev + od, full)
    for lex in range(lat.N):
        if lat.parity(*lat.coords(lex)) == 0:
            assert np.all(od[lex] == 0)
