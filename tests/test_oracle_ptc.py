"""Pins for the oracle's parallel-transport convolution layer and its gradients."""
import numpy as np
import pytest

import synth_inputs as si
from oracle import dirac, ptc
from oracle.lattice import Lattice


@pytest.fixture(scope="module")
def setup():
    lat = Lattice((2, 4, 2, 2))
    U = si.gauge_field(lat.dims, 0.3, seed=21)
    return lat, U


def _rand_w(rng, cout, cin):
    return 0.3 * (rng.standard_normal((9, cout, cin, 4, 4)) + 1j * rng.standard_normal((9, cout, cin, 4, 4)))


def test_wilson_weights_give_dslash(setup):
    lat, U = setup
    psi = si.gaussian_spinor(lat.dims, 1)
    out = ptc.forward(lat, U, ptc.wilson_weights(0.3), psi.reshape(1, lat.N, 4, 3))[0]
    assert np.max(np.abs(out - dirac.wilson_dslash(lat, U, psi, 0.3))) < 1e-14


def test_gauge_equivariance(setup):
    lat, U = setup
    rng = np.random.default_rng(0)
    W = _rand_w(rng, 2, 3)
    g = si.gauge_transform(lat.dims, seed=3)
    Ug = dirac.gauge_rotate(lat, U, g)
    phi = np.stack([si.gaussian_spinor(lat.dims, 10 + i) for i in range(3)])
    phig = np.stack([dirac.colour_rotate(lat, p, g) for p in phi])
    lhs = ptc.forward(lat, Ug, W, phig)
    rhs = np.stack([dirac.colour_rotate(lat, o, g) for o in ptc.forward(lat, U, W, phi)])
    assert np.max(np.abs(lhs - rhs)) < 1e-13


def test_backward_is_adjoint(setup):
    lat, U = setup
    rng = np.random.default_rng(1)
    W = _rand_w(rng, 2, 3)
    phi = np.stack([si.gaussian_spinor(lat.dims, 20 + i) for i in range(3)])
    g = np.stack([si.gaussian_spinor(lat.dims, 30 + i) for i in range(2)])
    g_in, _ = ptc.backward(lat, U, W, phi, g)
    assert abs(np.vdot(g, ptc.forward(lat, U, W, phi)) - np.vdot(g_in, phi)) < 1e-12 * abs(np.vdot(g_in, phi))


def test_weight_gradient_finite_difference(setup):
    lat, U = setup
    rng = np.random.default_rng(2)
    w1 = _rand_w(rng, 4, 1)
    w2 = _rand_w(rng, 1, 4)
    b = si.gaussian_spinor(lat.dims, 40)
    x = si.gaussian_spinor(lat.dims, 41)
    loss, (g1, g2) = ptc.net_loss_and_grad(lat, U, (w1, w2), b, x)
    h = 1e-6
    for (which, idx) in [(0, (0, 1, 0, 2, 3)), (0, (5, 3, 0, 0, 0)), (1, (8, 0, 2, 1, 1)), (1, (0, 0, 3, 3, 2))]:
        for unit in (1.0, 1j):
            ws = [w1.copy(), w2.copy()]
            ws[which][idx] += h * unit
            lp, _ = ptc.net_loss_and_grad(lat, U, tuple(ws), b, x)
            ws[which][idx] -= 2 * h * unit
            lm, _ = ptc.net_loss_and_grad(lat, U, tuple(ws), b, x)
            fd = (lp - lm) / (2 * h)
            grad = (g1, g2)[which][idx]
            an = grad.real if unit == 1.0 else grad.imag
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (which, idx, unit, fd, an)
