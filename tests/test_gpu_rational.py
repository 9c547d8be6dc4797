"""GPU rational sign (eq. 4-5, 12): multi-shift CG (single pass) and double
pass against the oracle's rational sign on the same field and low modes,
element by element, and against the exact sign of the dense H_w within the
measured delta of the rational function.  The oracle computes its own
coefficients (scipy's elliptic functions); nothing comes from the GPU path."""
import ctypes

import numpy as np
import pytest

import synth_inputs as si
from oracle import dense
from oracle import rational as ra
from oracle.lattice import Lattice

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from paper_1106_4964_amd import ovl  # noqa: E402

import gpu_util as gu  # noqa: E402

RHO = 1.5
F64 = ovl.OVL_F64


@pytest.fixture(scope="module")
def c1():
    dims = (4, 4, 4, 4)
    lat = Lattice(dims)
    U = si.gauge_field(dims, 0.3, 1)
    H = dense.dense_hw(lat, U, RHO)
    w, v = np.linalg.eigh(H)
    E = (v * np.where(w >= 0, 1.0, -1.0)) @ v.conj().T
    order = np.argsort(np.abs(w))
    return dict(dims=dims, lat=lat, U=U, E=E, w=w[order], v=v[:, order], hi=float(np.max(np.abs(w))) * 1.0001)


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("ell", [0, 12])
def test_rational_sign_matches_oracle(c1, method, ell):
    g = ovl.Geometry(c1["dims"])
    gauge = gu.make_gauge(g, c1["U"])
    N = c1["lat"].N
    if ell:
        V = np.ascontiguousarray(c1["v"][:, :ell].T).reshape(ell, N, 4, 3)
        lam = c1["w"][:ell].copy()
        lm = ovl.LowModes(g, gu.pack(g, V, F64, ell), lam)
        lo = abs(lam[-1])
    else:
        V, lam, lm = None, None, None
        lo = float(np.abs(c1["w"][0]))
    n = 8  # delta ~ 1e-8, far above the Krylov tolerance
    r = ovl.Rational(lo, c1["hi"], n)
    o = ra.make_rational(lo, c1["hi"], n)
    psi = si.gaussian_spinor(c1["dims"], 21)
    out = gu.empty_field(g, F64)
    st = ovl.RationalStats()
    rc = ovl.ovl_rational_sign_apply(out, gu.pack(g, psi, F64), gauge, RHO, r, lm, method, 1e-12, 2000,
                                     ctypes.byref(st), None)
    assert rc == 0
    got = gu.unpack(g, out, F64)
    want = ra.sign_apply_rational(c1["lat"], c1["U"], psi, RHO, o, V=V, lam=lam,
                                  method="multishift" if method == 0 else "double", tol=1e-12)
    err = gu.max_rel_err(got, want)
    exact = (c1["E"] @ psi.reshape(-1)).reshape(psi.shape)
    err_exact = np.linalg.norm(got - exact) / np.linalg.norm(psi)
    print("rational sign n=%d ell=%d method %d: %d steps, %d H_w applies; max rel err vs oracle %.2e, "
          "vs exact sign %.2e (delta %.2e)" % (n, ell, method, st.iterations, st.hw_applies, err, err_exact, r.delta))
    assert err < 1e-10
    assert err_exact <= 1.2 * r.delta + 1e-12
    # H_w applications: 2 per Krylov step and 1 for Q (double pass: both passes)
    want_hw = 2 * st.iterations + 1 if method == 0 else 2 * st.iterations + 2 * (st.iterations - 1) + 1
    assert st.hw_applies == want_hw


def test_rational_sign_edge_cases(c1):
    g = ovl.Geometry(c1["dims"])
    gauge = gu.make_gauge(g, c1["U"])
    r = ovl.Rational(float(np.abs(c1["w"][0])), c1["hi"], 8)
    zero = gu.pack(g, np.zeros((c1["lat"].N, 4, 3)), F64)
    out = gu.pack(g, np.ones((c1["lat"].N, 4, 3)), F64)
    st = ovl.RationalStats()
    for method in (0, 1):
        assert ovl.ovl_rational_sign_apply(out, zero, gauge, RHO, r, None, method, 1e-12, 100, ctypes.byref(st),
                                           None) == 0
        assert np.all(gu.unpack(g, out, F64) == 0.0)
    psi = gu.pack(g, si.gaussian_spinor(c1["dims"], 3), F64)
    for bad_method, bad_tol in ((2, 1e-12), (0, 0.0)):
        with pytest.raises(ovl.OvlError):
            ovl.ovl_rational_sign_apply(out, psi, gauge, RHO, r, None, bad_method, bad_tol, 100, ctypes.byref(st), None)
    with pytest.raises(ovl.OvlError):
        ovl.ovl_rational_sign_apply(psi, psi, gauge, RHO, r, None, 0, 1e-12, 100, ctypes.byref(st), None)
    # too few steps: a warning code, not an error
    assert ovl.ovl_rational_sign_apply(out, psi, gauge, RHO, r, None, 0, 1e-12, 3, ctypes.byref(st), None) == 1
