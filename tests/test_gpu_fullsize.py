"""Parity at the full lattice sizes of the measured workloads, in the launch
configuration the benchmark times (12 right-hand sides, F16 storage with
12-real links, autotuned stencil shapes): the oracle computes a few of the
batch's vectors in full and the GPU batch is compared on every site."""
import ctypes

import numpy as np
import pytest

import synth_inputs as si
from oracle import dirac, sign
from oracle.lattice import Lattice

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from paper_1106_4964_amd import ovl  # noqa: E402

import gpu_util as gu  # noqa: E402

F16, F64 = ovl.OVL_F16, ovl.OVL_F64
U16 = gu.UNIT_ROUNDOFF[F16]
RHO = 1.5
# Element-wise bounds (max over the 12 vectors of max|got - want| / max|want|)
# for F16 storage with FP32 arithmetic, about 2.5x the largest error measured
# on MI355X: H_w 6.3e-4, sign application (n = 4) 9.5e-4.
BOUND_HW_ELEMENTWISE = 1.5e-3
BOUND_SIGN_ELEMENTWISE = 2.5e-3


def _field(dims, seed=3):
    lat = Lattice(dims)
    U = si.gauge_field(dims, 0.25, seed)
    g = ovl.Geometry(dims)
    gauge = gu.make_gauge(g, U, [(F16, 1)])
    return lat, U, g, gauge


@pytest.fixture(scope="module")
def big():
    return _field((24, 24, 24, 64))


def test_hw_24x24x24x64_f16_12rhs(big):
    """H_w on 12 F16 vectors in the tuned shape, every vector compared with
    the oracle site by site (max |got - want| / max |want|)."""
    lat, U, g, gauge = big
    dims = lat.dims
    psi = np.stack([si.gaussian_spinor(dims, 800 + r) for r in range(12)])
    x = gu.pack(g, psi, F16, 12)
    y = gu.empty_field(g, F16, 12)
    ovl.ovl_hw_apply(y, x, gauge, RHO, F16, 12, None)  # tunes the shape
    ovl.ovl_hw_apply(y, x, gauge, RHO, F16, 12, None)
    shape = ovl.stencil_shape(g, F16, 1, 0, 12)
    got = gu.unpack(g, y, F16, 12)
    errs = []
    for r in range(12):
        errs.append(gu.max_rel_err(got[r], dirac.hw_apply(lat, U, psi[r], RHO)))
    print("H_w 24^3x64 F16, 12 rhs, shape %s: element-wise errors %s" % (shape, " ".join("%.2e" % e for e in errs)))
    assert max(errs) < BOUND_HW_ELEMENTWISE


def test_clenshaw_steps_24x24x24x64_f16_12rhs(big):
    """A sign application (n = 4) on the 12-rhs batch runs the Clenshaw-step
    stencils with 0 and 3 extra epilogue vectors at full size.  The inputs
    are psi_a + c_r psi_b (c_r = r - 5.5), so the oracle's recurrence on
    psi_a and psi_b gives all twelve expected outputs by linearity; each is
    compared site by site."""
    lat, U, g, gauge = big
    dims = lat.dims
    v0 = gu.pack(g, si.gaussian_spinor(dims, 17), F64)
    lam = ctypes.c_double()
    ovl.ovl_hw_bound(gauge, RHO, v0, 30, ctypes.byref(lam), None, None, None)
    lam_max = lam.value * 1.01
    s = ovl.Sign(0.2 * lam_max, lam_max, n=4)
    so = sign.SignApprox(lam_max=lam_max, eps=s.eps, coeffs=s.coeffs())
    pa, pb = si.gaussian_spinor(dims, 820), si.gaussian_spinor(dims, 821)
    coef = np.arange(12) - 5.5
    psi = pa[None] + coef[:, None, None, None] * pb[None]
    x = gu.pack(g, psi, F16, 12)
    del psi
    y = gu.empty_field(g, F16, 12)
    ovl.ovl_sign_apply(y, x, gauge, RHO, s, None, F16, 12, None)  # tunes the shapes
    ovl.ovl_stencil_timer(1)
    ovl.ovl_sign_apply(y, x, gauge, RHO, s, None, F16, 12, None)
    torch.cuda.synchronize()
    ovl.ovl_stencil_timer(0)
    n3, ms3 = ovl.stencil_timer_read(F16, 1, 3, 12)
    assert n3 >= 2
    got = gu.unpack(g, y, F16, 12)
    wa = sign.sign_apply(lat, U, pa, RHO, so)
    wb = sign.sign_apply(lat, U, pb, RHO, so)
    errs = [gu.max_rel_err(got[r], wa + coef[r] * wb) for r in range(12)]
    print("sign (n=4) 24^3x64 F16 12 rhs: element-wise errors %s; 3-vector stencil %d launches, %.1f us, shape %s"
          % (" ".join("%.2e" % e for e in errs), n3, 1e3 * ms3 / n3, ovl.stencil_shape(g, F16, 1, 3, 12)))
    assert max(errs) < BOUND_SIGN_ELEMENTWISE


def test_hw_32x32x32x64_f16_12rhs():
    lat, U, g, gauge = _field((32, 32, 32, 64), seed=5)
    dims = lat.dims
    psi = np.stack([si.gaussian_spinor(dims, 840 + r) for r in range(12)])
    x = gu.pack(g, psi, F16, 12)
    y = gu.empty_field(g, F16, 12)
    ovl.ovl_hw_apply(y, x, gauge, RHO, F16, 12, None)
    ovl.ovl_hw_apply(y, x, gauge, RHO, F16, 12, None)
    got = gu.unpack(g, y, F16, 12)
    want = dirac.hw_apply(lat, U, psi[3], RHO)
    err = gu.rel_err(got[3], want)
    print("H_w 32^3x64 F16 12 rhs: rel err %.2e, shape %s" % (err, ovl.stencil_shape(g, F16, 1, 0, 12)))
    assert err < 16 * U16 + 4e-7


def test_overlap_16x16x16x32_each_precision():
    """D(m) at 16^3x32 in FP64, FP32 and F16 storage against the oracle on
    the same coefficients (n = 20, no projection)."""
    dims = (16, 16, 16, 32)
    lat = Lattice(dims)
    U = si.gauge_field(dims, 0.25, 11)
    g = ovl.Geometry(dims)
    gauge = gu.make_gauge(g, U, [(ovl.OVL_F32, 1), (F16, 1)])
    v0 = gu.pack(g, si.gaussian_spinor(dims, 17), F64)
    lam = ctypes.c_double()
    ovl.ovl_hw_bound(gauge, RHO, v0, 30, ctypes.byref(lam), None, None, None)
    lam_max = lam.value * 1.01
    s = ovl.Sign(0.1 * lam_max, lam_max, n=20)
    so = sign.SignApprox(lam_max=lam_max, eps=s.eps, coeffs=s.coeffs())
    psi = si.gaussian_spinor(dims, 860)
    want = sign.overlap_apply(lat, U, psi, RHO, 0.01, so)
    for prec, bound in [(F64, 1e-12), (ovl.OVL_F32, 1e-5), (F16, 3e-2)]:
        y = gu.empty_field(g, prec)
        ovl.ovl_overlap_apply(y, gu.pack(g, psi, prec), gauge, RHO, 0.01, s, None, 0, prec, 1, None)
        err = gu.rel_err(gu.unpack(g, y, prec), want)
        print("D(m) 16^3x32 prec %d: rel err %.2e" % (prec, err))
        assert err < bound


def test_mixed_cg_16x16x16x32_one_rhs():
    """The 16^3x32 single-rhs case: 20 low modes from the GPU eigensolver,
    mixed CG (F16 inner, FP64 defect correction) at m = 0.01 to 1e-10, the
    solution judged by the oracle's own operator on the same coefficients
    and low modes."""
    dims = (16, 16, 16, 32)
    lat = Lattice(dims)
    U = si.gauge_field(dims, 0.25, 13)
    g = ovl.Geometry(dims)
    gauge = gu.make_gauge(g, U, [(F16, 1)])
    v0 = gu.pack(g, si.gaussian_spinor(dims, 17), F64)
    lam = ctypes.c_double()
    ovl.ovl_hw_bound(gauge, RHO, v0, 60, ctypes.byref(lam), None, None, None)
    lam_max = lam.value * (1 + 1e-6)
    ell, m_ = 20, 32
    V = gu.pack(g, np.stack([si.gaussian_spinor(dims, 2000 + i) for i in range(m_)]), F64, m_)
    lams = np.zeros(ell)
    est = ovl.EigStats()
    assert ovl.ovl_hw_eigs(gauge, RHO, ell, m_, V, lams, lam_max, 1e-11, 60, 30, ctypes.byref(est), None) == 0
    Vk = V[: ell * g.spinor_bytes(F64)]
    lm = ovl.LowModes(g, Vk, lams)
    s = ovl.Sign(abs(lams[-1]), lam_max, delta=1e-6)
    b = si.point_source(dims, 0, 0)[None]
    x = gu.pack(g, np.zeros_like(b), F64, 1)
    st = ovl.SolveStats()
    rc = ovl.ovl_cg_solve(x, gu.pack(g, b, F64, 1), 1, gauge, RHO, 0.01, s, lm, 1e-10, 20000,
                          ovl.SolveOpts(F16, 1e-2, 4, 1, 60), ctypes.byref(st), None)
    assert rc == 0 and st.true_residual[0] <= 1e-10
    so = sign.SignApprox(lam_max=lam_max, eps=s.eps, coeffs=s.coeffs())
    Vh = gu.unpack(g, Vk, F64, ell)
    xs = gu.unpack(g, x, F64)
    res = b[0] - sign.overlap_apply(lat, U, xs, RHO, 0.01, so, Vh, lams)
    rel = np.linalg.norm(res) / np.linalg.norm(b[0])
    print("16^3x32 mixed CG: n = %d, %d iterations, %d restarts, oracle residual %.2e"
          % (s.n, st.iterations, st.restarts, rel))
    assert rel <= 1.05e-10
