"""GPU overlap eigensolver (one chiral sector, Sec. V) and deflated CG
(eq. 9), judged by the oracle: eigenvalues against the dense eigensystem of
D built from the exact sign at 4^4, eigenvectors through the oracle's own
massless overlap on the same polynomial, and the deflated solve through the
oracle's D(m) with fewer iterations than the undeflated one."""
import ctypes

import numpy as np
import pytest

import synth_inputs as si
from oracle import dense, overlap_eigs as oe, sign
from oracle.lattice import Lattice

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from paper_1106_4964_amd import ovl  # noqa: E402

import gpu_util as gu  # noqa: E402

RHO = 1.5
F64, F32 = ovl.OVL_F64, ovl.OVL_F32


@pytest.fixture(scope="module")
def c1():
    dims = (4, 4, 4, 4)
    lat = Lattice(dims)
    U = si.gauge_field(dims, 0.3, 1)
    H = dense.dense_hw(lat, U, RHO)
    w, v = np.linalg.eigh(H)
    E = (v * np.where(w >= 0, 1.0, -1.0)) @ v.conj().T
    return dict(dims=dims, lat=lat, U=U, E=E, lo=float(np.min(np.abs(w))), hi=float(np.max(np.abs(w))) * 1.0001)


def _gpu_eigs(c1, g, gauge, s, ell, K, sector=1, tol=1e-10, prec=F64):
    V = gu.pack(g, np.stack([si.gaussian_spinor(c1["dims"], 300 + i) for i in range(2 * ell)]), F64, 2 * ell)
    d = np.zeros(4 * ell)
    nout = ctypes.c_int()
    st = ovl.EigStats()
    rc = ovl.ovl_overlap_eigs(gauge, RHO, s, None, prec, sector, ell, K, V, d, ctypes.byref(nout), tol, 60,
                              ctypes.byref(st), None)
    dc = d[: 2 * nout.value].view(np.complex128)
    return rc, V, dc, nout.value, st


@pytest.mark.parametrize("sector", [1, -1])
def test_overlap_eigs_against_dense(c1, sector):
    g = ovl.Geometry(c1["dims"])
    gauge = gu.make_gauge(g, c1["U"])
    s = ovl.Sign(c1["lo"], c1["hi"], n=200)
    ell = 10
    rc, V, d, n, st = _gpu_eigs(c1, g, gauge, s, ell, 48, sector)
    print("overlap eigs sector %+d: rc %d, %d pairs, %d restart cycles, %d D_w applies, max residual %.2e"
          % (sector, rc, n, st.iterations, st.hw_applies, st.max_residual))
    assert rc == 0 and n == 2 * ell
    # oracle: the same sector of the exact sign (dense), its pairs of D
    k_ref, V_ref = oe.sector_lowest_dense(c1["E"], c1["lat"].N, sector, ell)
    apply_E = lambda v: (c1["E"] @ v.reshape(-1)).reshape(v.shape)  # noqa: E731
    d_ref, _ = oe.overlap_pairs(apply_E, k_ref, V_ref, sector)
    assert np.max(np.abs(d - d_ref)) < 1e-9, (d, d_ref)
    # eigenvectors: D xi = d xi with the oracle's massless overlap on the same
    # polynomial, and orthonormal
    so = sign.make_sign(c1["lo"], c1["hi"], 200)
    Xi = gu.unpack(g, V[: n * g.spinor_bytes(F64)], F64, n)
    for i in range(n):
        r = sign.massless_overlap(c1["lat"], c1["U"], Xi[i], RHO, so) - d[i] * Xi[i]
        assert np.linalg.norm(r) < 1e-9
    Xf = Xi.reshape(n, -1)
    assert np.max(np.abs(Xf.conj() @ Xf.T - np.eye(n))) < 1e-9


@pytest.mark.parametrize("inner", [F64, F32])
def test_deflated_cg_fewer_iterations(c1, inner):
    g = ovl.Geometry(c1["dims"])
    gauge = gu.make_gauge(g, c1["U"], [(F32, 1)])
    s = ovl.Sign(c1["lo"], c1["hi"], n=200)
    ell = 12
    rc, V, d, n, st = _gpu_eigs(c1, g, gauge, s, ell, 48)
    assert rc == 0
    defl = ovl.Deflation(g, V, d)
    m, R = 0.01, 4
    b = gu.pack(g, si.point_sources(c1["dims"])[:R], F64, R)
    out = {}
    for name, df in (("plain", None), ("deflated", defl)):
        x = torch.zeros(g.spinor_bytes(F64, R), dtype=torch.uint8, device=gu.DEV)
        opts = ovl.SolveOpts(inner, 1e-3 if inner != F64 else 0.0, 0, 1, 60)
        opts.deflation = df.handle.value if df is not None else None
        stt = ovl.SolveStats()
        rc = ovl.ovl_cg_solve(x, b, R, gauge, RHO, m, s, None, 1e-10, 20000, opts, ctypes.byref(stt), None)
        assert rc == 0
        out[name] = (stt.iterations, stt.restarts, x, stt.deflation_dropped)
    print("4^4 CG m=0.01, inner %d: %d iterations plain, %d deflated (%d pairs of D)"
          % (inner, out["plain"][0], out["deflated"][0], n))
    assert out["deflated"][0] < 0.85 * out["plain"][0]
    assert out["deflated"][3] == 0  # good pairs are never dropped
    # the deflated solution is judged by the oracle's own D(m)
    so = sign.make_sign(c1["lo"], c1["hi"], 200)
    xs = gu.unpack(g, out["deflated"][2], F64, R)
    bs = si.point_sources(c1["dims"])[:R]
    for r in range(R):
        res = bs[r] - sign.overlap_apply(c1["lat"], c1["U"], xs[r], RHO, m, so)
        assert np.linalg.norm(res) / np.linalg.norm(bs[r]) <= 1.05e-10


def test_overlap_eigs_fp32_sign(c1):
    """The sector operator's sign applied with FP32 storage and arithmetic
    (the Lanczos basis and Rayleigh-Ritz in FP64): the pairs of D agree with
    the dense exact-sign ones to the FP32 level, the eigenvectors satisfy
    D xi = d xi through the oracle's overlap to ~1e-5, and they still deflate
    the FP64 CG (the defect correction makes up for their accuracy)."""
    g = ovl.Geometry(c1["dims"])
    gauge = gu.make_gauge(g, c1["U"], [(F32, 1)])
    s = ovl.Sign(c1["lo"], c1["hi"], n=200)
    ell = 10
    rc, V, d, n, st = _gpu_eigs(c1, g, gauge, s, ell, 48, 1, tol=1e-5, prec=F32)
    print("overlap eigs, FP32 sign: rc %d, %d pairs, %d restart cycles, max residual %.2e"
          % (rc, n, st.iterations, st.max_residual))
    assert rc == 0 and n == 2 * ell
    assert st.max_residual < 1e-4
    k_ref, V_ref = oe.sector_lowest_dense(c1["E"], c1["lat"].N, 1, ell)
    apply_E = lambda v: (c1["E"] @ v.reshape(-1)).reshape(v.shape)  # noqa: E731
    d_ref, _ = oe.overlap_pairs(apply_E, k_ref, V_ref, 1)
    assert np.max(np.abs(d - d_ref)) < 1e-5, (d, d_ref)
    so = sign.make_sign(c1["lo"], c1["hi"], 200)
    Xi = gu.unpack(g, V[: n * g.spinor_bytes(F64)], F64, n)
    for i in range(n):
        r = sign.massless_overlap(c1["lat"], c1["U"], Xi[i], RHO, so) - d[i] * Xi[i]
        assert np.linalg.norm(r) < 1e-4
    # the sector vectors are FP64-orthonormal; each partner u = P_-s eps v / sn
    # carries the sign's FP32 error divided by sn, so pairs are orthogonal to
    # each other only to that level
    Xf = Xi.reshape(n, -1)
    assert np.max(np.abs(Xf.conj() @ Xf.T - np.eye(n))) < 1e-4
    # deflation with these pairs: fewer iterations, same FP64 residual
    defl = ovl.Deflation(g, V, d)
    m, R = 0.01, 4
    b = gu.pack(g, si.point_sources(c1["dims"])[:R], F64, R)
    its = {}
    for name, df in (("plain", None), ("deflated", defl)):
        x = torch.zeros(g.spinor_bytes(F64, R), dtype=torch.uint8, device=gu.DEV)
        opts = ovl.SolveOpts(F32, 1e-3, 0, 1, 60)
        opts.deflation = df.handle.value if df is not None else None
        stt = ovl.SolveStats()
        assert ovl.ovl_cg_solve(x, b, R, gauge, RHO, m, s, None, 1e-10, 20000, opts, ctypes.byref(stt), None) == 0
        its[name] = stt.iterations
        if df is not None:
            xs = gu.unpack(g, x, F64, R)
            bs = si.point_sources(c1["dims"])[:R]
            for r in range(R):
                res = bs[r] - sign.overlap_apply(c1["lat"], c1["U"], xs[r], RHO, m, so)
                assert np.linalg.norm(res) / np.linalg.norm(bs[r]) <= 1.05e-10
    print("4^4 CG m=0.01, FP32 inner: %d iterations plain, %d deflated with FP32-sign pairs" % (its["plain"],
                                                                                               its["deflated"]))
    assert its["deflated"] < 0.85 * its["plain"]


def test_overlap_eigs_needs_the_precisions_links(c1):
    """A storage precision whose links the gauge field does not hold is an
    error, not a silent fallback."""
    g = ovl.Geometry(c1["dims"])
    gauge = gu.make_gauge(g, c1["U"])  # FP64 links only
    s = ovl.Sign(c1["lo"], c1["hi"], n=50)
    with pytest.raises(ovl.OvlError):
        _gpu_eigs(c1, g, gauge, s, 4, 24, 1, tol=1e-5, prec=ovl.OVL_F16)


def test_wrong_eigenpairs_are_dropped(c1):
    """A deflation whose pairs are not eigenpairs of D (random orthonormal
    vectors, |d| = 1e-3): eq. 9 then amplifies the wrong directions by
    1/|d(m)| ~ 90 and the first deflated cycle raises the residual.  The
    solve must notice, return to the x before that cycle, finish without
    deflation to the FP64 tolerance (judged by the oracle's D(m)) and say so."""
    g = ovl.Geometry(c1["dims"])
    gauge = gu.make_gauge(g, c1["U"], [(F32, 1)])
    s = ovl.Sign(c1["lo"], c1["hi"], n=200)
    rng = np.random.default_rng(5)
    nvec = 8
    N = c1["lat"].N
    A = rng.standard_normal((N * 12, nvec)) + 1j * rng.standard_normal((N * 12, nvec))
    Qm, _ = np.linalg.qr(A)
    Xi = np.ascontiguousarray(Qm.T).reshape(nvec, N, 4, 3)
    d = 1e-3 * np.exp(1j * rng.uniform(0, 2 * np.pi, nvec))
    V = gu.pack(g, Xi, F64, nvec)
    defl = ovl.Deflation(g, V, d)
    m, R = 0.01, 4
    bs = si.point_sources(c1["dims"])[:R]
    x = torch.zeros(g.spinor_bytes(F64, R), dtype=torch.uint8, device=gu.DEV)
    opts = ovl.SolveOpts(F32, 1e-3, 0, 1, 60)
    opts.deflation = defl.handle.value
    stt = ovl.SolveStats()
    rc = ovl.ovl_cg_solve(x, gu.pack(g, bs, F64, R), R, gauge, RHO, m, s, None, 1e-10, 20000, opts,
                          ctypes.byref(stt), None)
    print("wrong pairs: rc %d, %d iterations, %d cycles, deflation dropped %d"
          % (rc, stt.iterations, stt.restarts, stt.deflation_dropped))
    assert rc == 0
    assert stt.deflation_dropped == 1
    so = sign.make_sign(c1["lo"], c1["hi"], 200)
    xs = gu.unpack(g, x, F64, R)
    for r in range(R):
        res = bs[r] - sign.overlap_apply(c1["lat"], c1["U"], xs[r], RHO, m, so)
        assert np.linalg.norm(res) / np.linalg.norm(bs[r]) <= 1.05e-10


def _deflated_solve(c1, g, gauge, s, defl, rho=RHO, R=4, m=0.01):
    b = gu.pack(g, si.point_sources(c1["dims"])[:R], F64, R)
    x = torch.zeros(g.spinor_bytes(F64, R), dtype=torch.uint8, device=gu.DEV)
    opts = ovl.SolveOpts(F32, 1e-3, 0, 1, 60)
    opts.deflation = defl.handle.value if defl is not None else None
    stt = ovl.SolveStats()
    rc = ovl.ovl_cg_solve(x, b, R, gauge, rho, m, s, None, 1e-10, 20000, opts, ctypes.byref(stt), None)
    return rc, stt, gu.unpack(g, x, F64, R)


def _check_solution(c1, xs, m=0.01):
    so = sign.make_sign(c1["lo"], c1["hi"], 200)
    bs = si.point_sources(c1["dims"])[: len(xs)]
    for r in range(len(xs)):
        res = bs[r] - sign.overlap_apply(c1["lat"], c1["U"], xs[r], RHO, m, so)
        assert np.linalg.norm(res) / np.linalg.norm(bs[r]) <= 1.05e-10


def test_minimal_residual_deflation(c1):
    """ovl_deflation_prepare: the correction in span(Xi) that minimises the
    residual, with D(m) Xi from Z = D(0) Xi.  Accurate (FP64) pairs: the same
    iterations as eq. 9.  FP32-sign pairs: no more than eq. 9 with the same
    pairs.  Wrong pairs (random orthonormal vectors, |d| = 1e-3): the
    correction cannot raise the residual, so nothing is dropped.  Every
    solution meets 1e-10 through the oracle's D(m)."""
    g = ovl.Geometry(c1["dims"])
    gauge = gu.make_gauge(g, c1["U"], [(F32, 1)])
    s = ovl.Sign(c1["lo"], c1["hi"], n=200)
    ell = 10
    v64 = g.spinor_bytes(F64)
    res = {}
    for name, prec, tol in (("fp64 pairs", F64, 1e-10), ("fp32 pairs", F32, 1e-5)):
        rc, V, d, n, st = _gpu_eigs(c1, g, gauge, s, ell, 48, 1, tol=tol, prec=prec)
        assert rc == 0
        its = []
        for prepared in (False, True):
            defl = ovl.Deflation(g, V, d)
            if prepared:
                Z = torch.empty(n * v64, dtype=torch.uint8, device=gu.DEV)
                defl.prepare(gauge, RHO, s, None, Z)
            rc, stt, xs = _deflated_solve(c1, g, gauge, s, defl)
            assert rc == 0 and stt.deflation_dropped == 0
            _check_solution(c1, xs)
            its.append(stt.iterations)
        res[name] = its
    rng = np.random.default_rng(5)
    N = c1["lat"].N
    A = rng.standard_normal((N * 12, 8)) + 1j * rng.standard_normal((N * 12, 8))
    Xi = np.ascontiguousarray(np.linalg.qr(A)[0].T).reshape(8, N, 4, 3)
    defl = ovl.Deflation(g, gu.pack(g, Xi, F64, 8), 1e-3 * np.exp(1j * rng.uniform(0, 2 * np.pi, 8)))
    Z = torch.empty(8 * v64, dtype=torch.uint8, device=gu.DEV)
    defl.prepare(gauge, RHO, s, None, Z)
    rc, stt, xs = _deflated_solve(c1, g, gauge, s, defl)
    print("iterations (eq. 9, minimal residual):", res, "; wrong pairs prepared: %d, dropped %d"
          % (stt.iterations, stt.deflation_dropped))
    assert rc == 0 and stt.deflation_dropped == 0
    _check_solution(c1, xs)
    assert abs(res["fp64 pairs"][1] - res["fp64 pairs"][0]) <= 2
    assert res["fp32 pairs"][1] <= res["fp32 pairs"][0] + 1


def test_prepare_argument_errors(c1):
    g = ovl.Geometry(c1["dims"])
    gauge = gu.make_gauge(g, c1["U"], [(F32, 1)])
    s = ovl.Sign(c1["lo"], c1["hi"], n=50)
    rng = np.random.default_rng(1)
    N = c1["lat"].N
    A = rng.standard_normal((N * 12, 2)) + 1j * rng.standard_normal((N * 12, 2))
    V = gu.pack(g, np.ascontiguousarray(np.linalg.qr(A)[0].T).reshape(2, N, 4, 3), F64, 2)
    defl = ovl.Deflation(g, V, np.array([0.5 + 0.1j, 0.5 - 0.1j]))
    Z = torch.empty(2 * g.spinor_bytes(F64), dtype=torch.uint8, device=gu.DEV)
    with pytest.raises(ovl.OvlError):
        defl.prepare(gauge, 0.0, s, None, Z)  # rho <= 0
    with pytest.raises(ovl.OvlError):
        defl.prepare(gauge, RHO, s, None, V)  # Z aliasing Xi
    defl.prepare(gauge, RHO, s, None, Z)
    with pytest.raises(ovl.OvlError):
        _deflated_solve(c1, g, gauge, s, defl, rho=1.4)  # prepared with another rho
