"""GPU parity of geometry, packing and the Wilson stencil against the oracle."""
import ctypes

import numpy as np
import pytest

import synth_inputs as si
from oracle import dirac
from oracle.lattice import Lattice

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1106_4964_amd import ovl  # noqa: E402

import gpu_util as gu  # noqa: E402

SIZES = [(4, 4, 4, 4), (6, 6, 6, 8), (8, 6, 4, 10), (2, 2, 2, 2)]
PRECS = [ovl.OVL_F64, ovl.OVL_F32, ovl.OVL_F16, ovl.OVL_BF16]


@pytest.mark.parametrize("dims", SIZES)
def test_neighbor_table_bit_exact(dims):
    lat = Lattice(dims)
    g = ovl.Geometry(dims)
    dev = torch.empty((8, g.N), dtype=torch.int32, device=gu.DEV)
    ovl.ovl_geom_neighbors_device(g, dev, None)
    torch.cuda.synchronize()
    assert np.array_equal(dev.cpu().numpy(), lat.neighbor_table())


@pytest.mark.parametrize("prec", PRECS)
def test_pack_roundtrip(prec):
    dims = (6, 6, 6, 8)
    g = ovl.Geometry(dims)
    psi = np.stack([si.gaussian_spinor(dims, 5 + r) for r in range(3)])
    back = gu.unpack(g, gu.pack(g, psi, prec, 3), prec, 3)
    if prec == ovl.OVL_F64:
        assert np.array_equal(back, psi)
    else:
        assert gu.max_rel_err(back, psi) <= 2 * gu.UNIT_ROUNDOFF[prec] * np.max(np.abs(psi)) / np.max(np.abs(psi))
        # the even-odd reorder itself is exact: F32 equals a numpy float32 rounding
        if prec == ovl.OVL_F32:
            r = psi.real.astype(np.float32).astype(np.float64) + 1j * psi.imag.astype(np.float32).astype(np.float64)
            assert np.array_equal(back, r)


def _dslash_case(dims, prec, compress12, m, parity, seed=1, nrhs=1):
    lat = Lattice(dims)
    U = si.gauge_field(dims, 0.3, seed)
    psi = np.stack([si.gaussian_spinor(dims, 100 + seed + r) for r in range(nrhs)])
    g = ovl.Geometry(dims)
    reprs = [] if (prec == ovl.OVL_F64 and not compress12) else [(prec, compress12)]
    gauge = gu.make_gauge(g, U, reprs)
    inp = gu.pack(g, psi, prec, nrhs)
    out = gu.pack(g, np.zeros_like(psi), prec, nrhs)
    ovl.ovl_dslash(out, inp, gauge, m, parity, prec, nrhs, None)
    got = gu.unpack(g, out, prec, nrhs)
    if nrhs == 1:
        got = got[None]
    if parity == 2:
        want = np.stack([dirac.wilson_dslash(lat, U, p, m) for p in psi])
    else:
        want = np.stack([dirac.wilson_dslash_parity(lat, U, p, m, parity) for p in psi])
    return got, want


@pytest.mark.parametrize("dims", SIZES)
@pytest.mark.parametrize("m", [-1.5, 0.0, 0.1])
def test_dslash_f64_parity(dims, m):
    got, want = _dslash_case(dims, ovl.OVL_F64, 0, m, 2)
    assert gu.max_rel_err(got, want) < 1e-13


@pytest.mark.parametrize("parity", [0, 1])
def test_dslash_single_parity_leaves_other_half(parity):
    got, want = _dslash_case((6, 6, 6, 8), ovl.OVL_F64, 0, 0.1, parity)
    # the untouched half of `out` still holds the zeros it was packed with
    assert gu.max_rel_err(got, want) < 1e-13


def test_dslash_f64_compressed_links():
    got, want = _dslash_case((8, 6, 4, 10), ovl.OVL_F64, 1, -1.5, 2)
    assert gu.max_rel_err(got, want) < 1e-13


@pytest.mark.parametrize("prec", [ovl.OVL_F32, ovl.OVL_F16, ovl.OVL_BF16])
@pytest.mark.parametrize("compress12", [0, 1])
def test_dslash_low_precision_error(prec, compress12):
    got, want = _dslash_case((8, 6, 4, 10), prec, compress12, -1.5, 2)
    # storage rounding of input, links and output; FP32 arithmetic
    tol = 16 * gu.UNIT_ROUNDOFF[prec] + 4e-7
    err = gu.rel_err(got, want)
    print("prec", prec, "c12", compress12, "rel err", err)
    assert err < tol


def test_dslash_batch_equals_single():
    dims = (6, 6, 6, 8)
    got, want = _dslash_case(dims, ovl.OVL_F64, 0, 0.1, 2, nrhs=3)
    assert gu.max_rel_err(got, want) < 1e-13


def test_hw_apply_gamma5_hermitian():
    dims = (8, 6, 4, 10)
    lat = Lattice(dims)
    U = si.gauge_field(dims, 0.25, 3)
    psi = si.gaussian_spinor(dims, 7)
    g = ovl.Geometry(dims)
    gauge = gu.make_gauge(g, U)
    inp = gu.pack(g, psi, ovl.OVL_F64)
    out = gu.empty_field(g, ovl.OVL_F64)
    ovl.ovl_hw_apply(out, inp, gauge, 1.5, ovl.OVL_F64, 1, None)
    got = gu.unpack(g, out, ovl.OVL_F64)
    assert gu.max_rel_err(got, dirac.hw_apply(lat, U, psi, 1.5)) < 1e-13


def test_not_su3_rejected():
    dims = (4, 4, 4, 4)
    U = si.gauge_field(dims, 0.3, 1)
    U[5, 2] *= 1.01
    g = ovl.Geometry(dims)
    gauge = gu.make_gauge(g, U)
    with pytest.raises(ovl.OvlError) as e:
        gauge.set_repr(ovl.OVL_F16, 1)
    assert e.value.name == "OVL_E_NOT_SU3"
    gauge.set_repr(ovl.OVL_F16, 0)  # 18 reals need no SU(3) structure


def test_dslash_full_size_24x64():
    """The 24^3 x 64 lattice: GPU FP64 stencil against the oracle on every site."""
    dims = (24, 24, 24, 64)
    got, want = _dslash_case(dims, ovl.OVL_F64, 0, -1.5, 2, seed=5)
    assert gu.max_rel_err(got, want) < 1e-13


@pytest.mark.parametrize("prec", PRECS)
def test_every_vectors_per_thread_shape(prec):
    """Static shapes KR = 1..4 (batch sizes 1..4) and a tuned 12-rhs batch all
    give the same values as one-vector calls."""
    dims = (6, 6, 6, 8)
    lat = Lattice(dims)
    U = si.gauge_field(dims, 0.25, 4)
    g = ovl.Geometry(dims)
    gauge = gu.make_gauge(g, U, [] if prec == ovl.OVL_F64 else [(prec, 1)])
    psi = np.stack([si.gaussian_spinor(dims, 300 + r) for r in range(12)])
    inp = gu.pack(g, psi, prec, 12)
    vb = g.spinor_bytes(prec)
    single = gu.empty_field(g, prec, 12)
    ovl.ovl_stencil_tune(0)
    try:
        for r in range(12):
            ovl.ovl_dslash(single[r * vb:], inp[r * vb:], gauge, -0.3, 2, prec, 1, None)
        want = gu.unpack(g, single, prec, 12)
        for nrhs in (2, 3, 4):
            if prec == ovl.OVL_F64 and nrhs > 2:
                continue
            out = gu.empty_field(g, prec, nrhs)
            ovl.ovl_dslash(out, inp, gauge, -0.3, 2, prec, nrhs, None)
            got = gu.unpack(g, out, prec, nrhs)
            assert gu.max_rel_err(got, want[:nrhs]) <= 2 * gu.UNIT_ROUNDOFF[prec]
    finally:
        ovl.ovl_stencil_tune(1)
    out = gu.empty_field(g, prec, 12)
    ovl.ovl_dslash(out, inp, gauge, -0.3, 2, prec, 12, None)
    kr, bs, pipe, rin, tm = ovl.stencil_shape(g, prec, prec != ovl.OVL_F64, 0, 12)
    assert kr in (1, 2, 3, 4) and bs in (32, 64, 128, 256) and pipe in (0, 2, 3, 4) and rin in (0, 1)
    assert tm in (0, 1)
    got = gu.unpack(g, out, prec, 12)
    assert gu.max_rel_err(got, want) <= 2 * gu.UNIT_ROUNDOFF[prec]
    ref = dirac.wilson_dslash(lat, U, psi[5], -0.3)
    assert gu.rel_err(got[5], ref) < 16 * gu.UNIT_ROUNDOFF[prec] + 4e-7


def _shape_candidates(prec, nrhs):
    kmax = 2 if prec == ovl.OVL_F64 else 4
    out = []
    # block orders: by h, t-major, z-slabs of 2, 4 (ragged last slab on
    # Lz = 6), 5 (ragged) and 6 planes
    for tm in (0, 1, 2, 4, 5, 6):
        for kr in range(1, kmax + 1):
            if nrhs % kr:
                continue
            out += [(kr, 128, 0, 0, tm), (kr, 256, 0, 0, tm)]
            if nrhs > kr:
                out += [(kr, bs, 0, 1, tm) for bs in (32, 64) if bs * (nrhs // kr) <= 512]
        for dep in ((2,) if prec == ovl.OVL_F64 else (2, 3, 4)):
            out += [(1, 128, dep, 0, tm), (1, 256, dep, 0, tm)]
    return out


@pytest.mark.parametrize("prec", PRECS)
def test_every_pinned_shape(prec):
    """Every shape the tuner may pick (vectors per thread, side-by-side groups,
    pipelined loads), pinned in turn on a 12-rhs H_w batch, matches the same
    batch under the static default shape."""
    dims = (6, 6, 6, 10)
    U = si.gauge_field(dims, 0.25, 8)
    g = ovl.Geometry(dims)
    c12 = prec != ovl.OVL_F64
    gauge = gu.make_gauge(g, U, [(prec, 1)] if c12 else [])
    psi = np.stack([si.gaussian_spinor(dims, 500 + r) for r in range(12)])
    inp = gu.pack(g, psi, prec, 12)
    ovl.ovl_stencil_tune(0)
    try:
        ref = gu.empty_field(g, prec, 12)
        ovl.ovl_hw_apply(ref, inp, gauge, 1.4, prec, 12, None)
        want = gu.unpack(g, ref, prec, 12)
        for shape in _shape_candidates(prec, 12):
            ovl.stencil_set_shape(g, prec, c12, 0, 12, shape)
            assert ovl.stencil_shape(g, prec, c12, 0, 12) == shape
            out = gu.empty_field(g, prec, 12)
            ovl.ovl_hw_apply(out, inp, gauge, 1.4, prec, 12, None)
            got = gu.unpack(g, out, prec, 12)
            assert gu.max_rel_err(got, want) <= 2 * gu.UNIT_ROUNDOFF[prec], shape
        # unsupported block size, kr, block above 512 threads, pipelined kr > 1,
        # pipeline depth, rin flag, slab thicker than Lz = 6
        for bad in [(1, 96, 0, 0, 0), (5, 128, 0, 0, 0), (1, 64, 0, 1, 0), (2, 128, 2, 0, 0), (1, 128, 5, 0, 0),
                    (1, 128, 0, 2, 0), (1, 128, 0, 0, 7)]:
            with pytest.raises(ovl.OvlError):
                ovl.stencil_set_shape(g, prec, c12, 0, 12, bad)
    finally:
        ovl.ovl_stencil_tune(1)


def test_mem_stats_counts_links():
    """The library's device-memory accounting follows the packed links: the
    FP64 master copy (18 reals of 8 bytes per link) plus an F16 12-real copy
    (2 bytes per real), and both are returned when the gauge is destroyed."""
    dims = (4, 4, 4, 6)
    g = ovl.Geometry(dims)
    U = si.gauge_field(dims, 0.25, 8)
    # a first gauge leaves the workspace buffers its checks use in the pool
    del_me = gu.make_gauge(g, U, [(ovl.OVL_F16, 1)])
    del del_me
    live, peak = ctypes.c_int64(), ctypes.c_int64()
    ovl.ovl_mem_stats(None, None, 1)  # peak := live
    ovl.ovl_mem_stats(ctypes.byref(live), ctypes.byref(peak), 0)
    live0 = live.value
    assert peak.value == live0
    gauge = gu.make_gauge(g, U, [(ovl.OVL_F16, 1)])
    ovl.ovl_mem_stats(ctypes.byref(live), ctypes.byref(peak), 0)
    links = 4 * g.N * (18 * 8 + 12 * 2)
    assert live.value - live0 == links
    assert peak.value >= live.value
    del gauge
    ovl.ovl_mem_stats(ctypes.byref(live), ctypes.byref(peak), 0)
    assert live.value == live0
    assert peak.value >= live0 + links
