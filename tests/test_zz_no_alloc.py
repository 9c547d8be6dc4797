"""The allocation-free projection entry point against the allocating one.

ovl_lowmodes_project_noalloc keeps its scratch in a static per-device array
instead of the workspace pool.  Two calls in a row, the second on a smaller
input, must each reproduce ovl_lowmodes_project (bit-identical while the
split-K partial sums fit the array at full count, to rounding otherwise),
and no call may change the library's device-memory accounting.
"""
import ctypes

import numpy as np
import pytest

import synth_inputs as si

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from paper_1106_4964_amd import ovl  # noqa: E402

import gpu_util as gu  # noqa: E402


def _live_bytes():
    live = ctypes.c_int64()
    ovl.ovl_mem_stats(ctypes.byref(live), None, 0)
    return live.value


def _case(g, dims, ell, nrhs, prec, seed):
    V = si.orthonormal_spinors(dims, ell, seed=seed)
    lam = np.linspace(-0.9, 0.8, ell)
    lm = ovl.LowModes(g, gu.pack(g, V, ovl.OVL_F64, ell), lam)
    psi = np.stack([si.gaussian_spinor(dims, seed + 100 + r) for r in range(nrhs)])
    inp = gu.pack(g, psi, prec, nrhs)
    outs = [gu.empty_field(g, prec, nrhs) for _ in range(4)]
    return lm, inp, outs


def _run_pair(g, lm, inp, outs, prec, nrhs):
    ref_h, ref_w, got_h, got_w = outs
    ovl.ovl_lowmodes_project(lm, inp, ref_h, ref_w, prec, nrhs, None)
    torch.cuda.synchronize()
    before = _live_bytes()
    ovl.ovl_lowmodes_project_noalloc(lm, inp, got_h, got_w, prec, nrhs, None)
    torch.cuda.synchronize()
    assert _live_bytes() == before, "the no-alloc projection changed the library's device memory"
    return [gu.unpack(g, t, prec, nrhs).reshape(nrhs, -1) for t in (ref_h, ref_w, got_h, got_w)]


@pytest.mark.parametrize("prec", [ovl.OVL_F64, ovl.OVL_F16])
def test_noalloc_projection_two_calls(prec):
    dims = (6, 6, 6, 8)
    g = ovl.Geometry(dims)
    # first call: ell * nrhs = 2400 > 2044, so the static scratch holds fewer
    # K-blocks than the pooled path: equal to rounding
    lm1, inp1, outs1 = _case(g, dims, 200, 12, prec, seed=11)
    rh, rw, gh, gw = _run_pair(g, lm1, inp1, outs1, prec, 12)
    tol = 1e-13 if prec == ovl.OVL_F64 else 2.0 ** -10
    for r in range(12):
        assert gu.max_rel_err(gh[r], rh[r]) < tol
        assert gu.max_rel_err(gw[r], rw[r]) < tol
    # second call, smaller input (ell * nrhs = 63): the same K-blocks as the
    # pooled path, so bit-identical, and nothing left over from call 1 leaks in
    lm2, inp2, outs2 = _case(g, dims, 21, 3, prec, seed=23)
    rh, rw, gh, gw = _run_pair(g, lm2, inp2, outs2, prec, 3)
    assert np.array_equal(gh, rh) and np.array_equal(gw, rw)


def test_noalloc_projection_rejects_too_large():
    dims = (2, 2, 2, 2)
    g = ovl.Geometry(dims)
    ell = 1400  # ell * 12 = 16800 > 16131
    V = gu.empty_field(g, ovl.OVL_F64, ell)
    V.zero_()
    lm = ovl.LowModes(g, V, np.ones(ell))
    x = gu.empty_field(g, ovl.OVL_F64, 12)
    h = gu.empty_field(g, ovl.OVL_F64, 12)
    w = gu.empty_field(g, ovl.OVL_F64, 12)
    with pytest.raises(ovl.OvlError) as e:
        ovl.ovl_lowmodes_project_noalloc(lm, x, h, w, ovl.OVL_F64, 12, None)
    assert e.value.name == "OVL_E_ARG" and "16131" in str(e.value)
