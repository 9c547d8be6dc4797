"""CPU-side checks of the C-ABI library: it loads, exports every symbol the
header declares, and rejects bad arguments before touching the GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ovl.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ovl_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_1106_4964_amd import ovl

    names = declared_symbols()
    assert len(names) > 15
    missing = [n for n in names if not hasattr(ovl.lib, n)]
    assert not missing, missing
    # and the binding wraps each of them under the same name
    assert not [n for n in names if not hasattr(ovl, n)]


def test_geometry_errors_and_indices():
    from paper_1106_4964_amd import ovl

    for bad in [(3, 4, 4, 4), (4, 4, 4, 0), (4, 1, 4, 4)]:
        with pytest.raises(ovl.OvlError) as e:
            ovl.Geometry(bad)
        assert e.value.name == "OVL_E_DIMS"
    g = ovl.Geometry((4, 4, 4, 4))
    assert g.N == 256
    assert g.eo_index((1, 0, 0, 0)) == 128
    assert g.eo_index((3, 3, 3, 3)) == 127
    assert g.eo_index((1, 2, 3, 1)) == 188
    with pytest.raises(ovl.OvlError):
        g.eo_index((4, 0, 0, 0))


def test_spinor_bytes():
    from paper_1106_4964_amd import ovl

    g = ovl.Geometry((4, 4, 4, 6))
    assert g.spinor_bytes(ovl.OVL_F64) == 384 * 192
    assert g.spinor_bytes(ovl.OVL_F32, 12) == 12 * 384 * 96
    assert g.spinor_bytes(ovl.OVL_F16) == 384 * 48
    assert g.spinor_bytes(ovl.OVL_BF16) == 384 * 48
    with pytest.raises(ovl.OvlError):
        g.spinor_bytes(7)
    with pytest.raises(ovl.OvlError):
        g.spinor_bytes(ovl.OVL_F64, 0)


def test_null_and_alias_arguments_rejected_without_gpu():
    from paper_1106_4964_amd import ovl

    g = ovl.Geometry((4, 4, 4, 4))
    with pytest.raises(ovl.OvlError) as e:
        ovl.ovl_dslash(None, None, None, 0.0, 2, ovl.OVL_F64, 1, 0)
    assert e.value.name == "OVL_E_ARG"
    with pytest.raises(ovl.OvlError) as e:
        ovl.ovl_pack_spinor(g, 0x1000, 0x1000, ovl.OVL_F64, 1, 0)
    assert e.value.name == "OVL_E_ALIAS"
    with pytest.raises(ovl.OvlError) as e:
        ovl.ovl_convert(g, 0x1000, ovl.OVL_F64, 0x1000, ovl.OVL_F32, 1, 0)
    assert e.value.name == "OVL_E_ALIAS"


@pytest.mark.parametrize("n", [1, 2, 7, 40, 120])
def test_host_heev_against_numpy(n):
    """The host Jacobi eigensolver used by the GPU eigensolver, vs numpy.linalg.eigh."""
    import numpy as np

    from paper_1106_4964_amd import ovl

    rng = np.random.default_rng(n)
    a = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    h = a + a.conj().T
    if n > 5:
        h[0, 1] = h[1, 0] = 0.0  # a zero off-diagonal entry
    A = np.asfortranarray(h).astype(np.complex128)
    w = np.zeros(n)
    V = np.zeros((n, n), dtype=np.complex128, order="F")
    ovl.ovl_host_heev(n, A.ctypes.data, w, V.ctypes.data)
    wn = np.linalg.eigvalsh(h)
    assert np.max(np.abs(w - wn)) < 1e-12 * max(1.0, np.max(np.abs(wn)))
    assert np.max(np.abs(h @ V - V * w)) < 1e-11 * max(1.0, np.max(np.abs(wn)))
    assert np.max(np.abs(V.conj().T @ V - np.eye(n))) < 1e-13


@pytest.mark.parametrize("n,lo,hi", [(6, 0.2, 1.0), (8, 0.44, 6.3), (12, 0.05, 6.5)])
def test_rational_coefficients_match_the_oracle(n, lo, hi):
    """The library's Zolotarev coefficients (its own AGM elliptic functions)
    equal the oracle's (scipy's), and its measured delta matches (cases
    with delta far above rounding)."""
    from oracle import rational as ra
    from paper_1106_4964_amd import ovl

    r = ovl.Rational(lo, hi, n)
    o = ra.make_rational(lo, hi, n)
    assert np.max(np.abs(r.c / o.c - 1.0)) < 1e-10
    assert np.max(np.abs(r.b / o.b - 1.0)) < 1e-9
    assert abs(r.delta / ra.measure_delta(o) - 1.0) < 1e-3
    with pytest.raises(ovl.OvlError):
        ovl.Rational(lo, hi, 0)
    with pytest.raises(ovl.OvlError):
        ovl.Rational(hi, lo, 4)
