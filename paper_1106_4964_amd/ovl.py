"""ctypes binding of libovl.so (argument marshalling only).

Every `ovl_*` function here has the name and argument order of the C
function in include/ovl.h.  Pointer arguments accept a torch tensor (its
data_ptr is passed), a ctypes object, an int address, or None (NULL).  A
stream argument of None means torch's current HIP stream.  Negative status
codes raise OvlError; the function returns the (non-negative) status.

All compute runs in the HIP library.  If libovl.so is missing the import of
this module fails: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libovl.so")

OVL_F64, OVL_F32, OVL_F16, OVL_BF16 = 0, 1, 2, 3
PREC = {"f64": OVL_F64, "f32": OVL_F32, "f16": OVL_F16, "bf16": OVL_BF16}
OVL_OK = 0
OVL_W_NOT_CONVERGED = 1
ERRORS = {
    -1: "OVL_E_ARG", -2: "OVL_E_DIMS", -3: "OVL_E_PRECISION", -4: "OVL_E_ALIAS", -5: "OVL_E_HIP",
    -6: "OVL_E_NOT_SU3", -7: "OVL_E_BREAKDOWN", -8: "OVL_E_NAN", -9: "OVL_E_NOMEM", -10: "OVL_E_STATE",
}
OVL_MAX_RHS = 12


class OvlError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "?"), code, msg))
        self.code = code
        self.name = ERRORS.get(code, "?")


if not os.path.exists(LIB_PATH):
    raise ImportError(
        "libovl.so is not built (%s); run `python -m paper_1106_4964_amd.build` first" % LIB_PATH
    )


def _init_torch_device():
    """torch ships its own HIP runtime; libovl.so binds to whichever HIP
    runtime is already loaded.  The device must be initialised by torch
    before the library registers its kernels, or the two initialisations
    collide and the library sees no device."""
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.is_available():
        torch.cuda.init()


_init_torch_device()
lib = ctypes.CDLL(LIB_PATH)

P = ctypes.c_void_p
I = ctypes.c_int
D = ctypes.c_double
I64 = ctypes.c_int64
SZ = ctypes.c_size_t


ST = "stream"  # marker: a hipStream_t argument (None = torch's current stream)


class SolveOpts(ctypes.Structure):
    _fields_ = [
        ("inner_prec", ctypes.c_int),
        ("inner_tol", ctypes.c_double),
        ("graph_chunk", ctypes.c_int),
        ("check_every", ctypes.c_int),
        ("max_restarts", ctypes.c_int),
        ("harvest_x", ctypes.c_void_p),
        ("harvest_b", ctypes.c_void_p),
        ("harvest_cap", ctypes.c_int),
        ("inner_sign", ctypes.c_void_p),
        ("chiral", ctypes.c_int),
        ("deflation", ctypes.c_void_p),
        ("harvest_stride", ctypes.c_int),
        ("relax_signs", ctypes.c_void_p),
        ("n_relax", ctypes.c_int),
    ]


class EigStats(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int),
        ("hw_applies", ctypes.c_int64),
        ("max_residual", ctypes.c_double),
        ("seconds", ctypes.c_double),
    ]


class SolveStats(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int),
        ("restarts", ctypes.c_int),
        ("true_residual", ctypes.c_double * 12),
        ("seconds", ctypes.c_double),
        ("sign_applies", ctypes.c_int64),
        ("dslash_applies", ctypes.c_int64),
        ("fallback_used", ctypes.c_int),
        ("harvested", ctypes.c_int),
        ("deflation_dropped", ctypes.c_int),
    ]


def _sig(name, *args):
    fn = getattr(lib, name)
    fn.argtypes = list(args)
    fn.restype = I
    return fn


lib.ovl_last_error.restype = ctypes.c_char_p
lib.ovl_last_error.argtypes = []
lib.ovl_version.restype = I

_SIGS = {
    "ovl_geom_create": (P, P),
    "ovl_geom_destroy": (P,),
    "ovl_geom_volume": (P, P),
    "ovl_geom_eo_index": (P, P, P),
    "ovl_geom_neighbors_device": (P, P, ST),
    "ovl_spinor_bytes": (P, I, I, P),
    "ovl_pack_spinor": (P, P, P, I, I, ST),
    "ovl_unpack_spinor": (P, P, P, I, I, ST),
    "ovl_gauge_create": (P, P, ST, P),
    "ovl_gauge_set_repr": (P, I, I, ST),
    "ovl_gauge_destroy": (P,),
    "ovl_dslash": (P, P, P, D, I, I, I, ST),
    "ovl_hw_apply": (P, P, P, D, I, I, ST),
    "ovl_axpy": (P, P, P, P, I, I, ST),
    "ovl_xpay": (P, P, P, P, I, I, ST),
    "ovl_dot": (P, P, P, I, I, P, ST),
    "ovl_norm2": (P, P, I, I, P, ST),
    "ovl_convert": (P, P, I, P, I, I, ST),
    "ovl_sign_create": (D, D, D, I, P),
    "ovl_sign_destroy": (P,),
    "ovl_sign_info": (P, P, P, P),
    "ovl_sign_coeffs": (P, P, I),
    "ovl_lowmodes_create": (P, I, P, P, P),
    "ovl_lowmodes_destroy": (P,),
    "ovl_lowmodes_project": (P, P, P, P, I, I, ST),
    "ovl_lowmodes_project_noalloc": (P, P, P, P, I, I, ST),
    "ovl_sign_apply": (P, P, P, D, P, P, I, I, ST),
    "ovl_overlap_apply": (P, P, P, D, D, P, P, I, I, I, ST),
    "ovl_rational_create": (D, D, I, P),
    "ovl_rational_destroy": (P,),
    "ovl_rational_coeffs": (P, P, P, I, P, P),
    "ovl_rational_sign_apply": (P, P, P, D, P, P, I, D, I, P, ST),
    "ovl_cg_solve": (P, P, I, P, D, D, P, P, D, I, P, P, ST),
    "ovl_cg_multimass": (P, P, I, P, D, P, I, P, P, D, I, P, P, ST),
    "ovl_propagator": (P, P, P, D, P, P, I, I, ST),
    "ovl_counters": (P, P, I),
    "ovl_mem_stats": (P, P, I),
    "ovl_stencil_tune": (I,),
    "ovl_stencil_timer": (I,),
    "ovl_stencil_timer_read": (I, I, I, I, P, P),
    "ovl_stencil_shape": (P, I, I, I, I, P),
    "ovl_stencil_set_shape": (P, I, I, I, I, P),
    "ovl_hw_bound": (P, D, P, I, P, P, P, ST),
    "ovl_hw_eigs": (P, D, I, I, P, P, D, D, I, I, P, ST),
    "ovl_host_heev": (I, P, P, P),
    "ovl_overlap_eigs": (P, D, P, P, I, I, I, I, P, P, P, D, I, P, ST),
    "ovl_deflation_create": (P, I, P, P, P),
    "ovl_deflation_destroy": (P,),
    "ovl_deflation_prepare": (P, P, D, P, P, P, ST),
    "ovl_fgcr_solve": (P, P, I, P, D, D, P, P, P, I, D, I, P, P, ST),
    "ovl_net_create": (P, I, P),
    "ovl_net_destroy": (P,),
    "ovl_net_set_weights": (P, P, P),
    "ovl_net_get_weights": (P, P, P),
    "ovl_ptc_layer_forward": (P, P, I, P, I, P, ST),
    "ovl_ptc_layer_backward": (P, P, I, P, I, P, P, P, ST),
    "ovl_net_train": (P, P, P, P, I, I, I, D, P, P, ST),
    "ovl_net_apply": (P, P, P, P, ST),
}

EXPORTED = ["ovl_last_error", "ovl_version", "ovl_gauge_geom"] + list(_SIGS)


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "handle"):
        return x.handle.value
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    if isinstance(x, ctypes.c_void_p):
        return x.value
    if isinstance(x, ctypes.Structure):
        return ctypes.addressof(x)
    return ctypes.cast(x, ctypes.c_void_p).value


def _stream(s):
    if s is None:
        import torch

        return torch.cuda.current_stream().cuda_stream
    if hasattr(s, "cuda_stream"):
        return s.cuda_stream
    return int(s)


def _wrap(name, argtypes):
    fn = _sig(name, *[P if t is ST else t for t in argtypes])

    def call(*args):
        if len(args) != len(argtypes):
            raise TypeError("%s takes %d arguments (%d given)" % (name, len(argtypes), len(args)))
        conv = []
        for a, t in zip(args, argtypes):
            if t is ST:
                conv.append(_stream(a))
            elif t is P:
                conv.append(_ptr(a))
            else:
                conv.append(a)
        code = fn(*conv)
        if code < 0:
            raise OvlError(code, lib.ovl_last_error().decode())
        return code

    call.__name__ = name
    return call


for _n, _a in _SIGS.items():
    globals()[_n] = _wrap(_n, _a)

lib.ovl_gauge_geom.restype = P
lib.ovl_gauge_geom.argtypes = [P]


def ovl_gauge_geom(u):
    return lib.ovl_gauge_geom(_ptr(u))


def ovl_last_error():
    return lib.ovl_last_error().decode()


def ovl_version():
    return lib.ovl_version()


# ---------------------------------------------------------------------------
# Small RAII helpers around the handles (still only marshalling).
# ---------------------------------------------------------------------------
class Geometry:
    def __init__(self, dims):
        d = (ctypes.c_int32 * 4)(*[int(v) for v in dims])
        h = ctypes.c_void_p()
        ovl_geom_create(d, ctypes.byref(h))
        self.handle = h
        self.dims = tuple(int(v) for v in dims)
        n = ctypes.c_int64()
        ovl_geom_volume(h, ctypes.byref(n))
        self.N = n.value

    @property
    def _as_parameter_(self):
        return self.handle

    def spinor_bytes(self, prec, nrhs=1):
        b = ctypes.c_size_t()
        ovl_spinor_bytes(self.handle, prec, nrhs, ctypes.byref(b))
        return b.value

    def eo_index(self, xyzt):
        c = (ctypes.c_int32 * 4)(*xyzt)
        e = ctypes.c_int32()
        ovl_geom_eo_index(self.handle, c, ctypes.byref(e))
        return e.value

    def __del__(self, _lib=lib, _exiting=sys.is_finalizing):
        # at interpreter exit module globals may be gone and the process end
        # releases the device memory anyway
        if _exiting():
            return
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib.ovl_geom_destroy(self.handle)
            self.handle = None


class Gauge:
    """Packed gauge field.  `u_dev` is a device complex128 tensor [N,4,3,3]."""

    def __init__(self, geom: Geometry, u_dev, stream=None):
        h = ctypes.c_void_p()
        ovl_gauge_create(geom.handle, u_dev, stream, ctypes.byref(h))
        self.handle = h
        self.geom = geom

    @property
    def _as_parameter_(self):
        return self.handle

    def set_repr(self, prec, compress12, stream=None):
        ovl_gauge_set_repr(self.handle, prec, int(compress12), stream)

    def __del__(self, _lib=lib, _exiting=sys.is_finalizing):
        # at interpreter exit module globals may be gone and the process end
        # releases the device memory anyway
        if _exiting():
            return
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib.ovl_gauge_destroy(self.handle)
            self.handle = None


class Sign:
    """Polynomial sign approximation (order n, eps, measured delta)."""

    def __init__(self, lam_lo, lam_max, delta=1e-10, n=0):
        h = ctypes.c_void_p()
        ovl_sign_create(float(lam_lo), float(lam_max), float(delta), int(n), ctypes.byref(h))
        self.handle = h
        nn, eps, dl = ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
        ovl_sign_info(h, ctypes.byref(nn), ctypes.byref(eps), ctypes.byref(dl))
        self.n, self.eps, self.delta = nn.value, eps.value, dl.value
        self.lam_max = float(lam_max)

    def coeffs(self):
        c = np.zeros(self.n + 1)
        ovl_sign_coeffs(self.handle, c, self.n + 1)
        return c

    def __del__(self, _lib=lib, _exiting=sys.is_finalizing):
        # at interpreter exit module globals may be gone and the process end
        # releases the device memory anyway
        if _exiting():
            return
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib.ovl_sign_destroy(self.handle)
            self.handle = None


class RationalStats(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int),
        ("hw_applies", ctypes.c_int64),
        ("seconds", ctypes.c_double),
    ]


class Rational:
    """Zolotarev rational approximation of y^{-1/2} on [eps, 1] (host handle)."""

    def __init__(self, lam_lo, lam_max, n):
        h = ctypes.c_void_p()
        ovl_rational_create(float(lam_lo), float(lam_max), int(n), ctypes.byref(h))
        self.handle = h
        self.lam_max = float(lam_max)
        self.n = int(n)
        b, c = np.zeros(self.n), np.zeros(self.n)
        eps, dl = ctypes.c_double(), ctypes.c_double()
        ovl_rational_coeffs(self.handle, b, c, self.n, ctypes.byref(eps), ctypes.byref(dl))
        self.b, self.c, self.eps, self.delta = b, c, eps.value, dl.value

    def __del__(self, _lib=lib, _exiting=sys.is_finalizing):
        if _exiting():
            return
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib.ovl_rational_destroy(self.handle)
            self.handle = None


class LowModes:
    """Borrowed FP64 eigenvectors V (device, ell packed spinors) and eigenvalues."""

    def __init__(self, geom, V_dev, lam):
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        h = ctypes.c_void_p()
        ovl_lowmodes_create(geom.handle, len(lam), V_dev, lam, ctypes.byref(h))
        self.handle = h
        self.V = V_dev  # keep the borrowed buffer alive
        self.ell = len(lam)

    def __del__(self, _lib=lib, _exiting=sys.is_finalizing):
        # at interpreter exit module globals may be gone and the process end
        # releases the device memory anyway
        if _exiting():
            return
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib.ovl_lowmodes_destroy(self.handle)
            self.handle = None


class Net:
    """Two-layer PTC network 1 -> hidden -> 1 (weights held by the library)."""

    def __init__(self, geom, hidden=4):
        h = ctypes.c_void_p()
        ovl_net_create(geom.handle, hidden, ctypes.byref(h))
        self.handle = h
        self.hidden = hidden

    def set_weights(self, w1, w2):
        w1 = np.ascontiguousarray(w1, dtype=np.complex128)
        w2 = np.ascontiguousarray(w2, dtype=np.complex128)
        assert w1.size == 9 * self.hidden * 16 and w2.size == 9 * self.hidden * 16
        ovl_net_set_weights(self.handle, w1, w2)

    def get_weights(self):
        w1 = np.zeros((9, self.hidden, 1, 4, 4), dtype=np.complex128)
        w2 = np.zeros((9, 1, self.hidden, 4, 4), dtype=np.complex128)
        ovl_net_get_weights(self.handle, w1, w2)
        return w1, w2

    def __del__(self, _lib=lib, _exiting=sys.is_finalizing):
        # at interpreter exit module globals may be gone and the process end
        # releases the device memory anyway
        if _exiting():
            return
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib.ovl_net_destroy(self.handle)
            self.handle = None


class Deflation:
    """Borrowed FP64 eigenvectors Xi (device, n packed spinors) and complex eigenvalues d of D."""

    def __init__(self, geom, Xi_dev, d):
        d = np.ascontiguousarray(np.asarray(d, dtype=np.complex128))
        h = ctypes.c_void_p()
        ovl_deflation_create(geom.handle, len(d), Xi_dev, d.view(np.float64), ctypes.byref(h))
        self.handle = h
        self.Xi = Xi_dev  # keep the borrowed buffer alive
        self.n = len(d)
        self.Z = None

    def prepare(self, gauge, rho, sign, lowmodes, Z_dev, stream=None):
        """Minimal-residual form: Z = D(0) Xi into Z_dev (borrowed from then on)."""
        ovl_deflation_prepare(self, gauge, rho, sign, lowmodes, Z_dev, stream)
        self.Z = Z_dev

    def __del__(self, _lib=lib, _exiting=sys.is_finalizing):
        # at interpreter exit module globals may be gone and the process end
        # releases the device memory anyway
        if _exiting():
            return
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib.ovl_deflation_destroy(self.handle)
            self.handle = None


def stencil_shape(geom, prec, compress12, nextra, nrhs):
    """Tuned shape (kr, bs, pipe, rin, tm) of a stencil configuration, zeros if untuned."""
    sh = (ctypes.c_int * 5)()
    ovl_stencil_shape(geom, prec, int(compress12), nextra, nrhs, sh)
    return tuple(sh)


def stencil_set_shape(geom, prec, compress12, nextra, nrhs, shape):
    sh = (ctypes.c_int * 5)(*shape)
    ovl_stencil_set_shape(geom, prec, int(compress12), nextra, nrhs, sh)


def stencil_timer_read(prec, compress12, nextra, nrhs):
    """(launches, summed milliseconds) of one stencil configuration since the last clear."""
    n, ms = ctypes.c_int64(), ctypes.c_double()
    ovl_stencil_timer_read(prec, int(compress12), nextra, nrhs, ctypes.byref(n), ctypes.byref(ms))
    return n.value, ms.value
