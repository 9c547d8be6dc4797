"""Helpers for GPU tests: move seeded numpy fields through the C ABI."""
import numpy as np
import torch

from paper_1106_4964_amd import ovl

DEV = torch.device("cuda:0")


def stream():
    return torch.cuda.current_stream().cuda_stream


def to_dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def empty_field(geom, prec, nrhs=1) -> torch.Tensor:
    return torch.empty(geom.spinor_bytes(prec, nrhs), dtype=torch.uint8, device=DEV)


def pack(geom, aos: np.ndarray, prec, nrhs=1) -> torch.Tensor:
    src = to_dev(aos.astype(np.complex128))
    out = empty_field(geom, prec, nrhs)
    ovl.ovl_pack_spinor(geom, src, out, prec, nrhs, None)
    torch.cuda.synchronize()
    return out


def unpack(geom, dev: torch.Tensor, prec, nrhs=1) -> np.ndarray:
    out = torch.empty((nrhs, geom.N, 4, 3), dtype=torch.complex128, device=DEV)
    ovl.ovl_unpack_spinor(geom, dev, out, prec, nrhs, None)
    torch.cuda.synchronize()
    res = out.cpu().numpy()
    return res[0] if nrhs == 1 else res


def make_gauge(geom, U: np.ndarray, reprs=()):
    g = ovl.Gauge(geom, to_dev(U))
    for prec, c12 in reprs:
        g.set_repr(prec, c12)
    torch.cuda.synchronize()
    return g


def rel_err(got, want):
    return float(np.linalg.norm((np.asarray(got) - np.asarray(want)).ravel()) / np.linalg.norm(np.asarray(want).ravel()))


def max_rel_err(got, want):
    """Max |got - want| over elements, relative to max |want|."""
    return float(np.max(np.abs(np.asarray(got) - np.asarray(want))) / np.max(np.abs(np.asarray(want))))


# Unit roundoff of each storage precision: the tolerance of a low-precision
# stencil result is a small multiple of it (input, link and output rounding,
# each amplified by at most the O(10) norm of D_w relative to its output).
UNIT_ROUNDOFF = {ovl.OVL_F64: 2.0 ** -53, ovl.OVL_F32: 2.0 ** -24, ovl.OVL_F16: 2.0 ** -11, ovl.OVL_BF16: 2.0 ** -8}
