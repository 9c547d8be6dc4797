"""Gauge-equivariant parallel-transport convolution (PTC) layer (oracle).

Test infrastructure.  Not part of arXiv:1106.4964: a small learned
preconditioner for D(m) whose layers are built from the same parallel
transporters T_mu as the Wilson operator (eq. 2, without spin projector).

Layer (linear, no activation, so gauge equivariance is exact):
  phi_out[a](x) = sum_b sum_k W[k,a,b] (T_k phi_in[b])(x)
  k = 0 (identity), 1..4 (+x,+y,+z,+t), 5..8 (-x,-y,-z,-t)
  T_{+mu} phi(x) = U_mu(x) phi(x+mu),  T_{-mu} phi(x) = U_mu(x-mu)^dag phi(x-mu)
  W[k,a,b] is a complex 4x4 matrix acting on spin.
Shapes: phi [C, N, 4, 3], W [9, C_out, C_in, 4, 4].

Gradients use the convention grad z = dL/dRe z + i dL/dIm z for a real
loss L.  For phi_out = A phi_in the input gradient is A^dag g_out, with
T_{+mu}^dag = T_{-mu}; the weight gradient is
  G[k,a,b] = sum_x sum_colour g_out[a](x) (T_k phi_in[b](x))^dag   (4x4).
With one channel and W_0 = (4+m) 1, W_{+mu} = -(1-gamma_mu)/2,
W_{-mu} = -(1+gamma_mu)/2 the layer is D_w(m).
"""
from __future__ import annotations

import numpy as np

from . import dirac
from .lattice import Lattice

NPATH = 9


def path_transport(lat: Lattice, U, phi, k: int):
    """T_k phi for one channel (k as in the module docstring)."""
    if k == 0:
        return np.asarray(phi).reshape(lat.N, 4, 3).copy()
    d = (k - 1) if k <= 4 else (k - 5) + 4
    return dirac.transport(lat, U, phi, d)


def adjoint_path(k: int) -> int:
    if k == 0:
        return 0
    return k + 4 if k <= 4 else k - 4


def forward(lat: Lattice, U, W, phi_in):
    W = np.asarray(W)
    cout, cin = W.shape[1], W.shape[2]
    out = np.zeros((cout, lat.N, 4, 3), dtype=np.complex128)
    for b in range(cin):
        for k in range(NPATH):
            x = path_transport(lat, U, phi_in[b], k)
            for a in range(cout):
                out[a] += dirac.spin_mul(W[k, a, b], x)
    return out


def backward(lat: Lattice, U, W, phi_in, g_out):
    """Returns (g_in [C_in,N,4,3], g_W [9,C_out,C_in,4,4])."""
    W = np.asarray(W)
    cout, cin = W.shape[1], W.shape[2]
    g_in = np.zeros((cin, lat.N, 4, 3), dtype=np.complex128)
    g_W = np.zeros_like(W, dtype=np.complex128)
    for b in range(cin):
        for k in range(NPATH):
            x = path_transport(lat, U, phi_in[b], k)
            for a in range(cout):
                # sum over sites and colour of g_out[a][s,c] conj(x[t,c])
                g_W[k, a, b] = np.einsum("nsc,ntc->st", g_out[a], x.conj())
                y = dirac.spin_mul(W[k, a, b].conj().T, g_out[a])
                g_in[b] += path_transport(lat, U, y, adjoint_path(k))
    return g_in, g_W


def wilson_weights(m: float) -> np.ndarray:
    """Weights [9,1,1,4,4] that make one layer equal to D_w(m)."""
    W = np.zeros((NPATH, 1, 1, 4, 4), dtype=np.complex128)
    W[0, 0, 0] = (4.0 + m) * dirac.ID4
    for mu in range(4):
        W[1 + mu, 0, 0] = -0.5 * (dirac.ID4 - dirac.GAMMA[mu])
        W[5 + mu, 0, 0] = -0.5 * (dirac.ID4 + dirac.GAMMA[mu])
    return W


def net_forward(lat, U, weights, b):
    """Two-layer net 1 -> C -> 1 on a single field b [N,4,3]; returns
    (output [N,4,3], hidden [C,N,4,3])."""
    w1, w2 = weights
    h = forward(lat, U, w1, np.asarray(b).reshape(1, lat.N, 4, 3))
    out = forward(lat, U, w2, h)
    return out[0], h


def net_loss_and_grad(lat, U, weights, b, x):
    """L = ||M b - x||^2 / ||x||^2 and its weight gradients (g_w1, g_w2)."""
    w1, w2 = weights
    out, h = net_forward(lat, U, weights, b)
    xn2 = float(np.vdot(x, x).real)
    diff = out - np.asarray(x).reshape(lat.N, 4, 3)
    loss = float(np.vdot(diff, diff).real) / xn2
    g_out = (2.0 / xn2) * diff.reshape(1, lat.N, 4, 3)
    g_h, g_w2 = backward(lat, U, w2, h, g_out)
    _, g_w1 = backward(lat, U, w1, np.asarray(b).reshape(1, lat.N, 4, 3), g_h)
    return loss, (g_w1, g_w2)
