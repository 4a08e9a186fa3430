"""The P-predictor in float64 (oracle; test infrastructure only).

The paper parameterises the basis with a network followed by a thin QR
(Sec. 4, neural parameterisation; the prolongation is qf of the prediction).
The GPU build's network is a small CNN on the coefficient field:

    x_b   = [ (log a_b - mean) / std , Phi_k ]          (1 + k channels)
    P_hat = Phi_k + conv4(g(conv3(g(conv2(g(conv1(x_b)))))))
    P     = qf(P_hat)                                  (thin QR, diag(R) > 0)

with 3x3 'same' convolutions (cross-correlation, zero padding, bias), g the
erf-GELU, and Phi_k the k smoothest sine modes of the unit square
sin(i pi x) sin(j pi y) (ordered by i^2 + j^2, ties by i) at the cell centres,
scaled to unit 2-norm.  Parameters are one flat vector: for each layer
W (Cout, Cin, 3, 3) then b (Cout).

Steps are library primitives (torch's conv2d on the CPU in float64, numpy's
QR) and the formulas of the thin-QR backward and of Adam, written out.
"""
from __future__ import annotations

import math

import numpy as np
import torch

__all__ = ["smooth_modes", "sine_modes", "layer_shapes", "param_count", "cnn_input", "cnn_forward",
           "qf", "qr_backward", "adam_update"]


def smooth_modes(k: int):
    """The k pairs (i, j), i, j >= 1, with the smallest i^2 + j^2, ties by i."""
    pairs = sorted(((i * i + j * j, i, j) for i in range(1, 65) for j in range(1, 65)))
    return [(i, j) for _, i, j in pairs[:k]]


def sine_modes(N: int, k: int) -> np.ndarray:
    """Phi (N*N, k): column (i, j) = (2/N) sin(i pi x) sin(j pi y) at the cell
    centres x = (c + 1/2)/N, cell index x fastest."""
    c = (np.arange(N) + 0.5) / N
    cols = []
    for i, j in smooth_modes(k):
        cols.append((np.sin(j * np.pi * c)[:, None] * np.sin(i * np.pi * c)[None, :]).ravel() * (2.0 / N))
    return np.stack(cols, axis=1)


def layer_shapes(k: int, hidden: int):
    return [(hidden, 1 + k), (hidden, hidden), (hidden, hidden), (k, hidden)]


def param_count(k: int, hidden: int) -> int:
    return sum(co * ci * 9 + co for co, ci in layer_shapes(k, hidden))


def _unpack(params, k, hidden):
    out, off = [], 0
    p = torch.as_tensor(params, dtype=torch.float64)
    for co, ci in layer_shapes(k, hidden):
        W = p[off:off + co * ci * 9].reshape(co, ci, 3, 3)
        off += co * ci * 9
        b = p[off:off + co]
        off += co
        out.append((W, b))
    return out


def cnn_input(coef: np.ndarray, N: int, k: int) -> np.ndarray:
    """x (batch, 1 + k, N, N): standardised log a (population std) and Phi."""
    batch = coef.shape[0]
    la = np.log(coef.reshape(batch, N * N))
    mean = la.mean(axis=1, keepdims=True)
    std = np.sqrt(np.maximum((la * la).mean(axis=1, keepdims=True) - mean * mean, 0.0))
    std[std == 0] = 1.0
    phi = sine_modes(N, k)
    x = np.empty((batch, 1 + k, N, N))
    x[:, 0] = ((la - mean) / std).reshape(batch, N, N)
    x[:, 1:] = phi.T.reshape(1, k, N, N)
    return x


def cnn_forward(params, coef: np.ndarray, N: int, k: int, hidden: int, return_graph: bool = False):
    """P_hat (batch, N*N, k) in float64.  With return_graph, also the torch
    tensors (params leaf, P_hat) for gradients by autograd."""
    p = torch.tensor(np.asarray(params, dtype=np.float64), requires_grad=return_graph)
    layers = _unpack(p, k, hidden)
    h = torch.tensor(cnn_input(coef, N, k))
    for l, (W, b) in enumerate(layers):
        z = torch.nn.functional.conv2d(h, W, b, padding=1)
        h = torch.nn.functional.gelu(z) if l < 3 else z
    phi = torch.tensor(sine_modes(N, k))
    Phat = phi.unsqueeze(0) + h.reshape(h.shape[0], k, N * N).transpose(1, 2)
    if return_graph:
        return p, Phat
    return Phat.detach().numpy()


def qf(A: np.ndarray):
    """Thin QR with positive diagonal of R: (Q, R)."""
    Q, R = np.linalg.qr(A)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s[None, :], R * s[:, None]


def qr_backward(Q: np.ndarray, R: np.ndarray, gQ: np.ndarray) -> np.ndarray:
    """dL/dA for L depending on A only through Q = qf(A):
    dA = [gQ + Q copyltu(M)] R^-T,  M = -gQ^T Q,
    copyltu(M) = tril(M) + tril(M, -1)^T.  From dQ = dA R^-1 - Q dR R^-1 and
    Q^T dQ antisymmetric with R upper triangular (differentiating A = QR)."""
    M = -gQ.T @ Q
    C = np.tril(M) + np.tril(M, -1).T
    X = gQ + Q @ C
    return np.linalg.solve(R, X.T).T


def adam_update(p, g, m, v, lr, step, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam step; returns (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
