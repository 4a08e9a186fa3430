"""Pins for the oracle's P-predictor pieces (CPU only): the sine modes are
orthonormal and are the smoothest Dirichlet eigenvectors, the convolution is
a cross-correlation with the documented weight layout, the network reduces
to Phi + bias with zero weights, the thin-QR backward matches finite
differences and an independent autograd of a library QR, and Adam's first
step moves every parameter by lr against its gradient's sign."""
import numpy as np
import torch

import oracle as O
from oracle import predictor as PR


def test_sine_modes_orthonormal_and_smoothest():
    N, k = 24, 10
    Phi = PR.sine_modes(N, k)
    np.testing.assert_allclose(Phi.T @ Phi, np.eye(k), atol=1e-12)
    assert PR.smooth_modes(4) == [(1, 1), (1, 2), (2, 1), (2, 2)]
    # smoothness order: the Rayleigh quotients in the unit-coefficient FV
    # operator increase with i^2 + j^2
    A = O.fv_harmonic_2d(np.ones((N, N)))
    rq = [Phi[:, c] @ (A @ Phi[:, c]) for c in range(k)]
    ij = [i * i + j * j for i, j in PR.smooth_modes(k)]
    for a in range(k):
        for b in range(k):
            if ij[a] < ij[b]:
                assert rq[a] < rq[b]


def test_zero_weights_give_phi_plus_bias():
    N, k, hid = 16, 16, 16
    rng = np.random.default_rng(0)
    coef = np.exp(rng.standard_normal((2, N * N)))
    p = np.zeros(PR.param_count(k, hid))
    b4 = rng.standard_normal(k)
    p[-k:] = b4
    Phat = PR.cnn_forward(p, coef, N, k, hid)
    ref = PR.sine_modes(N, k)[None] + b4[None, None, :]
    np.testing.assert_allclose(Phat, np.broadcast_to(ref, Phat.shape), atol=1e-14)


def test_conv_is_cross_correlation_with_documented_layout():
    """A delta input through a single-channel 3x3 kernel reproduces the kernel
    flipped (cross-correlation): out[y, x] = sum W[dy, dx] in[y + dy - 1, x + dx - 1]."""
    W = torch.arange(9, dtype=torch.float64).reshape(1, 1, 3, 3)
    x = torch.zeros(1, 1, 5, 5, dtype=torch.float64)
    x[0, 0, 2, 2] = 1.0
    y = torch.nn.functional.conv2d(x, W, padding=1)[0, 0]
    np.testing.assert_array_equal(y[1:4, 1:4].numpy(), np.flip(W[0, 0].numpy()))


def test_input_channels():
    N, k = 16, 16
    coef = np.exp(np.random.default_rng(1).standard_normal((1, N * N)))
    x = PR.cnn_input(coef, N, k)
    assert abs(x[0, 0].mean()) < 1e-12 and abs(x[0, 0].std() - 1) < 1e-12
    np.testing.assert_allclose(x[0, 1:].reshape(k, -1).T, PR.sine_modes(N, k))


def test_qr_backward_finite_differences_and_autograd():
    rng = np.random.default_rng(2)
    n, k = 30, 5
    A = rng.standard_normal((n, k))
    W = rng.standard_normal((n, k))
    L = lambda M: float(np.sum(W * PR.qf(M)[0]) + 0.5 * np.sum(PR.qf(M)[0][:7] ** 2))
    Q, R = PR.qf(A)
    gQ = W.copy()
    gQ[:7] += Q[:7]
    gA = PR.qr_backward(Q, R, gQ)
    h = 1e-6
    fd = np.zeros_like(A)
    for idx in np.ndindex(*A.shape):
        Ap = A.copy(); Ap[idx] += h
        Am = A.copy(); Am[idx] -= h
        fd[idx] = (L(Ap) - L(Am)) / (2 * h)
    assert np.abs(gA - fd).max() <= 1e-7 * max(1.0, np.abs(gA).max())
    At = torch.tensor(A, requires_grad=True)
    Qt, Rt = torch.linalg.qr(At)
    s = torch.sign(torch.diagonal(Rt))
    Qt = Qt * s
    (torch.sum(torch.tensor(W) * Qt) + 0.5 * torch.sum(Qt[:7] ** 2)).backward()
    np.testing.assert_allclose(gA, At.grad.numpy(), atol=1e-12)


def test_adam_first_step_is_lr_sign():
    rng = np.random.default_rng(3)
    g = rng.standard_normal(50)
    p, m, v = PR.adam_update(np.zeros(50), g, np.zeros(50), np.zeros(50), 1e-3, 1)
    np.testing.assert_allclose(p, -1e-3 * np.sign(g), rtol=1e-6)
