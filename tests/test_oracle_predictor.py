"""Pins for the oracle's P-predictor pieces (CPU only): the sine modes are
orthonormal and are the smoothest Dirichlet eigenvectors, the network reduces
to Phi + bias with zero weights and equals the same network written out as
plain loops (cross-correlation, documented parameter order, GELU on layers 1-3
only), the thin-QR backward matches finite differences and an independent
autograd of a library QR, and Adam matches its unrolled moment sums over
several steps."""
import math

import numpy as np
import pytest
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


def _gelu_erf(z):
    return 0.5 * z * (1.0 + math.erf(z / math.sqrt(2.0)))


def _direct_cnn(params, x, k, hid):
    """The predictor written out with explicit loops (no library convolution):
    for each layer, out[o][y][x] = b[o] + sum_{i, dy, dx} W[o][i][dy][dx] *
    in[i][y + dy - 1][x + dx - 1] (zero outside the field), GELU after layers
    1-3 only; parameters consumed in the documented order (W (Cout, Cin, 3, 3)
    row-major, then b (Cout), layer by layer)."""
    C, N, _ = x.shape
    h = [[[float(x[c, yy, xx]) for xx in range(N)] for yy in range(N)] for c in range(C)]
    off = 0
    shapes = [(hid, 1 + k), (hid, hid), (hid, hid), (k, hid)]
    for layer, (co, ci) in enumerate(shapes):
        Wf = params[off:off + co * ci * 9]
        off += co * ci * 9
        bf = params[off:off + co]
        off += co
        out = []
        for o in range(co):
            plane = []
            for yy in range(N):
                row = []
                for xx in range(N):
                    s = float(bf[o])
                    for i in range(ci):
                        for dy in range(3):
                            for dx in range(3):
                                sy, sx = yy + dy - 1, xx + dx - 1
                                if 0 <= sy < N and 0 <= sx < N:
                                    s += float(Wf[((o * ci + i) * 3 + dy) * 3 + dx]) * h[i][sy][sx]
                    row.append(_gelu_erf(s) if layer < 3 else s)
                plane.append(row)
            out.append(plane)
        h = out
    return np.array(h)            # (k, N, N)


def test_cnn_forward_matches_direct_loops():
    """Distinct weights per (Cout, Cin, tap), a bias per layer, GELU on layers
    1-3 only, the residual Phi added: the oracle's forward equals the same
    network written out as loops.  A transposed (Cout, Cin) unpacking, a
    flipped kernel (convolution instead of cross-correlation), a GELU on layer
    4, a dropped bias or a missing residual each fail this."""
    N, k, hid, batch = 6, 2, 3, 2
    rng = np.random.default_rng(11)
    coef = np.exp(rng.standard_normal((batch, N * N)))
    p = rng.standard_normal(PR.param_count(k, hid)) * 0.7 + 0.05
    Phat = PR.cnn_forward(p, coef, N, k, hid)
    x = PR.cnn_input(coef, N, k)
    phi = PR.sine_modes(N, k)
    for b in range(batch):
        h4 = _direct_cnn(p, x[b], k, hid)                    # (k, N, N)
        ref = phi + h4.reshape(k, N * N).T
        np.testing.assert_allclose(Phat[b], ref, rtol=1e-12, atol=1e-12)
    # the layer-4 weights matter (a network reduced to its last bias would
    # differ), and so does every bias
    q = p.copy()
    n4 = k * hid * 9
    q[-k - n4:-k] = 0.0
    assert np.abs(PR.cnn_forward(q, coef, N, k, hid) - Phat).max() > 1e-2


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


def _adam_closed_form(g_seq, lr, b1, b2, eps):
    """Parameters after len(g_seq) steps from p = 0, m = v = 0, with the
    moments written as the exponentially weighted sums they unroll to:
    m_t = (1 - b1) sum_i b1^(t-i) g_i, v_t = (1 - b2) sum_i b2^(t-i) g_i^2,
    p_t = p_(t-1) - lr (m_t / (1 - b1^t)) / (sqrt(v_t / (1 - b2^t)) + eps)."""
    p = np.zeros_like(g_seq[0])
    for t in range(1, len(g_seq) + 1):
        m = (1 - b1) * sum(b1 ** (t - i) * g_seq[i - 1] for i in range(1, t + 1))
        v = (1 - b2) * sum(b2 ** (t - i) * g_seq[i - 1] ** 2 for i in range(1, t + 1))
        p = p - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
    return p


def test_adam_steps_two_and_three_closed_form():
    """Three steps with distinct gradients and distinct b1, b2 against the
    unrolled moment sums; a constant gradient moves every parameter by
    lr g / (|g| + eps) at every step (bias correction exact).  Swapped b1/b2,
    a wrong bias-correction exponent or a missing square fail this."""
    rng = np.random.default_rng(4)
    n, lr, b1, b2, eps = 40, 1e-2, 0.8, 0.95, 1e-8
    gs = [rng.standard_normal(n) for _ in range(3)]
    p, m, v = np.zeros(n), np.zeros(n), np.zeros(n)
    for t, g in enumerate(gs, start=1):
        p, m, v = PR.adam_update(p, g, m, v, lr, t, b1=b1, b2=b2, eps=eps)
        np.testing.assert_allclose(p, _adam_closed_form(gs[:t], lr, b1, b2, eps), rtol=1e-12, atol=1e-15)
    g = rng.standard_normal(n)
    p, m, v = np.zeros(n), np.zeros(n), np.zeros(n)
    for t in range(1, 4):
        p, m, v = PR.adam_update(p, g, m, v, lr, t, b1=b1, b2=b2, eps=eps)
        np.testing.assert_allclose(p, -t * lr * g / (np.abs(g) + eps), rtol=1e-12)


def _gpu_test_params(k, hid, seed):
    """The parameter draw of the GPU CNN tests (He-scaled weights, small biases)."""
    rng = np.random.default_rng(seed)
    parts = []
    for co, ci in PR.layer_shapes(k, hid):
        parts.append(rng.standard_normal(co * ci * 9) * np.sqrt(2.0 / (ci * 9)))
        parts.append(rng.standard_normal(co) * 0.1)
    return np.concatenate(parts).astype(np.float32)


@pytest.mark.parametrize("N,k,hid", [(32, 16, 16), (40, 16, 32), (48, 32, 32)])
def test_cnn_forward_bar_accepts_bf16_rounding_and_rejects_gross_errors(N, k, hid):
    """The CNN-forward parity bar (tests/_cnn_bar.py) on the GPU test's own
    inputs: a bfloat16 model of the GPU arithmetic passes it with room to
    spare, and an all-zero output, Phi alone, a zeroed last layer and a
    sign-flipped network all fail it."""
    import workloads as W
    from tests._cnn_bar import CNN_REL_TOL, U_BF16, bf16_forward, rel_errors
    p = _gpu_test_params(k, hid, 1)
    coef = np.stack([W.lognormal_field(10 + b, N).ravel() for b in range(2)])
    ref = PR.cnn_forward(p.astype(np.float64), coef, N, k, hid)
    phi = PR.sine_modes(N, k)
    em = rel_errors(bf16_forward(p, coef, N, k, hid), ref, phi)
    assert np.all(em <= CNN_REL_TOL / 4) and np.all(em >= U_BF16 / 4), em
    q = p.astype(np.float64)
    n4 = k * hid * 9
    q[-k - n4:-k] = 0.0
    mutants = {"zeros": np.zeros_like(ref), "phi only": np.broadcast_to(phi, ref.shape),
               "layer 4 zeroed": PR.cnn_forward(q, coef, N, k, hid), "sign flip": 2 * phi[None] - ref}
    for name, Y in mutants.items():
        assert np.all(rel_errors(Y, ref, phi) > 10 * CNN_REL_TOL), name
