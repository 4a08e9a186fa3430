"""The bar of the CNN-forward parity test and a bfloat16 model of the GPU
forward that calibrates it (test helpers; CPU).

The GPU forward rounds its input channels, its weights, every stored
pre-activation z_l and every GELU output to bfloat16 (unit roundoff
u = 2^-9) and accumulates in float32.  Its error is compared with the size of
what the network adds to the sine modes:

    err_b = ||P_hat_gpu,b - P_hat_ref,b||_F / ||P_hat_ref,b - Phi||_F

(per sample).  A model of that arithmetic (``bf16_forward``: torch float32
convolutions with the same roundings) gives err of about 2-3 u on the test
shapes (``tests/test_oracle_predictor.py`` prints and pins it); the bar
CNN_REL_TOL = 16 u ~ 0.031 leaves a factor of at least 5 for accumulation
order and the float32 erf, while every gross mistake of the forward puts err
near or above 1: an all-zero output, Phi alone (network dropped), a zeroed
last layer, a sign-flipped network (CPU test of the bar).
"""
import numpy as np
import torch

from oracle import predictor as PR

U_BF16 = 2.0 ** -9
CNN_REL_TOL = 16 * U_BF16


def rel_errors(Phat, ref, phi):
    """err_b for every sample; Phat, ref (batch, n, k), phi (n, k)."""
    Phat = np.asarray(Phat, dtype=np.float64)
    return np.array([np.linalg.norm(Phat[b] - ref[b]) / np.linalg.norm(ref[b] - phi)
                     for b in range(ref.shape[0])])


def _bf(t):
    return t.to(torch.bfloat16).to(torch.float32)


def bf16_forward(params, coef, N, k, hidden):
    """P_hat with the GPU forward's roundings (float32 accumulation)."""
    p = torch.tensor(np.asarray(params, dtype=np.float32))
    x = _bf(torch.tensor(PR.cnn_input(coef, N, k), dtype=torch.float32))
    off = 0
    h = x
    for l, (co, ci) in enumerate(PR.layer_shapes(k, hidden)):
        W = _bf(p[off:off + co * ci * 9].reshape(co, ci, 3, 3))
        off += co * ci * 9
        b = p[off:off + co]
        off += co
        z = torch.nn.functional.conv2d(h, W, None, padding=1) + b[None, :, None, None]
        if l < 3:
            h = _bf(torch.nn.functional.gelu(_bf(z)))
        else:
            h = z
    phi = torch.tensor(PR.sine_modes(N, k), dtype=torch.float32)
    return (phi.unsqueeze(0) + h.reshape(h.shape[0], k, N * N).transpose(1, 2)).double().numpy()
