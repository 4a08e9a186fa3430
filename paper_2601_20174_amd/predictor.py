"""Training and inference of the P-predictor (argument marshalling and the
loop only; every arithmetic step runs in libnlsp.so kernels).

One training step on a batch of fields:
    P_hat = CNN(coef; params)           cnn_fwd
    Q     = qf(P_hat)                   qr_thin_fwd (CholeskyQR2)
    L     = mean_b [ NLSS(Q_b; B_b)     subspace_loss_fwd with the NLSS column
                                        weights (k - j + 1)/k
                   + beta J_b(Q_b) / ||A_b^{1/2} B_b||_F^2 ]
                                        galerkin_term_fwd (the appendix's
                                        Galerkin-convergence objective, scaled
                                        by its value with no coarse space)
and the backward through subspace_loss_bwd, galerkin_term_bwd, qr_thin_bwd
and cnn_bwd, then one Adam step (adam_step).  B_b are the relaxed random
vectors of field b, A_b its operator (2-D finite volumes, coefficient a_b).
"""
from __future__ import annotations

import math
from typing import Optional

import torch

from . import api


class Predictor:
    def __init__(self, N: int, k: int, hidden: int = 32, seed: int = 0, device=None):
        self.N, self.k, self.hidden = N, k, hidden
        self.device = device or torch.device("cuda", torch.cuda.current_device())
        count = api.cnn_param_count(1, N, k, hidden)
        if count < 0:
            raise ValueError("unsupported predictor shape")
        g = torch.Generator(device="cpu").manual_seed(seed)
        parts = []
        for co, ci in [(hidden, 1 + k), (hidden, hidden), (hidden, hidden), (k, hidden)]:
            std = math.sqrt(2.0 / (ci * 9))
            parts.append(torch.randn(co * ci * 9, generator=g) * std)
            parts.append(torch.zeros(co))
        # the last layer starts at zero: P_hat = Phi_k at initialisation
        parts[-2].zero_()
        self.params = torch.cat(parts).to(torch.float32).to(self.device)
        assert self.params.numel() == count
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.steps = 0
        self._ws = {}

    def _workspace(self, batch: int) -> torch.Tensor:
        if batch not in self._ws:
            nb = api.cnn_workspace_bytes(batch, self.N, self.k, self.hidden)
            if nb == 0:
                raise ValueError("unsupported predictor shape")
            self._ws[batch] = torch.empty(nb, dtype=torch.uint8, device=self.device)
        return self._ws[batch]

    def nlss_weights(self) -> torch.Tensor:
        return torch.arange(self.k, 0, -1, dtype=torch.float32, device=self.device) / self.k

    def basis(self, coef: torch.Tensor, params: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Q = qf(P_hat) (batch, N*N, k) float32 for coef (batch, N*N) float64."""
        p = self.params if params is None else params
        ws = self._workspace(coef.shape[0])
        Phat = api.CnnPredictor.apply(p, coef, self.N, self.k, self.hidden, ws)
        return api.thin_q(Phat)

    def loss(self, coef: torch.Tensor, B: torch.Tensor, params: Optional[torch.Tensor] = None,
             beta: float = 1.0) -> torch.Tensor:
        """Mean over the batch of NLSS + beta J / ||A^{1/2} B||_F^2 (beta = 0:
        NLSS alone)."""
        Q = self.basis(coef, params)
        L = api.subspace_loss(Q, B, self.nlss_weights())
        if beta:
            op = api.Operator(api.OP_FV5, self.N, self.N, 1, coef.reshape(-1))   # batched coefficients
            J, _, E = api.galerkin_term(Q, B, op)
            L = L + beta * J / E
        return L.mean()

    def step(self, coef: torch.Tensor, B: torch.Tensor, lr: float = 1e-3, beta: float = 1.0) -> float:
        p = self.params.detach().requires_grad_(True)
        L = self.loss(coef, B, p, beta)
        L.backward()
        self.steps += 1
        api.adam_step(self.params, p.grad, self.m, self.v, lr, self.steps)
        return float(L.detach())
