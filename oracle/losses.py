"""Training objectives and their gradients in float64 (oracle; test
infrastructure only).

* Subspace loss  L(P; B) = ||B - P P^T B||_F^2 / ||B||_F^2.  For orthonormal P
  it equals 1 - J(P)/||B||_F^2 with J the projected energy of Sec. 4 (eq.
  subspace_energy); the appendix on optimality of smooth-error reduction gives
  the expansion.  Evaluated here from the definition for any P.
* NLSS loss (Sec. 4, eq. nlss_loss): (1/k) sum_l (1 - ||P_{1:l}^T S||^2/||S||^2).
* Column-weighted energy loss 1 - sum_j w_j ||p_j^T B||^2 / ||B||^2; with
  w_j = (k - j + 1)/k it is the NLSS loss for any P (prefix norms add up over
  columns), the weighted Ky Fan form stated after eq. nlss_loss.
* Captured energy Energy(r) = ||Q_r^T S||^2 / ||S||^2 (Sec. 4.1 diagnostic).
* Galerkin-convergence objective (appendix, "Galerkin Convergence"):
  J(P) = ||A^{1/2}(I - Pi_A(P)) S||_F^2, Pi_A(P) = P (P^T A P)^{-1} P^T A.
* The vector-Jacobian product of the Galerkin product A_c = P^T A P.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

__all__ = ["subspace_loss", "subspace_loss_grad", "nlss_loss", "nlss_weights",
           "weighted_energy_loss", "weighted_energy_loss_grad", "captured_energy",
           "galerkin_term", "galerkin_term_grad", "galerkin_term_dense",
           "galerkin_coarse_vjp"]


def subspace_loss(P: np.ndarray, B: np.ndarray) -> float:
    """||B - P (P^T B)||_F^2 / ||B||_F^2, straight from the definition."""
    Rm = B - P @ (P.T @ B)
    return float(np.sum(Rm * Rm) / np.sum(B * B))


def subspace_loss_grad(P: np.ndarray, B: np.ndarray) -> np.ndarray:
    """dL/dP for the loss above, valid for any (not necessarily orthonormal) P.

    With C = P^T B and G = P^T P,
      ||B - P C||^2 = ||B||^2 - 2 tr(C C^T) + tr(C^T G C),
    whose derivative is -4 B C^T + 2 P C C^T + 2 B C^T G, so
      dL/dP = -(2/||B||^2) [B C^T (2I - G) - P C C^T].
    """
    C = P.T @ B
    G = P.T @ P
    k = P.shape[1]
    bb = float(np.sum(B * B))
    return -(2.0 / bb) * (B @ C.T @ (2.0 * np.eye(k) - G) - P @ (C @ C.T))


def nlss_loss(P: np.ndarray, S: np.ndarray) -> float:
    """(1/k) sum_{l=1..k} (1 - ||P_{:, :l}^T S||_F^2 / ||S||_F^2)."""
    k = P.shape[1]
    ss = float(np.sum(S * S))
    tot = 0.0
    for l in range(1, k + 1):
        W = P[:, :l].T @ S
        tot += 1.0 - float(np.sum(W * W)) / ss
    return tot / k


def nlss_weights(k: int) -> np.ndarray:
    """w_j = (k - j + 1)/k, j = 1..k: column j lies in the prefixes l = j..k."""
    return (k - np.arange(k)) / float(k)


def weighted_energy_loss(P: np.ndarray, B: np.ndarray, w: np.ndarray) -> float:
    """1 - sum_j w_j ||p_j^T B||^2 / ||B||^2."""
    C = P.T @ B
    return float(1.0 - np.sum(w * np.sum(C * C, axis=1)) / np.sum(B * B))


def weighted_energy_loss_grad(P: np.ndarray, B: np.ndarray, w: np.ndarray) -> np.ndarray:
    """d/dP of the loss above: -(2/||B||^2) B C^T diag(w), C = P^T B."""
    C = P.T @ B
    return -(2.0 / float(np.sum(B * B))) * (B @ C.T) * w[None, :]


def captured_energy(Q: np.ndarray, S: np.ndarray, r: int) -> float:
    """Energy(r) = ||Q_{:, :r}^T S||_F^2 / ||S||_F^2."""
    W = Q[:, :r].T @ S
    return float(np.sum(W * W) / np.sum(S * S))


def galerkin_term_dense(A, P: np.ndarray, S: np.ndarray) -> float:
    """J(P) = ||A^{1/2} (I - P (P^T A P)^{-1} P^T A) S||_F^2 from the
    definition, with A^{1/2} from a dense eigendecomposition (small n only)."""
    Ad = A.toarray() if hasattr(A, "toarray") else np.asarray(A)
    lam, V = np.linalg.eigh(Ad)
    Ah = (V * np.sqrt(lam)) @ V.T
    Ac = P.T @ Ad @ P
    Pi = P @ np.linalg.solve(Ac, P.T @ Ad)
    E = Ah @ (S - Pi @ S)
    return float(np.sum(E * E))


def galerkin_term(A, P: np.ndarray, S: np.ndarray) -> float:
    """The same J(P) via the projector identity used in the appendix proof:
    J = tr(S^T A S) - tr(W^T A_c^{-1} W), W = P^T A S, A_c = P^T A P."""
    AS = A @ S
    W = P.T @ AS
    Ac = P.T @ (A @ P)
    cf = sla.cho_factor(0.5 * (Ac + Ac.T), lower=True)
    Z = sla.cho_solve(cf, W)
    return float(np.sum(S * AS) - np.sum(W * Z))


def galerkin_term_grad(A, P: np.ndarray, S: np.ndarray) -> np.ndarray:
    """dJ/dP = 2 A (P Z - S) Z^T with Z = A_c^{-1} P^T A S.

    From J = tr(S^T A S) - tr(W^T A_c^{-1} W): the W-dependence contributes
    -2 A S Z^T and the A_c-dependence +2 A P Z Z^T."""
    AS = A @ S
    AP = A @ P
    Ac = P.T @ AP
    cf = sla.cho_factor(0.5 * (Ac + Ac.T), lower=True)
    Z = sla.cho_solve(cf, P.T @ AS)
    return 2.0 * (AP @ (Z @ Z.T) - AS @ Z.T)


def galerkin_coarse_vjp(A, P: np.ndarray, gAc: np.ndarray) -> np.ndarray:
    """Vector-Jacobian product of A_c = P^T A P: for an upstream gradient
    G = dL/dA_c, dL/dP = A P (G + G^T) (A symmetric)."""
    return (A @ P) @ (gAc + gAc.T)
