"""Pins for the oracle's losses and gradients (CPU only): closed forms at the
SVD basis, the weighted Ky Fan identity, the first-order optimality of the
leading singular subspace, central finite differences and an independent
torch autograd evaluation."""
import numpy as np
import pytest
import torch

import oracle as O


def _S(seed=0, n=64, m=8):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, m)) @ np.diag(np.linspace(4, 0.3, m))


def test_losses_at_svd_basis_closed_form():
    S = _S()
    k = 4
    P, sigma = O.spectral_basis(S, k)
    tot = np.sum(sigma ** 2)
    np.testing.assert_allclose(O.subspace_loss(P, S), 1 - np.sum(sigma[:k] ** 2) / tot, atol=1e-14)
    ref = np.mean([1 - np.sum(sigma[:l] ** 2) / tot for l in range(1, k + 1)])
    np.testing.assert_allclose(O.nlss_loss(P, S), ref, atol=1e-14)
    np.testing.assert_allclose(O.captured_energy(P, S, 2), np.sum(sigma[:2] ** 2) / tot, atol=1e-14)


def test_nlss_weighted_ky_fan_identity():
    S = _S(1)
    k = 5
    P, _ = np.linalg.qr(np.random.default_rng(2).standard_normal((S.shape[0], k)))
    ss = np.sum(S * S)
    kyfan = sum((k - j) * P[:, j] @ S @ S.T @ P[:, j] for j in range(k))   # weight k-j+1, 1-based
    np.testing.assert_allclose(k * O.nlss_loss(P, S), k - kyfan / ss, atol=1e-13)


def test_riemannian_gradient_vanishes_at_leading_subspace():
    S = _S(2)
    P, _ = O.spectral_basis(S, 3)
    g = O.subspace_loss_grad(P, S)
    rg = g - P @ (P.T @ g)
    assert np.abs(rg).max() < 1e-13
    Pr, _ = np.linalg.qr(np.random.default_rng(3).standard_normal(P.shape))
    gr = O.subspace_loss_grad(Pr, S)
    assert np.abs(gr - Pr @ (Pr.T @ gr)).max() > 1e-3


def _fd(fun, P, h=1e-6):
    g = np.zeros_like(P)
    for idx in np.ndindex(*P.shape):
        Pp = P.copy(); Pp[idx] += h
        Pm = P.copy(); Pm[idx] -= h
        g[idx] = (fun(Pp) - fun(Pm)) / (2 * h)
    return g


def test_subspace_loss_gradient_finite_differences_and_autograd():
    S = _S(4)
    P = np.random.default_rng(5).standard_normal((64, 4))     # not orthonormal
    g = O.subspace_loss_grad(P, S)
    gfd = _fd(lambda Q: O.subspace_loss(Q, S), P)
    assert np.abs(g - gfd).max() <= 1e-7 * max(1.0, np.abs(g).max())
    Pt = torch.tensor(P, requires_grad=True)
    St = torch.tensor(S)
    l = ((St - Pt @ (Pt.T @ St)) ** 2).sum() / (St ** 2).sum()
    l.backward()
    np.testing.assert_allclose(g, Pt.grad.numpy(), atol=1e-12)


def test_weighted_energy_loss_is_nlss_for_any_P_and_its_gradient():
    S = _S(6)
    k = 5
    P = np.random.default_rng(7).standard_normal((64, k))      # not orthonormal
    w = O.nlss_weights(k)
    np.testing.assert_allclose(w, [5 / 5, 4 / 5, 3 / 5, 2 / 5, 1 / 5])
    # the prefix definition of eq. nlss_loss, summed term by term
    np.testing.assert_allclose(O.weighted_energy_loss(P, S, w), O.nlss_loss(P, S), rtol=1e-13)
    g = O.weighted_energy_loss_grad(P, S, w)
    gfd = _fd(lambda Q: O.nlss_loss(Q, S), P)
    assert np.abs(g - gfd).max() <= 1e-7 * max(1.0, np.abs(g).max())
    Pt = torch.tensor(P, requires_grad=True)
    St = torch.tensor(S)
    l = sum(1 - ((Pt[:, :j].T @ St) ** 2).sum() / (St ** 2).sum() for j in range(1, k + 1)) / k
    l.backward()
    np.testing.assert_allclose(g, Pt.grad.numpy(), atol=1e-12)
    # uniform weights 1 on orthonormal P give the plain subspace loss
    Q, _ = np.linalg.qr(P)
    np.testing.assert_allclose(O.weighted_energy_loss(Q, S, np.ones(k)), O.subspace_loss(Q, S), atol=1e-14)


def _small_spd(seed=0, N=6):
    rng = np.random.default_rng(seed)
    return O.fv_harmonic_2d(np.exp(rng.standard_normal((N, N))))


def test_galerkin_term_expansion_matches_definition_and_optimum():
    A = _small_spd()
    n = A.shape[0]
    rng = np.random.default_rng(1)
    S = O.relax(A, rng.standard_normal((n, 10)), 2 / 3, 3)
    k = 4
    P = rng.standard_normal((n, k))
    J = O.galerkin_term(A, P, S)
    np.testing.assert_allclose(J, O.galerkin_term_dense(A, P, S), rtol=1e-10)
    assert J >= 0
    # optimum: range(A^{1/2} P) = top-k left singular subspace of A^{1/2} S
    lam, V = np.linalg.eigh(A.toarray())
    Ah = (V * np.sqrt(lam)) @ V.T
    Ahi = (V / np.sqrt(lam)) @ V.T
    U, sig, _ = np.linalg.svd(Ah @ S, full_matrices=False)
    Popt = Ahi @ U[:, :k]
    Jopt = O.galerkin_term(A, Popt, S)
    np.testing.assert_allclose(Jopt, np.sum(sig[k:] ** 2), rtol=1e-9)
    for s in range(5):
        assert O.galerkin_term(A, np.random.default_rng(10 + s).standard_normal((n, k)), S) >= Jopt


def test_galerkin_gradients_finite_differences_and_autograd():
    A = _small_spd(2, N=5)
    n = A.shape[0]
    rng = np.random.default_rng(3)
    S = rng.standard_normal((n, 6))
    P = rng.standard_normal((n, 3))
    g = O.galerkin_term_grad(A, P, S)
    gfd = _fd(lambda Q: O.galerkin_term(A, Q, S), P)
    assert np.abs(g - gfd).max() <= 1e-6 * max(1.0, np.abs(g).max())
    At = torch.tensor(A.toarray())
    Pt = torch.tensor(P, requires_grad=True)
    Gc = torch.tensor(rng.standard_normal((3, 3)))
    Ac = Pt.T @ At @ Pt
    (Ac * Gc).sum().backward()
    np.testing.assert_allclose(O.galerkin_coarse_vjp(A, P, Gc.numpy()), Pt.grad.numpy(), atol=1e-12)
