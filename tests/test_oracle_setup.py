"""Pins for the oracle's setup phase: relaxation, spectral basis, Galerkin
operator (CPU only).  Checked against closed forms of the 5-point Poisson
problem, the Eckart-Young theorem and basis-independent invariants."""
import numpy as np
import pytest

import oracle as O
import workloads as W


def _sine_modes(N):
    """Orthonormal sine eigenvectors of poisson5(N), ordered by eigenvalue
    (ties broken by (i, j)), with eigenvalues."""
    h = 1.0 / (N + 1)
    x = np.arange(1, N + 1) * h
    modes = []
    for i in range(1, N + 1):
        for j in range(1, N + 1):
            lam = 4 - 2 * np.cos(i * np.pi * h) - 2 * np.cos(j * np.pi * h)
            v = np.outer(np.sin(j * np.pi * x), np.sin(i * np.pi * x)).ravel()
            modes.append((lam, i, j, v / np.linalg.norm(v)))
    modes.sort(key=lambda t: (t[0], t[1], t[2]))
    lam = np.array([m[0] for m in modes])
    V = np.stack([m[3] for m in modes], 1)
    return lam, V


def test_relaxation_on_eigenvector_is_exact_power():
    N, omega, s1 = 12, 2 / 3, 7
    A = O.poisson5(N)
    lam, V = _sine_modes(N)
    S0 = V[:, [0, 5, 100]]
    S = O.relax(A, S0, omega, s1)
    np.testing.assert_allclose(S, S0 * (1 - omega * lam[[0, 5, 100]] / 4) ** s1, atol=1e-14)


def test_basis_from_identity_is_smoothest_sine_modes():
    # S0 = I: S = (I - w A/4)^s1 is symmetric with singular values
    # |1 - w lambda/4|^s1, largest for the smoothest modes.  k=15 is a
    # valid cut for N=32 (lambda_15 < lambda_16).
    c = W.Cfg1()
    A = O.poisson5(c.N)
    S = O.relax(A, np.eye(c.n), c.omega, c.s1)
    lam, V = _sine_modes(c.N)
    for k in (15, 17):
        assert lam[k - 1] < lam[k] - 1e-9
        P, sigma = O.spectral_basis(S, k)
        sv = np.sort(np.abs(1 - c.omega * lam / 4) ** c.s1)[::-1]
        np.testing.assert_allclose(sigma[:k + 1], sv[:k + 1], rtol=1e-12)
        # sin of the largest principal angle between span(P) and the modes
        Vk = V[:, :k]
        assert np.linalg.norm(P - Vk @ (Vk.T @ P), 2) < 1e-10


def test_long_relaxation_captures_lowest_modes():
    c = W.Cfg1()
    A = O.poisson5(c.N)
    S = O.relax(A, c.S0(), c.omega, 200)
    P, _ = O.spectral_basis(S, c.k)
    _, V = _sine_modes(c.N)
    energy = np.sum((P.T @ V[:, :4]) ** 2, axis=0)
    assert energy.min() >= 0.99


def test_basis_eckart_young_and_orthonormality():
    rng = np.random.default_rng(3)
    S = rng.standard_normal((300, 20)) @ np.diag(np.linspace(3, 0.1, 20))
    for k in (1, 7, 19):
        P, sigma = O.spectral_basis(S, k)
        np.testing.assert_allclose(P.T @ P, np.eye(k), atol=1e-13)
        resid = np.linalg.norm(S - P @ (P.T @ S)) ** 2
        np.testing.assert_allclose(resid, np.sum(sigma[k:] ** 2), rtol=1e-10)
        # same subspace and singular values from the Gram eigenproblem
        w, Vg = np.linalg.eigh(S.T @ S)
        w, Vg = w[::-1], Vg[:, ::-1]
        np.testing.assert_allclose(sigma, np.sqrt(w), rtol=1e-10)
        U = S @ Vg[:, :k] / np.sqrt(w[:k])
        np.testing.assert_allclose(np.abs(np.diag(U.T @ P)), 1.0, atol=1e-10)
        # sign convention: largest-magnitude entry of every column positive
        for j in range(k):
            assert P[np.argmax(np.abs(P[:, j])), j] > 0


def test_galerkin_symmetric_spd_and_rotation():
    rng = np.random.default_rng(5)
    A = O.fv_harmonic_2d(np.exp(rng.standard_normal((9, 8))))
    S = O.relax(A, rng.standard_normal((72, 12)), 2 / 3, 10)
    P, _ = O.spectral_basis(S, 6)
    Y = A @ P
    Ac_raw = P.T @ Y
    assert np.abs(Ac_raw - Ac_raw.T).max() <= 1e-13 * np.abs(Ac_raw).max()
    Ac, L = O.galerkin(A, P)
    assert np.linalg.eigvalsh(Ac).min() > 0
    np.testing.assert_allclose(L @ L.T, Ac, atol=1e-13 * np.abs(Ac).max())
    Qm, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    Ac2, _ = O.galerkin(A, P @ Qm)
    np.testing.assert_allclose(Ac2, Qm.T @ Ac @ Qm, atol=1e-12)
    np.testing.assert_allclose(np.linalg.eigvalsh(Ac2), np.linalg.eigvalsh(Ac), rtol=1e-12)


def test_galerkin_on_exact_modes_is_diagonal_eigenvalues():
    N = 10
    A = O.poisson5(N)
    lam, V = _sine_modes(N)
    Ac, _ = O.galerkin(A, V[:, :8])
    np.testing.assert_allclose(Ac, np.diag(lam[:8]), atol=1e-13)


def test_not_spd_raises():
    A = O.poisson5(4)
    P = np.zeros((16, 2)); P[0, 0] = 1; P[0, 1] = 1      # rank deficient
    with pytest.raises(np.linalg.LinAlgError):
        O.galerkin(A, P)
