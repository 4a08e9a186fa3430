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


# ------------------------------------------------- randomized range finder
def _sin_theta(P, U):
    """sin of the largest principal angle between span(P) and span(U)
    (both orthonormal)."""
    return np.linalg.norm(P - U @ (U.T @ P), 2)


def test_randomized_basis_exact_on_low_rank():
    """S of exact rank 10 < l: range(S Omega) = range(S), so the randomized
    basis is the exact top-k singular subspace and the estimated singular
    values are the exact ones (library SVD), for any number of power steps."""
    rng = np.random.default_rng(80)
    n, m, r, k, l = 300, 40, 10, 6, 12
    sv = np.array([10.0, 7, 5, 3, 2, 1.5, 0.9, 0.5, 0.2, 0.1])
    U0, _ = np.linalg.qr(rng.standard_normal((n, r)))
    V0, _ = np.linalg.qr(rng.standard_normal((m, r)))
    S = (U0 * sv) @ V0.T
    Om = rng.standard_normal((m, l))
    for q in (0, 1, 2):
        P, sigma = O.randomized_basis(S, k, Om, q)
        np.testing.assert_allclose(P.T @ P, np.eye(k), atol=1e-13)
        assert _sin_theta(P, U0[:, :k]) < 1e-10
        np.testing.assert_allclose(sigma[:r], sv, rtol=1e-10)
        assert np.all(sigma[r:] < 1e-12 * sv[0])


def test_randomized_basis_full_sketch_equals_svd():
    """l = m with an invertible Omega: range(S Omega) = range(S) for a full
    rank S, so P spans the exact leading subspace (compared with the oracle's
    SVD route on a relaxed Poisson sample with a healthy gap at k)."""
    c = W.Cfg1()
    A = O.poisson5(c.N)
    S = O.relax(A, c.S0(), c.omega, c.s1)
    Pe, se = O.spectral_basis(S, c.k)
    assert se[c.k - 1] - se[c.k] > 1e-3 * se[0]
    Om = np.random.default_rng(81).standard_normal((c.m, c.m))
    P, sigma = O.randomized_basis(S, c.k, Om, 0)
    assert _sin_theta(P, Pe) < 1e-9
    np.testing.assert_allclose(sigma, se, rtol=1e-10)
    # same sign convention: equal columns, not only equal spans
    np.testing.assert_allclose(P, Pe, atol=1e-8)


def test_randomized_basis_depends_only_on_the_sketch_range():
    """Omega -> Omega G (G invertible l x l) leaves range(S Omega) and hence P
    unchanged; a transposed or mis-ordered product would not."""
    rng = np.random.default_rng(82)
    c = W.Cfg1()
    A = O.poisson5(c.N)
    S = O.relax(A, c.S0(), c.omega, c.s1)
    Om = rng.standard_normal((c.m, 24))
    G = rng.standard_normal((24, 24)) + 5 * np.eye(24)
    P1, s1 = O.randomized_basis(S, c.k, Om, 1)
    P2, s2 = O.randomized_basis(S, c.k, Om @ G, 1)
    assert _sin_theta(P1, P2) < 1e-9
    np.testing.assert_allclose(s1, s2, rtol=1e-10)


def test_randomized_basis_power_steps_approach_eckart_young():
    """With a decaying spectrum the projection residual ||S - P P^T S||_F
    never goes below the Eckart-Young optimum sqrt(sum_{j>k} sigma_j^2), and
    power steps bring it to that optimum (within 1e-3 relative at q = 4)."""
    rng = np.random.default_rng(83)
    n, m, k, l = 400, 60, 8, 14
    U0, _ = np.linalg.qr(rng.standard_normal((n, m)))
    V0, _ = np.linalg.qr(rng.standard_normal((m, m)))
    sv = 0.8 ** np.arange(m)
    S = (U0 * sv) @ V0.T
    opt = np.sqrt(np.sum(sv[k:] ** 2))
    Om = rng.standard_normal((m, l))
    res = []
    for q in (0, 1, 2, 4):
        P, _ = O.randomized_basis(S, k, Om, q)
        res.append(np.linalg.norm(S - P @ (P.T @ S)))
    assert all(r >= opt * (1 - 1e-12) for r in res)
    assert res[0] > res[-1]
    assert res[-1] <= opt * (1 + 1e-3)
