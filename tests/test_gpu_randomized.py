"""GPU parity of the randomized-sketch basis (setup_randomized_P) against
the oracle's randomized range finder on the same seeded inputs and the same
test matrix Omega, through the C ABI (marked gpu).

Both compute the same function of (S0, Omega): orth(.) differs (CholeskyQR2
on the GPU, Householder QR in the oracle) only by a rotation inside the
sketch's span, so the leading subspaces agree.  Bars: the estimated
singular values of B to 1e-9 (float64) / 2e-5 (mixed) relative; P^T P = I to
1e-12; the subspace within the gap-aware bound 100 eps sigma_1^2 / (gap
sigma_k) (the route through B B^T squares the singular values, as the Gram
route does), eps = 2^-52 or 2^-23."""
import numpy as np
import pytest
import torch

import oracle as O
from tests._cases import make_case, cuda, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2601_20174_amd as mod
    return mod


def _sin_theta(U, V):
    Qu, _ = np.linalg.qr(U)
    Qv, _ = np.linalg.qr(V)
    return np.linalg.norm(Qu - Qv @ (Qv.T @ Qu), 2)


@pytest.mark.parametrize("kind,size,m,k,l,q", [("poisson", (32, 32), 32, 16, 24, 0),
                                               ("poisson", (32, 32), 32, 16, 24, 2),
                                               ("fv5", (45, 38), 48, 20, 30, 1),
                                               ("q1", (40, 40), 64, 32, 42, 1),
                                               ("fv7", (17, 13), 40, 8, 16, 3)])
@pytest.mark.parametrize("prec", [0, 1])
def test_setup_randomized_P(nl, kind, size, m, k, l, q, prec):
    A, op, n = make_case(kind, 6, size)
    rng = np.random.default_rng(90)
    S0 = rng.standard_normal((n, m))
    Om = rng.standard_normal((m, l))
    omega, s1 = 2 / 3, 10
    S = O.relax(A, S0, omega, s1)
    Pr, sig_r = O.randomized_basis(S, k, Om, q)
    P, sig = nl.setup_randomized_P(op, cuda(S0), k, omega, s1, cuda(Om), q, prec)
    P, sig = host(P), host(sig)
    assert sig.shape == (l,)
    tol = 1e-9 if prec == 0 else 2e-5
    np.testing.assert_allclose(sig[:k + 1], sig_r[:k + 1], rtol=tol)
    np.testing.assert_allclose(P.T @ P, np.eye(k), atol=1e-12)
    eps = 2.0 ** -52 if prec == 0 else 2.0 ** -23
    gap = sig_r[k - 1] - sig_r[k]
    bound = 100 * eps * sig_r[0] ** 2 / max(gap * sig_r[k - 1], 1e-300)
    assert _sin_theta(P, Pr) <= max(bound, 1e-10), (_sin_theta(P, Pr), bound)
    for j in range(k):
        assert P[np.argmax(np.abs(P[:, j])), j] > 0


def test_randomized_full_sketch_matches_spectral_P(nl):
    """l = m: the sketch spans range(S) and the randomized basis spans the
    same subspace as setup_spectral_P's."""
    A, op, n = make_case("fv5", 11, (40, 40))
    rng = np.random.default_rng(91)
    S0 = rng.standard_normal((n, 32))
    Om = rng.standard_normal((32, 32))
    P1, s1 = nl.setup_spectral_P(op, cuda(S0), 12, 2 / 3, 10, 0)
    P2, s2 = nl.setup_randomized_P(op, cuda(S0), 12, 2 / 3, 10, cuda(Om), 0, 0)
    np.testing.assert_allclose(host(s2), host(s1), rtol=1e-9)
    assert _sin_theta(host(P1), host(P2)) < 1e-8


def test_randomized_rank_deficient_sketch(nl):
    """S0 = [X, X] (rank 8): a sketch of l = 12 columns is numerically of rank
    8, so setup_randomized_P returns NLSP_E_RANK (the oracle's B has
    sigma_9..12 at rounding level)."""
    A, op, n = make_case("poisson", 0, (30, 30))
    X = np.random.default_rng(92).standard_normal((n, 8))
    S0 = np.concatenate([X, X], axis=1)
    Om = np.random.default_rng(93).standard_normal((16, 12))
    _, sb = O.randomized_basis(O.relax(A, S0, 2 / 3, 10), 8, Om, 1)
    assert sb[8] <= 1e-12 * sb[0]
    for prec in (0, 1):
        with pytest.raises(nl.NlspError) as e:
            nl.setup_randomized_P(op, cuda(S0), 8, 2 / 3, 10, cuda(Om), 1, prec)
        assert e.value.status == nl.E_RANK
