"""Pins for the oracle's two-grid preconditioner and PCG (CPU only)."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from oracle.method import make_preconditioner
import workloads as W


def _problem(seed=0, N=7):
    rng = np.random.default_rng(seed)
    A = O.fv_harmonic_2d(np.exp(rng.standard_normal((N, N + 1))))
    S = O.relax(A, rng.standard_normal((A.shape[0], 12)), 2 / 3, 10)
    P, _ = O.spectral_basis(S, 5)
    Ac, L = O.galerkin(A, P)
    return A, P, Ac, L


def _dense_minv(A, P, L, omega, nu1, nu2):
    n = A.shape[0]
    return O.two_grid_apply(A, P, L, np.eye(n), omega, nu1, nu2)


def test_preconditioner_matches_error_propagation_form():
    # Two-grid textbook form: M^-1 = (I - E) A^-1 with
    # E = G^nu2 (I - P A_c^-1 P^T A) G^nu1, G = I - w D^-1 A.
    A, P, Ac, L = _problem()
    Ad = A.toarray()
    n = Ad.shape[0]
    omega = 2 / 3
    G = np.eye(n) - omega * Ad / Ad.diagonal()[:, None]
    Ec = np.eye(n) - P @ np.linalg.solve(Ac, P.T @ Ad)
    for nu1, nu2 in [(1, 1), (2, 2), (1, 0), (3, 1)]:
        E = np.linalg.matrix_power(G, nu2) @ Ec @ np.linalg.matrix_power(G, nu1)
        ref = (np.eye(n) - E) @ np.linalg.inv(Ad)
        np.testing.assert_allclose(_dense_minv(A, P, L, omega, nu1, nu2), ref, atol=1e-11)


def test_preconditioner_symmetric_positive_definite_iff_balanced():
    A, P, Ac, L = _problem(1)
    M = _dense_minv(A, P, L, 2 / 3, 1, 1)
    assert np.abs(M - M.T).max() <= 1e-13 * np.abs(M).max()
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0
    M10 = _dense_minv(A, P, L, 2 / 3, 1, 0)          # negative control
    assert np.abs(M10 - M10.T).max() > 1e-3 * np.abs(M10).max()


def test_coarse_correction_annihilates_range_and_is_a_norm_optimal():
    A, P, Ac, L = _problem(2)
    Ad = A.toarray()
    n = Ad.shape[0]
    C = _dense_minv(A, P, L, 2 / 3, 0, 0)            # nu=0: P A_c^-1 P^T
    Ec = np.eye(n) - C @ Ad
    rng = np.random.default_rng(0)
    y = rng.standard_normal(P.shape[1])
    assert np.linalg.norm(Ec @ (P @ y)) < 1e-12 * np.linalg.norm(P @ y)
    e = rng.standard_normal(n)
    LA = np.linalg.cholesky(Ad)                       # ||v||_A = ||LA^T v||
    yls, *_ = np.linalg.lstsq(LA.T @ P, LA.T @ e, rcond=None)
    best = np.linalg.norm(LA.T @ (e - P @ yls))
    got = np.sqrt((Ec @ e) @ Ad @ (Ec @ e))
    np.testing.assert_allclose(got, best, rtol=1e-10)


def test_preconditioner_depends_only_on_span():
    A, P, Ac, L = _problem(3)
    Qm, _ = np.linalg.qr(np.random.default_rng(1).standard_normal((5, 5)))
    P2 = P @ Qm
    _, L2 = O.galerkin(A, P2)
    np.testing.assert_allclose(_dense_minv(A, P, L, 2 / 3, 1, 1),
                               _dense_minv(A, P2, L2, 2 / 3, 1, 1), atol=1e-12)


def test_zero_rank_is_jacobi_polynomial():
    A, P, Ac, L = _problem(4)
    Ad = A.toarray()
    n = Ad.shape[0]
    omega, nu = 0.6, 2
    Dinv = np.diag(1 / Ad.diagonal())
    G = np.eye(n) - omega * Dinv @ Ad
    ref = sum(np.linalg.matrix_power(G, i) for i in range(2 * nu)) @ (omega * Dinv)
    np.testing.assert_allclose(_dense_minv(A, np.zeros((n, 0)), None, omega, nu, nu), ref,
                               atol=1e-12)


@pytest.mark.parametrize("kind", ["poisson", "fv", "q1"])
def test_pcg_against_dense_direct_solve(kind):
    rng = np.random.default_rng(11)
    A = {"poisson": O.poisson5(15), "fv": O.fv_harmonic_2d(np.exp(rng.standard_normal((16, 14)))),
         "q1": O.q1_aniso(18, 3e-3, 1.1)}[kind]
    n = A.shape[0]
    st = O.setup(A, rng.standard_normal((n, 16)), 8, 2 / 3, 10)
    f = rng.standard_normal((n, 2))
    res = O.pcg(A, f, make_preconditioner(A, st["P"], st["L"], 2 / 3, 1, 1), rtol=1e-10)
    xs = np.linalg.solve(A.toarray(), f)
    kappa = np.linalg.cond(A.toarray())
    assert (res.status == O.OK).all()
    assert (res.relres <= 1e-10).all()
    for j in range(2):
        err = np.linalg.norm(res.x[:, j] - xs[:, j]) / np.linalg.norm(xs[:, j])
        assert err <= kappa * 1e-10


def test_pcg_a_norm_error_monotone():
    A, P, Ac, L = _problem(5, N=12)
    f = np.random.default_rng(2).standard_normal(A.shape[0])
    xs = np.linalg.solve(A.toarray(), f)
    res = O.pcg(A, f, make_preconditioner(A, P, L, 2 / 3, 1, 1), rtol=1e-12, xstar=xs[:, None])
    an = res.history[0][1]
    assert len(an) > 5
    assert all(an[i + 1] <= an[i] * (1 + 1e-12) for i in range(len(an) - 1))


def test_plain_cg_terminates_within_distinct_eigenvalue_count():
    # Exact-arithmetic CG ends after at most d steps, d = number of distinct
    # eigenvalues of A (textbook).  The N=5 Poisson matrix has many repeats.
    A = O.poisson5(5)
    lam = np.linalg.eigvalsh(A.toarray())
    d = len(np.unique(np.round(lam, 10)))
    assert d < A.shape[0]
    f = np.random.default_rng(0).standard_normal(A.shape[0])
    res = O.pcg(A, f, None, rtol=1e-11)
    assert res.status[0] == O.OK and res.iters[0] <= d


def test_full_rank_coarse_space_converges_in_one_iteration():
    A = O.poisson5(6)
    n = A.shape[0]
    P, _ = np.linalg.qr(np.random.default_rng(0).standard_normal((n, n)))
    _, L = O.galerkin(A, P)
    f = np.random.default_rng(1).standard_normal(n)
    res = O.pcg(A, f, make_preconditioner(A, P, L, 2 / 3, 1, 1), rtol=1e-10)
    assert res.iters[0] == 1 and res.relres[0] < 1e-10


def test_scale_invariance_of_iterations():
    c = W.Cfg1()
    A = O.poisson5(c.N)
    st = O.setup(A, c.S0(), c.k, c.omega, c.s1)
    f = c.rhs()
    r1 = O.pcg(A, f, make_preconditioner(A, st["P"], st["L"], c.omega, 1, 1))
    A2 = 1e3 * A
    st2 = O.setup(A2, c.S0(), c.k, c.omega, c.s1)
    r2 = O.pcg(A2, 1e3 * f, make_preconditioner(A2, st2["P"], st2["L"], c.omega, 1, 1))
    assert r1.iters[0] == r2.iters[0]
    assert 45 <= r1.iters[0] <= 65          # two-grid beats plain CG (about 100) on cfg 1


def test_failure_statuses():
    A = O.poisson5(6)
    n = A.shape[0]
    f = np.ones(n)
    assert O.pcg(A, f, None, maxit=1).status[0] == O.NOT_CONVERGED
    fn = f.copy(); fn[3] = np.nan
    assert O.pcg(A, fn, None).status[0] == O.E_NONFINITE
    bad = A.copy().tolil(); bad[0, 0] = -10.0; bad = bad.tocsr()    # indefinite
    st = O.pcg(bad, np.eye(n)[:, 0] * 1.0, None, maxit=50).status[0]
    assert st in (O.E_BREAKDOWN, O.NOT_CONVERGED)
    z = O.pcg(A, np.zeros(n), None)
    assert z.iters[0] == 0 and z.relres[0] == 0 and z.status[0] == O.OK
