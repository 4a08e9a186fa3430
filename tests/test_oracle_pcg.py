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


def test_flexible_beta_equals_standard_beta_for_a_fixed_spd_preconditioner():
    """With a fixed symmetric positive definite M^-1 the new residual is
    M-orthogonal to the old one (r_new^T z_old = 0 in exact arithmetic), so the
    Polak-Ribiere beta (gamma' - r_new^T z_old) / gamma reduces to
    gamma' / gamma and both forms produce the same iterates: compared after
    every iteration (maxit = 1, 2, ...)."""
    A, P, Ac, L = _problem(6, N=10)
    Minv = make_preconditioner(A, P, L, 2 / 3, 1, 1)
    f = np.random.default_rng(7).standard_normal(A.shape[0])
    full = O.pcg(A, f, Minv, rtol=1e-10)
    assert full.status[0] == O.OK and full.iters[0] > 8
    for j in range(1, int(full.iters[0]) + 1):
        a = O.pcg(A, f, Minv, rtol=1e-10, maxit=j, flexible=False)
        b = O.pcg(A, f, Minv, rtol=1e-10, maxit=j, flexible=True)
        assert a.iters[0] == b.iters[0] == j
        np.testing.assert_allclose(b.x, a.x, rtol=0, atol=1e-10 * np.abs(a.x).max())
    # the flexible branch is live: with a nonsymmetric M^-1 (pre-smoothing only)
    # the two betas give different iterates
    Mns = make_preconditioner(A, P, L, 2 / 3, 1, 0)
    a = O.pcg(A, f, Mns, rtol=1e-10, maxit=6, flexible=False)
    b = O.pcg(A, f, Mns, rtol=1e-10, maxit=6, flexible=True)
    assert np.abs(a.x - b.x).max() > 1e-6 * np.abs(a.x).max()


class _OnceWrongProduct:
    """A sparse matrix whose `call`-th product A @ v carries an error of
    relative size `eps` (every other product is exact): makes the recursive
    residual drift away from the true residual f - A x."""

    def __init__(self, A, call, eps):
        self.A, self.call, self.eps, self.count = A, call, eps, 0
        self.shape = A.shape

    def __matmul__(self, v):
        self.count += 1
        out = self.A @ v
        if self.count == self.call:
            rng = np.random.default_rng(0)
            out = out + self.eps * np.linalg.norm(out) * rng.standard_normal(out.shape) / np.sqrt(out.size)
        return out


def test_residual_replacement_forced():
    """One inexact product A p early in the iteration: the recursive residual
    then meets the tolerance while the true residual does not, so the true
    residual replaces the recursive one and the iteration continues (the count
    goes on) until the true residual meets the tolerance."""
    A, P, Ac, L = _problem(8, N=10)
    Minv = make_preconditioner(A, P, L, 2 / 3, 1, 1)
    f = np.random.default_rng(9).standard_normal(A.shape[0])
    rtol = 1e-9
    clean = O.pcg(A, f, Minv, rtol=rtol)
    bad = _OnceWrongProduct(A, call=3, eps=1e-5)      # call 1: r0; call 2: q of iteration 1
    res = O.pcg(bad, f, Minv, rtol=rtol)
    assert res.status[0] == O.OK
    assert np.linalg.norm(f - A @ res.x[:, 0]) <= rtol * np.linalg.norm(f)
    h = res.history[0]
    # the replaced residual is far above the recursive one it replaces
    jumps = [i for i in range(1, len(h) - 1) if h[i + 1] > 100 * h[i]]
    assert len(jumps) == 1 and h[jumps[0]] <= rtol * np.linalg.norm(f)
    assert res.iters[0] > clean.iters[0] and res.iters[0] == len(h) - 1
    # the true residual at the replacement was far above the tolerance (a run
    # stopping on the recursive residual would have returned a wrong x), and
    # the restart from it converges in no more iterations than a fresh solve
    assert h[jumps[0] + 1] > 100 * rtol * np.linalg.norm(f)
    assert res.iters[0] - jumps[0] <= clean.iters[0]
