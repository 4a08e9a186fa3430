"""The method's steps in float64 (oracle; test infrastructure only).

Follows the NeuraLSP algorithm ("setup and one preconditioner application")
with the SVD-derived basis of Sec. 3 in place of the learned map:

  setup:  D = diag(A)
          S = (I - w D^-1 A)^{s1} S0                  (Sec. 3, near-nullspace vectors)
          P = leading k left singular vectors of S    (Sec. 3, Eckart-Young)
          A_c = P^T A P                               (algorithm setup; appendix eq. coarse_operator)
  apply:  z = 0; nu1 Jacobi sweeps; rho = b - A z;
          solve A_c e_c = P^T rho; z += P e_c; nu2 Jacobi sweeps
  solve:  preconditioned conjugate gradients (Hestenes-Stiefel) with the
          two-grid operator as M^-1 (Sec. 4.1, two-grid solver evaluation)

Where the paper leaves a choice open the oracle takes one reading, and the HIP
path takes the same one: relative residual ||f - A x||_2 / ||f||_2 per
right-hand side; iteration count = number of products A p; on meeting the
tolerance with the recursive residual the true residual is formed and, if it
fails, replaces the recursive one and the iteration restarts from it (beta = 0:
the old direction belongs to a residual up to 1/rtol times smaller and would
swamp the new one); multi-RHS means independent CG per column;
nu1 must equal nu2 (a symmetric preconditioner is needed by PCG).
"""
from __future__ import annotations

import dataclasses
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .operators import jacobi_diag

OK, NOT_CONVERGED = 0, 1
E_INVALID, E_NOT_SPD, E_BREAKDOWN, E_NONFINITE = -1, -2, -3, -4

__all__ = ["relax", "spectral_basis", "randomized_basis", "galerkin", "two_grid_apply", "pcg", "PCGResult",
           "setup", "OK", "NOT_CONVERGED", "E_INVALID", "E_NOT_SPD", "E_BREAKDOWN",
           "E_NONFINITE"]


def relax(A: sp.spmatrix, S0: np.ndarray, omega: float, s1: int) -> np.ndarray:
    """S = (I - w D^-1 A)^{s1} S0: s1 weighted-Jacobi sweeps of the
    homogeneous problem A s = 0 applied to every column (Sec. 3, near-nullspace
    vectors; algorithm setup)."""
    D = jacobi_diag(A)
    S = np.array(S0, dtype=np.float64, copy=True)
    for _ in range(s1):
        S = S - omega * (A @ S) / D[:, None]
    return S


def spectral_basis(S: np.ndarray, k: int):
    """P = U_k, the leading k left singular vectors of S (Sec. 3, SVD-centric
    construction: Eckart-Young-Mirsky).  Only span(P) is determined; each
    column is given the sign that makes its largest-magnitude entry positive
    (lowest index on ties).  Returns (P (n,k), sigma (all singular values,
    descending))."""
    U, sigma, _ = np.linalg.svd(np.asarray(S, dtype=np.float64), full_matrices=False)
    P = np.array(U[:, :k], copy=True)
    for j in range(k):
        i = int(np.argmax(np.abs(P[:, j])))
        if P[i, j] < 0:
            P[:, j] = -P[:, j]
    return P, sigma


def randomized_basis(S: np.ndarray, k: int, Omega: np.ndarray, q: int = 1):
    """P = leading k left singular vectors of S estimated by a randomized
    range finder (the RandomSVD baseline of the experimental setup; the
    sketching methods of Halko, Martinsson and Tropp 2011, cited in the related
    work): with a random test matrix Omega (m x l, l >= k, drawn by the caller),

      Y = S Omega,  Q_Y = orth(Y)
      q times:  Z = S^T Q_Y, Q_Z = orth(Z);  Y = S Q_Z, Q_Y = orth(Y)
      B = Q_Y^T S (l x m),  B = U_B diag(sigma) V_B^T
      P = Q_Y U_B[:, :k]

    (randomized subspace iteration, re-orthonormalised after every product,
    followed by the direct SVD of the small matrix B).  orth is a Householder
    QR.  Same sign convention as spectral_basis.  Returns (P (n, k), sigma
    (l,) the singular values of B, descending)."""
    S = np.asarray(S, dtype=np.float64)
    Y = S @ np.asarray(Omega, dtype=np.float64)
    Qy, _ = np.linalg.qr(Y)
    for _ in range(q):
        Qz, _ = np.linalg.qr(S.T @ Qy)
        Qy, _ = np.linalg.qr(S @ Qz)
    B = Qy.T @ S
    Ub, sigma, _ = np.linalg.svd(B, full_matrices=False)
    P = Qy @ Ub[:, :k]
    for j in range(k):
        i = int(np.argmax(np.abs(P[:, j])))
        if P[i, j] < 0:
            P[:, j] = -P[:, j]
    return P, sigma


def galerkin(A: sp.spmatrix, P: np.ndarray):
    """A_c = P^T A P (algorithm setup; Galerkin restriction R = P^T), made
    exactly symmetric, and its Cholesky factor L (A_c = L L^T).  A_c is SPD
    for SPD A and full-rank P (appendix, two-level subspace correction).
    Raises numpy.linalg.LinAlgError when A_c is not positive definite."""
    Y = A @ P
    Ac = P.T @ Y
    Ac = 0.5 * (Ac + Ac.T)
    L = np.linalg.cholesky(Ac)
    return Ac, L


def two_grid_apply(A: sp.spmatrix, P: np.ndarray, L: np.ndarray | None, b: np.ndarray,
                   omega: float, nu1: int, nu2: int, D: np.ndarray | None = None):
    """One application z = M^-1 b of the two-grid preconditioner (algorithm,
    "apply preconditioner to residual b"): z = 0; nu1 weighted-Jacobi sweeps on
    A z = b; rho = b - A z; solve A_c e_c = P^T rho (Cholesky); z += P e_c;
    nu2 sweeps starting from z.  ``b`` may be (n,) or (n, R) (columns are
    independent).  P with zero columns (or None) gives the smoother alone."""
    if D is None:
        D = jacobi_diag(A)
    b = np.asarray(b, dtype=np.float64)
    Dm = D if b.ndim == 1 else D[:, None]
    z = np.zeros_like(b)
    for _ in range(nu1):
        z = z + omega * (b - A @ z) / Dm
    if P is not None and P.shape[1] > 0:
        rho = b - A @ z
        c = P.T @ rho
        y = sla.solve_triangular(L, c, lower=True)
        e_c = sla.solve_triangular(L.T, y, lower=False)
        z = z + P @ e_c
    for _ in range(nu2):
        z = z + omega * (b - A @ z) / Dm
    return z


@dataclasses.dataclass
class PCGResult:
    x: np.ndarray            # (n, R)
    iters: np.ndarray        # (R,) int
    relres: np.ndarray       # (R,) true ||f - A x|| / ||f||
    status: np.ndarray       # (R,) int status code
    history: list            # per RHS: recursive ||r|| after each iteration (index 0 = r0)


def _pcg_one(A, f, x0, Minv, rtol, maxit, flexible, xstar=None):
    ff = float(np.linalg.norm(f))
    x = np.zeros_like(f) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    hist = []
    anorm = []
    if ff == 0.0:
        return np.zeros_like(f), 0, 0.0, OK, [0.0], anorm
    if not np.all(np.isfinite(f)):
        return x, 0, float("nan"), E_NONFINITE, hist, anorm
    tol = rtol * ff
    r = f - A @ x
    hist.append(float(np.linalg.norm(r)))
    if xstar is not None:
        e = xstar - x
        anorm.append(float(np.sqrt(max(e @ (A @ e), 0.0))))
    if hist[0] <= tol:
        return x, 0, hist[0] / ff, OK, hist, anorm
    z = Minv(r)
    gamma = float(r @ z)
    if not np.isfinite(gamma):
        return x, 0, float("nan"), E_NONFINITE, hist, anorm
    if gamma <= 0.0:
        return x, 0, float(np.linalg.norm(f - A @ x)) / ff, E_BREAKDOWN, hist, anorm
    p = z.copy()
    status = NOT_CONVERGED
    it = 0
    while it < maxit:
        q = A @ p
        delta = float(p @ q)
        if not np.isfinite(delta):
            status = E_NONFINITE
            break
        if delta <= 0.0:
            status = E_BREAKDOWN
            break
        alpha = gamma / delta
        x = x + alpha * p
        r = r - alpha * q
        it += 1
        rn = float(np.linalg.norm(r))
        hist.append(rn)
        if xstar is not None:
            e = xstar - x
            anorm.append(float(np.sqrt(max(e @ (A @ e), 0.0))))
        if not np.isfinite(rn):
            status = E_NONFINITE
            break
        restart = False
        if rn <= tol:
            rt = f - A @ x
            if float(np.linalg.norm(rt)) <= tol:
                status = OK
                break
            r = rt                                  # residual replacement ...
            restart = True                          # ... and a restart from it
        z_new = Minv(r)
        gamma_new = float(r @ z_new)
        if not np.isfinite(gamma_new):
            status = E_NONFINITE
            break
        if gamma_new <= 0.0:
            status = E_BREAKDOWN
            break
        if restart:
            beta = 0.0
        elif flexible:
            beta = (gamma_new - float(r @ z)) / gamma
        else:
            beta = gamma_new / gamma
        p = z_new + beta * p
        z = z_new
        gamma = gamma_new
    relres = float(np.linalg.norm(f - A @ x)) / ff
    return x, it, relres, status, hist, anorm


def pcg(A: sp.spmatrix, f: np.ndarray, Minv=None, rtol: float = 1e-8, maxit: int = 10000,
        x0: np.ndarray | None = None, flexible: bool = False, xstar=None) -> PCGResult:
    """Preconditioned CG (Hestenes-Stiefel) for every column of f independently.

    q = A p; delta = p^T q; alpha = gamma/delta; x += alpha p; r -= alpha q;
    stop when ||r|| <= rtol ||f|| and the true residual also passes (else the
    true residual replaces r and beta = 0 in the next update); z = M^-1 r;
    gamma' = r^T z; beta = gamma'/gamma
    (``flexible``: beta = (gamma' - r^T z_old)/gamma, Polak-Ribiere);
    p = z + beta p.  ``Minv`` defaults to the identity (plain CG).
    ``xstar`` (optional, (n,R)) records the A-norm error after every iteration
    in ``result.history`` entries as (residual_list, anorm_list) pairs.
    """
    f = np.asarray(f, dtype=np.float64)
    if f.ndim == 1:
        f = f[:, None]
    R = f.shape[1]
    if Minv is None:
        Minv = lambda v: v.copy()  # noqa: E731
    X = np.zeros_like(f)
    iters = np.zeros(R, dtype=np.int64)
    relres = np.zeros(R)
    status = np.zeros(R, dtype=np.int64)
    hist = []
    for j in range(R):
        xs = None if xstar is None else np.asarray(xstar)[:, j] if np.ndim(xstar) == 2 else xstar
        x, it, rr, st, h, an = _pcg_one(A, f[:, j], None if x0 is None else x0[:, j], Minv,
                                        rtol, maxit, flexible, xs)
        X[:, j] = x
        iters[j] = it
        relres[j] = rr
        status[j] = st
        hist.append((h, an) if xstar is not None else h)
    return PCGResult(X, iters, relres, status, hist)


def setup(A: sp.spmatrix, S0: np.ndarray, k: int, omega: float, s1: int):
    """The whole setup phase: relaxation, basis, Galerkin operator.
    Returns dict(S, P, sigma, Ac, L, D)."""
    S = relax(A, S0, omega, s1)
    P, sigma = spectral_basis(S, k)
    Ac, L = galerkin(A, P)
    return dict(S=S, P=P, sigma=sigma, Ac=Ac, L=L, D=jacobi_diag(A))


def make_preconditioner(A, P, L, omega, nu1, nu2):
    """M^-1 as a callable for ``pcg`` (nu1 must equal nu2 for PCG)."""
    D = jacobi_diag(A)
    return lambda b: two_grid_apply(A, P, L, b, omega, nu1, nu2, D)
