"""GPU parity of the operator and setup kernels against the FP64 oracle,
through the C ABI (marked gpu)."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import oracle as O
import workloads as W
from tests._cases import make_case, cuda, host, gpu_op

pytestmark = pytest.mark.gpu

KINDS = ["poisson", "fv5", "fv7", "q1"]


@pytest.fixture(scope="module")
def nl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2601_20174_amd as mod
    return mod


@pytest.mark.parametrize("kind", KINDS + ["poisson_big"])
@pytest.mark.parametrize("R", [1, 2, 3, 16])
def test_apply_operator(nl, kind, R):
    if kind == "poisson_big":   # several slabs of y-lines, lines split over blocks
        A, op, n = make_case("poisson", 1, (300, 70))
        x = np.random.default_rng(2).standard_normal((n, R))
        y = host(nl.apply_operator(op, cuda(x)))
        ref = A @ x
        scale = abs(A).sum(axis=1).A.ravel()[:, None] * np.abs(x).max()
        assert np.all(np.abs(y - ref) <= 1e-14 * scale)
        return
    A, op, n = make_case(kind, 1, (37, 29) if kind != "q1" else (41, 41))
    x = np.random.default_rng(2).standard_normal((n, R))
    y = host(nl.apply_operator(op, cuda(x)))
    ref = A @ x
    scale = abs(A).sum(axis=1).A.ravel()[:, None] * np.abs(x).max()
    assert np.all(np.abs(y - ref) <= 1e-14 * scale)


def test_q1_stencil_matches_oracle_assembly(nl):
    rng = np.random.default_rng(3)
    et = np.stack([10 ** rng.uniform(-3, 0, 8), rng.uniform(0, np.pi, 8)], 1)
    st = host(nl.q1_aniso_stencil(cuda(et)))
    side = 5
    c = 2 * side + 2                       # centre unknown of a 5x5 grid
    for s in range(8):
        row = O.q1_aniso(side, et[s, 0], et[s, 1]).toarray()[c].reshape(side, side)
        np.testing.assert_allclose(st[s].reshape(3, 3), row[1:4, 1:4], atol=1e-14)


@pytest.mark.parametrize("kind", ["fv5", "q1", "fv7", "poisson"])
@pytest.mark.parametrize("R", [2, 8])
def test_jacobi_sweep_f32(nl, kind, R):
    A, op, n = make_case(kind, 4, (33, 20) if kind != "q1" else (30, 30))
    rng = np.random.default_rng(5)
    b, x = rng.standard_normal((n, R)), rng.standard_normal((n, R))
    y = host(nl.jacobi_sweep_f32(op, 2 / 3, cuda(b, torch.float32), cuda(x, torch.float32)))
    D = A.diagonal()[:, None]
    xr = x.astype(np.float32).astype(np.float64)
    br = b.astype(np.float32).astype(np.float64)
    ref = xr + (2 / 3) * (br - A @ xr) / D
    assert np.abs(y - ref).max() <= 2e-5 * np.abs(ref).max()


def _fv7(nl, nx, ny, nz, seed, lognormal=False):
    rng = np.random.default_rng(seed)
    if lognormal:
        a = np.exp(rng.standard_normal((nz, ny, nx)))
    else:
        a = np.where(rng.integers(0, 2, size=(nz, ny, nx)) == 1, 1e3, 1.0)
    return O.fv_harmonic_3d(a), gpu_op(nl.OP_FV7, nx, ny, nz, a), nx * ny * nz


# 3-D FV7 with 2, 4 or 8 lanes of 16-byte vectors per row takes the z-march
# kernel: tiles of 16 x 8 cells, ragged in x, y and in the z-chunks (4 or 8
# planes), grids narrower than one tile, and two planes only
ZSHAPES = [(37, 29, 23), (16, 8, 4), (5, 3, 2), (50, 17, 9), (33, 9, 40)]


@pytest.mark.parametrize("shape", ZSHAPES)
@pytest.mark.parametrize("R", [4, 8, 16])
def test_apply_operator_fv7_zmarch(nl, shape, R):
    A, op, n = _fv7(nl, *shape, seed=sum(shape), lognormal=shape[0] % 2 == 1)
    x = np.random.default_rng(R).standard_normal((n, R))
    y = host(nl.apply_operator(op, cuda(x)))
    ref = A @ x
    scale = abs(A).sum(axis=1).A.ravel()[:, None] * np.abs(x).max()
    assert np.all(np.abs(y - ref) <= 1e-14 * scale)


@pytest.mark.parametrize("shape", ZSHAPES)
@pytest.mark.parametrize("R", [8, 16, 32])
def test_jacobi_sweep_f32_fv7_zmarch(nl, shape, R):
    A, op, n = _fv7(nl, *shape, seed=sum(shape) + 1, lognormal=shape[1] % 2 == 1)
    rng = np.random.default_rng(R)
    b, x = rng.standard_normal((n, R)), rng.standard_normal((n, R))
    y = host(nl.jacobi_sweep_f32(op, 2 / 3, cuda(b, torch.float32), cuda(x, torch.float32)))
    D = A.diagonal()[:, None]
    xr = x.astype(np.float32).astype(np.float64)
    br = b.astype(np.float32).astype(np.float64)
    ref = xr + (2 / 3) * (br - A @ xr) / D
    assert np.abs(y - ref).max() <= 2e-5 * np.abs(ref).max()


def test_fv7_operator_kernels_full_size(nl):
    """The 3-D benchmark workload (FV7, 128^3 cells, 16^3-cell blocks of a in
    {1, 1e3}, 16 right-hand sides) in the launch configuration the benchmark
    times: float64 y = A x and the float32 Jacobi sweep, every element against
    the oracle's assembled operator."""
    c4 = W.Cfg4()
    a = c4.coef()
    A = O.fv_harmonic_3d(a)
    op = gpu_op(nl.OP_FV7, c4.N, c4.N, c4.N, a)
    rng = np.random.default_rng(44)
    x = rng.standard_normal((c4.n, c4.R))
    y = host(nl.apply_operator(op, cuda(x)))
    ref = A @ x
    scale = abs(A).sum(axis=1).A.ravel()[:, None] * np.abs(x).max()
    assert np.all(np.abs(y - ref) <= 1e-14 * scale)
    del y, ref
    b = rng.standard_normal((c4.n, c4.R)).astype(np.float32)
    x32 = x.astype(np.float32)
    y = host(nl.jacobi_sweep_f32(op, 2 / 3, cuda(b, torch.float32), cuda(x32, torch.float32)))
    xr, br = x32.astype(np.float64), b.astype(np.float64)
    ref = xr + (2 / 3) * (br - A @ xr) / A.diagonal()[:, None]
    assert np.abs(y - ref).max() <= 2e-5 * np.abs(ref).max()


def _sin_theta(U, V):
    """sin of the largest principal angle between span(U) and span(V)."""
    Qu, _ = np.linalg.qr(U)
    Qv, _ = np.linalg.qr(V)
    return np.linalg.norm(Qu - Qv @ (Qv.T @ Qu), 2)


# m above 128: the eigensolver's multi-workgroup form (one launch per round)
@pytest.mark.parametrize("kind,size,m,k", [("poisson", (32, 32), 32, 16), ("fv5", (45, 38), 48, 20),
                                           ("q1", (40, 40), 64, 32), ("fv7", (17, 13), 40, 8),
                                           ("fv5", (45, 38), 150, 60), ("q1", (40, 40), 200, 90),
                                           ("fv7", (17, 13), 256, 64)])
@pytest.mark.parametrize("prec", [0, 1])
def test_setup_spectral_P(nl, kind, size, m, k, prec):
    A, op, n = make_case(kind, 6, size)
    S0 = np.random.default_rng(7).standard_normal((n, m))
    omega, s1 = 2 / 3, 10
    S = O.relax(A, S0, omega, s1)
    Pr, sig_r = O.spectral_basis(S, k)
    P, sig = nl.setup_spectral_P(op, cuda(S0), k, omega, s1, prec)
    P, sig = host(P), host(sig)
    # singular values: float64 Gram route loses ~eps*sigma_1^2/sigma_j^2 relative
    tol = 1e-9 if prec == 0 else 2e-5
    np.testing.assert_allclose(sig[:k + 1], sig_r[:k + 1], rtol=tol)
    np.testing.assert_allclose(P.T @ P, np.eye(k), atol=1e-12)
    # gap-aware subspace bound (Wedin), safety factor 10
    eps = 2.0 ** -52 if prec == 0 else 2.0 ** -23
    gap = sig_r[k - 1] - sig_r[k]
    bound = 10 * eps * sig_r[0] ** 2 / max(gap * sig_r[k - 1], 1e-300) * 10
    assert _sin_theta(P, Pr) <= max(bound, 1e-10)
    # sign convention where columns are determined (simple, separated sigmas)
    for j in range(k):
        assert P[np.argmax(np.abs(P[:, j])), j] > 0


@pytest.mark.parametrize("k", [16, 40])
@pytest.mark.parametrize("nu", [1, 2])
def test_galerkin_float_basis_only(nl, k, nu):
    """Only the float32 smoothed basis asked for: on 3-D FV7 grids the last
    float64 sweep stores it rounded; it equals the float32 rounding of the
    float64 basis bit for bit, and the factors are unchanged."""
    A, op, n = make_case("fv7", 8, (17, 13))
    S = O.relax(A, np.random.default_rng(9).standard_normal((n, 2 * k)), 2 / 3, 10)
    Pr, _ = O.spectral_basis(S, k)
    M = nl.galerkin_coarse(op, cuda(Pr), 2 / 3, nu, q64=True, q32=True)
    M32 = nl.galerkin_coarse(op, cuda(Pr), 2 / 3, nu, q64=False, q32=True)
    assert torch.equal(M32.Q32, M.Q64.float())
    assert torch.equal(M32.Q32, M.Q32)
    assert torch.equal(M32.Ac, M.Ac) and torch.equal(M32.Linv, M.Linv)


# k above 64: the row-by-row triangular inverse in LDS
@pytest.mark.parametrize("kind,size,k", [("poisson", (32, 32), 16), ("fv5", (45, 38), 20),
                                         ("q1", (40, 40), 17), ("fv7", (17, 13), 8),
                                         ("fv5", (45, 38), 100), ("fv7", (17, 13), 128)])
@pytest.mark.parametrize("nu", [1, 2])
def test_galerkin_coarse(nl, kind, size, k, nu):
    A, op, n = make_case(kind, 8, size)
    S = O.relax(A, np.random.default_rng(9).standard_normal((n, 2 * k)), 2 / 3, 10)
    Pr, _ = O.spectral_basis(S, k)
    Ac_r, L_r = O.galerkin(A, Pr)
    M = nl.galerkin_coarse(op, cuda(Pr), 2 / 3, nu)
    Ac, L, Linv = host(M.Ac), host(M.L), host(M.Linv)
    np.testing.assert_allclose(Ac, Ac_r, atol=1e-13 * np.abs(Ac_r).max())
    assert np.array_equal(Ac, Ac.T)
    np.testing.assert_allclose(L, L_r, atol=1e-12 * np.abs(L_r).max())
    kp = nl.nlsp_padded_rank(k)
    np.testing.assert_allclose(Linv[:k, :k] @ L, np.eye(k), atol=1e-11)
    assert np.all(Linv[k:, :] == 0) and np.all(Linv[:, k:] == 0)
    D = A.diagonal()[:, None]
    Qr = Pr.copy()
    for _ in range(nu):
        Qr = Qr - (2 / 3) * (A @ Qr) / D
    Q64, Q32 = host(M.Q64), host(M.Q32)
    assert Q64.shape == (n, kp)
    np.testing.assert_allclose(Q64[:, :k], Qr, atol=1e-14 * np.abs(Qr).max() * 8)
    assert np.all(Q64[:, k:] == 0)
    np.testing.assert_allclose(Q32[:, :k], Qr, atol=1e-6 * np.abs(Qr).max())
