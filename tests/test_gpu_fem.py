"""GPU parity of the P1 finite-element path (the paper's own discretisation:
jittered Delaunay meshes, the five benchmark families, identity rows on the
Dirichlet boundary) against the float64 oracle, through the C ABI (marked
gpu): the assembled compressed-row matrix, its application and Jacobi sweep,
the spectral basis, and PCG at the paper's settings (K = 72 smoothed vectors,
k = 48, nu = 5, omega = 0.66, rtol 1e-6).

Bars: assembly to 1e-13 of the largest entry and exactly symmetric (the
oracle sums the same terms in another order); y = A x to 1e-14 relative; the
float32 sweep to 2e-5 of the largest entry; the basis as test_gpu_kernels
(singular values, gap-aware subspace bound); PCG float64 form iterations
within +-1 of the oracle, mixed forms the solution bar
||x - x_oracle|| <= 2 rtol ||f|| / lambda_min(A), true relative residual
<= rtol in every form."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as sla
import torch

import oracle as O
from oracle.method import make_preconditioner
import workloads as W
from tests._cases import cuda, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2601_20174_amd as mod
    return mod


def _fem(nl, N, fam, seed):
    pts, tris, bnd = W.p1_mesh(seed, N)
    kt, sK, sM = W.p1_coefficients(fam, seed + 1, len(tris), N)
    A = O.p1_fem(pts, tris, kt, sK, sM, bnd)
    op = nl.p1_operator(pts, tris, bnd, cuda(kt), sK, sM)
    return A, op, pts.shape[0]


@pytest.mark.parametrize("fam", W.P1_FAMILIES)
@pytest.mark.parametrize("N", [9, 64])
def test_p1_assembly(nl, fam, N):
    A, op, n = _fem(nl, N, fam, 100 + N)
    rp, ci, v = host(op.row_ptr), host(op.col_idx), host(op.coef)
    B = sp.csr_matrix((v, ci, rp), shape=(n, n))
    assert abs(B - A).max() <= 1e-13 * abs(A).max()
    assert abs(B - B.T).max() == 0.0
    assert nl.nlsp_operator_size(op) == n


def test_csr_apply_and_sweep(nl):
    A, op, n = _fem(nl, 20, "anisotropic", 7)
    rng = np.random.default_rng(8)
    for R in (1, 3):
        x = rng.standard_normal((n, R))
        y = host(nl.apply_operator(op, cuda(x)))
        ref = A @ x
        assert np.abs(y - ref).max() <= 1e-14 * np.abs(ref).max() * 8
        b = rng.standard_normal((n, R)).astype(np.float32)
        x32 = x.astype(np.float32)
        ys = host(nl.jacobi_sweep_f32(op, 0.66, cuda(b, torch.float32), cuda(x32, torch.float32)))
        xr, br = x32.astype(np.float64), b.astype(np.float64)
        refs = xr + 0.66 * (br - A @ xr) / A.diagonal()[:, None]
        assert np.abs(ys - refs).max() <= 2e-5 * np.abs(refs).max()


def _sin_theta(U, V):
    Qu, _ = np.linalg.qr(U)
    Qv, _ = np.linalg.qr(V)
    return np.linalg.norm(Qu - Qv @ (Qv.T @ Qu), 2)


@pytest.mark.parametrize("fam", W.P1_FAMILIES)
@pytest.mark.parametrize("prec", [0, 1])
def test_p1_setup_spectral_P(nl, fam, prec):
    A, op, n = _fem(nl, 24, fam, 30)
    m, k, omega, s1 = 40, 16, 0.66, 10
    S0 = np.random.default_rng(31).standard_normal((n, m))
    Pr, sig_r = O.spectral_basis(O.relax(A, S0, omega, s1), k)
    P, sig = nl.setup_spectral_P(op, cuda(S0), k, omega, s1, prec)
    P, sig = host(P), host(sig)
    np.testing.assert_allclose(sig[:k + 1], sig_r[:k + 1], rtol=1e-9 if prec == 0 else 2e-5)
    eps = 2.0 ** -52 if prec == 0 else 2.0 ** -23
    bound = 100 * eps * sig_r[0] ** 2 / max((sig_r[k - 1] - sig_r[k]) * sig_r[k - 1], 1e-300)
    assert _sin_theta(P, Pr) <= max(bound, 1e-10)


@pytest.mark.parametrize("fam", W.P1_FAMILIES)
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_p1_pcg_paper_settings(nl, fam, prec):
    """The paper's PCG settings on a 33 x 33-vertex jittered mesh (n = 1089):
    the oracle's basis from 72 relaxed vectors, k = 48, nu = 5 sweeps with
    omega = 0.66, rtol 1e-6, in every precision form."""
    c = W.CfgFem(N=32)
    A, op, n = _fem(nl, c.N, fam, 50)
    S0 = np.random.default_rng(51).standard_normal((n, c.m))
    st = O.setup(A, S0, c.k, c.omega, c.s1)
    f = np.random.default_rng(52).standard_normal((n, 2))
    res = O.pcg(A, f, make_preconditioner(A, st["P"], st["L"], c.omega, c.nu, c.nu), rtol=c.rtol,
                flexible=(prec != 0))
    M = nl.galerkin_coarse(op, cuda(st["P"]), c.omega, c.nu)
    u, info, rc = nl.pcg_solve(op, M, cuda(f), prec=prec, rtol=c.rtol)
    assert rc == nl.OK
    u = host(u)
    lam = float(sla.eigsh(A, k=1, sigma=0, which="LM", return_eigenvectors=False)[0])
    for j in range(f.shape[1]):
        true_rel = np.linalg.norm(f[:, j] - A @ u[:, j]) / np.linalg.norm(f[:, j])
        assert info[j].status == nl.OK and true_rel <= c.rtol * 1.0001, (j, info[j], true_rel)
        if prec == 0:
            assert abs(info[j].iters - res.iters[j]) <= 1, (j, info[j].iters, res.iters[j])
        else:
            assert np.linalg.norm(u[:, j] - res.x[:, j]) <= 2 * c.rtol * np.linalg.norm(f[:, j]) / lam
