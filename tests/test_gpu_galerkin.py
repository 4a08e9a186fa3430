"""GPU parity of the batched Galerkin product A_c = P^T A P and its backward
A P (G + G^T) against the FP64 oracle, through the C ABI (marked gpu).

Tolerance (derived from the arithmetic).  Y = A P is formed in float32 from
the float64 stencil (coefficients rounded to float32, harmonic means and the
row sum in float32): |dY| <= 16 u (|A| |P|), u = 2^-24.  A_c accumulates
P^T Y in float32 MFMA over at most n rows (n/4 + 8 roundings) and adds slabs
in float64: |dA_c| <= (n/4 + 8) u |P|^T |Y| + |P|^T |dY|.  The backward
accumulates Y (G + G^T) in float32 over kp terms: |dgP| <= (|dY| + (kp/4 + 8) u
|Y|) |G + G^T|.  Tests require twice these bounds."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests._cases import host

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def nl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2601_20174_amd as mod
    return mod


def _batch(nl, kind, batch, seed):
    """(list of oracle operators, batched GPU Operator, n)"""
    rng = np.random.default_rng(seed)
    if kind == "fv5":
        nx, ny = 37, 29
        coefs = [np.exp(rng.standard_normal((ny, nx))) for _ in range(batch)]
        As = [O.fv_harmonic_2d(c) for c in coefs]
        op = nl.Operator(nl.OP_FV5, nx, ny, 1, torch.tensor(np.concatenate([c.ravel() for c in coefs]),
                                                            dtype=torch.float64, device="cuda"))
        return As, op, nx * ny
    if kind == "grf":
        N = 48
        coefs = [W.lognormal_field(seed + b, N) for b in range(batch)]
        As = [O.fv_harmonic_2d(c) for c in coefs]
        op = nl.Operator(nl.OP_FV5, N, N, 1, torch.tensor(np.concatenate([c.ravel() for c in coefs]),
                                                          dtype=torch.float64, device="cuda"))
        return As, op, N * N
    if kind == "fv7":
        nx, ny, nz = 9, 7, 5
        coefs = [np.where(rng.integers(0, 2, (nz, ny, nx)) == 1, 1e3, 1.0) for _ in range(batch)]
        As = [O.fv_harmonic_3d(c) for c in coefs]
        op = nl.Operator(nl.OP_FV7, nx, ny, nz, torch.tensor(np.concatenate([c.ravel() for c in coefs]),
                                                             dtype=torch.float64, device="cuda"))
        return As, op, nx * ny * nz
    if kind == "q1":
        side = 23
        et = np.stack([10 ** rng.uniform(-3, 0, batch), rng.uniform(0, np.pi, batch)], 1)
        st = nl.q1_aniso_stencil(torch.tensor(et, dtype=torch.float64, device="cuda"))
        As = [O.q1_aniso(side, et[b, 0], et[b, 1]) for b in range(batch)]
        op = nl.Operator(nl.OP_STENCIL9, side, side, 1, st.reshape(-1).contiguous())
        return As, op, side * side
    if kind == "poisson":
        nx, ny = 31, 17
        return [O.poisson5(nx, ny)] * batch, nl.Operator(nl.OP_POISSON5, nx, ny), nx * ny
    raise ValueError(kind)


def _bounds(A, P, G):
    aA, aP = abs(A), np.abs(P)
    n, k = P.shape
    AP = aA @ aP
    dY = 16 * U32 * AP
    Y = np.abs(A @ P)
    dAc = (n / 4 + 8) * U32 * (aP.T @ Y) + aP.T @ dY
    kp = (k + 15) // 16 * 16
    S = np.abs(G + G.T)
    dgP = (dY + (kp / 4 + 8) * U32 * Y) @ S
    return dAc, dgP


@pytest.mark.parametrize("kind", ["fv5", "grf", "fv7", "q1", "poisson"])
@pytest.mark.parametrize("k", [5, 16, 20])
def test_galerkin_fwd_bwd(nl, kind, k):
    batch = 3
    As, op, n = _batch(nl, kind, batch, 11)
    rng = np.random.default_rng(7)
    P32 = np.stack([np.linalg.qr(rng.standard_normal((n, k)))[0] for _ in range(batch)]).astype(np.float32)
    G32 = rng.standard_normal((batch, k, k)).astype(np.float32)
    Pt = torch.tensor(P32, device="cuda")
    Ac, Y = nl.galerkin_fwd(op, Pt)
    gP = host(nl.galerkin_bwd(Y, torch.tensor(G32, device="cuda")))
    Ac = host(Ac)
    for b in range(batch):
        A, P, G = As[b], P32[b].astype(np.float64), G32[b].astype(np.float64)
        ref = P.T @ (A @ P)
        dAc, dgP = _bounds(A, P, G)
        assert np.all(np.abs(Ac[b] - ref) <= 2 * dAc + np.abs(ref) * U32), (b, np.abs(Ac[b] - ref).max())
        assert np.array_equal(Ac[b], Ac[b].T)
        gref = O.galerkin_coarse_vjp(A, P, G)
        assert np.all(np.abs(gP[b] - gref) <= 2 * dgP), (b, np.abs(gP[b] - gref).max())


def test_galerkin_eigenvalues_match_oracle_setup(nl):
    """A_c of an orthonormal basis from the oracle's own spectral setup: the
    float32 product reproduces the oracle's float64 Galerkin operator."""
    As, op, n = _batch(nl, "grf", 2, 3)
    Ps = []
    for b in range(2):
        S0 = W.normal_block(100 + b, n, 24)
        st = O.setup(As[b], S0, 12, 2 / 3, 10)
        Ps.append(st["P"])
    P32 = np.stack(Ps).astype(np.float32)
    Ac, _ = nl.galerkin_fwd(op, torch.tensor(P32, device="cuda"))
    for b in range(2):
        P = P32[b].astype(np.float64)
        ref = P.T @ (As[b] @ P)
        ev, evr = np.linalg.eigvalsh(host(Ac)[b].astype(np.float64)), np.linalg.eigvalsh(ref)
        assert np.allclose(ev, evr, rtol=1e-5, atol=0)


def test_autograd_and_directional_finite_difference(nl):
    """torch.autograd through GalerkinProduct matches galerkin_bwd, and a
    central difference of L(P) = <W, A_c(P)> along a random direction V
    matches <dL/dP, V> (float32 arithmetic: relative 1e-3)."""
    As, op, n = _batch(nl, "fv5", 2, 5)
    rng = np.random.default_rng(9)
    P32 = (rng.standard_normal((2, n, 8)) / np.sqrt(n)).astype(np.float32)
    Wt = torch.tensor(rng.standard_normal((2, 8, 8)).astype(np.float32), device="cuda")
    Pt = torch.tensor(P32, device="cuda", requires_grad=True)
    Ac = nl.galerkin_product(Pt, op)
    (Ac * Wt).sum().backward()
    _, Y = nl.galerkin_fwd(op, Pt.detach())
    assert torch.equal(Pt.grad, nl.galerkin_bwd(Y, Wt))
    V = torch.tensor(rng.standard_normal(P32.shape).astype(np.float32), device="cuda")
    h = 1e-2
    Lp = (nl.galerkin_fwd(op, Pt.detach() + h * V)[0].double() * Wt.double()).sum()
    Lm = (nl.galerkin_fwd(op, Pt.detach() - h * V)[0].double() * Wt.double()).sum()
    fd = float((Lp - Lm) / (2 * h))
    an = float((Pt.grad.double() * V.double()).sum())
    assert abs(fd - an) <= 1e-3 * max(1.0, abs(an))


def test_subspace_loss_directional_finite_difference(nl):
    rng = np.random.default_rng(4)
    n, k, m = 900, 8, 24
    B = torch.tensor(rng.standard_normal((2, n, m)).astype(np.float32), device="cuda")
    Pt = torch.tensor((rng.standard_normal((2, n, k)) / np.sqrt(n)).astype(np.float32), device="cuda",
                      requires_grad=True)
    nl.subspace_loss(Pt, B).sum().backward()
    # direction scaled like P; step 3e-2: central-difference truncation 1e-3
    # (float64 evaluation of the same data), float32 loss noise below that
    V = torch.tensor((rng.standard_normal((2, n, k)) / np.sqrt(n)).astype(np.float32), device="cuda")
    h = 3e-2
    Lp = nl.subspace_loss_fwd(Pt.detach() + h * V, B)[0].double().sum()
    Lm = nl.subspace_loss_fwd(Pt.detach() - h * V, B)[0].double().sum()
    fd = float((Lp - Lm) / (2 * h))
    an = float((Pt.grad.double() * V.double()).sum())
    assert abs(fd - an) <= 1e-2 * abs(an)


def test_invalid(nl):
    As, op, n = _batch(nl, "fv5", 2, 1)
    with pytest.raises(ValueError):
        nl.galerkin_fwd(op, torch.zeros(3, n, 4, device="cuda"))    # only 2 coefficient fields
    with pytest.raises(nl.NlspError):
        nl.galerkin_fwd(op, torch.zeros(2, n, 65, device="cuda"))   # k > 64


# ------------------------------------------------- Galerkin-convergence term
def _gterm_bounds(A, P, S):
    """First-order worst-case bounds of the GPU's J and dJ/dP (float32 stencil
    and MFMA products over n/4 + 8 steps, slab sums and the small solves in
    float64, M rounded to float32 and X M accumulated over (m + k)/4 + 8 steps):
      |dAS| <= 16 u |A||S|,  |dAP| <= 16 u |A||P|,  g = (n/4 + 8) u
      |dW| <= g |P|^T|AS| + |P|^T|dAS|,  |dAc| <= g |P|^T|AP| + |P|^T|dAP|
      |dJ| <= sum |S||dAS| + 2 <|Z|, |dW|> + <|Z||Z|^T, |dAc|> + u |J|
      |dZ| <= |Ac^-1| (|dW| + |dAc||Z|)
      |dgrad| <= 2 (|dAP||ZZ^T| + |AP| (|dZ||Z|^T + |Z||dZ|^T) + |dAS||Z|^T
                 + |AS||dZ|^T) + ((m + k)/4 + 9) u |X||M|,  X = [AS | AP]."""
    n, k = P.shape
    m = S.shape[1]
    aA, aP, aS = abs(A), np.abs(P), np.abs(S)
    AS, AP = A @ S, A @ P
    dAS, dAP = 16 * U32 * (aA @ aS), 16 * U32 * (aA @ aP)
    g = (n / 4 + 8) * U32
    dW = g * (aP.T @ np.abs(AS)) + aP.T @ dAS
    dAc = g * (aP.T @ np.abs(AP)) + aP.T @ dAP
    Ac = P.T @ AP
    Acinv = np.linalg.inv(0.5 * (Ac + Ac.T))
    Z = Acinv @ (P.T @ AS)
    aZ = np.abs(Z)
    J = float(np.sum(S * AS) - np.sum((P.T @ AS) * Z))
    dJ = np.sum(aS * dAS) + 2 * np.sum(aZ * dW) + np.sum((aZ @ aZ.T) * dAc) + U32 * abs(J)
    dZ = np.abs(Acinv) @ (dW + dAc @ aZ)
    M = np.vstack([-2 * Z.T, 2 * Z @ Z.T])
    X = np.hstack([AS, AP])
    dg = 2 * (dAP @ np.abs(Z @ Z.T) + np.abs(AP) @ (dZ @ aZ.T + aZ @ dZ.T) + dAS @ aZ.T + np.abs(AS) @ dZ.T)
    dg = dg + ((m + k) / 4 + 9) * U32 * (np.abs(X) @ np.abs(M))
    return dJ, dg


@pytest.mark.parametrize("kind", ["fv5", "grf", "fv7", "q1", "poisson"])
@pytest.mark.parametrize("k,m", [(5, 7), (16, 24), (12, 60)])
def test_galerkin_term_fwd_bwd(nl, kind, k, m):
    batch = 3
    As, op, n = _batch(nl, kind, batch, 21)
    rng = np.random.default_rng(17)
    P32 = np.stack([np.linalg.qr(rng.standard_normal((n, k)))[0] for _ in range(batch)]).astype(np.float32)
    S32 = rng.standard_normal((batch, n, m)).astype(np.float32)
    gJ = torch.linspace(0.5, 1.5, batch, dtype=torch.float32, device="cuda")
    J, bad, saved, E = nl.galerkin_term_fwd(op, torch.tensor(P32, device="cuda"), torch.tensor(S32, device="cuda"))
    gP = host(nl.galerkin_term_bwd(op, k, m, saved, gJ))
    J, bad, gJh, E = host(J), host(bad), host(gJ), host(E)
    assert np.all(bad == 0)
    for b in range(batch):
        A, P, S = As[b], P32[b].astype(np.float64), S32[b].astype(np.float64)
        ref = O.galerkin_term(A, P, S)
        gref = O.galerkin_term_grad(A, P, S)
        dJ, dg = _gterm_bounds(A, P, S)
        assert abs(J[b] - ref) <= 2 * dJ, (b, J[b], ref, dJ)
        # E = tr(S^T A S) = J with no coarse space (float32 stencil products)
        Eref = float(np.sum(S * (A @ S)))
        dE = np.sum(np.abs(S) * (16 * U32 * (abs(A) @ np.abs(S)))) + U32 * abs(Eref)
        assert abs(E[b] - Eref) <= 2 * dE, (b, E[b], Eref, dE)
        err = np.abs(gP[b] - gJh[b] * gref)
        assert np.all(err <= 2 * gJh[b] * dg + 1e-30), (b, err.max(), (gJh[b] * dg).max())


def test_galerkin_term_autograd_and_optimum(nl):
    """Autograd through GalerkinTerm equals galerkin_term_bwd; at the top-k
    left singular subspace of A^{1/2} S the GPU's J is the oracle's minimum,
    below J at a random basis (the appendix's optimality statement)."""
    As, op, n = _batch(nl, "grf", 2, 31)
    k, m = 6, 16
    rng = np.random.default_rng(3)
    S32 = rng.standard_normal((2, n, m)).astype(np.float32)
    P32 = np.stack([np.linalg.qr(rng.standard_normal((n, k)))[0] for _ in range(2)]).astype(np.float32)
    Pt = torch.tensor(P32, device="cuda", requires_grad=True)
    St = torch.tensor(S32, device="cuda")
    J, bad, _ = nl.galerkin_term(Pt, St, op)
    (J * torch.tensor([1.0, 2.0], device="cuda")).sum().backward()
    _, _, saved, _ = nl.galerkin_term_fwd(op, Pt.detach(), St)
    assert torch.equal(Pt.grad, nl.galerkin_term_bwd(op, k, m, saved, torch.tensor([1.0, 2.0], device="cuda")))
    # the optimum: P* = A^{-1/2} U_k spans the Galerkin-optimal subspace
    Popt = []
    for b in range(2):
        Ad = As[b].toarray()
        lam, V = np.linalg.eigh(Ad)
        Ah = (V * np.sqrt(lam)) @ V.T
        U = np.linalg.svd(Ah @ S32[b].astype(np.float64), full_matrices=False)[0][:, :k]
        Popt.append(np.linalg.qr(np.linalg.solve(Ah, U))[0])
    Jo = host(nl.galerkin_term_fwd(op, torch.tensor(np.stack(Popt).astype(np.float32), device="cuda"), St)[0])
    Jr = host(J.detach())
    for b in range(2):
        P = Popt[b].astype(np.float32).astype(np.float64)
        Jref = O.galerkin_term(As[b], P, S32[b].astype(np.float64))
        assert abs(Jo[b] - Jref) <= 2 * _gterm_bounds(As[b], P, S32[b].astype(np.float64))[0]
        assert Jo[b] < Jr[b]
