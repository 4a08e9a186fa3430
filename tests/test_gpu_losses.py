"""GPU parity of the subspace-loss forward/backward kernels against the FP64
oracle, through the C ABI (marked gpu).

Tolerance (derived from the arithmetic).  The kernels form T = P^T [B | P]
with float32 MFMA over row slabs (each output entry accumulates in float32
over at most `n` rows, four products per step) and add slabs in float64, so
every entry of T carries an error of at most g_T = (n/4 + 8) u (|P|^T [|B| |P|])
with u = 2^-24 (Higham's gamma bound for a length-(n/4 + 8) float32 sum).  The
loss and the backward's small matrix are formed from T in float64, and the
backward's products [B | P] M again accumulate in float32 over m + k terms.
The tests propagate these bounds to first order with absolute values
(`_bounds`) and require the GPU to be within twice that of the oracle,
computed in float64 from the same float32 inputs.  A dropped term, a sign or
an index error is O(1) of the loss and fails."""
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


def _inputs(seed, batch, n, k, m, ortho=True):
    Ps, Bs = [], []
    for b in range(batch):
        Bm = W.normal_block(W.seed_for(5, 1, seed * 100 + b), n, m) @ np.diag(np.linspace(3.0, 0.2, m))
        Pm = W.normal_block(W.seed_for(5, 2, seed * 100 + b), n, k)
        if ortho:
            Pm, _ = np.linalg.qr(Pm)
        else:
            Pm = Pm / np.sqrt(n)
        Ps.append(Pm.astype(np.float32))
        Bs.append(Bm.astype(np.float32))
    return np.stack(Ps), np.stack(Bs)


def _bounds(P, B, w):
    """First-order worst-case error bounds of the loss and of dL/dP (see the
    module docstring); P, B are float64 copies of the float32 inputs."""
    n, k = P.shape
    m = B.shape[1]
    gT = (n / 4 + 8) * U32
    aP, aB = np.abs(P), np.abs(B)
    dC = gT * (aP.T @ aB)
    dG = gT * (aP.T @ aP)
    C, G = P.T @ B, P.T @ P
    bb = np.sum(B * B)
    dbb = (n + 8) * U32 * bb
    if w is None:
        H = C @ C.T
        dH = np.abs(C) @ dC.T + dC @ np.abs(C).T
        lt = -2 * np.trace(H) + np.sum(G * H)
        dl = 2 * np.trace(dH) + np.sum(dG * np.abs(H)) + np.sum(np.abs(G) * dH)
        dL = dl / bb + abs(lt) * dbb / bb ** 2
        M1 = -(2 / bb) * C.T @ (2 * np.eye(k) - G)
        M2 = (2 / bb) * H
        dM1 = (2 / bb) * (dC.T @ np.abs(2 * np.eye(k) - G) + np.abs(C).T @ dG) + np.abs(M1) * (dbb / bb + U32)
        dM2 = (2 / bb) * dH + np.abs(M2) * (dbb / bb + U32)
        X, M, dM = np.hstack([B, P]), np.vstack([M1, M2]), np.vstack([dM1, dM2])
    else:
        H = np.sum(C * C, axis=1)
        dH = 2 * np.sum(np.abs(C) * dC, axis=1)
        lt = np.sum(w * H)
        dL = np.sum(np.abs(w) * dH) / bb + abs(lt) * dbb / bb ** 2
        M = -(2 / bb) * C.T * w[None, :]
        dM = (2 / bb) * dC.T * np.abs(w)[None, :] + np.abs(M) * (dbb / bb + U32)
        X = B
    gX = (X.shape[1] / 4 + 8) * U32
    dgP = gX * (np.abs(X) @ np.abs(M)) + np.abs(X) @ dM
    return dL, dgP


CASES = [  # batch, n, k, m: ragged n, k, m not multiples of 16, several slabs
    (3, 200, 5, 7),
    (2, 1000, 32, 64),
    (4, 129, 16, 16),
    (2, 3001, 20, 100),
    (1, 777, 64, 128),
]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("ortho", [True, False])
def test_subspace_loss_fwd_bwd(nl, case, weighted, ortho):
    batch, n, k, m = case
    P32, B32 = _inputs(1, batch, n, k, m, ortho)
    w = O.nlss_weights(k).astype(np.float32) if weighted else None
    Pt, Bt = torch.tensor(P32, device="cuda"), torch.tensor(B32, device="cuda")
    wt = torch.tensor(w, device="cuda") if weighted else None
    loss, saved = nl.subspace_loss_fwd(Pt, Bt, wt)
    g = torch.linspace(0.5, 2.0, batch, dtype=torch.float32, device="cuda")
    gP = host(nl.subspace_loss_bwd(Pt, Bt, saved, g))
    loss = host(loss)
    for b in range(batch):
        P, B = P32[b].astype(np.float64), B32[b].astype(np.float64)
        if weighted:
            w64 = w.astype(np.float64)
            ref = O.weighted_energy_loss(P, B, w64)
            gref = O.weighted_energy_loss_grad(P, B, w64)
        else:
            ref = O.subspace_loss(P, B)
            gref = O.subspace_loss_grad(P, B)
        dL, dgP = _bounds(P, B, w.astype(np.float64) if weighted else None)
        gb = float(host(g)[b])
        assert abs(loss[b] - ref) <= 2 * dL + abs(ref) * U32, (b, loss[b], ref, dL)
        err = np.abs(gP[b] - gb * gref)
        assert np.all(err <= 2 * gb * dgP + 1e-30), (b, err.max(), (gb * dgP).min())


def test_nlss_weights_give_nlss_loss(nl):
    """With colw_j = (k - j + 1)/k the weighted loss is the NLSS loss of the
    paper's prefix definition (evaluated by the oracle term by term)."""
    batch, n, k, m = 2, 500, 12, 24
    P32, B32 = _inputs(2, batch, n, k, m, True)
    w = torch.tensor(O.nlss_weights(k).astype(np.float32), device="cuda")
    loss, _ = nl.subspace_loss_fwd(torch.tensor(P32, device="cuda"), torch.tensor(B32, device="cuda"), w)
    for b in range(batch):
        ref = O.nlss_loss(P32[b].astype(np.float64), B32[b].astype(np.float64))
        assert abs(float(host(loss)[b]) - ref) <= 1e-5


def test_autograd_function_and_determinism(nl):
    batch, n, k, m = 3, 640, 16, 32
    P32, B32 = _inputs(3, batch, n, k, m, False)
    Pt = torch.tensor(P32, device="cuda", requires_grad=True)
    Bt = torch.tensor(B32, device="cuda")
    L = nl.subspace_loss(Pt, Bt)
    (L * torch.arange(1, batch + 1, device="cuda", dtype=torch.float32)).sum().backward()
    g1 = Pt.grad.clone()
    loss, saved = nl.subspace_loss_fwd(Pt.detach(), Bt)
    g2 = nl.subspace_loss_bwd(Pt.detach(), Bt, saved, torch.arange(1, batch + 1, device="cuda",
                                                                    dtype=torch.float32))
    assert torch.equal(L.detach(), loss)
    assert torch.equal(g1, g2)


def test_invalid_arguments(nl):
    P = torch.zeros(1, 100, 65, device="cuda")     # k > 64
    B = torch.zeros(1, 100, 8, device="cuda")
    with pytest.raises(nl.NlspError):
        nl.subspace_loss_fwd(P, B)


@pytest.mark.slow
def test_full_size_batch(nl):
    """64 fields of 128^2 unknowns, k = 32, m = 64: every loss and the
    gradients of four samples against the oracle."""
    batch, n, k, m = 64, 128 * 128, 32, 64
    P32, B32 = _inputs(4, batch, n, k, m, True)
    Pt, Bt = torch.tensor(P32, device="cuda"), torch.tensor(B32, device="cuda")
    loss, saved = nl.subspace_loss_fwd(Pt, Bt)
    ones = torch.ones(batch, device="cuda")
    gP = nl.subspace_loss_bwd(Pt, Bt, saved, ones)
    loss = host(loss)
    for b in range(batch):
        P, B = P32[b].astype(np.float64), B32[b].astype(np.float64)
        dL, _ = _bounds(P, B, None)
        assert abs(loss[b] - O.subspace_loss(P, B)) <= 2 * dL + 1e-7
    for b in (0, 17, 40, 63):
        P, B = P32[b].astype(np.float64), B32[b].astype(np.float64)
        _, dgP = _bounds(P, B, None)
        assert np.all(np.abs(host(gP[b]) - O.subspace_loss_grad(P, B)) <= 2 * dgP)


def _energy_bound(P, S):
    """First-order bound on Energy(r) from the product bound of T = P^T S
    (module docstring) and a float32 sum bound on ||S||^2."""
    n = P.shape[0]
    g = (n / 4 + 8) * U32
    T = P.T @ S
    dT = g * (np.abs(P).T @ np.abs(S))
    de = np.sum(2.0 * np.abs(T) * dT + dT * dT, axis=1)
    bb = float(np.sum(S * S))
    E = np.cumsum(np.sum(T * T, axis=1)) / bb
    return np.cumsum(de) / bb + E * (n + 8) * U32


@pytest.mark.parametrize("n,k,m", [(1000, 5, 7), (4099, 16, 64), (2311, 40, 33)])
def test_captured_energy(nl, n, k, m):
    """Energy_b(r) of the leading r columns of orthonormal bases against the
    oracle's captured_energy, r = 1..k, one basis per sample; the curve is
    non-decreasing and ends at the energy of the whole basis."""
    rng = np.random.default_rng(n + k)
    batch = 3
    Ps, Ss = [], []
    for b in range(batch):
        S = rng.standard_normal((n, m)) * np.exp(-0.1 * np.arange(m))[None, :]
        Q, _ = np.linalg.qr(rng.standard_normal((n, k)) + S[:, :1])
        Ps.append(Q.astype(np.float32))
        Ss.append(S.astype(np.float32))
    P32, S32 = np.stack(Ps), np.stack(Ss)
    E = host(nl.captured_energy(torch.tensor(P32, device="cuda"), torch.tensor(S32, device="cuda")))
    assert E.shape == (batch, k) and E.dtype == np.float64
    for b in range(batch):
        P64, S64 = P32[b].astype(np.float64), S32[b].astype(np.float64)
        ref = np.array([O.captured_energy(P64, S64, r) for r in range(1, k + 1)])
        tol = 2.0 * _energy_bound(P64, S64) + 1e-15
        assert np.all(np.abs(E[b] - ref) <= tol), np.max(np.abs(E[b] - ref) / tol)
        assert np.all(np.diff(E[b]) >= 0.0)


def test_captured_energy_svd_prefix(nl):
    """For the leading left singular vectors of S the curve is the prefix sums
    of sigma^2 over their total (Eckart-Young), up to the float32 rounding of
    the basis."""
    rng = np.random.default_rng(11)
    n, m, k = 3000, 48, 24
    S = rng.standard_normal((n, m)) * np.exp(-0.15 * np.arange(m))[None, :]
    U, sig, _ = np.linalg.svd(S, full_matrices=False)
    P32, S32 = U[:, :k].astype(np.float32)[None], S.astype(np.float32)[None]
    E = host(nl.captured_energy(torch.tensor(P32, device="cuda"), torch.tensor(S32, device="cuda")))[0]
    closed = np.cumsum(sig[:k] ** 2) / np.sum(sig ** 2)
    assert np.max(np.abs(E - closed)) <= 1e-5
