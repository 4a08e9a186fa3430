"""Failure statuses forced from the inputs, through the C ABI (marked gpu).
Each premise is pinned on the oracle first (the exact rank, the singular
coarse matrix, the indefinite operator); every kernel still runs to its
normal end, only the status differs."""
import numpy as np
import pytest
import torch

import oracle as O
from tests._cases import make_case, cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2601_20174_amd as mod
    return mod


@pytest.mark.parametrize("prec", [0, 1])
def test_duplicated_vectors_give_rank_error(nl, prec):
    """S0 = [X, X] with 8 distinct columns has rank 8, and relaxation is
    linear, so S has rank 8 too: asking for k = 12 leaves sigma_12 = 0 in
    exact arithmetic and setup_spectral_P returns NLSP_E_RANK."""
    A, op, n = make_case("poisson", 0, (30, 30))
    X = np.random.default_rng(70).standard_normal((n, 8))
    S0 = np.concatenate([X, X], axis=1)
    _, sig = O.spectral_basis(O.relax(A, S0, 2 / 3, 10), 12)
    assert sig[11] <= 1e-13 * sig[0] and sig[7] > 1e-3 * sig[0]
    with pytest.raises(nl.NlspError) as e:
        nl.setup_spectral_P(op, cuda(S0), 12, 2 / 3, 10, prec)
    assert e.value.status == nl.E_RANK
    # the same vectors with k at their rank are fine
    P, _ = nl.setup_spectral_P(op, cuda(S0), 8, 2 / 3, 10, prec)
    assert torch.isfinite(P).all()


def test_rank_deficient_basis_gives_not_spd(nl):
    """A basis with a zero column makes A_c = P^T A P singular (a zero row and
    column): the oracle's Cholesky fails and galerkin_coarse returns
    NLSP_E_NOT_SPD."""
    A, op, n = make_case("fv5", 71, (33, 27))
    S = O.relax(A, np.random.default_rng(72).standard_normal((n, 16)), 2 / 3, 10)
    P, _ = O.spectral_basis(S, 8)
    P[:, 3] = 0.0
    with pytest.raises(np.linalg.LinAlgError):
        O.galerkin(A, P)
    with pytest.raises(nl.NlspError) as e:
        nl.galerkin_coarse(op, cuda(P), 2 / 3, 1)
    assert e.value.status == nl.E_NOT_SPD


@pytest.mark.parametrize("prec", [0, 1])
def test_negative_definite_operator_breaks_down(nl, prec):
    """PCG on -A (negative definite) with the preconditioner built for A:
    p^T (-A) p < 0 at the first step (or r^T z <= 0 before it), so every
    right-hand side ends with NLSP_E_BREAKDOWN; plain CG in the oracle breaks
    down on the same operator."""
    A, op, n = make_case("poisson", 0, (30, 30))
    S = O.relax(A, np.random.default_rng(73).standard_normal((n, 16)), 2 / 3, 10)
    P, _ = O.spectral_basis(S, 8)
    M = nl.galerkin_coarse(op, cuda(P), 2 / 3, 1)
    neg = torch.tensor([0.0, 1.0, 0.0, 1.0, -4.0, 1.0, 0.0, 1.0, 0.0], dtype=torch.float64, device="cuda")
    op_neg = nl.Operator(nl.OP_STENCIL9, 30, 30, 1, neg)
    f = np.random.default_rng(74).standard_normal((n, 2))
    res = O.pcg(-A, f)
    assert np.all(res.status == O.E_BREAKDOWN)
    u, info, rc = nl.pcg_solve(op_neg, M, cuda(f), prec=prec)
    assert rc == nl.E_BREAKDOWN
    for inf in info:
        assert inf.status == nl.E_BREAKDOWN and inf.iters <= 1, inf
    assert torch.isfinite(u).all()
