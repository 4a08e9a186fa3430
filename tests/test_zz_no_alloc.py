"""The non-allocating solve entry point (pcg_solve_noalloc, for callers that
cannot allocate device memory) against pcg_solve on the same inputs, through
the C ABI: two calls in a row, the second on a smaller system, so the second
runs on scratch memory that still holds the first call's state.  Both entry
points run the same kernels (direct launches against graph replay), so the
solutions, iteration counts and statuses must agree exactly."""
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


def _case(nl, kind, seed, size, m, k, R):
    A, op, n = make_case(kind, seed, size)
    S = O.relax(A, np.random.default_rng(seed + 1).standard_normal((n, m)), 2 / 3, 10)
    P, _ = O.spectral_basis(S, k)
    M = nl.galerkin_coarse(op, cuda(P), 2 / 3, 1)
    f = np.random.default_rng(seed + 2).standard_normal((n, R))
    return A, op, M, f


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_noalloc_matches_pcg_solve(nl, prec):
    big = _case(nl, "grf", 60, (96, 96), 32, 16, 3)
    small = _case(nl, "fv5", 63, (40, 30), 16, 8, 2)
    for A, op, M, f in (big, small):
        print(f"pcg_solve_noalloc prec={prec} n={f.shape[0]} R={f.shape[1]}", flush=True)
        u_ref, info_ref, rc_ref = nl.pcg_solve(op, M, cuda(f), prec=prec)
        u = torch.zeros_like(u_ref)
        info, rc = nl.pcg_solve_noalloc(op, M, cuda(f), u, prec=prec)
        torch.cuda.synchronize()
        assert rc == rc_ref == nl.OK
        for a, b in zip(info, info_ref):
            assert (a.iters, a.status) == (b.iters, b.status), (a, b)
            assert a.relres == b.relres
        assert torch.equal(u, u_ref)
        uh = host(u)
        for j in range(f.shape[1]):
            assert np.linalg.norm(f[:, j] - A @ uh[:, j]) / np.linalg.norm(f[:, j]) <= 1e-8 * 1.0001
