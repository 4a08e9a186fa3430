"""GPU against oracle at the configurations the benchmark times (marked gpu).

* The batched anisotropic workload: one system of each grid side drawn by the
  workload generator (64, 96, 128, 192, 256), k = 32, m = 64, 8 right-hand
  sides, the tuned tile the benchmark uses (1024 rows per workgroup), GPU
  setup as in the benchmark.  The oracle runs its own setup (SVD of its own
  relaxed vectors) and its own PCG, so an error in either GPU setup or solve
  shows.
* The 2-D log-normal workload at full size (512 x 512, m = 128, k = 64).

Bars: float64 form, iterations within +-1 of the oracle and a true relative
residual <= rtol; mixed forms (float32 or float16 basis), true relative
residual <= rtol and ||x - x_oracle|| <= 2 rtol ||f|| / lambda_min(A)."""
import numpy as np
import pytest
import scipy.sparse.linalg as sla
import torch

import oracle as O
from oracle.method import make_preconditioner
import workloads as W
from tests._cases import gpu_op, cuda, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2601_20174_amd as mod
    return mod


def _lam_min(A):
    return float(sla.eigsh(A, k=1, sigma=0, which="LM", return_eigenvectors=False)[0])


def _bars(nl, A, f, u, infos, res, cols, prec, rtol, lam):
    for j in cols:
        inf = infos[j]
        true_rel = np.linalg.norm(f[:, j] - A @ u[:, j]) / np.linalg.norm(f[:, j])
        assert inf.status == nl.OK, (j, inf)
        assert true_rel <= rtol * 1.0001, (j, true_rel)
        i = cols.index(j)
        if prec == nl.FP64:
            assert abs(inf.iters - res.iters[i]) <= 1, (j, inf.iters, res.iters[i])
        else:
            err = np.linalg.norm(u[:, j] - res.x[:, i])
            assert err <= 2 * rtol * np.linalg.norm(f[:, j]) / lam, (j, err)


@pytest.fixture(scope="module")
def aniso(nl):
    """One system per grid side of the batched workload, its GPU coarse space
    (float64 setup, as the benchmark) and the oracle's own setup."""
    c3 = W.Cfg3()
    side, eps, theta = c3.systems()
    picks = [int(np.flatnonzero(side == s)[0]) for s in c3.sides]
    st = nl.q1_aniso_stencil(torch.tensor(np.stack([eps[picks], theta[picks]], 1), dtype=torch.float64,
                                          device="cuda"))
    ops, S0s, out = [], [], []
    for j, i in enumerate(picks):
        sd = int(side[i])
        n = sd * sd
        ops.append(nl.Operator(nl.OP_STENCIL9, sd, sd, 1, st[j].contiguous()))
        S0s.append(c3.S0(i, n))
    Ms = nl.setup_many(ops, [cuda(s) for s in S0s], c3.k, c3.omega, c3.s1, c3.nu, nl.FP64, workers=4)
    torch.cuda.synchronize()
    for j, i in enumerate(picks):
        sd = int(side[i])
        A = O.q1_aniso(sd, eps[i], theta[i])
        stg = O.setup(A, S0s[j], c3.k, c3.omega, c3.s1)
        f = c3.rhs(i, sd * sd)
        res = O.pcg(A, f, make_preconditioner(A, stg["P"], stg["L"], c3.omega, c3.nu, c3.nu), rtol=c3.rtol)
        out.append(dict(A=A, op=ops[j], M=Ms[j], f=f, res=res, lam=_lam_min(A)))
    return c3, out


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_batched_anisotropic_benchmark_configuration(nl, aniso, prec):
    c3, syss = aniso
    systems = [nl.System(s["op"], s["M"], cuda(s["f"]), torch.zeros(s["f"].shape, dtype=torch.float64,
                                                                     device="cuda")) for s in syss]
    print(f"batched anisotropic, prec={prec}, sides {[s['op'].nx for s in syss]}, rows_per_block=1024",
          flush=True)
    infos, rc = nl.pcg_solve_batched(systems, prec=prec, rtol=c3.rtol, rows_per_block=1024)
    assert rc == nl.OK
    for s, sysm, inf in zip(syss, systems, infos):
        _bars(nl, s["A"], s["f"], host(sysm.u), inf, s["res"], list(range(c3.R)), prec, c3.rtol, s["lam"])


def test_log_normal_full_size(nl):
    """512 x 512 cells, m = 128, k = 64: float64 and mixed GPU paths (GPU
    setup in each precision, as the benchmark) against the oracle's setup and
    PCG on the same seeded inputs."""
    c = W.Cfg2()
    a = c.coef()
    A = O.fv_harmonic_2d(a)
    S0h, f = c.S0(), c.rhs()
    op = gpu_op(nl.OP_FV5, c.N, c.N, 1, a)
    stg = O.setup(A, S0h, c.k, c.omega, c.s1)
    res = O.pcg(A, f, make_preconditioner(A, stg["P"], stg["L"], c.omega, c.nu, c.nu), rtol=c.rtol)
    lam = _lam_min(A)
    S0 = cuda(S0h)
    for prec in (nl.FP64, nl.MIXED, nl.MIXED_F16):
        print(f"log-normal 512^2, prec={prec}", flush=True)
        P, sigma = nl.setup_spectral_P(op, S0, c.k, c.omega, c.s1, min(prec, nl.MIXED))
        np.testing.assert_allclose(host(sigma)[:c.k + 1], stg["sigma"][:c.k + 1], rtol=1e-4)
        M = nl.galerkin_coarse(op, P, c.omega, c.nu)
        u, info, rc = nl.pcg_solve(op, M, cuda(f), prec=prec, rtol=c.rtol)
        assert rc == nl.OK
        _bars(nl, A, f, host(u).reshape(f.shape), info, res, [0], prec, c.rtol, lam)
