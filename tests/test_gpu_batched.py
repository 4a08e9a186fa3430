"""GPU parity of the batched solve (many systems of different sizes in the
same launches, hipGraph replay, tuned tiles), through the C ABI (marked gpu).

Bars: with the default tile every system is partitioned exactly as by
pcg_solve, so the batched solve must reproduce the single-system solves bit
for bit; with other tiles the reductions are ordered differently, and the
float64 form must keep the iteration count within +-1 of the FP64 oracle with
a true relative residual <= rtol per right-hand side (mixed form: true
relative residual <= rtol)."""
import numpy as np
import pytest
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


SIDES = [24, 31, 40, 17, 50, 33]


def _batch(nl, R, k=12, m=24, seed=0, sides=SIDES, zero_col=False):
    """Anisotropic Q1 systems (one (eps, theta) per system), GPU setup."""
    rng = np.random.default_rng(seed)
    et = np.stack([10 ** rng.uniform(-2, 0, len(sides)), rng.uniform(0, np.pi, len(sides))], 1)
    st = nl.q1_aniso_stencil(torch.tensor(et, dtype=torch.float64, device="cuda"))
    out = []
    for i, side in enumerate(sides):
        n = side * side
        op = nl.Operator(nl.OP_STENCIL9, side, side, 1, st[i].contiguous())
        S0 = cuda(W.normal_block(W.seed_for(3, 1, 10 * seed + i), n, m))
        P, _ = nl.setup_spectral_P(op, S0, k, 2 / 3, 10, nl.FP64)
        M = nl.galerkin_coarse(op, P, 2 / 3, 1)
        f = W.normal_block(W.seed_for(3, 2, 10 * seed + i), n, R)
        if zero_col and i == 2:
            f[:, 1] = 0.0
        A = O.q1_aniso(side, et[i, 0], et[i, 1])
        out.append((A, op, M, P, f))
    return out


def _systems(nl, batch):
    return [nl.System(op, M, cuda(f), torch.zeros(f.shape, dtype=torch.float64, device="cuda"))
            for (_, op, M, _, f) in batch]


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("R", [1, 3, 8])
def test_default_tile_matches_single_system_bitwise(nl, prec, R):
    batch = _batch(nl, R, zero_col=(R == 3))
    systems = _systems(nl, batch)
    infos, rc = nl.pcg_solve_batched(systems, prec=prec, rtol=1e-8, check_every=8)
    assert rc == nl.OK
    for (A, op, M, _, f), s, inf in zip(batch, systems, infos):
        u1, info1, rc1 = nl.pcg_solve(op, M, cuda(f), prec=prec, rtol=1e-8, check_every=8)
        assert torch.equal(s.u, u1.reshape(s.u.shape))
        for a, b in zip(inf, info1):
            assert (a.iters, a.status, a.relres) == (b.iters, b.status, b.relres)


@pytest.mark.parametrize("R,k", [(16, 50), (8, 30), (8, 50)])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_matrix_core_batch(nl, prec, R, k):
    """16 right-hand sides with kp = 64, 8 with kp = 32 and 64: the batch takes
    the matrix-core basis passes; with the default tile it reproduces the
    single-system solves bit for bit, and every right-hand side reaches the
    tolerance."""
    batch = _batch(nl, R, k=k, m=64, sides=[24, 31, 40, 50])
    systems = _systems(nl, batch)
    infos, rc = nl.pcg_solve_batched(systems, prec=prec, rtol=1e-8, check_every=8)
    assert rc == nl.OK
    for (A, op, M, _, f), s, inf in zip(batch, systems, infos):
        u1, info1, rc1 = nl.pcg_solve(op, M, cuda(f), prec=prec, rtol=1e-8, check_every=8)
        assert torch.equal(s.u, u1.reshape(s.u.shape))
        u = host(s.u).reshape(f.shape)
        for j, a in enumerate(inf):
            true_rel = np.linalg.norm(f[:, j] - A @ u[:, j]) / np.linalg.norm(f[:, j])
            assert a.status == nl.OK, (j, a)
            assert true_rel <= 1e-8 * 1.0001, (j, true_rel)


@pytest.mark.parametrize("R,k,sides,rows", [
    (16, 50, [64, 96, 40], 2048),    # 96 lines in runs of 64: a workgroup spans two x-segments; 40 has no whole segments
    (8, 30, [128, 64, 50], 1408),    # runs of 22 lines: the x-segment changes inside a workgroup's run
    (8, 50, [64, 128], 512),
])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_line_march_against_oracle(nl, prec, R, k, sides, rows):
    """Matrix-core batches of 9-point systems whose x-lines split into whole
    chunks: the matvec kernel (every precision) and the float-basis update
    kernel march each x-segment through y with their operands in an LDS ring
    (workgroups whose run of lines crosses a segment boundary, and systems
    without whole segments, take the gather path in the same launch).  Every
    right-hand side reaches the tolerance, in the oracle's PCG iteration count
    (float64: +-1; mixed forms: the flexible variant's, within 5 %), and the
    batch equals the single-system solves with the same tile."""
    batch = _batch(nl, R, k=k, m=64, sides=sides, seed=5)
    systems = _systems(nl, batch)
    infos, rc = nl.pcg_solve_batched(systems, prec=prec, rtol=1e-8, rows_per_block=rows)
    assert rc == nl.OK
    for (A, op, M, P, f), s, inf in zip(batch, systems, infos):
        one = _systems(nl, [(A, op, M, P, f)])
        _, rc1 = nl.pcg_solve_batched(one, prec=prec, rtol=1e-8, rows_per_block=rows)
        assert rc1 == nl.OK and torch.equal(s.u, one[0].u)
        u = host(s.u)
        _, L = O.galerkin(A, host(P))
        res = O.pcg(A, f, make_preconditioner(A, host(P), L, 2 / 3, 1, 1), rtol=1e-8, flexible=(prec != 0))
        for c in range(R):
            rel = np.linalg.norm(f[:, c] - A @ u[:, c]) / np.linalg.norm(f[:, c])
            assert inf[c].status == nl.OK, (c, inf[c])
            assert rel <= 1e-8 * 1.0001, (c, rel)
            bar = 1 if prec == 0 else max(2, 0.05 * res.iters[c])
            assert abs(inf[c].iters - res.iters[c]) <= bar, (c, inf[c].iters, res.iters[c])


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("rows", [128, 512, 2048])
def test_tiles_against_oracle(nl, prec, rows):
    R = 8
    batch = _batch(nl, R, seed=1)
    systems = _systems(nl, batch)
    infos, rc = nl.pcg_solve_batched(systems, prec=prec, rtol=1e-8, rows_per_block=rows)
    assert rc == nl.OK
    for (A, op, M, P, f), s, inf in zip(batch, systems, infos):
        u = host(s.u)
        Ph = host(P)
        _, L = O.galerkin(A, Ph)
        res = O.pcg(A, f, make_preconditioner(A, Ph, L, 2 / 3, 1, 1), rtol=1e-8, flexible=(prec != 0))
        for c in range(R):
            rel = np.linalg.norm(f[:, c] - A @ u[:, c]) / np.linalg.norm(f[:, c])
            assert inf[c].status == nl.OK
            assert rel <= 1e-8 * 1.0001
            if prec == 0:
                assert abs(inf[c].iters - res.iters[c]) <= 1, (c, inf[c].iters, res.iters[c])
            else:
                assert abs(inf[c].iters - res.iters[c]) <= max(2, 0.05 * res.iters[c])


def test_deterministic_and_graph_replay_matches_direct_launches(nl):
    """Two graph-replayed batched solves are bit-identical, and equal to the
    single-system solves (direct launches, no graph)."""
    batch = _batch(nl, 2, seed=2)
    s1 = _systems(nl, batch)
    s2 = _systems(nl, batch)
    i1, _ = nl.pcg_solve_batched(s1, prec=1, rows_per_block=0, check_every=6)
    i2, _ = nl.pcg_solve_batched(s2, prec=1, rows_per_block=0, check_every=6)
    for a, b in zip(s1, s2):
        assert torch.equal(a.u, b.u)


def test_tuner_picks_a_candidate_and_leaves_u(nl):
    batch = _batch(nl, 8, seed=3, sides=[23, 30, 41, 18])
    systems = _systems(nl, batch)
    assert nl.pcg_solve_batched_tuned(systems, prec=1) is None
    for s in systems:
        s.u.fill_(0.25)
    best, times = nl.pcg_solve_batched_tune(systems, prec=1, iters=8)
    assert best in times and len(times) >= 4 and all(t > 0 for t in times.values())
    for s in systems:
        assert torch.all(s.u == 0.25)
    # the choice is recorded for this batch shape (and only for it)
    assert nl.pcg_solve_batched_tuned(systems, prec=1) == best
    assert nl.pcg_solve_batched_tuned(systems, prec=0) is None
    assert nl.pcg_solve_batched_tuned(systems[:3], prec=1) is None
    assert nl.pcg_solve_batched_tuned(systems[::-1], prec=1) is None
    for s in systems:
        s.u.zero_()
    infos, rc = nl.pcg_solve_batched(systems, prec=1, rows_per_block=best)
    assert rc == nl.OK
    u_best = [s.u.clone() for s in systems]
    for s in systems:
        s.u.zero_()
    infos2, rc2 = nl.pcg_solve_batched(systems, prec=1, rows_per_block=nl.TUNED)
    assert rc2 == nl.OK
    for a, s in zip(u_best, systems):
        assert torch.equal(a, s.u)
    for a, b in zip(infos, infos2):
        assert [(x.iters, x.relres) for x in a] == [(x.iters, x.relres) for x in b]
    # an untuned shape under TUNED runs the default plan
    sub = systems[:2]
    for s in sub:
        s.u.zero_()
    i3, _ = nl.pcg_solve_batched(sub, prec=1, rows_per_block=nl.TUNED)
    u3 = [s.u.clone() for s in sub]
    for s in sub:
        s.u.zero_()
    i4, _ = nl.pcg_solve_batched(sub, prec=1, rows_per_block=0)
    for a, s in zip(u3, sub):
        assert torch.equal(a, s.u)


def test_invalid(nl):
    batch = _batch(nl, 2, seed=4, sides=[20, 21])
    systems = _systems(nl, batch)
    systems[1].M = nl.galerkin_coarse(batch[1][1], batch[1][3][:, :8].contiguous(), 2 / 3, 1)   # other k
    with pytest.raises(nl.NlspError):
        nl.pcg_solve_batched(systems)


def test_setup_many_matches_sequential_setup(nl):
    """setup_many (systems spread over worker threads and streams) returns the
    coarse spaces of one setup_spectral_P + galerkin_coarse per system, bit for
    bit, in the order of the systems."""
    rng = np.random.default_rng(3)
    sides = [24, 31, 40, 17, 50, 33, 29]
    et = np.stack([10 ** rng.uniform(-2, 0, len(sides)), rng.uniform(0, np.pi, len(sides))], 1)
    st = nl.q1_aniso_stencil(torch.tensor(et, dtype=torch.float64, device="cuda"))
    ops, S0s = [], []
    for i, side in enumerate(sides):
        n = side * side
        ops.append(nl.Operator(nl.OP_STENCIL9, side, side, 1, st[i].contiguous()))
        S0s.append(cuda(W.normal_block(W.seed_for(3, 1, 70 + i), n, 24)))
    Ms = nl.setup_many(ops, S0s, 12, 2 / 3, 10, 1, nl.FP64, workers=3)
    torch.cuda.synchronize()
    for op, S0, M in zip(ops, S0s, Ms):
        P, _ = nl.setup_spectral_P(op, S0, 12, 2 / 3, 10, nl.FP64)
        M1 = nl.galerkin_coarse(op, P, 2 / 3, 1)
        for a, b in ((M.Ac, M1.Ac), (M.L, M1.L), (M.Linv, M1.Linv), (M.Q64, M1.Q64), (M.Q32, M1.Q32)):
            assert torch.equal(a, b)


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_device_loop_matches_host_polled_solve(nl, prec):
    """The device-loop form enqueues the same kernels as the host-polled
    solve up to convergence and then only launches that exit at once: when no
    residual replacement was needed (equal iteration counts), u and every
    per-RHS record agree bit for bit, and the zero right-hand side is solved
    by u = 0 from a nonzero guess."""
    R = 3
    batch = _batch(nl, R, seed=5, zero_col=True)
    s1 = _systems(nl, batch)
    s2 = _systems(nl, batch)
    for a, b in zip(s1, s2):
        a.u.fill_(0.5)
        b.u.fill_(0.5)
    infos, rc = nl.pcg_solve_batched(s1, prec=prec, rtol=1e-8)
    assert rc == nl.OK
    dev_info = nl.pcg_solve_batched_async(s2, prec=prec, rtol=1e-8, maxit=400)
    torch.cuda.synchronize()
    infos2 = nl.rhs_info_from_device(dev_info, len(s2), R)
    for a, b, ia, ib in zip(s1, s2, infos, infos2):
        assert [(x.iters, x.status, x.relres) for x in ia] == [(x.iters, x.status, x.relres) for x in ib]
        assert torch.equal(a.u, b.u)
    assert torch.all(s2[2].u[:, 1] == 0.0)


def test_device_loop_budget_reports_not_converged(nl):
    """A budget below the iterations needed stops every right-hand side at
    maxit with NOT_CONVERGED and its true relative residual."""
    R = 2
    batch = _batch(nl, R, seed=6, sides=[30, 41])
    systems = _systems(nl, batch)
    info = nl.rhs_info_from_device(nl.pcg_solve_batched_async(systems, prec=1, rtol=1e-8, maxit=5), 2, R)
    for (A, op, M, P, f), s, inf in zip(batch, systems, info):
        u = host(s.u)
        for c in range(R):
            true_rel = np.linalg.norm(f[:, c] - A @ u[:, c]) / np.linalg.norm(f[:, c])
            assert inf[c].iters == 5 and inf[c].status == nl.NOT_CONVERGED
            assert abs(inf[c].relres - true_rel) <= 1e-9 * max(1.0, true_rel)


def test_device_loop_captured_in_a_graph(nl):
    """The device-loop solve captured in a graph (workspace and record buffer
    allocated beforehand) and replayed three times, with eager work and
    synchronisations between the replays: every replay equals the eager
    device-loop solve bit for bit."""
    R = 8
    batch = _batch(nl, R, seed=7, sides=[24, 31, 40, 50])
    systems = _systems(nl, batch)
    nsys = len(systems)
    nb = nl.pcg_solve_batched_workspace_bytes(systems, nl.MIXED)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    info = torch.empty(nsys * R * nl.api.RHS_INFO_BYTES, dtype=torch.uint8, device="cuda")
    nl.pcg_solve_batched_async(systems, prec=nl.MIXED, maxit=120, workspace=ws, info=info)
    torch.cuda.synchronize()
    u_ref = [s.u.clone() for s in systems]
    info_ref = info.clone()
    assert all(x.status == nl.OK for si in nl.rhs_info_from_device(info_ref, nsys, R) for x in si)
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    for s in systems:
        s.u.zero_()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=side):
        nl.pcg_solve_batched_async(systems, prec=nl.MIXED, maxit=120, workspace=ws, info=info)
    torch.cuda.synchronize()
    for rep in range(3):
        for s in systems:
            s.u.zero_()
        info.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, s in zip(u_ref, systems):
            assert torch.equal(a, s.u), rep
        assert torch.equal(info, info_ref), rep
