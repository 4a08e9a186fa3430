"""The C-ABI library on the host (no GPU needed): it loads, exports every
function that include/nlsp.h declares, and its host-side entry points and
argument validation behave as documented.  Nothing here launches a kernel:
every call below either is pure host code or is rejected by validation,
which runs before any HIP call."""
import ctypes
import glob
import os
import re
import subprocess

import pytest

from conftest import ROOT

HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


def declared_functions():
    names = []
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        for m in re.finditer(r"^[A-Za-z_][\w \t\*]*?\b([A-Za-z_]\w*)\s*\(", text, flags=re.M):
            if m.group(0).lstrip().startswith(("typedef", "#", "return")):
                continue
            names.append(m.group(1))
    return names


@pytest.fixture(scope="module")
def lib():
    from paper_2601_20174_amd import _lib, build
    if not os.path.exists(_lib.LIB_PATH):
        build.build()
    return _lib.load()


def test_header_declares_functions():
    names = declared_functions()
    assert len(names) == len(set(names))
    for must in ("setup_spectral_P", "galerkin_coarse", "pcg_solve", "nlsp_status_string"):
        assert must in names


def test_binding_covers_header():
    from paper_2601_20174_amd import _lib
    assert set(declared_functions()) == set(_lib.SIGNATURES)


def test_every_declared_symbol_exported(lib):
    from paper_2601_20174_amd import _lib
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if ln.strip()}
    for name in declared_functions():
        assert name in exported, name
        assert getattr(lib, name) is not None


def test_status_strings(lib):
    from paper_2601_20174_amd import api
    seen = set()
    for name in ("NLSP_OK", "NLSP_NOT_CONVERGED", "NLSP_E_INVALID", "NLSP_E_NOT_SPD", "NLSP_E_BREAKDOWN",
                 "NLSP_E_NONFINITE", "NLSP_E_WORKSPACE", "NLSP_E_HIP", "NLSP_E_RANK"):
        code = getattr(api, name[5:]) if hasattr(api, name[5:]) else None
        if code is None:
            continue
        s = lib.nlsp_status_string(code).decode()
        assert s == name
        seen.add(code)
    assert len(seen) >= 8
    assert lib.nlsp_status_string(12345).decode() == "NLSP_UNKNOWN_STATUS"


def test_padded_rank(lib):
    for k, kp in [(1, 16), (16, 16), (17, 32), (32, 32), (48, 64), (64, 64), (65, 128), (128, 128),
                  (129, 256), (256, 256)]:
        assert lib.nlsp_padded_rank(k) == kp
    for k in (0, -3, 257):
        assert lib.nlsp_padded_rank(k) == -1


def _op(kind, nx, ny, nz=1, coef=None):
    from paper_2601_20174_amd import _lib
    return _lib.NlspOperator(kind, nx, ny, nz, coef)


def test_operator_size(lib):
    from paper_2601_20174_amd import api
    fake = ctypes.c_void_p(0x1000)  # never dereferenced by the size query
    assert lib.nlsp_operator_size(ctypes.byref(_op(api.OP_POISSON5, 7, 5))) == 35
    assert lib.nlsp_operator_size(ctypes.byref(_op(api.OP_FV5, 8, 4, 1, fake))) == 32
    assert lib.nlsp_operator_size(ctypes.byref(_op(api.OP_FV7, 4, 3, 2, fake))) == 24
    assert lib.nlsp_operator_size(ctypes.byref(_op(api.OP_STENCIL9, 9, 9, 1, fake))) == 81
    # invalid: missing coefficients, empty grid, unknown kind, n >= 2^31, null
    assert lib.nlsp_operator_size(ctypes.byref(_op(api.OP_FV5, 8, 4))) == -1
    assert lib.nlsp_operator_size(ctypes.byref(_op(api.OP_POISSON5, 0, 4))) == -1
    assert lib.nlsp_operator_size(ctypes.byref(_op(99, 4, 4, 1, fake))) == -1
    assert lib.nlsp_operator_size(ctypes.byref(_op(api.OP_FV7, 2048, 1024, 1024, fake))) == -1
    assert lib.nlsp_operator_size(None) == -1


def test_workspace_queries(lib):
    from paper_2601_20174_amd import api
    op = ctypes.byref(_op(api.OP_POISSON5, 64, 64))
    a = lib.setup_spectral_P_workspace_bytes(op, 32, 16, api.FP64)
    b = lib.setup_spectral_P_workspace_bytes(op, 32, 16, api.MIXED)
    assert a > 0 and b > 0 and a % 256 == 0
    assert lib.setup_spectral_P_workspace_bytes(op, 8, 16, api.FP64) == 0      # m < k
    assert lib.setup_spectral_P_workspace_bytes(op, 300, 16, api.FP64) == 0    # m > 256
    assert lib.setup_spectral_P_workspace_bytes(op, 32, 16, 7) == 0            # bad precision
    assert lib.galerkin_coarse_workspace_bytes(op, 16) > 0
    assert lib.galerkin_coarse_workspace_bytes(op, 0) == 0
    w1 = lib.pcg_solve_workspace_bytes(op, 16, 1)
    w8 = lib.pcg_solve_workspace_bytes(op, 16, 8)
    assert 0 < w1 < w8
    assert lib.pcg_solve_workspace_bytes(op, 16, 17) == 0                       # R > 16
    assert lib.pcg_solve_workspace_bytes(op, 256, 16) == 0                      # kp * R > 2048


def test_cnn_shape_limits(lib):
    """Predictor shapes the library accepts: k and the hidden width multiples
    of 16 up to 64, and at most 16 (16-channel output, 16-channel input)
    tile pairs in the first layer's weight gradient."""
    from paper_2601_20174_amd import api
    assert api.cnn_param_count(2, 32, 32, 32) == (33 * 32 + 32 * 32 * 2 + 32 * 32) * 9 + 3 * 32 + 32
    assert api.cnn_param_count(2, 32, 48, 64) > 0          # 4 x 4 tile pairs
    assert api.cnn_param_count(2, 32, 64, 48) > 0          # 3 x 5
    assert api.cnn_param_count(2, 32, 64, 64) == -1        # 4 x 5
    assert api.cnn_workspace_bytes(2, 32, 64, 64) == 0
    assert api.cnn_param_count(2, 32, 24, 32) == -1        # k not a multiple of 16
    assert api.cnn_param_count(2, 8, 32, 32) == -1         # grid smaller than a tile


def test_solver_workspace_holds_face_weights_for_matrix_core_form(lib):
    """A finite-volume operator solved in the matrix-core form (16 right-hand
    sides with k padded to 64 or 128: k in 33 .. 128; 8 with k padded to 32 or
    64: k in 17 .. 64) gets 3 n float64 + 3 n float32 face weights in the
    solver workspace; other operators and the other forms do not."""
    from paper_2601_20174_amd import api
    fake = ctypes.c_void_p(0x1000)  # never dereferenced by the size query
    fv7 = ctypes.byref(_op(api.OP_FV7, 8, 8, 8, fake))       # n = 512
    fv5 = ctypes.byref(_op(api.OP_FV5, 32, 16, 1, fake))     # n = 512
    p5 = ctypes.byref(_op(api.OP_POISSON5, 32, 16))          # n = 512
    n = 512
    for k in (40, 64, 100, 128):
        base = lib.pcg_solve_workspace_bytes(p5, k, 16)
        assert base > 0
        assert lib.pcg_solve_workspace_bytes(fv7, k, 16) == base + 3 * n * (8 + 4)
        assert lib.pcg_solve_workspace_bytes(fv5, k, 16) == base + 3 * n * (8 + 4)
    for k in (20, 32, 50, 64):
        base = lib.pcg_solve_workspace_bytes(p5, k, 8)
        assert lib.pcg_solve_workspace_bytes(fv7, k, 8) == base + 3 * n * (8 + 4)
    for k, R in ((100, 8), (16, 8), (32, 16), (16, 16), (64, 1), (64, 4)):
        assert lib.pcg_solve_workspace_bytes(fv7, k, R) == lib.pcg_solve_workspace_bytes(p5, k, R)


def test_validation_rejects_before_any_gpu_call(lib):
    """Invalid arguments come back as NLSP_E_INVALID / NLSP_E_WORKSPACE on a
    machine without a GPU, i.e. validation precedes every HIP call."""
    from paper_2601_20174_amd import _lib, api
    fake = ctypes.c_void_p(0x1000)
    op = ctypes.byref(_op(api.OP_POISSON5, 16, 16))
    bad = ctypes.byref(_op(api.OP_FV5, 16, 16))  # no coefficients
    E_INV, E_WS = api.E_INVALID, api.E_WORKSPACE
    assert lib.apply_operator(op, fake, fake, 1, None) == E_INV              # x == y
    assert lib.apply_operator(bad, fake, ctypes.c_void_p(0x2000), 1, None) == E_INV
    assert lib.apply_operator(op, None, fake, 1, None) == E_INV
    assert lib.jacobi_sweep_f32(op, 0.0, fake, fake, ctypes.c_void_p(0x2000), 1, None) == E_INV
    assert lib.q1_aniso_stencil(0, fake, fake, None) == E_INV
    sig = ctypes.c_void_p(0x3000)
    assert lib.setup_spectral_P(op, None, 32, 16, 2 / 3, 10, api.FP64, fake, sig, None, 0, None) == E_INV
    assert lib.setup_spectral_P(op, fake, 8, 16, 2 / 3, 10, api.FP64, fake, sig, None, 0, None) == E_INV
    assert lib.setup_spectral_P(op, fake, 32, 16, -1.0, 10, api.FP64, fake, sig, None, 0, None) == E_INV
    assert lib.setup_spectral_P(op, fake, 32, 16, 2 / 3, 10, api.FP64, fake, sig, None, 0, None) == E_WS
    # randomized sketch: k <= l <= m, 0 <= q <= 8
    assert lib.setup_randomized_P(op, fake, 32, 16, 2 / 3, 10, fake, 12, 1, api.FP64, fake, sig, None, 0,
                                  None) == E_INV
    assert lib.setup_randomized_P(op, fake, 32, 16, 2 / 3, 10, fake, 40, 1, api.FP64, fake, sig, None, 0,
                                  None) == E_INV
    assert lib.setup_randomized_P(op, fake, 32, 16, 2 / 3, 10, fake, 24, 9, api.FP64, fake, sig, None, 0,
                                  None) == E_INV
    assert lib.setup_randomized_P(op, fake, 32, 16, 2 / 3, 10, None, 24, 1, api.FP64, fake, sig, None, 0,
                                  None) == E_INV
    assert lib.setup_randomized_P(op, fake, 32, 16, 2 / 3, 10, fake, 24, 1, api.FP64, fake, sig, None, 0,
                                  None) == E_WS
    assert lib.setup_randomized_P_workspace_bytes(op, 32, 16, 12, api.FP64) == 0
    assert lib.setup_randomized_P_workspace_bytes(op, 32, 16, 24, api.MIXED) > \
        lib.setup_randomized_P_workspace_bytes(op, 32, 16, 24, api.FP64) // 2
    assert lib.galerkin_coarse(op, fake, 16, 2 / 3, 0, fake, fake, fake, fake, None, None, 0, None) == E_INV
    assert lib.galerkin_coarse(op, fake, 16, 2 / 3, 1, fake, fake, fake, None, None, None, 0, None) == E_INV
    assert lib.galerkin_coarse(op, fake, 16, 2 / 3, 1, fake, fake, fake, fake, None, None, 0, None) == E_WS
    M = _lib.NlspTwoLevel(16, 1, 2 / 3, api.MIXED, fake, None, fake)
    opts = _lib.NlspPcgOpts(1e-8, 100, 0, 8, None)
    info = (_lib.NlspRhsInfo * 16)()
    u = ctypes.c_void_p(0x4000)
    assert lib.pcg_solve(op, ctypes.byref(M), fake, u, 17, ctypes.byref(opts), info, None, 0, None) == E_INV
    M_noq = _lib.NlspTwoLevel(16, 1, 2 / 3, api.MIXED, fake, fake, None)
    assert lib.pcg_solve(op, ctypes.byref(M_noq), fake, u, 1, ctypes.byref(opts), info, None, 0, None) == E_INV
    opts_bad = _lib.NlspPcgOpts(0.0, 100, 0, 8, None)
    assert lib.pcg_solve(op, ctypes.byref(M), fake, u, 1, ctypes.byref(opts_bad), info, None, 0, None) == E_INV
    assert lib.pcg_solve(op, ctypes.byref(M), fake, u, 1, ctypes.byref(opts), info, None, 0, None) == E_WS
    # the non-allocating solve: its scratch array holds 256 MiB; a 128^3
    # system with k = 128 and 16 right-hand sides needs more
    assert lib.pcg_solve_noalloc(op, ctypes.byref(M_noq), fake, u, 1, ctypes.byref(opts), info, None) == E_INV
    big = ctypes.byref(_op(api.OP_POISSON5, 2048, 1024))
    Mbig = _lib.NlspTwoLevel(128, 1, 2 / 3, api.MIXED, fake, None, fake)
    assert lib.pcg_solve_noalloc(big, ctypes.byref(Mbig), fake, u, 16, ctypes.byref(opts), info, None) == E_WS
    tm_b = _lib.NlspKernelTiming(1, 1, 0.0, 0)
    opts_tm_b = _lib.NlspPcgOpts(1e-8, 100, 0, 8, ctypes.pointer(tm_b))
    # batched: tile below -1, the tuned-tile query's arguments
    sysb = (_lib.NlspSystem * 1)(_lib.NlspSystem(_op(api.OP_POISSON5, 16, 16), M, fake, u))
    assert lib.pcg_solve_batched(1, sysb, 1, -2, ctypes.byref(opts), info, None, 0, None) == E_INV
    assert lib.pcg_solve_batched_workspace_bytes(1, sysb, 1, -2) == 0
    rpb = ctypes.c_int(0)
    assert lib.pcg_solve_batched_tuned(0, sysb, 1, ctypes.byref(rpb)) == E_INV
    assert lib.pcg_solve_batched_tuned(1, sysb, 0, ctypes.byref(rpb)) == E_INV
    assert lib.pcg_solve_batched_tuned(1, sysb, 1, None) == E_INV
    # device loop: a record array is required, timing is not supported
    assert lib.pcg_solve_batched_async(1, sysb, 1, 0, ctypes.byref(opts), None, None, 0, None) == E_INV
    assert lib.pcg_solve_batched_async(1, sysb, 1, 0, ctypes.byref(opts_tm_b), fake, None, 0, None) == E_INV
    assert lib.pcg_solve_batched_async(1, sysb, 1, 0, ctypes.byref(opts), fake, None, 0, None) == E_WS
    tm = _lib.NlspKernelTiming(1, 1, 0.0, 0)
    opts_tm = _lib.NlspPcgOpts(1e-8, 100, 0, 8, ctypes.pointer(tm))
    assert lib.pcg_solve_noalloc(op, ctypes.byref(M), fake, u, 1, ctypes.byref(opts_tm), info, None) == E_INV


def test_binding_checks_shapes_before_any_launch(lib):
    """The binding compares every buffer's rows with the operator's size (and
    the coefficient count with the operator kind) before a pointer reaches the
    library, which cannot see buffer lengths.  CPU tensors suffice: each check
    raises before the tensor's device is looked at."""
    import torch
    from paper_2601_20174_amd import api
    n = 16 * 16
    op = api.Operator(api.OP_POISSON5, 16, 16)
    x = torch.zeros(n + 1, 2, dtype=torch.float64)
    with pytest.raises(ValueError, match="rows"):
        api.apply_operator(op, x)
    with pytest.raises(ValueError, match="columns"):
        api.apply_operator(op, torch.zeros(n, 2, dtype=torch.float64), torch.zeros(n, 3, dtype=torch.float64))
    with pytest.raises(ValueError, match="coefficients"):
        api.apply_operator(api.Operator(api.OP_FV5, 16, 16, 1, torch.ones(n - 1, dtype=torch.float64)),
                           torch.zeros(n, dtype=torch.float64))
    with pytest.raises(ValueError, match="coefficients"):
        api.apply_operator(api.Operator(api.OP_STENCIL9, 16, 16, 1, torch.ones(8, dtype=torch.float64)),
                           torch.zeros(n, dtype=torch.float64))
    with pytest.raises(ValueError, match="coefficients"):
        api.apply_operator(api.Operator(api.OP_FV7, 8, 8, 8, None), torch.zeros(512, dtype=torch.float64))
    with pytest.raises(ValueError, match="rows"):
        api.jacobi_sweep_f32(op, 2 / 3, torch.zeros(n - 1, dtype=torch.float32), torch.zeros(n, dtype=torch.float32))
    with pytest.raises(ValueError, match="rows"):
        api.setup_spectral_P(op, torch.zeros(n - 2, 32, dtype=torch.float64), 16, 2 / 3, 10)
    with pytest.raises(ValueError, match="rows"):
        api.galerkin_coarse(op, torch.zeros(n + 16, 16, dtype=torch.float64), 2 / 3)
    kp = api.nlsp_padded_rank(16)
    M = api.TwoLevel(16, 1, 2 / 3, torch.zeros(16, 16, dtype=torch.float64), torch.zeros(16, 16, dtype=torch.float64),
                     torch.zeros(kp, kp, dtype=torch.float64), None, torch.zeros(n, kp, dtype=torch.float32))
    with pytest.raises(ValueError, match="rows"):
        api.pcg_solve(op, M, torch.zeros(n - 1, dtype=torch.float64), prec=api.MIXED)
    with pytest.raises(ValueError, match="columns"):
        api.pcg_solve(op, M, torch.zeros(n, 2, dtype=torch.float64), torch.zeros(n, 3, dtype=torch.float64),
                      prec=api.MIXED)
    with pytest.raises(ValueError, match="no basis"):
        api.pcg_solve(op, M, torch.zeros(n, dtype=torch.float64), prec=api.FP64)
    small = api.Operator(api.OP_POISSON5, 8, 8)
    with pytest.raises(ValueError, match="another system"):
        api.pcg_solve(small, M, torch.zeros(64, dtype=torch.float64), prec=api.MIXED)
    sysA = api.System(op, M, torch.zeros(n, 2, dtype=torch.float64), torch.zeros(n, 2, dtype=torch.float64))
    sysB = api.System(op, M, torch.zeros(n, 2, dtype=torch.float64), torch.zeros(n - 1, 2, dtype=torch.float64))
    with pytest.raises(ValueError, match="rows"):
        api.pcg_solve_batched([sysA, sysB])
    sysC = api.System(op, M, torch.zeros(n, 3, dtype=torch.float64), torch.zeros(n, 3, dtype=torch.float64))
    with pytest.raises(ValueError, match="same number"):
        api.pcg_solve_batched([sysA, sysC])


def test_p1_pattern_on_the_host(lib):
    """p1_pattern (host code): the compressed rows hold exactly the couplings
    of the oracle's assembled P1 matrix, with ascending columns, a lone
    diagonal in every boundary row, and per entry the element contributions
    in increasing triangle order (codes 9 t + 3 a + b whose vertex pair is
    the entry's)."""
    import numpy as np
    import oracle as O
    import workloads as W
    N = 6
    pts, tris, bnd = W.p1_mesh(77, N)
    kt, sK, sM = W.p1_coefficients("screened_poisson", 78, len(tris), N)
    npt, nt = len(pts), len(tris)
    nnz, nc = ctypes.c_int64(0), ctypes.c_int64(0)
    assert lib.p1_pattern(npt, nt, tris.ctypes.data, bnd.ctypes.data, ctypes.byref(nnz), ctypes.byref(nc),
                          None, None, None, None) == 0
    rp = np.empty(npt + 1, np.int32)
    ci = np.empty(nnz.value, np.int32)
    cp = np.empty(nnz.value + 1, np.int32)
    cl = np.empty(nc.value, np.int32)
    assert lib.p1_pattern(npt, nt, tris.ctypes.data, bnd.ctypes.data, ctypes.byref(nnz), ctypes.byref(nc),
                          rp.ctypes.data, ci.ctypes.data, cp.ctypes.data, cl.ctypes.data) == 0
    A = O.p1_fem(pts, tris, kt, sK, sM, bnd).tocsr()
    A.sort_indices()
    assert rp[0] == 0 and rp[-1] == nnz.value and np.all(np.diff(rp) >= 1)
    for i in range(npt):
        cols = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(cols) > 0)
        if bnd[i]:
            assert list(cols) == [i]
        assert set(A.indices[A.indptr[i]:A.indptr[i + 1]]) <= set(cols)
        for e in range(rp[i], rp[i + 1]):
            codes = cl[cp[e]:cp[e + 1]]
            assert np.all(np.diff(codes) > 0)
            for code in codes:
                t, a, b = code // 9, (code % 9) // 3, code % 3
                assert (tris[t, a], tris[t, b]) == (i, ci[e])
    inner = bnd == 0
    assert nc.value == sum(int(inner[v].sum()) ** 2 for v in tris)
    # a vertex index out of range is rejected
    bad = tris.copy()
    bad[0, 0] = npt
    assert lib.p1_pattern(npt, nt, bad.ctypes.data, bnd.ctypes.data, ctypes.byref(nnz), ctypes.byref(nc),
                          None, None, None, None) == -1
