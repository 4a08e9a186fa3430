"""Python binding of the C ABI: argument marshalling only.

Every function has the name of its C entry point, takes torch tensors that
live on the GPU, allocates outputs and workspace with torch (device memory
only; torch provides memory and the current stream) and calls the library.
No arithmetic of the method happens here.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import List, Optional

import torch

from . import _lib

OK, NOT_CONVERGED = 0, 1
E_INVALID, E_NOT_SPD, E_BREAKDOWN, E_NONFINITE, E_WORKSPACE, E_HIP, E_RANK = -1, -2, -3, -4, -5, -6, -7
FP64, MIXED, MIXED_F16 = 0, 1, 2
OP_POISSON5, OP_FV5, OP_FV7, OP_STENCIL9, OP_CSR = 0, 1, 2, 3, 4


class NlspError(RuntimeError):
    def __init__(self, fn: str, status: int):
        self.status = status
        super().__init__(f"{fn}: {status_string(status)} ({status})")


def _L():
    return _lib.load()


def status_string(status: int) -> str:
    return _L().nlsp_status_string(int(status)).decode()


def _check(fn: str, rc: int, allow=(OK,)):
    if rc not in allow:
        raise NlspError(fn, rc)
    return rc


def _dev(t: torch.Tensor, dtype, name: str) -> int:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


def _op_checked(op: "Operator") -> "Operator":
    """A single-system operator whose coefficient array holds exactly what its
    kind reads (the library cannot see buffer lengths)."""
    if op.nx < 1 or op.ny < 1 or op.nz < 1:
        raise ValueError(f"operator extents must be positive, got {op.nx} x {op.ny} x {op.nz}")
    if op.kind == OP_CSR:
        if op.ny != 1 or op.nz != 1:
            raise ValueError("a compressed-row operator has nx = n rows and ny = nz = 1")
        if op.row_ptr is None or op.col_idx is None or op.coef is None:
            raise ValueError("a compressed-row operator needs row_ptr, col_idx and coef")
        if op.row_ptr.numel() != op.n + 1 or op.col_idx.numel() != op.coef.numel():
            raise ValueError(f"compressed rows: row_ptr must hold {op.n + 1} entries and col_idx as many as coef")
        return op
    per = {OP_FV5: op.n, OP_FV7: op.n, OP_STENCIL9: 9}.get(op.kind)
    if per is not None and (op.coef is None or op.coef.numel() != per):
        got = None if op.coef is None else op.coef.numel()
        raise ValueError(f"operator kind {op.kind} needs {per} coefficients, got {got}")
    return op


def _rows(t: torch.Tensor, n: int, name: str, cols: Optional[int] = None):
    """Checks that t is (n,) or (n, cols) before its pointer reaches a kernel."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dim() not in (1, 2) or t.shape[0] != n:
        raise ValueError(f"{name} must have {n} rows, got shape {tuple(t.shape)}")
    c = 1 if t.dim() == 1 else t.shape[1]
    if cols is not None and c != cols:
        raise ValueError(f"{name} must have {cols} columns, got shape {tuple(t.shape)}")
    return c


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _workspace(nbytes: int, device) -> torch.Tensor:
    # torch's caching allocator returns 512-byte aligned blocks
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


@dataclasses.dataclass
class Operator:
    """Operator descriptor (see nlsp_operator).  ``coef`` is a GPU float64
    tensor: the cell coefficient a for OP_FV5/OP_FV7, 9 stencil values for
    OP_STENCIL9, None for OP_POISSON5, the values for OP_CSR (with row_ptr
    (n + 1) and col_idx (nnz) int32 GPU tensors; nx = n, ny = nz = 1)."""
    kind: int
    nx: int
    ny: int
    nz: int = 1
    coef: Optional[torch.Tensor] = None
    row_ptr: Optional[torch.Tensor] = None
    col_idx: Optional[torch.Tensor] = None

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def device(self):
        return self.coef.device if self.coef is not None else torch.device("cuda", torch.cuda.current_device())

    def c(self) -> _lib.NlspOperator:
        ptr = _dev(self.coef, torch.float64, "coef") if self.coef is not None else None
        rp = _dev(self.row_ptr, torch.int32, "row_ptr") if self.row_ptr is not None else None
        ci = _dev(self.col_idx, torch.int32, "col_idx") if self.col_idx is not None else None
        return _lib.NlspOperator(self.kind, self.nx, self.ny, self.nz, ptr, rp, ci)


def nlsp_operator_size(op: Operator) -> int:
    return int(_L().nlsp_operator_size(ctypes.byref(op.c())))


def nlsp_padded_rank(k: int) -> int:
    return int(_L().nlsp_padded_rank(int(k)))


def p1_operator(points, tris, boundary, ktensor: torch.Tensor, sK: float, sM: float, device=None) -> Operator:
    """The P1 finite-element operator A = sK K + sM M of a triangulation as an
    OP_CSR descriptor: p1_pattern on the host (points, tris, boundary are
    numpy arrays: (np, 2) float64, (nt, 3) int32, (np,) uint8), its arrays
    copied to the GPU, then p1_assemble there.  ktensor (nt, 3) float64 on the
    GPU: [Kxx, Kxy, Kyy] per triangle."""
    import numpy as np
    tris = np.ascontiguousarray(tris, dtype=np.int32)
    bnd = np.ascontiguousarray(boundary, dtype=np.uint8)
    pts = np.ascontiguousarray(points, dtype=np.float64)
    npt, nt = pts.shape[0], tris.shape[0]
    if pts.shape != (npt, 2) or tris.shape != (nt, 3) or bnd.shape != (npt,):
        raise ValueError("points (np, 2), tris (nt, 3) and boundary (np,) expected")
    if tuple(ktensor.shape) != (nt, 3):
        raise ValueError("ktensor must be (nt, 3)")
    L = _L()
    nnz, nc = ctypes.c_int64(0), ctypes.c_int64(0)
    _check("p1_pattern", L.p1_pattern(npt, nt, tris.ctypes.data, bnd.ctypes.data, ctypes.byref(nnz),
                                      ctypes.byref(nc), None, None, None, None))
    rp = np.empty(npt + 1, dtype=np.int32)
    ci = np.empty(nnz.value, dtype=np.int32)
    cp = np.empty(nnz.value + 1, dtype=np.int32)
    cl = np.empty(max(nc.value, 1), dtype=np.int32)
    _check("p1_pattern", L.p1_pattern(npt, nt, tris.ctypes.data, bnd.ctypes.data, ctypes.byref(nnz),
                                      ctypes.byref(nc), rp.ctypes.data, ci.ctypes.data, cp.ctypes.data,
                                      cl.ctypes.data))
    dev = ktensor.device if device is None else device
    g = {name: torch.from_numpy(a).to(dev) for name, a in
         (("rp", rp), ("ci", ci), ("cp", cp), ("cl", cl), ("pts", pts), ("tris", tris), ("bnd", bnd))}
    vals = torch.empty(nnz.value, dtype=torch.float64, device=dev)
    _check("p1_assemble", L.p1_assemble(npt, nt, g["pts"].data_ptr(), g["tris"].data_ptr(),
                                        _dev(ktensor, torch.float64, "ktensor"), float(sK), float(sM),
                                        g["bnd"].data_ptr(), g["rp"].data_ptr(), g["ci"].data_ptr(),
                                        g["cp"].data_ptr(), g["cl"].data_ptr(), vals.data_ptr(), _stream()))
    return Operator(OP_CSR, npt, 1, 1, vals, g["rp"], g["ci"])


def q1_aniso_stencil(eps_theta: torch.Tensor) -> torch.Tensor:
    """(nsys, 2) [eps, theta] -> (nsys, 9) stencils."""
    nsys = eps_theta.shape[0]
    out = torch.empty((nsys, 9), dtype=torch.float64, device=eps_theta.device)
    _check("q1_aniso_stencil", _L().q1_aniso_stencil(nsys, _dev(eps_theta, torch.float64, "eps_theta"),
                                                     _dev(out, torch.float64, "stencil"), _stream()))
    return out


def stream_copy(src: torch.Tensor, dst: torch.Tensor) -> torch.Tensor:
    """dst = src with the library's plain copy kernel (both contiguous GPU
    tensors of the same size, a multiple of 16 bytes)."""
    nb = src.numel() * src.element_size()
    if not (src.is_cuda and dst.is_cuda and src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("src and dst must be contiguous GPU tensors")
    if dst.numel() * dst.element_size() != nb:
        raise ValueError("src and dst differ in size")
    _check("stream_copy", _L().stream_copy(src.data_ptr(), dst.data_ptr(), nb, _stream()))
    return dst


def apply_operator(op: Operator, x: torch.Tensor, y: Optional[torch.Tensor] = None) -> torch.Tensor:
    R = _rows(x, _op_checked(op).n, "x")
    if y is None:
        y = torch.empty_like(x)
    _rows(y, op.n, "y", R)
    _check("apply_operator", _L().apply_operator(ctypes.byref(op.c()), _dev(x, torch.float64, "x"),
                                                 _dev(y, torch.float64, "y"), R, _stream()))
    return y


def jacobi_sweep_f32(op: Operator, omega: float, b: torch.Tensor, x: torch.Tensor,
                     y: Optional[torch.Tensor] = None) -> torch.Tensor:
    R = _rows(x, _op_checked(op).n, "x")
    _rows(b, op.n, "b", R)
    if y is None:
        y = torch.empty_like(x)
    _rows(y, op.n, "y", R)
    _check("jacobi_sweep_f32", _L().jacobi_sweep_f32(
        ctypes.byref(op.c()), float(omega), _dev(b, torch.float32, "b"), _dev(x, torch.float32, "x"),
        _dev(y, torch.float32, "y"), R, _stream()))
    return y


def setup_spectral_P_workspace_bytes(op: Operator, m: int, k: int, prec: int) -> int:
    return int(_L().setup_spectral_P_workspace_bytes(ctypes.byref(op.c()), m, k, prec))


def setup_spectral_P(op: Operator, S0: torch.Tensor, k: int, omega: float, s1: int,
                     prec: int = FP64, workspace: Optional[torch.Tensor] = None):
    """Returns (P (n,k) float64, sigma (m,) float64)."""
    if S0.dim() != 2:
        raise ValueError("S0 must be (n, m)")
    n, m = S0.shape
    _rows(S0, _op_checked(op).n, "S0", m)
    P = torch.empty((n, k), dtype=torch.float64, device=S0.device)
    sigma = torch.empty((m,), dtype=torch.float64, device=S0.device)
    nb = setup_spectral_P_workspace_bytes(op, m, k, prec)
    if nb == 0:
        raise NlspError("setup_spectral_P_workspace_bytes", E_INVALID)
    ws = workspace if workspace is not None else _workspace(nb, S0.device)
    rc = _L().setup_spectral_P(ctypes.byref(op.c()), _dev(S0, torch.float64, "S0"), m, k,
                               float(omega), int(s1), int(prec), _dev(P, torch.float64, "P"),
                               _dev(sigma, torch.float64, "sigma"), ws.data_ptr(), ws.numel(),
                               _stream())
    _check("setup_spectral_P", rc)
    return P, sigma


def setup_randomized_P_workspace_bytes(op: Operator, m: int, k: int, l: int, prec: int) -> int:
    return int(_L().setup_randomized_P_workspace_bytes(ctypes.byref(op.c()), m, k, l, prec))


def setup_randomized_P(op: Operator, S0: torch.Tensor, k: int, omega: float, s1: int, Omega: torch.Tensor,
                       q: int = 1, prec: int = FP64, workspace: Optional[torch.Tensor] = None):
    """Randomized-sketch basis; Omega (m, l) float64 is the caller's random
    test matrix.  Returns (P (n,k) float64, sigma (l,) float64)."""
    if S0.dim() != 2 or Omega.dim() != 2:
        raise ValueError("S0 must be (n, m) and Omega (m, l)")
    n, m = S0.shape
    _rows(S0, _op_checked(op).n, "S0", m)
    _rows(Omega, m, "Omega")
    l = Omega.shape[1]
    P = torch.empty((n, k), dtype=torch.float64, device=S0.device)
    sigma = torch.empty((l,), dtype=torch.float64, device=S0.device)
    nb = setup_randomized_P_workspace_bytes(op, m, k, l, prec)
    if nb == 0:
        raise NlspError("setup_randomized_P_workspace_bytes", E_INVALID)
    ws = workspace if workspace is not None else _workspace(nb, S0.device)
    rc = _L().setup_randomized_P(ctypes.byref(op.c()), _dev(S0, torch.float64, "S0"), m, k, float(omega),
                                 int(s1), _dev(Omega, torch.float64, "Omega"), l, int(q), int(prec),
                                 _dev(P, torch.float64, "P"), _dev(sigma, torch.float64, "sigma"),
                                 ws.data_ptr(), ws.numel(), _stream())
    _check("setup_randomized_P", rc)
    return P, sigma


@dataclasses.dataclass
class TwoLevel:
    """The solver's coarse-space factors (nlsp_two_level) and A_c, L."""
    k: int
    nu: int
    omega: float
    Ac: torch.Tensor
    L: torch.Tensor
    Linv: torch.Tensor
    Q64: Optional[torch.Tensor]
    Q32: Optional[torch.Tensor]

    def c(self, prec: int) -> _lib.NlspTwoLevel:
        return _lib.NlspTwoLevel(
            self.k, self.nu, float(self.omega), int(prec), _dev(self.Linv, torch.float64, "Linv"),
            _dev(self.Q64, torch.float64, "Q64") if self.Q64 is not None else None,
            _dev(self.Q32, torch.float32, "Q32") if self.Q32 is not None else None)


def _two_level_checked(M: TwoLevel, n: int, prec: int) -> TwoLevel:
    """The stored basis the solve reads has n rows and the padded rank."""
    kp = nlsp_padded_rank(M.k)
    Q = M.Q64 if prec == FP64 else M.Q32
    if Q is None:
        raise ValueError("the coarse space holds no basis of the requested precision")
    if tuple(Q.shape) != (n, kp) or tuple(M.Linv.shape) != (kp, kp):
        raise ValueError(f"coarse space shaped for another system: Q {tuple(Q.shape)}, expected ({n}, {kp})")
    return M


def galerkin_coarse_workspace_bytes(op: Operator, k: int) -> int:
    return int(_L().galerkin_coarse_workspace_bytes(ctypes.byref(op.c()), k))


def galerkin_coarse(op: Operator, P: torch.Tensor, omega: float, nu: int = 1, q64: bool = True,
                    q32: bool = True, workspace: Optional[torch.Tensor] = None) -> TwoLevel:
    if P.dim() != 2:
        raise ValueError("P must be (n, k)")
    n, k = P.shape
    _rows(P, _op_checked(op).n, "P", k)
    kp = nlsp_padded_rank(k)
    dev = P.device
    Ac = torch.empty((k, k), dtype=torch.float64, device=dev)
    L = torch.empty((k, k), dtype=torch.float64, device=dev)
    Linv = torch.empty((kp, kp), dtype=torch.float64, device=dev)
    Q64 = torch.empty((n, kp), dtype=torch.float64, device=dev) if q64 else None
    Q32 = torch.empty((n, kp), dtype=torch.float32, device=dev) if q32 else None
    nb = galerkin_coarse_workspace_bytes(op, k)
    if nb == 0:
        raise NlspError("galerkin_coarse_workspace_bytes", E_INVALID)
    ws = workspace if workspace is not None else _workspace(nb, dev)
    rc = _L().galerkin_coarse(ctypes.byref(op.c()), _dev(P, torch.float64, "P"), k, float(omega),
                              int(nu), Ac.data_ptr(), L.data_ptr(), Linv.data_ptr(),
                              Q64.data_ptr() if Q64 is not None else None,
                              Q32.data_ptr() if Q32 is not None else None, ws.data_ptr(),
                              ws.numel(), _stream())
    _check("galerkin_coarse", rc)
    return TwoLevel(k, nu, omega, Ac, L, Linv, Q64, Q32)


def pcg_solve_workspace_bytes(op: Operator, k: int, R: int) -> int:
    return int(_L().pcg_solve_workspace_bytes(ctypes.byref(op.c()), k, R))


@dataclasses.dataclass
class RhsInfo:
    iters: int
    status: int
    relres: float


def setup_many(ops: List[Operator], S0s: List[torch.Tensor], k: int, omega: float, s1: int, nu: int = 1,
               prec: int = FP64, workers: int = 4, q64: bool = True, q32: bool = True) -> List[TwoLevel]:
    """setup_spectral_P + galerkin_coarse for many systems (Algorithm 1's setup
    per system), `workers` systems at a time: each worker thread issues its
    systems on a stream of its own (default priority), so the small kernels of
    different systems overlap on the device (each setup call waits for its own
    stream before it returns its status).  `prec` is the setup's precision;
    q64 / q32 select the stored bases as in galerkin_coarse.  Returns the
    coarse spaces in the order of `ops`; the caller's current stream waits for
    all of them."""
    from concurrent.futures import ThreadPoolExecutor
    if len(ops) != len(S0s):
        raise ValueError("ops and S0s differ in length")
    if not ops:
        return []
    dev = S0s[0].device
    workers = max(1, min(workers, len(ops)))
    cur = torch.cuda.current_stream(dev)
    streams = [torch.cuda.Stream(device=dev) for _ in range(workers)]
    for st in streams:
        st.wait_stream(cur)
    out: List[Optional[TwoLevel]] = [None] * len(ops)

    def run(w: int):
        with torch.cuda.stream(streams[w]):
            for i in range(w, len(ops), workers):
                P, _ = setup_spectral_P(ops[i], S0s[i], k, omega, s1, prec)
                out[i] = galerkin_coarse(ops[i], P, omega, nu, q64=q64, q32=q32)

    with ThreadPoolExecutor(workers) as ex:
        for fut in [ex.submit(run, w) for w in range(workers)]:
            fut.result()
    for st in streams:
        cur.wait_stream(st)
    return out   # type: ignore[return-value]


def pcg_solve(op: Operator, M: TwoLevel, f: torch.Tensor, u: Optional[torch.Tensor] = None,
              prec: int = FP64, rtol: float = 1e-8, maxit: int = 10000, flexible: Optional[bool] = None,
              check_every: int = 32, workspace: Optional[torch.Tensor] = None,
              timing: Optional[dict] = None):
    """Returns (u, [RhsInfo per RHS], status).  ``f`` is (n,) or (n, R).
    ``timing`` = {"phase": 1|2, "every": int} asks the library to time one
    kernel (1 the update kernel, 2 the matvec kernel) with hipEvents attached to its dispatches; on return it also holds
    "total_ms" and "launches"."""
    squeeze = f.dim() == 1
    R = _rows(f, _op_checked(op).n, "f")
    _two_level_checked(M, op.n, prec)
    f2 = f.reshape(f.shape[0], -1)
    if u is None:
        u = torch.zeros_like(f2)
    else:
        _rows(u, op.n, "u", R)
        u = u.reshape(f2.shape)
    if flexible is None:
        flexible = prec != FP64
    nb = pcg_solve_workspace_bytes(op, M.k, R)
    if nb == 0:
        raise NlspError("pcg_solve_workspace_bytes", E_INVALID)
    ws = workspace if workspace is not None else _workspace(nb, f.device)
    tm = None
    if timing is not None:
        tm = _lib.NlspKernelTiming(int(timing.get("phase", 0)), int(timing.get("every", 1)), 0.0, 0)
    opts = _lib.NlspPcgOpts(float(rtol), int(maxit), 1 if flexible else 0, int(check_every),
                            ctypes.pointer(tm) if tm is not None else None)
    info = (_lib.NlspRhsInfo * R)()
    Mc = M.c(prec)
    rc = _L().pcg_solve(ctypes.byref(op.c()), ctypes.byref(Mc), _dev(f2, torch.float64, "f"),
                        _dev(u, torch.float64, "u"), R, ctypes.byref(opts), info, ws.data_ptr(),
                        ws.numel(), _stream())
    _check("pcg_solve", rc, allow=(OK, NOT_CONVERGED, E_BREAKDOWN, E_NONFINITE))
    if tm is not None:
        timing["total_ms"] = tm.total_ms
        timing["launches"] = tm.launches
    infos: List[RhsInfo] = [RhsInfo(info[i].iters, info[i].status, info[i].relres) for i in range(R)]
    return (u.reshape(f.shape) if squeeze else u), infos, rc


NOALLOC_SCRATCH_BYTES = 256 << 20   # NLSP_NOALLOC_SCRATCH_BYTES


def pcg_solve_noalloc(op: Operator, M: TwoLevel, f: torch.Tensor, u: torch.Tensor, prec: int = FP64,
                      rtol: float = 1e-8, maxit: int = 10000, flexible: Optional[bool] = None,
                      check_every: int = 32):
    """pcg_solve through the library's non-allocating entry point: the
    workspace is the library's own device scratch array, so the C call
    allocates nothing; ``u`` (n,) or (n, R), the initial guess, is updated in
    place.  Returns ([RhsInfo per RHS], status)."""
    R = _rows(f, _op_checked(op).n, "f")
    _rows(u, op.n, "u", R)
    _two_level_checked(M, op.n, prec)
    if flexible is None:
        flexible = prec != FP64
    opts = _lib.NlspPcgOpts(float(rtol), int(maxit), 1 if flexible else 0, int(check_every), None)
    info = (_lib.NlspRhsInfo * R)()
    Mc = M.c(prec)
    rc = _L().pcg_solve_noalloc(ctypes.byref(op.c()), ctypes.byref(Mc), _dev(f, torch.float64, "f"),
                                _dev(u, torch.float64, "u"), R, ctypes.byref(opts), info, _stream())
    _check("pcg_solve_noalloc", rc, allow=(OK, NOT_CONVERGED, E_BREAKDOWN, E_NONFINITE))
    return [RhsInfo(info[i].iters, info[i].status, info[i].relres) for i in range(R)], rc


# ------------------------------------------------------------ training losses
def subspace_loss_saved_bytes(batch: int, n: int, k: int, m: int) -> int:
    return int(_L().subspace_loss_saved_bytes(batch, n, k, m))


def subspace_loss_workspace_bytes(batch: int, n: int, k: int, m: int) -> int:
    return int(_L().subspace_loss_workspace_bytes(batch, n, k, m))


def _loss_dims(P: torch.Tensor, B: torch.Tensor):
    if P.dim() != 3 or B.dim() != 3 or P.shape[:2] != B.shape[:2]:
        raise ValueError("P must be (batch, n, k) and B (batch, n, m)")
    return P.shape[0], P.shape[1], P.shape[2], B.shape[2]


def subspace_loss_fwd(P: torch.Tensor, B: torch.Tensor, colw: Optional[torch.Tensor] = None,
                      workspace: Optional[torch.Tensor] = None):
    """Per-sample loss (batch,) float32 and the `saved` buffer for the backward."""
    batch, n, k, m = _loss_dims(P, B)
    nb = subspace_loss_saved_bytes(batch, n, k, m)
    if nb == 0:
        raise NlspError("subspace_loss_saved_bytes", E_INVALID)
    saved = torch.empty(nb, dtype=torch.uint8, device=P.device)
    loss = torch.empty(batch, dtype=torch.float32, device=P.device)
    wb = subspace_loss_workspace_bytes(batch, n, k, m)
    ws = workspace if workspace is not None else _workspace(wb, P.device)
    cw = _dev(colw, torch.float32, "colw") if colw is not None else None
    rc = _L().subspace_loss_fwd(batch, n, k, m, _dev(P, torch.float32, "P"), _dev(B, torch.float32, "B"), cw,
                                loss.data_ptr(), saved.data_ptr(), nb, ws.data_ptr(), ws.numel(), _stream())
    _check("subspace_loss_fwd", rc)
    return loss, saved


def subspace_loss_bwd(P: torch.Tensor, B: torch.Tensor, saved: torch.Tensor, gloss: torch.Tensor,
                      gP: Optional[torch.Tensor] = None) -> torch.Tensor:
    batch, n, k, m = _loss_dims(P, B)
    if gP is None:
        gP = torch.empty_like(P)
    rc = _L().subspace_loss_bwd(batch, n, k, m, _dev(P, torch.float32, "P"), _dev(B, torch.float32, "B"),
                                saved.data_ptr(), saved.numel(), _dev(gloss, torch.float32, "gloss"),
                                _dev(gP, torch.float32, "gP"), _stream())
    _check("subspace_loss_bwd", rc)
    return gP


def captured_energy(P: torch.Tensor, S: torch.Tensor, workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Energy_b(r) = ||P_b[:, :r]^T S_b||_F^2 / ||S_b||_F^2 for r = 1..k, as a
    (batch, k) float64 tensor: the captured energy of the leading r columns
    (prefix truncation of an ordered basis; orthonormal P)."""
    batch, n, k, m = _loss_dims(P, S)
    wb = int(_L().captured_energy_workspace_bytes(batch, n, k, m))
    if wb == 0:
        raise NlspError("captured_energy_workspace_bytes", E_INVALID)
    ws = workspace if workspace is not None else _workspace(wb, P.device)
    energy = torch.empty(batch, k, dtype=torch.float64, device=P.device)
    rc = _L().captured_energy(batch, n, k, m, _dev(P, torch.float32, "P"), _dev(S, torch.float32, "S"),
                              energy.data_ptr(), ws.data_ptr(), ws.numel(), _stream())
    _check("captured_energy", rc)
    return energy


class SubspaceLoss(torch.autograd.Function):
    """Per-sample subspace (or, with colw, column-weighted / NLSS) loss with
    the library's backward; B and colw receive no gradient."""

    @staticmethod
    def forward(ctx, P, B, colw=None):
        P = P.contiguous()
        B = B.contiguous()
        loss, saved = subspace_loss_fwd(P, B, colw)
        ctx.save_for_backward(P, B, saved)
        return loss

    @staticmethod
    def backward(ctx, gloss):
        P, B, saved = ctx.saved_tensors
        gP = subspace_loss_bwd(P, B, saved, gloss.contiguous().to(torch.float32))
        return gP, None, None


def subspace_loss(P: torch.Tensor, B: torch.Tensor, colw: Optional[torch.Tensor] = None) -> torch.Tensor:
    return SubspaceLoss.apply(P, B, colw)


# ------------------------------------------------------------ Galerkin product
def galerkin_fwd_workspace_bytes(batch: int, op: Operator, k: int) -> int:
    return int(_L().galerkin_fwd_workspace_bytes(batch, ctypes.byref(op.c()), k))


def galerkin_bwd_workspace_bytes(batch: int, n: int, k: int) -> int:
    return int(_L().galerkin_bwd_workspace_bytes(batch, n, k))


def galerkin_fwd(op: Operator, P: torch.Tensor):
    """A_c = P^T A P per sample, P (batch, n, k) float32; ``op`` carries the
    batched coefficients (batch x n for FV5/FV7).  Returns (Ac, Y = A P)."""
    if P.dim() != 3:
        raise ValueError("P must be (batch, n, k)")
    batch, n, k = P.shape
    if n != nlsp_operator_size(op):
        raise ValueError("P rows must match the operator size")
    per = {OP_FV5: n, OP_FV7: n, OP_STENCIL9: 9}.get(op.kind, 0)
    if per and (op.coef is None or op.coef.numel() < batch * per):
        raise ValueError(f"batched coefficients: need {batch} x {per} values")
    Ac = torch.empty(batch, k, k, dtype=torch.float32, device=P.device)
    Y = torch.empty_like(P)
    nb = galerkin_fwd_workspace_bytes(batch, op, k)
    if nb == 0:
        raise NlspError("galerkin_fwd_workspace_bytes", E_INVALID)
    ws = _workspace(nb, P.device)
    rc = _L().galerkin_fwd(batch, ctypes.byref(op.c()), _dev(P, torch.float32, "P"), k, Ac.data_ptr(),
                           Y.data_ptr(), ws.data_ptr(), ws.numel(), _stream())
    _check("galerkin_fwd", rc)
    return Ac, Y


def galerkin_bwd(Y: torch.Tensor, gAc: torch.Tensor) -> torch.Tensor:
    batch, n, k = Y.shape
    gP = torch.empty_like(Y)
    nb = galerkin_bwd_workspace_bytes(batch, n, k)
    if nb == 0:
        raise NlspError("galerkin_bwd_workspace_bytes", E_INVALID)
    ws = _workspace(nb, Y.device)
    rc = _L().galerkin_bwd(batch, n, k, _dev(Y, torch.float32, "Y"), _dev(gAc, torch.float32, "gAc"),
                           gP.data_ptr(), ws.data_ptr(), ws.numel(), _stream())
    _check("galerkin_bwd", rc)
    return gP


class GalerkinProduct(torch.autograd.Function):
    """A_c = P^T A P (batched) with the library's backward A P (G + G^T)."""

    @staticmethod
    def forward(ctx, P, op):
        Ac, Y = galerkin_fwd(op, P.contiguous())
        ctx.save_for_backward(Y)
        return Ac

    @staticmethod
    def backward(ctx, gAc):
        (Y,) = ctx.saved_tensors
        return galerkin_bwd(Y, gAc.contiguous().to(torch.float32)), None


def galerkin_product(P: torch.Tensor, op: Operator) -> torch.Tensor:
    return GalerkinProduct.apply(P, op)


# ------------------------------------------------- Galerkin-convergence term
def galerkin_term_saved_bytes(batch: int, op: Operator, k: int, m: int) -> int:
    return int(_L().galerkin_term_saved_bytes(batch, ctypes.byref(op.c()), k, m))


def galerkin_term_workspace_bytes(batch: int, op: Operator, k: int, m: int) -> int:
    return int(_L().galerkin_term_workspace_bytes(batch, ctypes.byref(op.c()), k, m))


def galerkin_term_fwd(op: Operator, P: torch.Tensor, S: torch.Tensor):
    """J_b = ||A^{1/2}(I - P A_c^{-1} P^T A) S||_F^2 per sample, P (batch, n, k)
    and S (batch, n, m) float32; ``op`` carries the batched coefficients.
    Returns (J, bad, saved, E) with E_b = ||A^{1/2} S_b||_F^2."""
    if P.dim() != 3 or S.dim() != 3 or P.shape[:2] != S.shape[:2]:
        raise ValueError("P must be (batch, n, k) and S (batch, n, m)")
    batch, n, k = P.shape
    m = S.shape[2]
    if n != nlsp_operator_size(op):
        raise ValueError("rows must match the operator size")
    per = {OP_FV5: n, OP_FV7: n, OP_STENCIL9: 9}.get(op.kind, 0)
    if per and (op.coef is None or op.coef.numel() < batch * per):
        raise ValueError(f"batched coefficients: need {batch} x {per} values")
    sb = galerkin_term_saved_bytes(batch, op, k, m)
    nb = galerkin_term_workspace_bytes(batch, op, k, m)
    if sb == 0 or nb == 0:
        raise NlspError("galerkin_term_workspace_bytes", E_INVALID)
    J = torch.empty(batch, dtype=torch.float32, device=P.device)
    E = torch.empty(batch, dtype=torch.float32, device=P.device)
    bad = torch.empty(batch, dtype=torch.int32, device=P.device)
    saved = _workspace(sb, P.device)
    ws = _workspace(nb, P.device)
    rc = _L().galerkin_term_fwd(batch, ctypes.byref(op.c()), _dev(P, torch.float32, "P"),
                                _dev(S, torch.float32, "S"), k, m, J.data_ptr(), E.data_ptr(), bad.data_ptr(),
                                saved.data_ptr(), saved.numel(), ws.data_ptr(), ws.numel(), _stream())
    _check("galerkin_term_fwd", rc)
    return J, bad, saved, E


def galerkin_term_bwd(op: Operator, k: int, m: int, saved: torch.Tensor, gJ: torch.Tensor) -> torch.Tensor:
    batch = gJ.numel()
    n = nlsp_operator_size(op)
    gP = torch.empty(batch, n, k, dtype=torch.float32, device=saved.device)
    rc = _L().galerkin_term_bwd(batch, ctypes.byref(op.c()), k, m, saved.data_ptr(),
                                _dev(gJ, torch.float32, "gJ"), gP.data_ptr(), _stream())
    _check("galerkin_term_bwd", rc)
    return gP


class GalerkinTerm(torch.autograd.Function):
    """J(P) per sample with the library's backward (E = ||A^{1/2} S||_F^2
    and the flags receive no gradient)."""

    @staticmethod
    def forward(ctx, P, S, op):
        J, bad, saved, E = galerkin_term_fwd(op, P.contiguous(), S.contiguous())
        ctx.op, ctx.k, ctx.m = op, P.shape[2], S.shape[2]
        ctx.save_for_backward(saved)
        ctx.mark_non_differentiable(bad, E)
        return J, bad, E

    @staticmethod
    def backward(ctx, gJ, gbad, gE):
        (saved,) = ctx.saved_tensors
        return galerkin_term_bwd(ctx.op, ctx.k, ctx.m, saved, gJ.contiguous().to(torch.float32)), None, None


def galerkin_term(P: torch.Tensor, S: torch.Tensor, op: Operator):
    """Returns (J, bad, E); J is differentiable in P."""
    return GalerkinTerm.apply(P, S, op)


# ------------------------------------------------------------ batched solve
@dataclasses.dataclass
class System:
    """One system of a batch: operator, its two-level factors, right-hand
    sides f (n, R) and solution u (n, R), float64 GPU tensors."""
    op: Operator
    M: TwoLevel
    f: torch.Tensor
    u: torch.Tensor


def _systems(systems: List[System], prec: int):
    arr = (_lib.NlspSystem * len(systems))()
    R = None
    for i, s in enumerate(systems):
        Ri = _rows(s.f, _op_checked(s.op).n, f"systems[{i}].f")
        if R is None:
            R = Ri
        if Ri != R:
            raise ValueError("every system needs the same number of right-hand sides")
        _rows(s.u, s.op.n, f"systems[{i}].u", R)
        _two_level_checked(s.M, s.op.n, prec)
    for i, s in enumerate(systems):
        arr[i] = _lib.NlspSystem(s.op.c(), s.M.c(prec), _dev(s.f, torch.float64, "f"),
                                 _dev(s.u, torch.float64, "u"))
    return arr, R


def _opts(rtol, maxit, flexible, check_every):
    return _lib.NlspPcgOpts(float(rtol), int(maxit), 1 if flexible else 0, int(check_every), None)


def pcg_solve_batched_workspace_bytes(systems: List[System], prec: int, rows_per_block: int = 0) -> int:
    arr, R = _systems(systems, prec)
    return int(_L().pcg_solve_batched_workspace_bytes(len(systems), arr, R, int(rows_per_block)))


TUNED = -1   # rows_per_block: the tile pcg_solve_batched_tune chose for this batch shape


def pcg_solve_batched(systems: List[System], prec: int = MIXED, rtol: float = 1e-8, maxit: int = 10000,
                      flexible: Optional[bool] = None, check_every: int = 32, rows_per_block: int = 0,
                      workspace: Optional[torch.Tensor] = None):
    """Solves every system in place (s.u); returns ([[RhsInfo] per system], status).
    rows_per_block = TUNED takes the tile recorded by pcg_solve_batched_tune for
    a batch of this shape (the default plan if there is none)."""
    arr, R = _systems(systems, prec)
    if flexible is None:
        flexible = prec != FP64
    nb = _L().pcg_solve_batched_workspace_bytes(len(systems), arr, R, int(rows_per_block))
    if nb == 0:
        raise NlspError("pcg_solve_batched_workspace_bytes", E_INVALID)
    ws = workspace if workspace is not None else _workspace(nb, systems[0].f.device)
    info = (_lib.NlspRhsInfo * (len(systems) * R))()
    opts = _opts(rtol, maxit, flexible, check_every)
    rc = _L().pcg_solve_batched(len(systems), arr, R, int(rows_per_block), ctypes.byref(opts), info,
                                ws.data_ptr(), ws.numel(), _stream())
    _check("pcg_solve_batched", rc, allow=(OK, NOT_CONVERGED, E_BREAKDOWN, E_NONFINITE))
    out = [[RhsInfo(info[i * R + c].iters, info[i * R + c].status, info[i * R + c].relres) for c in range(R)]
           for i in range(len(systems))]
    return out, rc


RHS_INFO_BYTES = ctypes.sizeof(_lib.NlspRhsInfo)


def pcg_solve_batched_async(systems: List[System], prec: int = MIXED, rtol: float = 1e-8, maxit: int = 1000,
                            flexible: Optional[bool] = None, rows_per_block: int = 0,
                            workspace: Optional[torch.Tensor] = None, info: Optional[torch.Tensor] = None):
    """The batched solve with its loop on the device: enqueues a fixed budget
    of `maxit` iterations on the current stream and returns at once, so it can
    be captured in a CUDA/HIP graph (pass `workspace` and `info`, allocated
    beforehand, to keep the call free of allocations).  Returns the device
    tensor of per-RHS records (decode with rhs_info_from_device after the
    stream has run)."""
    arr, R = _systems(systems, prec)
    if flexible is None:
        flexible = prec != FP64
    nb = _L().pcg_solve_batched_workspace_bytes(len(systems), arr, R, int(rows_per_block))
    if nb == 0:
        raise NlspError("pcg_solve_batched_workspace_bytes", E_INVALID)
    dev = systems[0].f.device
    ws = workspace if workspace is not None else _workspace(nb, dev)
    need = len(systems) * R * RHS_INFO_BYTES
    if info is None:
        info = torch.empty(need, dtype=torch.uint8, device=dev)
    if not info.is_cuda or info.dtype != torch.uint8 or info.numel() < need or info.data_ptr() % 8 != 0:
        raise ValueError(f"info must be a GPU uint8 tensor of at least {need} bytes, 8-byte aligned")
    opts = _opts(rtol, maxit, flexible, 1)
    rc = _L().pcg_solve_batched_async(len(systems), arr, R, int(rows_per_block), ctypes.byref(opts),
                                      info.data_ptr(), ws.data_ptr(), ws.numel(), _stream())
    _check("pcg_solve_batched_async", rc)
    return info


def rhs_info_from_device(info: torch.Tensor, nsys: int, R: int) -> List[List[RhsInfo]]:
    """Decodes the device records of pcg_solve_batched_async (copies to the host)."""
    raw = bytes(info[: nsys * R * RHS_INFO_BYTES].cpu().numpy().tobytes())
    recs = (_lib.NlspRhsInfo * (nsys * R)).from_buffer_copy(raw)
    return [[RhsInfo(recs[i * R + c].iters, recs[i * R + c].status, recs[i * R + c].relres) for c in range(R)]
            for i in range(nsys)]


def pcg_solve_batched_tune(systems: List[System], prec: int = MIXED, rtol: float = 1e-8, iters: int = 16,
                           flexible: Optional[bool] = None):
    """Times `iters` iterations per candidate tile (u is left untouched);
    returns (best rows_per_block, {rows_per_block: ms})."""
    arr, R = _systems(systems, prec)
    if flexible is None:
        flexible = prec != FP64
    ncand = _L().pcg_solve_batched_tune_candidates(R, None)
    cand = (ctypes.c_int * ncand)()
    _L().pcg_solve_batched_tune_candidates(R, cand)
    nb = _L().pcg_solve_batched_tune_workspace_bytes(len(systems), arr, R)
    if nb == 0:
        raise NlspError("pcg_solve_batched_tune_workspace_bytes", E_INVALID)
    ws = _workspace(nb, systems[0].f.device)
    best = ctypes.c_int(0)
    ms = (ctypes.c_double * ncand)()
    opts = _opts(rtol, 10000, flexible, iters)
    rc = _L().pcg_solve_batched_tune(len(systems), arr, R, ctypes.byref(opts), int(iters), ctypes.byref(best), ms,
                                     ws.data_ptr(), ws.numel(), _stream())
    _check("pcg_solve_batched_tune", rc)
    return best.value, {int(cand[i]): float(ms[i]) for i in range(ncand)}


def pcg_solve_batched_tuned(systems: List[System], prec: int = MIXED) -> Optional[int]:
    """The tile recorded by pcg_solve_batched_tune for a batch of this shape
    on the current device, or None."""
    arr, R = _systems(systems, prec)
    rpb = ctypes.c_int(0)
    rc = _L().pcg_solve_batched_tuned(len(systems), arr, R, ctypes.byref(rpb))
    if rc < 0:
        _check("pcg_solve_batched_tuned", rc)
    return rpb.value if rc == 1 else None


# ------------------------------------------------------------ thin QR
def qr_thin_workspace_bytes(batch: int, n: int, k: int) -> int:
    return int(_L().qr_thin_workspace_bytes(batch, n, k))


def qr_thin_fwd(A: torch.Tensor, workspace: Optional[torch.Tensor] = None):
    """Q, R, bad for A (batch, n, k) float32: A = Q R, R (batch, k, k) float64."""
    batch, n, k = A.shape
    Q = torch.empty_like(A)
    R = torch.empty(batch, k, k, dtype=torch.float64, device=A.device)
    bad = torch.empty(batch, dtype=torch.int32, device=A.device)
    nb = qr_thin_workspace_bytes(batch, n, k)
    if nb == 0:
        raise NlspError("qr_thin_workspace_bytes", E_INVALID)
    ws = workspace if workspace is not None else _workspace(nb, A.device)
    rc = _L().qr_thin_fwd(batch, n, k, _dev(A, torch.float32, "A"), Q.data_ptr(), R.data_ptr(), bad.data_ptr(),
                          ws.data_ptr(), ws.numel(), _stream())
    _check("qr_thin_fwd", rc)
    return Q, R, bad


def qr_thin_bwd(Q: torch.Tensor, R: torch.Tensor, gQ: torch.Tensor, workspace: Optional[torch.Tensor] = None):
    batch, n, k = Q.shape
    gA = torch.empty_like(Q)
    nb = qr_thin_workspace_bytes(batch, n, k)
    ws = workspace if workspace is not None else _workspace(nb, Q.device)
    rc = _L().qr_thin_bwd(batch, n, k, _dev(Q, torch.float32, "Q"), _dev(R, torch.float64, "R"),
                          _dev(gQ, torch.float32, "gQ"), gA.data_ptr(), ws.data_ptr(), ws.numel(), _stream())
    _check("qr_thin_bwd", rc)
    return gA


class ThinQ(torch.autograd.Function):
    """Q factor of the thin QR (CholeskyQR2) with the library's backward."""

    @staticmethod
    def forward(ctx, A):
        Q, R, bad = qr_thin_fwd(A.contiguous())
        ctx.save_for_backward(Q, R)
        return Q

    @staticmethod
    def backward(ctx, gQ):
        Q, R = ctx.saved_tensors
        return qr_thin_bwd(Q, R, gQ.contiguous().to(torch.float32))


def thin_q(A: torch.Tensor) -> torch.Tensor:
    return ThinQ.apply(A)


# ------------------------------------------------------------ P-predictor CNN
def _cnn_shape(batch: int, N: int, k: int, hidden: int):
    return _lib.NlspCnnShape(int(batch), int(N), int(k), int(hidden))


def cnn_param_count(batch: int, N: int, k: int, hidden: int = 32) -> int:
    return int(_L().cnn_param_count(ctypes.byref(_cnn_shape(batch, N, k, hidden))))


def cnn_workspace_bytes(batch: int, N: int, k: int, hidden: int = 32) -> int:
    return int(_L().cnn_workspace_bytes(ctypes.byref(_cnn_shape(batch, N, k, hidden))))


def cnn_fwd(params: torch.Tensor, coef: torch.Tensor, N: int, k: int, hidden: int, workspace: torch.Tensor):
    """P_hat (batch, N*N, k) float32 from coef (batch, N*N) float64; the
    workspace keeps the activations for cnn_bwd."""
    batch = coef.shape[0]
    Phat = torch.empty(batch, N * N, k, dtype=torch.float32, device=coef.device)
    sh = _cnn_shape(batch, N, k, hidden)
    rc = _L().cnn_fwd(ctypes.byref(sh), _dev(params, torch.float32, "params"), _dev(coef, torch.float64, "coef"),
                      Phat.data_ptr(), workspace.data_ptr(), workspace.numel(), _stream())
    _check("cnn_fwd", rc)
    return Phat


def cnn_bwd(params: torch.Tensor, gPhat: torch.Tensor, N: int, k: int, hidden: int, workspace: torch.Tensor):
    batch = gPhat.shape[0]
    g = torch.empty_like(params)
    sh = _cnn_shape(batch, N, k, hidden)
    rc = _L().cnn_bwd(ctypes.byref(sh), _dev(params, torch.float32, "params"), _dev(gPhat, torch.float32, "gPhat"),
                      g.data_ptr(), workspace.data_ptr(), workspace.numel(), _stream())
    _check("cnn_bwd", rc)
    return g


class CnnPredictor(torch.autograd.Function):
    """P_hat = CNN(coef; params) with the library's backward for params."""

    @staticmethod
    def forward(ctx, params, coef, N, k, hidden, workspace):
        ctx.meta = (N, k, hidden, workspace)
        ctx.save_for_backward(params)
        return cnn_fwd(params.contiguous(), coef, N, k, hidden, workspace)

    @staticmethod
    def backward(ctx, gPhat):
        (params,) = ctx.saved_tensors
        N, k, hidden, ws = ctx.meta
        return cnn_bwd(params, gPhat.contiguous().to(torch.float32), N, k, hidden, ws), None, None, None, None, None


def adam_step(params: torch.Tensor, grads: torch.Tensor, m: torch.Tensor, v: torch.Tensor, lr: float, step: int,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    rc = _L().adam_step(params.numel(), _dev(params, torch.float32, "params"), _dev(grads, torch.float32, "grads"),
                        _dev(m, torch.float32, "m"), _dev(v, torch.float32, "v"), float(lr), float(beta1),
                        float(beta2), float(eps), int(step), _stream())
    _check("adam_step", rc)
