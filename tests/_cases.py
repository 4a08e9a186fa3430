"""Shared builders for GPU parity tests: the same seeded inputs as an oracle
operator (scipy sparse) and as a GPU operator descriptor."""
import numpy as np
import torch

import oracle as O
import workloads as W


def gpu_op(kind, nx, ny, nz=1, coef=None):
    import paper_2601_20174_amd as nl
    c = None if coef is None else torch.tensor(np.ascontiguousarray(coef).ravel(), dtype=torch.float64,
                                               device="cuda")
    return nl.Operator(kind, nx, ny, nz, c)


def make_case(kind: str, seed: int = 0, size=(37, 29)):
    """Returns (A_oracle, gpu Operator, n).  Sizes are deliberately ragged."""
    import paper_2601_20174_amd as nl
    rng = np.random.default_rng(seed)
    if kind == "poisson":
        nx, ny = size
        return O.poisson5(nx, ny), gpu_op(nl.OP_POISSON5, nx, ny), nx * ny
    if kind == "fv5":
        nx, ny = size
        a = np.exp(rng.standard_normal((ny, nx)))
        return O.fv_harmonic_2d(a), gpu_op(nl.OP_FV5, nx, ny, 1, a), nx * ny
    if kind == "grf":
        N = size[0]
        a = W.lognormal_field(seed, N)
        return O.fv_harmonic_2d(a), gpu_op(nl.OP_FV5, N, N, 1, a), N * N
    if kind == "fv7":
        nx, ny = size
        nz = 7
        a = np.where(rng.integers(0, 2, size=(nz, ny, nx)) == 1, 1e3, 1.0)
        return O.fv_harmonic_3d(a), gpu_op(nl.OP_FV7, nx, ny, nz, a), nx * ny * nz
    if kind == "q1":
        side = size[0]
        eps, theta = 10 ** rng.uniform(-3, 0), rng.uniform(0, np.pi)
        st = nl.q1_aniso_stencil(torch.tensor([[eps, theta]], dtype=torch.float64, device="cuda"))
        op = nl.Operator(nl.OP_STENCIL9, side, side, 1, st.reshape(9).contiguous())
        return O.q1_aniso(side, eps, theta), op, side * side
    raise ValueError(kind)


def cuda(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    return t.detach().cpu().numpy()
