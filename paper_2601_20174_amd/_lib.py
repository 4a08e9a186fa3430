"""ctypes declarations of the C ABI in include/nlsp.h.

The shared library ``libnlsp.so`` is built in-tree by
``paper_2601_20174_amd.build.build()``.  Loading fails loudly when it is
missing: there is no CPU fallback anywhere in the package.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnlsp.so")

c_int, c_double, c_size_t, c_void_p, c_int64 = (ctypes.c_int, ctypes.c_double, ctypes.c_size_t,
                                                 ctypes.c_void_p, ctypes.c_int64)


class NlspOperator(ctypes.Structure):
    _fields_ = [("kind", c_int), ("nx", c_int), ("ny", c_int), ("nz", c_int), ("coef", c_void_p),
                ("row_ptr", c_void_p), ("col_idx", c_void_p)]


class NlspTwoLevel(ctypes.Structure):
    _fields_ = [("k", c_int), ("nu", c_int), ("omega", c_double), ("prec", c_int),
                ("Linv", c_void_p), ("Q64", c_void_p), ("Q32", c_void_p)]


class NlspKernelTiming(ctypes.Structure):
    _fields_ = [("phase", c_int), ("every", c_int), ("total_ms", c_double), ("launches", c_int)]


class NlspPcgOpts(ctypes.Structure):
    _fields_ = [("rtol", c_double), ("maxit", c_int), ("flexible", c_int), ("check_every", c_int),
                ("timing", ctypes.POINTER(NlspKernelTiming))]


class NlspSystem(ctypes.Structure):
    _fields_ = [("A", NlspOperator), ("M", NlspTwoLevel), ("f", c_void_p), ("u", c_void_p)]


class NlspCnnShape(ctypes.Structure):
    _fields_ = [("batch", c_int), ("N", c_int), ("k", c_int), ("hidden", c_int)]


class NlspRhsInfo(ctypes.Structure):
    _fields_ = [("iters", c_int), ("status", c_int), ("relres", c_double)]


POP = ctypes.POINTER(NlspOperator)

# name -> (restype, argtypes); every symbol declared in include/nlsp.h
SIGNATURES = {
    "nlsp_status_string": (ctypes.c_char_p, [c_int]),
    "nlsp_operator_size": (c_int64, [POP]),
    "nlsp_padded_rank": (c_int, [c_int]),
    "q1_aniso_stencil": (c_int, [c_int, c_void_p, c_void_p, c_void_p]),
    "p1_pattern": (c_int, [c_int, c_int, c_void_p, c_void_p, ctypes.POINTER(c_int64), ctypes.POINTER(c_int64),
                           c_void_p, c_void_p, c_void_p, c_void_p]),
    "p1_assemble": (c_int, [c_int, c_int, c_void_p, c_void_p, c_void_p, c_double, c_double, c_void_p, c_void_p,
                            c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "stream_copy": (c_int, [c_void_p, c_void_p, c_int64, c_void_p]),
    "apply_operator": (c_int, [POP, c_void_p, c_void_p, c_int, c_void_p]),
    "jacobi_sweep_f32": (c_int, [POP, c_double, c_void_p, c_void_p, c_void_p, c_int, c_void_p]),
    "setup_spectral_P_workspace_bytes": (c_size_t, [POP, c_int, c_int, c_int]),
    "setup_spectral_P": (c_int, [POP, c_void_p, c_int, c_int, c_double, c_int, c_int, c_void_p,
                                 c_void_p, c_void_p, c_size_t, c_void_p]),
    "setup_randomized_P_workspace_bytes": (c_size_t, [POP, c_int, c_int, c_int, c_int]),
    "setup_randomized_P": (c_int, [POP, c_void_p, c_int, c_int, c_double, c_int, c_void_p, c_int, c_int,
                                   c_int, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "galerkin_coarse_workspace_bytes": (c_size_t, [POP, c_int]),
    "galerkin_coarse": (c_int, [POP, c_void_p, c_int, c_double, c_int, c_void_p, c_void_p,
                                c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "pcg_solve_workspace_bytes": (c_size_t, [POP, c_int, c_int]),
    "pcg_solve": (c_int, [POP, ctypes.POINTER(NlspTwoLevel), c_void_p, c_void_p, c_int,
                          ctypes.POINTER(NlspPcgOpts), ctypes.POINTER(NlspRhsInfo), c_void_p,
                          c_size_t, c_void_p]),
    "pcg_solve_noalloc": (c_int, [POP, ctypes.POINTER(NlspTwoLevel), c_void_p, c_void_p, c_int,
                                  ctypes.POINTER(NlspPcgOpts), ctypes.POINTER(NlspRhsInfo), c_void_p]),
    "subspace_loss_saved_bytes": (c_size_t, [c_int, c_int, c_int, c_int]),
    "subspace_loss_workspace_bytes": (c_size_t, [c_int, c_int, c_int, c_int]),
    "subspace_loss_fwd": (c_int, [c_int, c_int, c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p,
                                  c_void_p, c_size_t, c_void_p, c_size_t, c_void_p]),
    "subspace_loss_bwd": (c_int, [c_int, c_int, c_int, c_int, c_void_p, c_void_p, c_void_p, c_size_t,
                                  c_void_p, c_void_p, c_void_p]),
    "captured_energy_workspace_bytes": (c_size_t, [c_int, c_int, c_int, c_int]),
    "captured_energy": (c_int, [c_int, c_int, c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t,
                                c_void_p]),
    "galerkin_fwd_workspace_bytes": (c_size_t, [c_int, POP, c_int]),
    "galerkin_fwd": (c_int, [c_int, POP, c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "galerkin_bwd_workspace_bytes": (c_size_t, [c_int, c_int, c_int]),
    "galerkin_bwd": (c_int, [c_int, c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "galerkin_term_saved_bytes": (c_size_t, [c_int, POP, c_int, c_int]),
    "galerkin_term_workspace_bytes": (c_size_t, [c_int, POP, c_int, c_int]),
    "galerkin_term_fwd": (c_int, [c_int, POP, c_void_p, c_void_p, c_int, c_int, c_void_p, c_void_p, c_void_p,
                                  c_void_p, c_size_t, c_void_p, c_size_t, c_void_p]),
    "galerkin_term_bwd": (c_int, [c_int, POP, c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p]),
    "pcg_solve_batched_workspace_bytes": (c_size_t, [c_int, ctypes.POINTER(NlspSystem), c_int, c_int]),
    "pcg_solve_batched": (c_int, [c_int, ctypes.POINTER(NlspSystem), c_int, c_int, ctypes.POINTER(NlspPcgOpts),
                                  ctypes.POINTER(NlspRhsInfo), c_void_p, c_size_t, c_void_p]),
    "pcg_solve_batched_tune_candidates": (c_int, [c_int, ctypes.POINTER(c_int)]),
    "pcg_solve_batched_tune_workspace_bytes": (c_size_t, [c_int, ctypes.POINTER(NlspSystem), c_int]),
    "pcg_solve_batched_tune": (c_int, [c_int, ctypes.POINTER(NlspSystem), c_int, ctypes.POINTER(NlspPcgOpts),
                                       c_int, ctypes.POINTER(c_int), ctypes.POINTER(c_double), c_void_p,
                                       c_size_t, c_void_p]),
    "pcg_solve_batched_tuned": (c_int, [c_int, ctypes.POINTER(NlspSystem), c_int, ctypes.POINTER(c_int)]),
    "pcg_solve_batched_async": (c_int, [c_int, ctypes.POINTER(NlspSystem), c_int, c_int, ctypes.POINTER(NlspPcgOpts),
                                        c_void_p, c_void_p, c_size_t, c_void_p]),
    "qr_thin_workspace_bytes": (c_size_t, [c_int, c_int, c_int]),
    "qr_thin_fwd": (c_int, [c_int, c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t,
                            c_void_p]),
    "qr_thin_bwd": (c_int, [c_int, c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t,
                            c_void_p]),
    "cnn_param_count": (c_int64, [ctypes.POINTER(NlspCnnShape)]),
    "cnn_workspace_bytes": (c_size_t, [ctypes.POINTER(NlspCnnShape)]),
    "cnn_fwd": (c_int, [ctypes.POINTER(NlspCnnShape), c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "cnn_bwd": (c_int, [ctypes.POINTER(NlspCnnShape), c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "adam_step": (c_int, [c_int64, c_void_p, c_void_p, c_void_p, c_void_p, ctypes.c_float, ctypes.c_float,
                          ctypes.c_float, ctypes.c_float, c_int, c_void_p]),
}

_LIB = None


def load():
    """Load libnlsp.so once and declare every exported function."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run paper_2601_20174_amd.build.build() "
                           "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib
