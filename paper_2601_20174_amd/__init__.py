"""MI355X (gfx950) spectral two-level preconditioned conjugate gradients.

The method (NeuraLSP, SVD-derived basis): relax random vectors with weighted
Jacobi, take the leading left singular subspace of the result as the
prolongation P, form the Galerkin operator A_c = P^T A P and precondition CG
with the two-grid cycle (Jacobi smoothing + coarse correction).  All
arithmetic runs in the HIP library libnlsp.so (C ABI in include/nlsp.h); this
package only marshals torch tensors into it.
"""
from .api import (  # noqa: F401
    OK, NOT_CONVERGED, E_INVALID, E_NOT_SPD, E_BREAKDOWN, E_NONFINITE, E_WORKSPACE, E_HIP, E_RANK,
    FP64, MIXED, MIXED_F16, OP_POISSON5, OP_FV5, OP_FV7, OP_STENCIL9, OP_CSR, NlspError, Operator, TwoLevel, RhsInfo,
    status_string, nlsp_operator_size, nlsp_padded_rank, p1_operator, q1_aniso_stencil, stream_copy, apply_operator,
    jacobi_sweep_f32, setup_spectral_P_workspace_bytes, setup_spectral_P, setup_randomized_P_workspace_bytes,
    setup_randomized_P,
    galerkin_coarse_workspace_bytes, galerkin_coarse, setup_many, pcg_solve_workspace_bytes, pcg_solve, pcg_solve_noalloc,
    subspace_loss_saved_bytes, subspace_loss_workspace_bytes, subspace_loss_fwd, subspace_loss_bwd,
    SubspaceLoss, subspace_loss, captured_energy, galerkin_fwd_workspace_bytes, galerkin_bwd_workspace_bytes, galerkin_fwd,
    galerkin_bwd, GalerkinProduct, galerkin_product, galerkin_term_saved_bytes, galerkin_term_workspace_bytes,
    galerkin_term_fwd, galerkin_term_bwd, GalerkinTerm, galerkin_term, System, pcg_solve_batched_workspace_bytes,
    pcg_solve_batched, pcg_solve_batched_tune, pcg_solve_batched_tuned, TUNED, pcg_solve_batched_async, rhs_info_from_device, qr_thin_workspace_bytes, qr_thin_fwd, qr_thin_bwd, ThinQ, thin_q,
    cnn_param_count, cnn_workspace_bytes, cnn_fwd, cnn_bwd, CnnPredictor, adam_step,
)
