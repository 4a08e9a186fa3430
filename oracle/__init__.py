"""FP64 CPU oracle for the spectral two-level preconditioned CG method.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this
package.  The product path (``paper_2601_20174_amd``) never imports it, and
this package imports nothing from the product path: the two share only the
seeded input generators in ``workloads``.

The oracle is deliberately plain and slow: sparse matrices assembled from the
defining formulas, library primitives (sparse mat-vec, LAPACK SVD and
Cholesky) as single steps, and the algorithm's steps written in the paper's
order and notation (the NeuraLSP algorithm: setup, then one preconditioner
application per PCG iteration).  Everything is float64.

Modules
-------
operators  assembly of the SPD operator A for each workload family
method     relaxation, spectral basis (SVD and randomized range finder),
           Galerkin coarse operator, two-grid
           preconditioner, PCG
losses     subspace loss, NLSS loss, Galerkin-convergence objective and
           their gradients
"""
from .operators import (poisson5, fv_harmonic_2d, fv_harmonic_3d, q1_aniso_element,
                        q1_aniso, p1_element, p1_fem, jacobi_diag)
from .method import (relax, spectral_basis, randomized_basis, galerkin, two_grid_apply, pcg, PCGResult,
                     setup, NOT_CONVERGED, OK, E_BREAKDOWN, E_NONFINITE, E_NOT_SPD,
                     E_INVALID)
from . import predictor
from .losses import (subspace_loss, subspace_loss_grad, nlss_loss, nlss_weights,
                     weighted_energy_loss, weighted_energy_loss_grad, captured_energy,
                     galerkin_term, galerkin_term_grad, galerkin_term_dense,
                     galerkin_coarse_vjp)

__all__ = [
    "predictor",
    "poisson5", "fv_harmonic_2d", "fv_harmonic_3d", "q1_aniso_element", "q1_aniso", "p1_element", "p1_fem",
    "jacobi_diag", "relax", "spectral_basis", "randomized_basis", "galerkin", "two_grid_apply", "pcg",
    "PCGResult", "setup", "OK", "NOT_CONVERGED", "E_BREAKDOWN", "E_NONFINITE",
    "E_NOT_SPD", "E_INVALID", "subspace_loss", "subspace_loss_grad", "nlss_loss",
    "nlss_weights", "weighted_energy_loss", "weighted_energy_loss_grad",
    "captured_energy", "galerkin_term", "galerkin_term_grad", "galerkin_term_dense",
    "galerkin_coarse_vjp",
]
