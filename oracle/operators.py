"""Assembly of the sparse SPD operator A (oracle; test infrastructure only).

The paper poses D[u] = f on the unit square with homogeneous Dirichlet data and
solves the discretised system A u = f (Sec. 3, "PDE Discretization and Linear
Systems"); its benchmarks use P1 finite elements with Dirichlet rows (appendix,
benchmark PDE families).  The workloads here are structured-grid members of the
same families, each assembled from its defining formula into a
``scipy.sparse.csr_matrix``:

* ``poisson5``       5-point Laplacian T(x)I + I(x)T, T = tridiag(-1, 2, -1).
* ``fv_harmonic_2d`` cell-centred finite volumes for -div(a grad u), face
                     transmissibility = harmonic mean of the two cell values,
                     Dirichlet wall half a cell away (boundary face 2 a_P).
* ``fv_harmonic_3d`` the same rules in 3-D (7-point).
* ``q1_aniso``       bilinear (Q1) finite elements for -div(K grad u) with a
                     constant tensor K = R(theta) diag(1, eps) R(theta)^T on a
                     uniform grid; boundary nodes eliminated (9-point).
* ``p1_fem``         the paper's own discretisation (FEM dataset appendix):
                     linear (P1) elements on a triangulation, stiffness
                     |T| g_i^T K_T g_j and mass |T|/12 [2 1 1; 1 2 1; 1 1 2]
                     per triangle, A = sK K + sM M, Dirichlet vertices by
                     zeroing their rows and columns with a unit diagonal.

Unknowns are ordered x fastest: index = x + nx*(y + ny*z).  No 1/h^2 or area
scaling is applied (PCG iterates are invariant under A -> cA, f -> cf).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

__all__ = ["poisson5", "fv_harmonic_2d", "fv_harmonic_3d", "q1_aniso_element",
           "q1_aniso", "p1_element", "p1_fem", "jacobi_diag"]


def poisson5(N: int, Ny: int | None = None) -> sp.csr_matrix:
    """Constant-coefficient 5-point Poisson on an N x Ny interior grid."""
    Ny = N if Ny is None else Ny

    def T(m):
        return sp.diags([-np.ones(m - 1), 2.0 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1])

    A = sp.kron(sp.identity(Ny), T(N)) + sp.kron(T(Ny), sp.identity(N))
    return sp.csr_matrix(A)


def _harmonic(a, b):
    return 2.0 * a * b / (a + b)


def _assemble_faces(n, diag, rows, cols, vals):
    """A = diag + sum over interior faces of t*(e_P - e_Q)(e_P - e_Q)^T."""
    r = np.concatenate([np.arange(n), rows, cols])
    c = np.concatenate([np.arange(n), cols, rows])
    v = np.concatenate([diag, -vals, -vals])
    return sp.csr_matrix(sp.coo_matrix((v, (r, c)), shape=(n, n)))


def fv_harmonic_2d(a: np.ndarray) -> sp.csr_matrix:
    """Cell-centred FV operator for -div(a grad u), a indexed [y, x]."""
    a = np.asarray(a, dtype=np.float64)
    ny, nx = a.shape
    n = nx * ny
    idx = np.arange(n).reshape(ny, nx)
    diag = np.zeros((ny, nx))
    rows, cols, vals = [], [], []
    # x-faces between (y, x) and (y, x+1)
    t = _harmonic(a[:, :-1], a[:, 1:])
    diag[:, :-1] += t
    diag[:, 1:] += t
    rows.append(idx[:, :-1].ravel()); cols.append(idx[:, 1:].ravel()); vals.append(t.ravel())
    # y-faces between (y, x) and (y+1, x)
    t = _harmonic(a[:-1, :], a[1:, :])
    diag[:-1, :] += t
    diag[1:, :] += t
    rows.append(idx[:-1, :].ravel()); cols.append(idx[1:, :].ravel()); vals.append(t.ravel())
    # Dirichlet wall faces: transmissibility 2 a_P (distance h/2)
    diag[:, 0] += 2.0 * a[:, 0]
    diag[:, -1] += 2.0 * a[:, -1]
    diag[0, :] += 2.0 * a[0, :]
    diag[-1, :] += 2.0 * a[-1, :]
    return _assemble_faces(n, diag.ravel(), np.concatenate(rows), np.concatenate(cols),
                           np.concatenate(vals))


def fv_harmonic_3d(a: np.ndarray) -> sp.csr_matrix:
    """Cell-centred FV operator (7-point) for -div(a grad u), a indexed [z, y, x]."""
    a = np.asarray(a, dtype=np.float64)
    nz, ny, nx = a.shape
    n = a.size
    idx = np.arange(n).reshape(nz, ny, nx)
    diag = np.zeros_like(a)
    rows, cols, vals = [], [], []
    for axis in range(3):
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(None, -1)
        hi[axis] = slice(1, None)
        lo, hi = tuple(lo), tuple(hi)
        t = _harmonic(a[lo], a[hi])
        diag[lo] += t
        diag[hi] += t
        rows.append(idx[lo].ravel()); cols.append(idx[hi].ravel()); vals.append(t.ravel())
        first = [slice(None)] * 3
        last = [slice(None)] * 3
        first[axis] = 0
        last[axis] = -1
        diag[tuple(first)] += 2.0 * a[tuple(first)]
        diag[tuple(last)] += 2.0 * a[tuple(last)]
    return _assemble_faces(n, diag.ravel(), np.concatenate(rows), np.concatenate(cols),
                           np.concatenate(vals))


def q1_aniso_element(eps: float, theta: float) -> np.ndarray:
    """4x4 Q1 element stiffness int grad(phi_i)^T K grad(phi_j) on a square
    element, by 2x2 Gauss quadrature (exact for bilinears).  In 2-D the result
    does not depend on the element size.  Local node order: (0,0), (1,0),
    (1,1), (0,1)."""
    c, s = np.cos(theta), np.sin(theta)
    # R(theta) diag(1, eps) R(theta)^T written out, so that K12 == K21 exactly
    K = np.array([[c * c + eps * s * s, (1.0 - eps) * c * s],
                  [(1.0 - eps) * c * s, s * s + eps * c * c]])
    g = 0.5 / np.sqrt(3.0)
    pts = [0.5 - g, 0.5 + g]
    Ke = np.zeros((4, 4))
    for xi in pts:
        for eta in pts:
            # reference gradients of (1-xi)(1-eta), xi(1-eta), xi*eta, (1-xi)eta
            G = np.array([[-(1 - eta), -(1 - xi)],
                          [(1 - eta), -xi],
                          [eta, xi],
                          [-eta, (1 - xi)]])
            Ke += 0.25 * G @ K @ G.T
    return 0.5 * (Ke + Ke.T)      # the integrand is symmetric; remove rounding asymmetry


def q1_aniso(side: int, eps: float, theta: float) -> sp.csr_matrix:
    """Q1 FEM operator on a (side+2)^2 node grid of the unit square with the
    boundary nodes eliminated (Dirichlet): side^2 unknowns, 9-point."""
    Ke = q1_aniso_element(eps, theta)
    nn = side + 2
    node = np.arange(nn * nn).reshape(nn, nn)          # [y, x]
    ey, ex = np.meshgrid(np.arange(nn - 1), np.arange(nn - 1), indexing="ij")
    ey, ex = ey.ravel(), ex.ravel()
    loc = np.stack([node[ey, ex], node[ey, ex + 1], node[ey + 1, ex + 1], node[ey + 1, ex]], 1)
    r = np.repeat(loc, 4, axis=1).ravel()
    c = np.tile(loc, (1, 4)).ravel()
    v = np.tile(Ke.ravel(), ey.size)
    Afull = sp.csr_matrix(sp.coo_matrix((v, (r, c)), shape=(nn * nn, nn * nn)))
    interior = node[1:-1, 1:-1].ravel()
    return sp.csr_matrix(Afull[interior][:, interior])


def p1_element(p: np.ndarray, K: np.ndarray):
    """Local stiffness and mass matrices of one linear triangle (FEM dataset
    appendix): vertices p (3, 2) counter-clockwise, tensor K (2, 2).  The
    basis gradients are constant: with 2|T| = (x1-x0)(y2-y0) - (x2-x0)(y1-y0),
    grad phi_a = (y_{a+1} - y_{a+2}, x_{a+2} - x_{a+1}) / (2|T|) (indices mod
    3).  Returns (K_T (3, 3) = |T| g K g^T, M_T (3, 3) = |T|/12 [2 1 1; 1 2 1;
    1 1 2])."""
    x, y = p[:, 0], p[:, 1]
    a2 = (x[1] - x[0]) * (y[2] - y[0]) - (x[2] - x[0]) * (y[1] - y[0])
    area = 0.5 * a2
    g = np.empty((3, 2))
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        g[a] = [(y[b] - y[c]) / a2, (x[c] - x[b]) / a2]
    Ke = np.empty((3, 3))
    for a in range(3):
        for b in range(3):
            Ke[a, b] = area * (g[a] @ K @ g[b])
    Me = area / 12.0 * np.array([[2.0, 1.0, 1.0], [1.0, 2.0, 1.0], [1.0, 1.0, 2.0]])
    return Ke, Me


def p1_fem(points: np.ndarray, tris: np.ndarray, ktensor: np.ndarray, sK: float, sM: float,
           boundary: np.ndarray) -> sp.csr_matrix:
    """A = sK K + sM M assembled over the triangles (element by element, plain
    sums), then every boundary vertex's row and column set to zero and its
    diagonal to one (the appendix's Dirichlet treatment).  ktensor (nt, 3)
    holds [Kxx, Kxy, Kyy] per triangle."""
    n = points.shape[0]
    rows, cols, vals = [], [], []
    for t in range(tris.shape[0]):
        idx = tris[t]
        K = np.array([[ktensor[t, 0], ktensor[t, 1]], [ktensor[t, 1], ktensor[t, 2]]])
        Ke, Me = p1_element(points[idx], K)
        Ae = sK * Ke + sM * Me
        for a in range(3):
            for b in range(3):
                rows.append(idx[a])
                cols.append(idx[b])
                vals.append(Ae[a, b])
    A = sp.csr_matrix(sp.coo_matrix((vals, (rows, cols)), shape=(n, n)))
    keep = sp.diags((boundary == 0).astype(np.float64))
    A = keep @ A @ keep + sp.diags((boundary != 0).astype(np.float64))
    A = sp.csr_matrix(A)
    A.eliminate_zeros()
    return A


def jacobi_diag(A: sp.spmatrix) -> np.ndarray:
    """D = diag(A) (the algorithm's setup step)."""
    return np.asarray(A.diagonal(), dtype=np.float64)
