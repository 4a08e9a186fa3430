"""Pins for the oracle's operator assembly (CPU only).

Each check is fixed by mathematics independent of the assembly code: hand
computations (tests/golden), textbook stencils, closed-form eigenpairs."""
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_blocks(name):
    blocks, cur, key = {}, None, None
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.replace("-", "").replace(" ", "").replace(".", "").isdigit():
            cur.append([float(v) for v in line.split()])
        else:
            key = line
            cur = blocks.setdefault(key, [])
    return {k: np.array(v) for k, v in blocks.items()}


def _read_matrix(name):
    rows = [list(map(float, l.split())) for l in open(os.path.join(GOLD, name))
            if l.strip() and not l.startswith("#")]
    return np.array(rows)


def _all_ops():
    rng = np.random.default_rng(7)
    yield "poisson", O.poisson5(6, 5)
    yield "fv2", O.fv_harmonic_2d(np.exp(rng.standard_normal((5, 7))))
    yield "fv3", O.fv_harmonic_3d(np.exp(rng.standard_normal((3, 4, 5))))
    yield "q1", O.q1_aniso(6, 1e-3, 0.7)
    yield "q1b", O.q1_aniso(5, 0.3, 2.9)


@pytest.mark.parametrize("name,A", list(_all_ops()))
def test_symmetric_exactly_and_spd(name, A):
    D = A - A.T
    assert abs(D).max() == 0.0
    np.linalg.cholesky(A.toarray())          # raises if not SPD


def test_poisson_closed_form_eigenpairs():
    N = 9
    h = 1.0 / (N + 1)
    A = O.poisson5(N)
    x = np.arange(1, N + 1) * h
    for i, j in [(1, 1), (2, 5), (9, 3)]:
        v = np.outer(np.sin(j * np.pi * x), np.sin(i * np.pi * x)).ravel()  # [y, x]
        lam = 4 - 2 * np.cos(i * np.pi * h) - 2 * np.cos(j * np.pi * h)
        np.testing.assert_allclose(A @ v, lam * v, atol=1e-13)


def test_fv_hand_computed_two_cells():
    A = O.fv_harmonic_2d(np.array([[1.0, 3.0]]))
    np.testing.assert_allclose(A.toarray(), _read_matrix("fv_two_cells.txt"), rtol=0, atol=1e-15)


def test_fv_constant_coefficient_is_laplacian_plus_wall_faces():
    N = 6
    A = O.fv_harmonic_2d(np.ones((N, N)))
    walls = np.zeros((N, N))
    walls[:, 0] += 1; walls[:, -1] += 1; walls[0, :] += 1; walls[-1, :] += 1
    # unit transmissibility inside, 2 at a wall: 5-point Laplacian + 1 per wall face
    ref = O.poisson5(N) + sp.diags(walls.ravel())
    assert abs(A - ref).max() < 1e-15
    A3 = O.fv_harmonic_3d(np.ones((3, 4, 5)))
    assert np.allclose(A3.diagonal().reshape(3, 4, 5)[1, 1, 1:-1], 6.0)
    assert np.allclose(A3.diagonal().reshape(3, 4, 5)[0, 0, 0], 9.0)
    assert np.allclose(A3.sum(axis=1).A.ravel().reshape(3, 4, 5)[1, 1, 1:-1], 0.0)


def test_fv_scaling_and_harmonic_face():
    rng = np.random.default_rng(1)
    a = np.exp(rng.standard_normal((4, 5)))
    A = O.fv_harmonic_2d(a)
    assert abs(O.fv_harmonic_2d(3.0 * a) - 3.0 * A).max() < 1e-12
    # face between cells (y=2,x=1) and (y=2,x=2)
    i, j = 2 * 5 + 1, 2 * 5 + 2
    assert np.isclose(-A[i, j], 2 * a[2, 1] * a[2, 2] / (a[2, 1] + a[2, 2]), rtol=1e-15)


def test_q1_element_textbook_blocks():
    g = _read_blocks("q1_element_laplace.txt")
    eps = 0.37
    Ke = O.q1_aniso_element(eps, 0.0)
    np.testing.assert_allclose(6 * Ke, g["xx"] + eps * g["yy"], atol=1e-13)
    # a quarter turn swaps the roles of x and y
    Ke90 = O.q1_aniso_element(eps, np.pi / 2)
    np.testing.assert_allclose(6 * Ke90, eps * g["xx"] + g["yy"], atol=1e-13)
    # rows sum to zero, one-dimensional kernel (constants)
    rng = np.random.default_rng(0)
    Kr = O.q1_aniso_element(1e-2, rng.uniform(0, np.pi))
    np.testing.assert_allclose(Kr.sum(1), 0, atol=1e-14)
    w = np.linalg.eigvalsh(Kr)
    assert abs(w[0]) < 1e-14 and w[1] > 1e-6


def test_q1_isotropic_is_textbook_nine_point():
    side = 7
    A = O.q1_aniso(side, 1.0, 1.234).toarray()
    c = 3 * side + 3                        # an interior unknown away from the boundary
    row = A[c].reshape(side, side)
    np.testing.assert_allclose(row[2:5, 2:5], [[-1 / 3, -1 / 3, -1 / 3],
                                               [-1 / 3, 8 / 3, -1 / 3],
                                               [-1 / 3, -1 / 3, -1 / 3]], atol=1e-14)
    assert np.count_nonzero(np.abs(row) > 1e-15) == 9


# ------------------------------------------------------------- P1 elements
def _grid_mesh(N, flip_pattern=False):
    """Uniform right-triangle mesh of [0,1]^2 (no jitter): each square split by
    one diagonal (alternating directions with flip_pattern), CCW triangles."""
    h = 1.0 / N
    j, i = np.meshgrid(np.arange(N + 1), np.arange(N + 1), indexing="ij")
    pts = np.stack([i.ravel() * h, j.ravel() * h], 1)
    tris = []
    for jj in range(N):
        for ii in range(N):
            a, b = ii + (N + 1) * jj, ii + 1 + (N + 1) * jj
            c, d = ii + (N + 1) * (jj + 1), ii + 1 + (N + 1) * (jj + 1)
            if flip_pattern and (ii + jj) % 2:
                tris += [[a, b, c], [b, d, c]]
            else:
                tris += [[a, b, d], [a, d, c]]
    ii, jj = i.ravel(), j.ravel()
    bnd = ((ii == 0) | (ii == N) | (jj == 0) | (jj == N)).astype(np.uint8)
    return pts, np.array(tris, dtype=np.int32), bnd


def test_p1_reference_element():
    """Reference triangle (0,0), (1,0), (0,1), K = I: the textbook local
    stiffness 1/2 [[2,-1,-1],[-1,1,0],[-1,0,1]] and mass 1/24 [[2,1,1],...]."""
    Ke, Me = O.p1_element(np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]), np.eye(2))
    np.testing.assert_allclose(Ke, 0.5 * np.array([[2, -1, -1], [-1, 1, 0], [-1, 0, 1]]), atol=1e-15)
    np.testing.assert_allclose(Me, np.array([[2, 1, 1], [1, 2, 1], [1, 1, 2]]) / 24.0, atol=1e-15)


@pytest.mark.parametrize("flip", [False, True])
def test_p1_right_triangles_give_the_five_point_stencil(flip):
    """On a uniform right-triangle mesh, P1 with K = diag(kx, ky) is the
    5-point stencil 2kx + 2ky, -kx (x-neighbours), -ky (y-neighbours), for
    either diagonal of each square (the diagonal coupling vanishes)."""
    N, kx, ky = 8, 3.0, 0.5
    pts, tris, bnd = _grid_mesh(N, flip)
    kt = np.tile([kx, 0.0, ky], (len(tris), 1))
    A = O.p1_fem(pts, tris, kt, 1.0, 0.0, bnd).toarray()
    for j in range(1, N):
        for i in range(1, N):
            r = i + (N + 1) * j
            row = np.zeros((N + 1) ** 2)
            row[r] = 2 * kx + 2 * ky
            for di, dj, v in ((1, 0, -kx), (-1, 0, -kx), (0, 1, -ky), (0, -1, -ky)):
                c = (i + di) + (N + 1) * (j + dj)
                if not bnd[c]:
                    row[c] = v
            np.testing.assert_allclose(A[r], row, atol=1e-14)
    for r in np.flatnonzero(bnd):
        e = np.zeros((N + 1) ** 2)
        e[r] = 1.0
        np.testing.assert_array_equal(A[r], e)
        np.testing.assert_array_equal(A[:, r], e)


def test_p1_stiffness_kills_linears_and_mass_integrates():
    """Without Dirichlet rows, on a jittered mesh with random tensors: every
    row of the stiffness sums to 0 (constants) ; with K = I the interior rows
    vanish on the nodal values of x and of y (linear functions are discrete
    harmonic); the mass matrix sums to the area 1."""
    N = 10
    pts, tris, bnd = W.p1_mesh(40, N)
    nt = len(tris)
    kt, _, _ = W.p1_coefficients("anisotropic", 41, nt, N)
    none = np.zeros_like(bnd)
    K = O.p1_fem(pts, tris, kt, 1.0, 0.0, none)
    assert np.abs(K @ np.ones(len(pts))).max() < 1e-10 * abs(K).max()
    K1 = O.p1_fem(pts, tris, np.tile([1.0, 0.0, 1.0], (nt, 1)), 1.0, 0.0, none)
    inner = np.flatnonzero(bnd == 0)
    for c in range(2):
        assert np.abs((K1 @ pts[:, c])[inner]).max() < 1e-12
    M = O.p1_fem(pts, tris, kt, 0.0, 1.0, none)
    assert abs(M.sum() - 1.0) < 1e-13


def test_p1_mesh_and_families_are_spd():
    """The jittered mesh: boundary fixed, interior jitter within
    min(0.35 h, 0.49 d), triangles counter-clockwise covering the unit area;
    every family's matrix is symmetric positive definite (Cholesky)."""
    N = 12
    pts, tris, bnd = W.p1_mesh(42, N)
    h = 1.0 / N
    j, i = np.meshgrid(np.arange(N + 1), np.arange(N + 1), indexing="ij")
    grid = np.stack([i.ravel() * h, j.ravel() * h], 1)
    d = np.minimum(np.minimum(grid[:, 0], 1 - grid[:, 0]), np.minimum(grid[:, 1], 1 - grid[:, 1]))
    assert np.all(np.abs(pts - grid).max(1) <= np.minimum(0.35 * h, 0.49 * d) + 1e-15)
    p0, p1, p2 = pts[tris[:, 0]], pts[tris[:, 1]], pts[tris[:, 2]]
    a2 = (p1[:, 0] - p0[:, 0]) * (p2[:, 1] - p0[:, 1]) - (p2[:, 0] - p0[:, 0]) * (p1[:, 1] - p0[:, 1])
    assert np.all(a2 > 0) and abs(0.5 * a2.sum() - 1.0) < 1e-12
    for fam in W.P1_FAMILIES:
        kt, sK, sM = W.p1_coefficients(fam, 43, len(tris), N)
        A = O.p1_fem(pts, tris, kt, sK, sM, bnd)
        assert abs(A - A.T).max() <= 1e-14 * abs(A).max()
        np.linalg.cholesky(A.toarray())
