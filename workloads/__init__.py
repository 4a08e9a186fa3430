"""Seeded synthetic inputs for the spectral two-level PCG workloads.

This module is the only code shared by the FP64 oracle (``oracle/``) and the
HIP path (``paper_2601_20174_amd``).  It draws random numbers and coefficient
fields; it holds none of the method's arithmetic (no operator assembly, no
relaxation, no basis, no solver).  Every draw is a pure function of its seed,
so the oracle and the GPU side see bit-identical inputs.

Seeds follow one rule: ``1000*cfg + {0: coefficient field, 1: S0, 2: RHS}``,
with member ``i`` of a batch (fields, systems) offset by ``10*i``.

Workload families (structured-grid stand-ins for the paper's P1-FEM families on
jittered Delaunay meshes of the unit square, Sec. 4.1 and the appendix on
benchmark PDEs):

* ``poisson``    constant-coefficient Poisson, 5-point, interior grid N x N.
* ``grf``        log-normal diffusion a = exp(g), g a Gaussian random field
                 with squared-exponential covariance, cell-centred grid.
* ``aniso``      a batch of rotated anisotropic tensors, one (eps, theta) per
                 system, and a grid side per system.
* ``checker3d``  a 3-D piecewise-constant coefficient, 16^3-cell blocks drawn
                 i.i.d. from {1, 1e3}.
* ``p1``         the paper's own families on unstructured meshes (the FEM
                 dataset appendix): a jittered Delaunay triangulation of the
                 unit square and, per triangle, the coefficient draws of the
                 diffusion, anisotropic, screened Poisson, heat and wave
                 benchmarks.  The mesh and the draws only: assembly of the
                 stiffness and mass matrices is the method's (oracle and GPU
                 each do their own).
"""
from __future__ import annotations

import dataclasses
import numpy as np

__all__ = [
    "seed_for", "normal_block", "uniform_block", "grf_field", "lognormal_field",
    "checkerboard_3d", "aniso_batch", "p1_mesh", "p1_coefficients", "P1_FAMILIES", "Cfg1", "Cfg2",
    "Cfg3", "Cfg4", "Cfg5", "CfgPaper", "CfgFem", "CONFIGS",
]

COEF, S0, RHS = 0, 1, 2


def seed_for(cfg: int, what: int, member: int = 0) -> int:
    """Seed of one draw: 1000*cfg + what + 10*member."""
    return 1000 * int(cfg) + int(what) + 10 * int(member)


def normal_block(seed: int, rows: int, cols: int) -> np.ndarray:
    """(rows, cols) float64 N(0,1), row-major (cols fastest)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((rows, cols))


def uniform_block(seed: int, rows: int, cols: int, lo=-1.0, hi=1.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(rows, cols))


def grf_field(seed: int, N: int, corr_len: float = 0.1, sigma: float = 1.0) -> np.ndarray:
    """Stationary Gaussian random field on the N x N cell centres of [0,1]^2.

    Covariance C(d) = sigma^2 exp(-d^2 / (2 corr_len^2)).  Sampled exactly by
    circulant embedding on a 2N x 2N torus of side 2 (the covariance has
    decayed to exp(-50) at distance 1, so the embedding is non-negative up to
    rounding), then cropped to the first N x N cells.  Returns (N, N) with
    index [y, x].
    """
    M = 2 * N
    h = 1.0 / N
    idx = np.arange(M)
    d1 = np.minimum(idx, M - idx) * h
    d2 = d1[:, None] ** 2 + d1[None, :] ** 2
    c = sigma * sigma * np.exp(-d2 / (2.0 * corr_len * corr_len))
    lam = np.fft.fft2(c).real
    lam = np.clip(lam, 0.0, None)
    rng = np.random.default_rng(seed)
    xi = rng.standard_normal((M, M))
    g = np.fft.ifft2(np.sqrt(lam) * np.fft.fft2(xi)).real
    return np.ascontiguousarray(g[:N, :N])


def lognormal_field(seed: int, N: int, corr_len=0.1, sigma=1.0) -> np.ndarray:
    """a = exp(g) for the GRF above; (N, N) float64, index [y, x]."""
    return np.exp(grf_field(seed, N, corr_len, sigma))


def iid_lognormal_field(seed: int, N: int, sigma: float) -> np.ndarray:
    """Cell-wise i.i.d. kappa = exp(eta), eta ~ N(0, sigma^2) (the paper's
    diffusion family draws one such value per triangle)."""
    rng = np.random.default_rng(seed)
    return np.exp(sigma * rng.standard_normal((N, N)))


def checkerboard_3d(seed: int, N: int = 128, blocks: int = 8, lo=1.0, hi=1e3,
                    strict: bool = False) -> np.ndarray:
    """(N, N, N) float64 coefficient, index [z, y, x], constant on blocks of
    (N/blocks)^3 cells.  Each block value is drawn i.i.d. from {lo, hi}; with
    ``strict`` the parity pattern (bi+bj+bk) mod 2 is used instead."""
    assert N % blocks == 0
    b = N // blocks
    if strict:
        bi = np.indices((blocks, blocks, blocks)).sum(axis=0) % 2
        vals = np.where(bi == 1, hi, lo)
    else:
        rng = np.random.default_rng(seed)
        vals = np.where(rng.integers(0, 2, size=(blocks,) * 3) == 1, hi, lo)
    return np.ascontiguousarray(np.repeat(np.repeat(np.repeat(vals, b, 0), b, 1), b, 2)
                                .astype(np.float64))


ANISO_SIDES = (64, 96, 128, 192, 256)


def aniso_batch(seed: int, nsys: int, sides=ANISO_SIDES):
    """Per-system (side, eps, theta): side ~ U(sides), eps = 10^U(-3,0),
    theta ~ U(0, pi).  Returns three arrays of length nsys."""
    rng = np.random.default_rng(seed)
    side = rng.choice(np.asarray(sides, dtype=np.int64), size=nsys)
    eps = 10.0 ** rng.uniform(-3.0, 0.0, size=nsys)
    theta = rng.uniform(0.0, np.pi, size=nsys)
    return side, eps, theta


# ------------------------------------------------------ unstructured meshes
def p1_mesh(seed: int, N: int):
    """Jittered Delaunay triangulation of [0,1]^2 (the FEM dataset appendix,
    common mesh setup): the (N+1)^2 grid points (i/N, j/N), vertex index
    i + (N+1) j; boundary vertices fixed, interior vertex p moved by
    xi ~ U([-e, e]^2) with e = min(0.35 h, 0.49 d), h = 1/N, d the distance
    of p to the boundary; Delaunay triangulation of the moved points;
    triangles of near-zero signed area (|2 area| <= 1e-12 h^2) removed; every
    triangle ordered counter-clockwise.
    Returns (points (np, 2) float64, tris (nt, 3) int32, boundary (np,) uint8)."""
    from scipy.spatial import Delaunay
    h = 1.0 / N
    j, i = np.meshgrid(np.arange(N + 1), np.arange(N + 1), indexing="ij")
    i, j = i.ravel(), j.ravel()
    pts = np.stack([i * h, j * h], axis=1)
    bnd = ((i == 0) | (i == N) | (j == 0) | (j == N)).astype(np.uint8)
    d = np.minimum(np.minimum(pts[:, 0], 1.0 - pts[:, 0]), np.minimum(pts[:, 1], 1.0 - pts[:, 1]))
    e = np.minimum(0.35 * h, 0.49 * d)
    rng = np.random.default_rng(seed)
    xi = rng.uniform(-1.0, 1.0, size=pts.shape) * e[:, None]
    pts = pts + xi * (bnd == 0)[:, None]
    tris = Delaunay(pts).simplices.astype(np.int64)
    p0, p1, p2 = pts[tris[:, 0]], pts[tris[:, 1]], pts[tris[:, 2]]
    a2 = (p1[:, 0] - p0[:, 0]) * (p2[:, 1] - p0[:, 1]) - (p2[:, 0] - p0[:, 0]) * (p1[:, 1] - p0[:, 1])
    keep = np.abs(a2) > 1e-12 * h * h
    tris, a2 = tris[keep], a2[keep]
    flip = a2 < 0
    tris[flip, 1], tris[flip, 2] = tris[flip, 2].copy(), tris[flip, 1].copy()
    return np.ascontiguousarray(pts), np.ascontiguousarray(tris.astype(np.int32)), bnd


P1_FAMILIES = ("diffusion", "anisotropic", "screened_poisson", "heat", "wave")


def p1_coefficients(family: str, seed: int, nt: int, N: int):
    """Per-triangle coefficient draws of one benchmark family (FEM dataset
    appendix): returns (ktensor (nt, 3) = [Kxx, Kxy, Kyy] of the diffusion
    tensor per triangle, sK, sM) for the matrix A = sK K(ktensor) + sM M.
      diffusion         kappa_T = exp(eta), eta ~ N(0, 1.5^2); A = K
      anisotropic       theta_T ~ U(0, pi), K_T = R diag(1e3, 1) R^T; A = K
      screened_poisson  kappa_T = exp(N(0, 1)), alpha = 10^U(0, 2); A = K + alpha M
      heat              kappa_T = exp(N(0, 1)), dt = 10^U(-2, 0); A = M + dt K
      wave              kappa_T = exp(N(0, 1.5^2)), c = 10^U(2, 3),
                        dt ~ U(h, 2h); A = M + (c dt)^2 K"""
    rng = np.random.default_rng(seed)
    h = 1.0 / N
    if family == "anisotropic":
        th = rng.uniform(0.0, np.pi, size=nt)
        c, s = np.cos(th), np.sin(th)
        kt = np.stack([1e3 * c * c + s * s, (1e3 - 1.0) * c * s, 1e3 * s * s + c * c], axis=1)
        return kt, 1.0, 0.0
    sig = 1.5 if family in ("diffusion", "wave") else 1.0
    kappa = np.exp(rng.normal(0.0, sig, size=nt))
    kt = np.stack([kappa, np.zeros(nt), kappa], axis=1)
    if family == "diffusion":
        return kt, 1.0, 0.0
    if family == "screened_poisson":
        return kt, 1.0, float(10.0 ** rng.uniform(0.0, 2.0))
    if family == "heat":
        return kt, float(10.0 ** rng.uniform(-2.0, 0.0)), 1.0
    if family == "wave":
        c = 10.0 ** rng.uniform(2.0, 3.0)
        dt = rng.uniform(h, 2.0 * h)
        return kt, float((c * dt) ** 2), 1.0
    raise ValueError(family)


# ---------------------------------------------------------------- configurations
@dataclasses.dataclass(frozen=True)
class Cfg1:
    """2-D Poisson, 5-point, 32x32 interior (n=1024); m=32, s1=10, w=2/3, k=16,
    one RHS f ~ U(-1,1), nu1=nu2=1, rtol 1e-8."""
    cfg: int = 1
    N: int = 32
    m: int = 32
    k: int = 16
    s1: int = 10
    omega: float = 2.0 / 3.0
    nu: int = 1
    R: int = 1
    rtol: float = 1e-8

    @property
    def n(self):
        return self.N * self.N

    def S0(self):
        return normal_block(seed_for(self.cfg, S0), self.n, self.m)

    def rhs(self):
        return uniform_block(seed_for(self.cfg, RHS), self.n, self.R)


@dataclasses.dataclass(frozen=True)
class Cfg2:
    """2-D log-normal diffusion on N x N cells (512^2 at full size), a = exp(g),
    GRF corr. length 0.1, sigma 1; m=128, k=64, f ~ N(0,1)."""
    cfg: int = 2
    N: int = 512
    m: int = 128
    k: int = 64
    s1: int = 10
    omega: float = 2.0 / 3.0
    nu: int = 1
    R: int = 1
    rtol: float = 1e-8
    corr_len: float = 0.1
    sigma: float = 1.0

    @property
    def n(self):
        return self.N * self.N

    def coef(self):
        return lognormal_field(seed_for(self.cfg, COEF), self.N, self.corr_len, self.sigma)

    def S0(self):
        return normal_block(seed_for(self.cfg, S0), self.n, self.m)

    def rhs(self):
        return normal_block(seed_for(self.cfg, RHS), self.n, self.R)


@dataclasses.dataclass(frozen=True)
class Cfg3:
    """Batch of anisotropic Q1 systems: side ~ U{64..256}, eps ~ logU(1e-3,1),
    theta ~ U(0,pi); k=32, m=64, 8 RHS ~ N(0,1) per system."""
    cfg: int = 3
    nsys: int = 256
    m: int = 64
    k: int = 32
    s1: int = 10
    omega: float = 2.0 / 3.0
    nu: int = 1
    R: int = 8
    rtol: float = 1e-8
    sides: tuple = ANISO_SIDES

    def systems(self):
        return aniso_batch(seed_for(self.cfg, COEF), self.nsys, self.sides)

    def S0(self, i, n):
        return normal_block(seed_for(self.cfg, S0, i), n, self.m)

    def rhs(self, i, n):
        return normal_block(seed_for(self.cfg, RHS, i), n, self.R)


@dataclasses.dataclass(frozen=True)
class Cfg4:
    """3-D block coefficient (16^3-cell blocks, a in {1,1e3}) on N^3 cells
    (128^3 at full size); m=256, k=128, 16 RHS ~ N(0,1)."""
    cfg: int = 4
    N: int = 128
    blocks: int = 8
    m: int = 256
    k: int = 128
    s1: int = 10
    omega: float = 2.0 / 3.0
    nu: int = 1
    R: int = 16
    rtol: float = 1e-8

    @property
    def n(self):
        return self.N ** 3

    def coef(self):
        return checkerboard_3d(seed_for(self.cfg, COEF), self.N, self.blocks)

    def S0(self):
        return normal_block(seed_for(self.cfg, S0), self.n, self.m)

    def rhs(self):
        return normal_block(seed_for(self.cfg, RHS), self.n, self.R)


@dataclasses.dataclass(frozen=True)
class Cfg5:
    """Training batch: 64 log-normal fields at 128^2 (config-2 generator),
    m=64 relaxed vectors, k=32."""
    cfg: int = 5
    batch: int = 64
    N: int = 128
    m: int = 64
    k: int = 32
    s1: int = 10
    omega: float = 2.0 / 3.0

    def coef(self, i):
        return lognormal_field(seed_for(self.cfg, COEF, i), self.N)

    def S0(self, i):
        return normal_block(seed_for(self.cfg, S0, i), self.N * self.N, self.m)


@dataclasses.dataclass(frozen=True)
class CfgPaper:
    """Paper-shaped run (context only): i.i.d. cell-wise kappa = exp(N(0,1.5^2))
    on 65^2 unknowns, K=72 test vectors, k=48, nu=5, omega=0.66, rtol 1e-6
    (Sec. 4.1 settings)."""
    cfg: int = 9
    N: int = 65
    m: int = 72
    k: int = 48
    s1: int = 10
    omega: float = 0.66
    nu: int = 5
    R: int = 1
    rtol: float = 1e-6

    @property
    def n(self):
        return self.N * self.N

    def coef(self):
        return iid_lognormal_field(seed_for(self.cfg, COEF), self.N, 1.5)

    def S0(self):
        return normal_block(seed_for(self.cfg, S0), self.n, self.m)

    def rhs(self):
        return normal_block(seed_for(self.cfg, RHS), self.n, self.R)


@dataclasses.dataclass(frozen=True)
class CfgFem:
    """The paper's own workload shape: P1 finite elements on a jittered
    Delaunay mesh of [0,1]^2 with (N+1)^2 vertices (N = 64: n = 4225), one of
    the five benchmark families, identity rows for the Dirichlet boundary;
    K = 72 smoothed test vectors, rank k = 48, nu = 5 sweeps with omega = 0.66,
    relative tolerance 1e-6 (the paper's PCG settings)."""
    cfg: int = 6
    N: int = 64
    m: int = 72
    k: int = 48
    s1: int = 10
    omega: float = 0.66
    nu: int = 5
    R: int = 1
    rtol: float = 1e-6

    @property
    def n(self):
        return (self.N + 1) ** 2

    def mesh(self, i: int = 0):
        return p1_mesh(seed_for(self.cfg, COEF, i), self.N)

    def coefficients(self, family: str, nt: int, i: int = 0):
        return p1_coefficients(family, seed_for(self.cfg, COEF, i) + 5 + 100 * P1_FAMILIES.index(family), nt,
                               self.N)

    def S0(self, i: int = 0):
        return normal_block(seed_for(self.cfg, S0, i), self.n, self.m)

    def rhs(self, i: int = 0):
        return normal_block(seed_for(self.cfg, RHS, i), self.n, self.R)


CONFIGS = {1: Cfg1, 2: Cfg2, 3: Cfg3, 4: Cfg4, 5: Cfg5, 6: CfgFem, 9: CfgPaper}
