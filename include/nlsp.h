/*
 * nlsp.h - C ABI of the MI355X (gfx950) spectral two-level PCG library.
 *
 * The library solves A u = f for a sparse SPD operator A (Sec. 3, "PDE
 * discretization and linear systems") with conjugate gradients preconditioned
 * by the two-grid cycle of the NeuraLSP algorithm ("setup and one
 * preconditioner application"): nu weighted-Jacobi sweeps, a Galerkin coarse
 * correction with A_c = P^T A P, and nu more sweeps.  The prolongation P is the
 * leading k-dimensional left singular subspace of relaxed random vectors
 * S = (I - w D^-1 A)^{s1} S0 (Sec. 3, near-nullspace vectors and SVD-centric
 * construction).
 *
 * Conventions shared by every entry point
 *   - Buffers marked "device" are device pointers owned by the caller; the
 *     library never frees them.  Host arrays are marked "host".
 *   - Dense matrices are row-major.  Vectors of R right-hand sides are (n, R)
 *     with the R values of one unknown contiguous.  Unknowns are numbered
 *     x fastest: i = x + nx*(y + ny*z).
 *   - Scratch memory comes from a caller-provided device workspace whose size
 *     is returned by the matching *_workspace_bytes query (256-byte aligned
 *     base required).  The library allocates no device memory.
 *   - All work is enqueued on `stream` (a hipStream_t; NULL = default stream).
 *     Functions that must return a status computed on the device synchronise
 *     that stream before returning; this is stated per function.
 *   - Arguments are validated on the host before any HIP call; invalid
 *     arguments return NLSP_E_INVALID and enqueue nothing.
 *   - No function throws, aborts or exits.  Every function returns an
 *     nlsp_status value (int).
 */
#ifndef NLSP_H
#define NLSP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
enum nlsp_status {
  NLSP_OK = 0,
  NLSP_NOT_CONVERGED = 1,   /* warning: maxit reached; outputs valid, info filled */
  NLSP_E_INVALID = -1,      /* bad argument (checked on the host)               */
  NLSP_E_NOT_SPD = -2,      /* Cholesky of A_c or of a Gram matrix failed       */
  NLSP_E_BREAKDOWN = -3,    /* p^T A p <= 0 or r^T M^-1 r <= 0 in PCG           */
  NLSP_E_NONFINITE = -4,    /* NaN/Inf in a PCG scalar                          */
  NLSP_E_WORKSPACE = -5,    /* workspace too small or misaligned                */
  NLSP_E_HIP = -6,          /* a HIP runtime call failed                        */
  NLSP_E_RANK = -7          /* relaxed vectors numerically rank-deficient       */
};

/* Human-readable name of a status code (static string). */
const char* nlsp_status_string(int status);

/* ------------------------------------------------------------ operators */
/* Matrix-free SPD operators on structured grids (the paper's PDE families are
 * P1 FEM on meshes of the unit square; these are structured members of the
 * same families, homogeneous Dirichlet boundary eliminated, no 1/h^2 scale). */
enum nlsp_op_kind {
  NLSP_OP_POISSON5 = 0,   /* 2-D 5-point Laplacian: 4 on the diagonal, -1 per neighbour; coef unused */
  NLSP_OP_FV5 = 1,        /* 2-D cell-centred FV for -div(a grad u): face weight = harmonic mean
                             2 a_P a_Q / (a_P + a_Q); wall face 2 a_P.  coef = a, (ny, nx) */
  NLSP_OP_FV7 = 2,        /* the same in 3-D, 7-point; coef = a, (nz, ny, nx) */
  NLSP_OP_STENCIL9 = 3,   /* 2-D constant 9-point stencil; coef = 9 doubles c[(dy+1)*3 + (dx+1)],
                             (A u)_(x,y) = sum c[..] u_(x+dx, y+dy), terms outside the grid dropped */
  NLSP_OP_CSR = 4         /* a general sparse SPD matrix in compressed rows (e.g. the P1 finite
                             elements of p1_assemble): n = nx rows (ny = nz = 1); row_ptr (n + 1)
                             and col_idx (nnz) int32, coef = values (nnz) float64; every row holds
                             its diagonal entry, which must be positive */
};

typedef struct {
  int kind;               /* enum nlsp_op_kind */
  int nx, ny, nz;         /* unknowns per axis; nz = 1 for 2-D kinds; NLSP_OP_CSR: nx = n, ny = nz = 1 */
  const double* coef;     /* device; see kind; NULL for NLSP_OP_POISSON5 */
  const int* row_ptr;     /* device, NLSP_OP_CSR only (else ignored) */
  const int* col_idx;     /* device, NLSP_OP_CSR only (else ignored) */
} nlsp_operator;

/* Number of unknowns n = nx*ny*nz, or -1 for an invalid descriptor. */
int64_t nlsp_operator_size(const nlsp_operator* A);

/* Build the 9-point stencil of bilinear (Q1) finite elements for
 * -div(K grad u), K = R(theta) diag(1, eps) R(theta)^T constant per system, on a
 * uniform grid with the boundary eliminated (element stiffness by 2x2 Gauss
 * quadrature; the anisotropic diffusion family of the paper's appendix, with
 * one tensor per system).
 *   eps_theta  device, (nsys, 2): eps > 0, theta
 *   stencil    device, (nsys, 9): output, layout of NLSP_OP_STENCIL9
 * Asynchronous. */
int q1_aniso_stencil(int nsys, const double* eps_theta, double* stencil, void* stream);

/* ------------------------------------------------- P1 finite elements */
/* The paper's own discretisation (FEM dataset appendix): linear elements on a
 * triangulation with per-triangle tensor K_T, local stiffness
 * |T| g_a^T K_T g_b (g the constant basis gradients) and mass
 * |T|/12 [2 1 1; 1 2 1; 1 1 2], A = sK K + sM M, Dirichlet vertices by zeroing
 * their rows and columns and a unit diagonal.  Built in two calls:
 *
 * p1_pattern (host): the compressed-row pattern of A and, for every stored
 * entry, the list of element contributions to it (code 9 t + 3 a + b:
 * triangle t, local row a, local column b), in increasing triangle order.  A
 * boundary vertex's row holds only its diagonal; couplings to it are dropped.
 *   tris      host (nt, 3) vertex indices, counter-clockwise
 *   boundary  host (np) 1 for a Dirichlet vertex
 *   nnz, ncontrib   host out: sizes (call with the four arrays NULL first)
 *   row_ptr (np + 1), col_idx (nnz), cptr (nnz + 1), clist (ncontrib): host
 *   outputs, or all NULL for the sizes only
 * Columns of a row ascend.  Returns NLSP_E_INVALID for an index out of range
 * or sizes beyond int32. */
int p1_pattern(int np, int nt, const int* tris, const unsigned char* boundary, int64_t* nnz,
               int64_t* ncontrib, int* row_ptr, int* col_idx, int* cptr, int* clist);

/* p1_assemble (device): the values of A on the pattern above, one thread
 * per row summing its contributions in the listed order (deterministic;
 * every local matrix is formed in a form symmetric in a, b, so A is exactly
 * symmetric).
 *   points   device (np, 2) float64      tris   device (nt, 3) int32
 *   ktensor  device (nt, 3) float64: [Kxx, Kxy, Kyy] per triangle
 *   sK, sM   stiffness and mass scales   boundary device (np) uint8
 *   row_ptr, col_idx, cptr, clist   device copies of p1_pattern's outputs
 *   vals     device (nnz) float64, output (coef of an NLSP_OP_CSR operator)
 * Asynchronous on `stream`. */
int p1_assemble(int np, int nt, const double* points, const int* tris, const double* ktensor, double sK,
                double sM, const unsigned char* boundary, const int* row_ptr, const int* col_idx,
                const int* cptr, const int* clist, double* vals, void* stream);

/* dst = src for `bytes` bytes (a multiple of 16; both 16-byte aligned, device):
 * the plainest streaming kernel (one 16-byte vector per thread, non-temporal
 * stores), the practical HBM ceiling against which the benchmark reports its
 * bandwidth-bound kernels.  Asynchronous on `stream`. */
int stream_copy(const void* src, void* dst, int64_t bytes, void* stream);

/* y = A x in float64 for R right-hand sides; x, y device (n, R).  Asynchronous. */
int apply_operator(const nlsp_operator* A, const double* x, double* y, int R, void* stream);

/* One weighted-Jacobi sweep y = x + w D^-1 (b - A x) for R right-hand sides,
 * float32 vectors and arithmetic (the smoother of the algorithm's
 * preconditioner application); b, x, y device (n, R) float32, x != y.
 * Asynchronous. */
int jacobi_sweep_f32(const nlsp_operator* A, double omega, const float* b, const float* x,
                     float* y, int R, void* stream);

/* --------------------------------------------------------------- precision */
enum nlsp_precision {
  NLSP_FP64 = 0,     /* everything in float64 */
  NLSP_MIXED = 1,    /* relaxation, smoother and P/Q products in float32; PCG
                        recurrences, dot products, reductions, Cholesky and the
                        orthonormalisation of P in float64 */
  NLSP_MIXED_F16 = 2 /* pcg_solve only: as NLSP_MIXED, with the coarse term
                        Q A_c^-1 Q^T applied as W W^T, W = Q L^-T, and W
                        stored once in float16, scaled by a power of two so
                        its largest entry is just below 1 (formed from Q32 and
                        L^-1 once per solve; products and sums as
                        NLSP_MIXED).  One rounded matrix serves restriction
                        and prolongation, so the preconditioner stays
                        symmetric.  Halves the basis traffic, the largest part
                        of an iteration's bytes (the paper's rank control as a
                        bandwidth control, Sec. 4) */
};

/* ------------------------------------------------------------ setup: P */
/* Padded rank used by the solver's coarse-space buffers: the smallest power of
 * two >= max(k, 16).  Returns -1 if k < 1 or k > 256. */
int nlsp_padded_rank(int k);

size_t setup_spectral_P_workspace_bytes(const nlsp_operator* A, int m, int k, int prec);

/* Spectral prolongation (Sec. 3; algorithm setup):
 *   S = (I - w D^-1 A)^{s1} S0               relaxation of m random vectors
 *   G = S^T S, G = V diag(lambda) V^T         Gram matrix and its eigenpairs
 *   P0 = S V_k diag(lambda_k)^{-1/2}          leading left singular vectors
 *   P  = CholeskyQR2(P0)                      re-orthonormalised in float64
 * Span(P) is the dominant k-dimensional left singular subspace of S
 * (Eckart-Young); each column is signed so that its largest-magnitude entry
 * is positive.
 *   S0     device (n, m) float64, read only
 *   m, k   1 <= k <= m <= 256, m <= n
 *   omega  Jacobi damping, 0 < omega
 *   s1     relaxation sweeps, s1 >= 0
 *   prec   NLSP_FP64: S kept in float64; NLSP_MIXED: S relaxed in float32
 *   P      device (n, k) float64, output, P^T P = I
 *   sigma  device (m,) float64, output: singular values of S, descending
 * Synchronises `stream`; returns NLSP_E_RANK when sigma_k <= 1e-6 sigma_1
 * (S is then numerically of rank < k: the Gram route resolves singular values
 * only down to about sqrt(eps) sigma_1, and P is not meaningful) and
 * NLSP_E_NOT_SPD when an orthonormalisation Gram matrix is not positive
 * definite. */
int setup_spectral_P(const nlsp_operator* A, const double* S0, int m, int k, double omega,
                     int s1, int prec, double* P, double* sigma, void* ws, size_t ws_bytes,
                     void* stream);

size_t setup_randomized_P_workspace_bytes(const nlsp_operator* A, int m, int k, int l, int prec);

/* Spectral prolongation from a randomized sketch of the relaxed vectors (the
 * RandomSVD baseline of the experimental setup: randomized range finder with
 * subspace iteration, Halko, Martinsson and Tropp 2011, cited in the related
 * work):
 *   S = (I - w D^-1 A)^{s1} S0                relaxation, as setup_spectral_P
 *   Y = S Omega, Q_Y = orth(Y)                sketch of the range of S
 *   q times: Q_Z = orth(S^T Q_Y), Q_Y = orth(S Q_Z)   subspace iteration
 *   B = Q_Y^T S = U_B diag(sigma) V_B^T        (through B B^T, l x l)
 *   P = CholeskyQR2(Q_Y U_B[:, :k])           signs as setup_spectral_P
 * orth is CholeskyQR2 in float64.  The eigenproblem is l x l instead of m x m.
 *   S0     device (n, m) float64, read only
 *   Omega  device (m, l) float64, read only: the random test matrix (drawn by
 *          the caller, e.g. N(0, 1) entries)
 *   m, k, l  1 <= k <= l <= m <= 256, m <= n
 *   q      subspace-iteration steps, 0 <= q <= 8
 *   omega, s1, prec   as setup_spectral_P
 *   P      device (n, k) float64, output, P^T P = I
 *   sigma  device (l,) float64, output: singular values of B, descending
 *          (estimates of the leading singular values of S)
 * Synchronises `stream`; returns NLSP_E_RANK when a sketch is numerically of
 * rank < l or sigma_k <= 1e-6 sigma_1, NLSP_E_NOT_SPD when the final
 * orthonormalisation fails. */
int setup_randomized_P(const nlsp_operator* A, const double* S0, int m, int k, double omega,
                       int s1, const double* Omega, int l, int q, int prec, double* P,
                       double* sigma, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------- setup: coarse */
size_t galerkin_coarse_workspace_bytes(const nlsp_operator* A, int k);

/* Galerkin coarse operator and the solver's coarse-space factors (algorithm
 * setup; appendix, two-level subspace correction):
 *   A_c  = P^T A P (exactly symmetric: its upper triangle, mirrored), A_c = L L^T (Cholesky)
 *   Linv = L^{-1}, zero-padded to (kp, kp), kp = nlsp_padded_rank(k)
 *   Q    = (I - w D^-1 A)^nu P, zero-padded to (n, kp)
 * With these the two-grid preconditioner of the algorithm (nu pre- and nu
 * post-sweeps, z = 0 start) equals, in exact arithmetic,
 *   M^-1 r = J_{2nu} r + Q A_c^-1 Q^T r,
 * where J_{2nu} r is 2 nu weighted-Jacobi sweeps on A z = r from z = 0.
 *   P     device (n, k) float64, full column rank
 *   Ac    device (k, k) float64, output
 *   L     device (k, k) float64, output (lower triangle; upper set to 0)
 *   Linv  device (kp, kp) float64, output
 *   Q64   device (n, kp) float64 output, or NULL
 *   Q32   device (n, kp) float32 output, or NULL (at least one of Q64/Q32)
 * Synchronises `stream`; returns NLSP_E_NOT_SPD when A_c is not positive
 * definite. */
int galerkin_coarse(const nlsp_operator* A, const double* P, int k, double omega, int nu,
                    double* Ac, double* L, double* Linv, double* Q64, float* Q32,
                    void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- solve */
typedef struct {
  int k;                 /* coarse rank (k >= 1) */
  int nu;                /* smoothing sweeps, nu1 = nu2 = nu >= 1 */
  double omega;          /* Jacobi damping used to build Q */
  int prec;              /* NLSP_FP64 reads Q64, NLSP_MIXED and NLSP_MIXED_F16 read Q32 */
  const double* Linv;    /* device (kp, kp) from galerkin_coarse */
  const double* Q64;     /* device (n, kp) or NULL */
  const float* Q32;      /* device (n, kp) or NULL */
} nlsp_two_level;

/* Optional event timing of one of the solver's two per-iteration kernels:
 *   1  update: convergence test, beta, p^T q, alpha, p <- z + beta p,
 *      q <- w + beta q, x += alpha p, r -= alpha q, coarse coefficients,
 *      smoother and prolongation z = J r + Q c, r^T z, ||r||^2, p^T q
 *      (for nu > 1: its update phase)
 *   2  matvec: w = A z, (Q A_c^-1)^T w, z^T w, z^T q + p^T w
 * one launch in `every` carries a start and a stop hipEvent attached to its
 * own dispatch (hipExtLaunchKernelGGL), so the events take the dispatch's
 * begin and end timestamps and no marker packet is inserted between kernels. */
typedef struct {
  int phase;             /* 1 or 2; 0 = no timing */
  int every;             /* time one launch in `every` (>= 1) */
  double total_ms;       /* out: summed duration of the timed launches */
  int launches;          /* out: number of timed launches */
} nlsp_kernel_timing;

typedef struct {
  double rtol;           /* stop when ||f - A u||_2 <= rtol ||f||_2 (per RHS) */
  int maxit;             /* iteration cap (products A p), >= 1 */
  int flexible;          /* 0: beta = r'z / r_old'z_old; 1: Polak-Ribiere beta */
  int check_every;       /* iterations enqueued between host convergence polls (>= 1) */
  nlsp_kernel_timing* timing;  /* host, optional (NULL): per-kernel event timing */
} nlsp_pcg_opts;

typedef struct {
  int iters;             /* number of products A p performed */
  int status;            /* NLSP_OK, NLSP_NOT_CONVERGED, NLSP_E_BREAKDOWN or NLSP_E_NONFINITE */
  double relres;         /* true ||f - A u||_2 / ||f||_2 at exit, float64 */
} nlsp_rhs_info;

size_t pcg_solve_workspace_bytes(const nlsp_operator* A, int k, int R);

/* Preconditioned conjugate gradients (Hestenes-Stiefel; Sec. 4.1 two-grid
 * solver evaluation) with the two-level preconditioner above, independently
 * for each of R right-hand sides.  On meeting the tolerance with the
 * recursive residual the true residual f - A u is formed; if it fails it
 * replaces the recursive one and the iteration continues.
 *   f     device (n, R) float64
 *   u     device (n, R) float64: initial guess in, solution out
 *   info  host array of R records, output
 * Returns the worst per-RHS status (errors before NOT_CONVERGED before OK).
 * Synchronises `stream` (convergence is polled from the host). */
int pcg_solve(const nlsp_operator* A, const nlsp_two_level* M, const double* f, double* u,
              int R, const nlsp_pcg_opts* opts, nlsp_rhs_info* info, void* ws,
              size_t ws_bytes, void* stream);

/* Size of the device scratch array behind pcg_solve_noalloc (256 MiB; e.g.
 * 149 MiB for n = 512^2, k = 64, R = 1). */
#define NLSP_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)

/* pcg_solve for callers that cannot allocate device memory (code between
 * graph captures, serving loops that forbid allocation): the same solve, the
 * same kernels and results, with the workspace taken from a device array of
 * NLSP_NOALLOC_SCRATCH_BYTES inside the library instead of a caller buffer.
 *   A, M, f, u, R, info   as pcg_solve; the caller owns f, u and info
 *   opts                  as pcg_solve; opts->timing must be NULL
 * Calls no hipMalloc/hipFree and instantiates no graph (iterations are
 * launched directly).  The scratch array is per GPU (the one current at the
 * call, which must be the device of `stream`), held by the library until the
 * process ends; its device address is looked up once per device.  Calls on
 * one GPU share it: two calls that overlap on that GPU (different streams or
 * threads) race and give undefined results; calls in sequence are fine (each
 * clears what must start at zero).
 * Returns NLSP_E_WORKSPACE, enqueueing nothing, when
 * pcg_solve_workspace_bytes(A, M->k, R) exceeds NLSP_NOALLOC_SCRATCH_BYTES;
 * NLSP_E_INVALID as pcg_solve, or if opts->timing is set; NLSP_E_HIP if the
 * scratch address cannot be obtained.  Otherwise as pcg_solve (synchronises
 * `stream`). */
int pcg_solve_noalloc(const nlsp_operator* A, const nlsp_two_level* M, const double* f, double* u,
                      int R, const nlsp_pcg_opts* opts, nlsp_rhs_info* info, void* stream);

/* One system of a batch: its operator, its two-level preconditioner (from
 * setup_spectral_P + galerkin_coarse) and its right-hand sides. */
typedef struct {
  nlsp_operator A;
  nlsp_two_level M;      /* k, nu and prec must be equal across the batch */
  const double* f;       /* device (n_i, R) float64 */
  double* u;             /* device (n_i, R) float64: initial guess in, solution out */
} nlsp_system;

size_t pcg_solve_batched_workspace_bytes(int nsys, const nlsp_system* sys, int R, int rows_per_block);

/* pcg_solve for a batch of independent systems of different sizes, each with
 * R right-hand sides, in the same kernel launches: every iteration is one
 * launch of each solver kernel over the workgroups of all systems (a system
 * whose right-hand sides have stopped exits at once).  Without opts->timing
 * the check_every iterations between host polls (made even) are captured
 * once in a hipGraph and replayed.
 *   sys             host array of nsys descriptors
 *   rows_per_block  rows of a system per workgroup (0 = one workgroup per
 *                   NT / R rows, capped at 512 per system); pick it with
 *                   pcg_solve_batched_tune; -1 = the tile that tuner chose
 *                   for a batch of this shape on the current device (0 if
 *                   it has not been tuned in this process)
 *   info            host array of nsys * R records, system-major
 * Returns the worst per-RHS status.  Synchronises `stream`. */
int pcg_solve_batched(int nsys, const nlsp_system* sys, int R, int rows_per_block,
                      const nlsp_pcg_opts* opts, nlsp_rhs_info* info, void* ws, size_t ws_bytes,
                      void* stream);

/* The batched solve with its loop on the device (for callers that capture
 * it in a graph or cannot wait on the host): the same kernels as
 * pcg_solve_batched, but a fixed budget of opts->maxit iterations is enqueued
 * on `stream` (maxit + 1 update and maxit matvec launches) and nothing is
 * read back: no host synchronisation, host-to-device copy, memory fill or
 * allocation happens (descriptors travel as kernel arguments).  A system
 * whose right-hand sides have all stopped leaves the remaining launches at
 * their first instructions, so choose maxit near the iterations expected.
 * There is no residual replacement: a right-hand side whose recursive
 * residual passed and whose true residual did not is NOT_CONVERGED.
 *   info_dev  DEVICE array of nsys * R records (system-major), written by the
 *             last kernel of the solve
 *   opts->timing must be NULL; check_every is not used
 * Returns NLSP_OK once everything is enqueued (or NLSP_E_INVALID /
 * NLSP_E_WORKSPACE / NLSP_E_HIP); the per-RHS statuses are in info_dev.  The
 * workspace is sized by pcg_solve_batched_workspace_bytes and must not be
 * shared with another solve in flight. */
int pcg_solve_batched_async(int nsys, const nlsp_system* sys, int R, int rows_per_block,
                            const nlsp_pcg_opts* opts, nlsp_rhs_info* info_dev, void* ws, size_t ws_bytes,
                            void* stream);

/* Autotuner of the batched solve's tile (rows of a system per workgroup):
 * times `iters` iterations of pcg_solve_batched (on copies of the initial
 * guesses held in the workspace; the caller's u is not modified) for each
 * candidate of pcg_solve_batched_tune_candidates and returns the fastest.
 *   ms  host array of candidate times (ms), or NULL
 * Synchronises `stream`. */
int pcg_solve_batched_tune_candidates(int R, int* rows_per_block);
size_t pcg_solve_batched_tune_workspace_bytes(int nsys, const nlsp_system* sys, int R);
int pcg_solve_batched_tune(int nsys, const nlsp_system* sys, int R, const nlsp_pcg_opts* opts,
                           int iters, int* best_rows_per_block, double* ms, void* ws,
                           size_t ws_bytes, void* stream);

/* The tuner's choice is recorded for the process, keyed by the batch shape:
 * the current device, the basis precision, R, k, nu and each system's
 * operator kind and size, in order (a later tune of the same shape replaces
 * it).  Returns 1 and the recorded tile in *rows_per_block, 0 when this shape
 * has not been tuned, NLSP_E_INVALID on bad arguments.  Thread-safe. */
int pcg_solve_batched_tuned(int nsys, const nlsp_system* sys, int R, int* rows_per_block);

/* ------------------------------------------------------- training losses */
/* Subspace loss of a batch of predicted bases against relaxed samples (Sec. 4,
 * projected energy eq. subspace_energy and the NLSS loss eq. nlss_loss; the
 * loss form follows the appendix on optimality of smooth-error reduction):
 *   colw == NULL  L_b = ||B_b - P_b P_b^T B_b||_F^2 / ||B_b||_F^2, evaluated
 *                 through C = P^T B and G = P^T P, so valid for any P
 *   colw != NULL  L_b = 1 - sum_j colw_j ||p_j^T B_b||^2 / ||B_b||_F^2; with
 *                 colw_j = (k - j + 1)/k this equals the NLSS loss for any P
 *   P     device (batch, n, k) float32        B  device (batch, n, m) float32
 *   colw  device (k) float32 or NULL          loss  device (batch) float32
 *   saved device, >= subspace_loss_saved_bytes, 256-byte aligned: written by
 *         the forward (per sample the float64 loss, then the backward's small
 *         matrix), read by the backward; owned by the caller
 * Limits: 1 <= k <= 64, 1 <= m <= 256 (else NLSP_E_INVALID).  Products are
 * float32 MFMA over row slabs; slabs are added in float64 in a fixed order,
 * so results are bit-reproducible.  Asynchronous on `stream`. */
size_t subspace_loss_saved_bytes(int batch, int n, int k, int m);
size_t subspace_loss_workspace_bytes(int batch, int n, int k, int m);
int subspace_loss_fwd(int batch, int n, int k, int m, const float* P, const float* B,
                      const float* colw, float* loss, void* saved, size_t saved_bytes,
                      void* ws, size_t ws_bytes, void* stream);

/* Gradient of the forward's loss: gP_b = gloss_b * dL_b/dP_b, with
 *   plain     dL/dP = -(2/||B||^2) [B C^T (2I - G) - P C C^T]
 *   weighted  dL/dP = -(2/||B||^2) B C^T diag(colw)
 *   saved  device, as written by subspace_loss_fwd for the same P, B, colw
 *   gloss  device (batch) float32          gP  device (batch, n, k) float32
 * Asynchronous on `stream`. */
int subspace_loss_bwd(int batch, int n, int k, int m, const float* P, const float* B,
                      const void* saved, size_t saved_bytes, const float* gloss, float* gP,
                      void* stream);

/* Captured energy of a batch of ordered bases under prefix truncation (Sec. 5,
 * Quantitative Results: the energy-gap figure E_SVD(r) - E_model(r); the
 * captured energy Tr(P^T S S^T P) of the appendix's Ky Fan argument):
 *   energy[b][r-1] = ||P_b[:, :r]^T S_b||_F^2 / ||S_b||_F^2,  r = 1 .. k
 * (the fraction of ||S_b||_F^2 that the first r columns capture when P_b has
 * orthonormal columns).  Truncating a basis to its first r columns needs no
 * call: pass P[:, :r] wherever a basis is taken.
 *   P  device (batch, n, k) float32      S  device (batch, n, m) float32
 *   energy  device (batch, k) float64
 * Limits as subspace_loss_fwd.  The products P^T S are the forward's float32
 * MFMA products with float64 slab sums; row energies and prefix sums in
 * float64, fixed order.  Asynchronous on `stream`. */
size_t captured_energy_workspace_bytes(int batch, int n, int k, int m);
int captured_energy(int batch, int n, int k, int m, const float* P, const float* S, double* energy, void* ws,
                    size_t ws_bytes, void* stream);

/* Galerkin product of a batch of bases with a batch of operators (Algorithm 1
 * coarse operator; appendix "Two-Level Subspace Correction", coarse-operator
 * equation), for training through A_c:
 *   Y_b = A_b P_b,  A_c,b = (P_b^T Y_b + Y_b^T P_b) / 2
 *   A     host descriptor shared by the batch (kind, grid); its coefficients
 *         are batched: FV5/FV7 coef = batch x n doubles, STENCIL9 coef =
 *         batch x 9 doubles, POISSON5 none
 *   P     device (batch, n, k) float32     Ac  device (batch, k, k) float32
 *   Y     device (batch, n, k) float32, output, kept by the caller for the
 *         backward
 * Limits: 1 <= k <= 64, n k < 2^31.  Float32 stencil and MFMA products,
 * slab sums in float64.  Asynchronous on `stream`. */
size_t galerkin_fwd_workspace_bytes(int batch, const nlsp_operator* A, int k);
int galerkin_fwd(int batch, const nlsp_operator* A, const float* P, int k, float* Ac, float* Y,
                 void* ws, size_t ws_bytes, void* stream);

/* Backward of the Galerkin product: with G_b = dL/dA_c,b (upstream),
 * dL/dP_b = A_b P_b (G_b + G_b^T) = Y_b (G_b + G_b^T)   (A_b symmetric).
 *   Y    device (batch, n, k) float32 from galerkin_fwd
 *   gAc  device (batch, k, k) float32      gP  device (batch, n, k) float32
 * Asynchronous on `stream`. */
size_t galerkin_bwd_workspace_bytes(int batch, int n, int k);
int galerkin_bwd(int batch, int n, int k, const float* Y, const float* gAc, float* gP, void* ws,
                 size_t ws_bytes, void* stream);

/* Galerkin-convergence term (Sec. 4 and the appendix's Galerkin objective,
 * the projected energy that the Galerkin coarse space minimises) for a batch:
 *   J_b(P) = ||A_b^{1/2} (I - P (P^T A_b P)^{-1} P^T A_b) S_b||_F^2
 *          = tr(S^T A S) - tr(W^T A_c^{-1} W),   W = P^T A S,  A_c = P^T A P,
 *   dJ_b/dP_b = 2 [A P Z Z^T - A S Z^T],  Z = A_c^{-1} W   (A_b symmetric).
 *   A      host descriptor with batched coefficients, as for galerkin_fwd
 *   P      device (batch, n, k) float32      S  device (batch, n, m) float32
 *   J      device (batch) float32            bad device (batch) int: 1 where
 *          P^T A P was not positive definite (J and M of that sample invalid)
 *   E      device (batch) float32 or NULL: tr(S^T A S) = ||A^{1/2} S||_F^2,
 *          the value of J with no coarse space (the scale of the term in a
 *          training loss)
 *   saved  device, galerkin_term_saved_bytes: [A S | A P] (float32) and the
 *          backward's small matrix, written by the forward, read by the
 *          backward (caller-owned, 256-byte aligned)
 * Limits: 1 <= k <= 64, m + k <= 256, k m <= 4096, n (m + k) < 2^31.  Float32
 * stencil and MFMA products, slab sums, Cholesky and the k x m solves in
 * float64.  Asynchronous on `stream`. */
size_t galerkin_term_saved_bytes(int batch, const nlsp_operator* A, int k, int m);
size_t galerkin_term_workspace_bytes(int batch, const nlsp_operator* A, int k, int m);
int galerkin_term_fwd(int batch, const nlsp_operator* A, const float* P, const float* S, int k, int m, float* J,
                      float* E, int* bad, void* saved, size_t saved_bytes, void* ws, size_t ws_bytes,
                      void* stream);
/* dL/dP_b = gJ_b dJ_b/dP_b from `saved` (gJ device (batch) float32, gP device
 * (batch, n, k) float32).  Asynchronous on `stream`. */
int galerkin_term_bwd(int batch, const nlsp_operator* A, int k, int m, const void* saved, const float* gJ,
                      float* gP, void* stream);

/* Thin QR of a batch of n x k matrices (the qf() of Sec. 4 that makes the
 * predicted basis orthonormal): A = Q R, R upper triangular with positive
 * diagonal, by CholeskyQR2 (Gram matrix in float64 from float32 MFMA
 * products, Cholesky, triangular inverse; twice).
 *   A    device (batch, n, k) float32      Q  device (batch, n, k) float32
 *   R    device (batch, k, k) float64      bad device (batch) int: set to 1
 *        where a Gram matrix was not positive definite (A rank deficient)
 * Limits: 1 <= k <= 64, k <= n.  Asynchronous on `stream`. */
size_t qr_thin_workspace_bytes(int batch, int n, int k);
int qr_thin_fwd(int batch, int n, int k, const float* A, float* Q, double* R, int* bad, void* ws,
                size_t ws_bytes, void* stream);

/* Backward of Q = qf(A) for an upstream gradient gQ (R receives none):
 *   gA = [gQ + Q copyltu(-gQ^T Q)] R^-T,
 * copyltu(M) = the symmetric matrix with the lower triangle of M.
 * Asynchronous on `stream`. */
int qr_thin_bwd(int batch, int n, int k, const float* Q, const double* R, const float* gQ, float* gA,
                void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------- P-predictor CNN */
/* A small convolutional predictor of the basis (Sec. 4, neural
 * parameterisation + thin QR; here a CNN on the coefficient field):
 *   P_hat_b = Phi_k + conv4(g(conv3(g(conv2(g(conv1(x_b))))))),
 *   x_b = [ (log a_b - mean) / std , Phi_k ]   (1 + k channels per cell),
 * 3x3 'same' convolutions with zero padding and bias, width `hidden`, g =
 * erf-GELU, Phi_k the k smoothest sine modes sin(i pi x) sin(j pi y) of the
 * unit square (by i^2 + j^2, ties by i) at the cell centres, unit 2-norm.
 * Fields are N x N cells, numbered x fastest (as the operators).
 * Parameters (float32, one vector): for l = 1..4, W_l (Cout, Cin, 3, 3) then
 * b_l (Cout).  Arithmetic: bfloat16 activations and weights in the
 * convolutions, float32 accumulation, float32 output and gradients.
 * Limits: k and hidden multiples of 16, <= 64; N >= 16;
 * ceil((1 + k) / 16) * hidden / 16 <= 16 (so k = 64 with hidden = 64 is
 * rejected). */
typedef struct {
  int batch;             /* fields */
  int N;                 /* cells per side */
  int k;                 /* basis columns */
  int hidden;            /* channels of the hidden layers */
} nlsp_cnn_shape;

int64_t cnn_param_count(const nlsp_cnn_shape* shape);   /* -1 if the shape is invalid */
size_t cnn_workspace_bytes(const nlsp_cnn_shape* shape);

/* P_hat (batch, N*N, k) float32 from params and the cell coefficients
 * coef (batch, N*N) float64 (device).  The workspace keeps the activations
 * for cnn_bwd.  Asynchronous on `stream`. */
int cnn_fwd(const nlsp_cnn_shape* shape, const float* params, const double* coef, float* Phat,
            void* ws, size_t ws_bytes, void* stream);

/* Gradient of the parameters (written, not accumulated) for an upstream
 * gradient gPhat (batch, N*N, k); `ws` must hold the activations of the
 * cnn_fwd call with the same params.  Asynchronous on `stream`. */
int cnn_bwd(const nlsp_cnn_shape* shape, const float* params, const float* gPhat, float* gparams,
            void* ws, size_t ws_bytes, void* stream);

/* One bias-corrected Adam step (step >= 1) on `count` float32 parameters;
 * m and v are the caller's moment buffers (zero before step 1). */
int adam_step(int64_t count, float* params, const float* grads, float* m, float* v, float lr,
              float beta1, float beta2, float eps, int step, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* NLSP_H */
