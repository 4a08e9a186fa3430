// Setup of the spectral two-level preconditioner on gfx950:
//   relaxation S = (I - w D^-1 A)^{s1} S0       (Sec. 3, near-nullspace vectors)
//   Gram G = S^T S (float64 MFMA), G = V L V^T   (Sec. 3, SVD-centric construction)
//   P0 = S V_k L_k^{-1/2}, CholeskyQR2 -> P      (orthonormal basis, float64)
//   A_c = P^T (A P), L = chol(A_c), L^-1, Q = (I - w D^-1 A)^nu P
//                                                 (algorithm setup: Galerkin operator)
#include <cmath>
#include <vector>

#include "device_common.hpp"
#include "host_common.hpp"

namespace nlsp {

typedef double d4_t __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------ stencil rows
// Coefficients of row i of A in nine fixed slots (slot 0 the diagonal for the
// 5/7-point kinds, the stencil position for the 9-point kind); an absent
// neighbour has weight 0 and column i, so every slot can be read unguarded.
struct Row9 {
  double c[9];
  int64_t j[9];
};

NLSP_DEV void row_coeffs(const OpDev& op, int64_t i, Row9& rw) {
  // branch-free: absent neighbours get weight 0 and column i, and their
  // coefficient loads read row i, so all loads of the row issue together
  int x, y, z;
  decompose(op, i, x, y, z);
  const int nx = op.nx, ny = op.ny;
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    rw.c[t] = 0.0;
    rw.j[t] = i;
  }
  if (op.kind == NLSP_OP_STENCIL9) {
    const auto c = op.coef;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int t = (dy + 1) * 3 + (dx + 1);
        const bool ok = y + dy >= 0 && y + dy < ny && x + dx >= 0 && x + dx < nx;
        rw.c[t] = ok ? c[t] : 0.0;
        rw.j[t] = ok ? i + dx + (int64_t)dy * nx : i;
      }
    return;
  }
  const int64_t sxy = (int64_t)nx * ny;
  const bool in[6] = {x > 0, x < nx - 1, y > 0, y < ny - 1, z > 0, z < op.nz - 1};
  const int64_t nb[6] = {i - 1, i + 1, i - nx, i + nx, i - sxy, i + sxy};
  const int nf = (op.kind == NLSP_OP_FV7) ? 6 : 4;
  if (op.kind == NLSP_OP_POISSON5) {
    rw.c[0] = 4.0;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      rw.c[1 + f] = in[f] ? -1.0 : 0.0;
      rw.j[1 + f] = in[f] ? nb[f] : i;
    }
    return;
  }
  const auto a = op.coef;
  const double aP = a[i];
  double d = 0.0;
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    if (f >= nf) break;
    const int64_t j = in[f] ? nb[f] : i;
    const double t = harmonic<double>(aP, a[j]);
    d += in[f] ? t : 2.0 * aP;
    rw.c[1 + f] = in[f] ? -t : 0.0;
    rw.j[1 + f] = j;
  }
  rw.c[0] = d;
}

// the diagonal entry of a row from its coefficients (the centre slot)
NLSP_DEV double row_center(const OpDev& op, const Row9& rw) {
  return (op.kind == NLSP_OP_STENCIL9) ? rw.c[4] : rw.c[0];
}

// Multi-column stencil pass over (n, m) row-major blocks.  One wave per
// unknown (the row's coefficients are computed once per wave), lanes over
// the m columns (coalesced).
//   mode 0: out = in - w D^-1 (A in)     (Jacobi relaxation of A s = 0)
//   mode 1: out = A in
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_stencil_cols(OpDev op, int m, double omega, int mode,
                                                      const TI* __restrict__ in,
                                                      TO* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  if (i >= op.n) return;
  Row9 rw;
  row_coeffs(op, i, rw);
  const double scale = (mode == 0) ? omega / row_center(op, rw) : 0.0;
  for (int col = lane; col < m; col += 64) {
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < 9; ++t) s += rw.c[t] * (double)in[rw.j[t] * m + col];
    const double v = (mode == 0) ? (double)in[i * m + col] - scale * s : s;
    out[i * m + col] = (TO)v;
  }
}

// Row-blocked form of the same passes for 16-byte column vectors (VW columns
// per lane): a workgroup owns TR consecutive rows (consecutive workgroups on
// one XCD, so the rows' y- and z-neighbours were read by the same L2), forms
// each row's coefficients once into LDS, then streams the (row, column
// vector) items, two per thread with every load issued before the arithmetic.
// Only the operator's NSL slots are read (5, 7 or 9, in the order of
// k_stencil_cols); coefficients and sums in float64 as there.
constexpr int COLS_NT = 256, COLS_TR = 128;

template <typename T, int VW>
struct ColVec {
  using V = T __attribute__((ext_vector_type(VW)));
};

template <typename T, int VW, int NSL>
__global__ __launch_bounds__(COLS_NT) void k_cols(OpDev op, int mp, int TR, FastDiv fcv, double omega, int mode,
                                                 const T* __restrict__ in, T* __restrict__ out) {
  using V = typename ColVec<T, VW>::V;
  constexpr int CS = NSL == 9 ? 4 : 0;   // the centre slot
  __shared__ double sc[COLS_TR][NSL];
  __shared__ int sj[COLS_TR][NSL];       // neighbour row minus the row
  __shared__ double ssc[COLS_TR];        // omega / a_ii (mode 0)
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t r0 = (int64_t)lb * TR;
  const int nrows = (int)min((int64_t)TR, op.n - r0);
  for (int t = threadIdx.x; t < nrows; t += COLS_NT) {
    Row9 rw;
    row_coeffs(op, r0 + t, rw);
#pragma unroll
    for (int q = 0; q < NSL; ++q) {
      sc[t][q] = rw.c[q];
      sj[t][q] = (int)(rw.j[q] - (r0 + t));
    }
    ssc[t] = (mode == 0) ? omega / row_center(op, rw) : 0.0;
  }
  __syncthreads();
  const int CV = (int)fcv.d;
  const int total = nrows * CV;
  for (int b0 = threadIdx.x; b0 < total; b0 += 2 * COLS_NT) {
    int rl[2];
    int64_t g[2];
    V v[2][NSL];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int idx = min(b0 + h * COLS_NT, total - 1);   // a spare item repeats the last one
      rl[h] = (int)fdiv((uint32_t)idx, fcv);
      g[h] = (r0 + rl[h]) * mp + (int64_t)(idx - rl[h] * CV) * VW;
#pragma unroll
      for (int q = 0; q < NSL; ++q)
        v[h][q] = *reinterpret_cast<const V*>(in + g[h] + (int64_t)sj[rl[h]][q] * mp);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (b0 + h * COLS_NT >= total) break;
      V o;
#pragma unroll
      for (int e = 0; e < VW; ++e) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < NSL; ++q) acc += sc[rl[h]][q] * (double)v[h][q][e];
        o[e] = (T)((mode == 0) ? (double)v[h][CS][e] - ssc[rl[h]] * acc : acc);
      }
      *reinterpret_cast<V*>(out + g[h]) = o;
    }
  }
}

// The multi-column pass for a compressed-row operator: one wave per row
// (its entries read once per wave), lanes over the m columns; float64
// coefficients and sums, modes as k_stencil_cols.
template <typename T>
__global__ __launch_bounds__(256) void k_csr_cols(OpDev op, int m, double omega, int mode, const T* __restrict__ in,
                                                  T* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  if (i >= op.n) return;
  const int e0 = op.rp[i], e1 = op.rp[i + 1];
  double dg = 0.0;
  for (int e = e0; e < e1; ++e)
    if (op.ci[e] == (int)i) dg = op.coef[e];
  const double scale = (mode == 0) ? omega / dg : 0.0;
  for (int col = lane; col < m; col += 64) {
    double s = 0.0;
    for (int e = e0; e < e1; ++e) s += op.coef[e] * (double)in[(int64_t)op.ci[e] * m + col];
    const double v = (mode == 0) ? (double)in[i * m + col] - scale * s : s;
    out[i * m + col] = (T)v;
  }
}

// Column-slab z-march over a 3-D FV7 operator (in the operator kernels'
// source): false when the shape does not fit it.
template <typename T>
bool zmarch_cols(const OpDev& op, int mode, double omega, int ld, const T* in, T* out, hipStream_t s);
// its float32 relaxation sweep reading float64 rows, and its float64 sweep
// storing float32 rows
bool zmarch_cols_relax_f64in(const OpDev& op, double omega, int ld, const double* in, float* out, hipStream_t s);
bool zmarch_cols_relax_f32out(const OpDev& op, double omega, int ld, const double* in, float* out, hipStream_t s);

// the multi-column pass over (n, mp) blocks: the column-slab z-march on 3-D
// FV7 grids (each row read from HBM once, where k_cols re-reads the z
// neighbours' planes, which have left the L2 by then: 3-D setup with m = 256
// on 128^3 cells 59.6 -> 51.5 ms mixed, 77.0 -> 58.2 ms float64), k_cols when
// the rows are whole 16-byte vectors, k_stencil_cols otherwise (k_csr_cols
// for compressed rows)
template <typename T>
inline void launch_cols(const OpDev& op, int mp, double omega, int mode, const T* in, T* out, hipStream_t s) {
  if (op.kind == NLSP_OP_CSR) {
    hipLaunchKernelGGL(k_csr_cols<T>, dim3(ceil_div(op.n, 4)), dim3(256), 0, s, op, mp, omega, mode, in, out);
    return;
  }
  if (zmarch_cols<T>(op, mode, omega, mp, in, out, s)) return;
  constexpr int VW = 16 / sizeof(T);
  const bool al = reinterpret_cast<uintptr_t>(in) % 16 == 0 && reinterpret_cast<uintptr_t>(out) % 16 == 0;
  if (mp % VW != 0 || !al || op.n * mp >= (int64_t(1) << 31)) {
    hipLaunchKernelGGL((k_stencil_cols<T, T>), dim3(ceil_div(op.n, 4)), dim3(256), 0, s, op, mp, omega, mode,
                       in, out);
    return;
  }
  const int CV = mp / VW;
  const int TR = std::max(1, std::min(COLS_TR, 2048 / CV));
  const unsigned nb = (unsigned)ceil_div(op.n, TR);
  const FastDiv f = make_fastdiv((uint32_t)CV);
  switch (op.kind) {
    case NLSP_OP_STENCIL9:
      hipLaunchKernelGGL((k_cols<T, VW, 9>), dim3(nb), dim3(COLS_NT), 0, s, op, mp, TR, f, omega, mode, in, out);
      break;
    case NLSP_OP_FV7:
      hipLaunchKernelGGL((k_cols<T, VW, 7>), dim3(nb), dim3(COLS_NT), 0, s, op, mp, TR, f, omega, mode, in, out);
      break;
    default:
      hipLaunchKernelGGL((k_cols<T, VW, 5>), dim3(nb), dim3(COLS_NT), 0, s, op, mp, TR, f, omega, mode, in, out);
  }
}

// --------------------------------------------------------------- MFMA Gram
// Partial cross products C = X^T Y over a slice of rows, X (n, a), Y (n, b)
// row-major, a and b multiples of 16.  v_mfma_f64_16x16x4f64: lane l supplies
// A[l%16][l/16] and B[l/16][l%16] and receives D[4*v + l/16][l%16], v < 4
// (the float64 variant interleaves output rows; checked on the device).
// With A[i][kk] = X[r0+kk][16I+i] and B[kk][j] = Y[r0+kk][16J+j] both operands
// are "row r0 + l/16, column l%16 of a 4 x 16 block".  Tiles are dealt
// round-robin to the waves; `sym` keeps only tiles with I <= J (X == Y).
constexpr int GS_ROWS = 16;   // rows per staged slab (4 MFMA k-steps)
constexpr int GS_MAXV = 2;    // 16-byte vectors per thread and slab (host-checked)
template <typename T>
struct GsVec {
  static constexpr int VE = 16 / sizeof(T);
  using V = T __attribute__((ext_vector_type(VE)));
};
// LDS row stride (doubles): a row of 8a bytes that is a multiple of 256
// bytes gets 16 doubles of padding, so consecutive rows start 128 bytes apart
// modulo the 256-byte bank row
__host__ __device__ inline int gs_stride(int a) { return a + ((a * 8) % 256 == 0 ? 16 : 0); }
inline size_t gs_lds_bytes(int a, int b, int sym) {
  return sizeof(double) * GS_ROWS * (gs_stride(a) + (sym == 1 ? 0 : gs_stride(b)));
}

template <typename T, int MAXT>
__global__ __launch_bounds__(1024) void k_gram_partial(const T* __restrict__ X,
                                                       const T* __restrict__ Y, int64_t n, int a,
                                                       int b, int sym, int64_t rows_per_wg,
                                                       double* __restrict__ part) {
  extern __shared__ double gsh[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
  const int TA = a / 16, TB = b / 16;
  // sym 1: X^T X (Y = X, loaded once); sym 2: X^T Y whose result is known to
  // be symmetric; both compute the upper triangle of tiles only
  const bool tri = sym != 0, one = sym == 1;
  const int ntiles = tri ? TA * (TA + 1) / 2 : TA * TB;
  // tiles in a fixed order (row-major; upper triangle with sym), dealt
  // round-robin: slot q of this wave holds tile wave + q * nwave.  Decoded per
  // slot with a compile-time slot index, so the list stays in registers.
  int tI[MAXT], tJ[MAXT];
  const int nt = wave < ntiles ? min(MAXT, (ntiles - wave + nwave - 1) / nwave) : 0;
#pragma unroll
  for (int q = 0; q < MAXT; ++q) {
    const int cnt = min(wave + q * nwave, ntiles - 1);
    int I, J;
    if (tri) {
      int rem = cnt, row = 0;
      while (rem >= TA - row) { rem -= TA - row; ++row; }
      I = row;
      J = row + rem;
    } else {
      I = cnt / TB;
      J = cnt % TB;
    }
    tI[q] = I;
    tJ[q] = J;
  }
  d4_t acc[MAXT];
#pragma unroll
  for (int q = 0; q < MAXT; ++q) acc[q] = d4_t{0.0, 0.0, 0.0, 0.0};
  // Row slabs of GS_ROWS rows of X (and Y) are staged in LDS as float64 with
  // coalesced 16-byte loads; the next slab is loaded into registers while the
  // MFMAs consume the current one.  Rows past the slice are zero.  LDS rows
  // are padded so that the four 128-byte row segments an MFMA operand read
  // touches fall on alternating bank halves.
  using V = typename GsVec<T>::V;
  constexpr int VE = GsVec<T>::VE;
  const int sa = gs_stride(a), sb = one ? 0 : gs_stride(b);
  double* Xs = gsh;
  double* Ys = one ? gsh : gsh + GS_ROWS * sa;
  const int nva = GS_ROWS * a / VE, nvb = one ? 0 : GS_ROWS * b / VE;   // vectors per slab
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg;
  const int64_t r1 = min(n, r0 + rows_per_wg);
  V reg[GS_MAXV];
  auto fetch = [&](int64_t row0) {
#pragma unroll
    for (int u = 0; u < GS_MAXV; ++u) {
      const int v = threadIdx.x + u * blockDim.x;
      V x = V{};
      if (v < nva) {
        const int rr = v * VE / a;
        if (row0 + rr < r1) x = *reinterpret_cast<const V*>(X + row0 * a + (int64_t)v * VE);
      } else if (v < nva + nvb) {
        const int w = v - nva, rr = w * VE / b;
        if (row0 + rr < r1) x = *reinterpret_cast<const V*>(Y + row0 * b + (int64_t)w * VE);
      }
      reg[u] = x;
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int u = 0; u < GS_MAXV; ++u) {
      const int v = threadIdx.x + u * blockDim.x;
      if (v < nva) {
        const int e = v * VE, rr = e / a, cc = e - rr * a;
#pragma unroll
        for (int c = 0; c < VE; ++c) Xs[rr * sa + cc + c] = (double)reg[u][c];
      } else if (v < nva + nvb) {
        const int e = (v - nva) * VE, rr = e / b, cc = e - rr * b;
#pragma unroll
        for (int c = 0; c < VE; ++c) Ys[rr * sb + cc + c] = (double)reg[u][c];
      }
    }
  };
  const int kr = lane >> 4, kc = lane & 15;
  const int ldy = one ? sa : sb;
  if (r0 < r1) {
    fetch(r0);
    stage();
  }
  __syncthreads();
  for (int64_t row0 = r0; row0 < r1; row0 += GS_ROWS) {
    const bool more = row0 + GS_ROWS < r1;
    if (more) fetch(row0 + GS_ROWS);
#pragma unroll 1
    for (int ks = 0; ks < GS_ROWS / 4; ++ks) {
      const double* xr = Xs + (4 * ks + kr) * sa + kc;
      const double* yr = Ys + (4 * ks + kr) * ldy + kc;
#pragma unroll
      for (int q = 0; q < MAXT; ++q) {
        if (q < nt) {
          const double av = xr[16 * tI[q]];
          const double bv = yr[16 * tJ[q]];
          acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[q], 0, 0, 0);
        }
      }
    }
    __syncthreads();
    if (more) stage();
    __syncthreads();
  }
  double* P = part + (int64_t)blockIdx.x * a * b;
#pragma unroll
  for (int q = 0; q < MAXT; ++q) {
    if (q < nt) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * tI[q] + 4 * v + kr, j = 16 * tJ[q] + kc;
        P[(int64_t)i * b + j] = acc[q][v];
      }
    }
  }
}

// Sum of the nwg partial products, fixed order.  A block owns 64 stored
// elements (e = i b + j; with sym only tiles I <= J are stored, each written
// to (i, j) and (j, i)); its four waves sum the partials w = q, q + 4, ... for
// q = wave (eight loads in flight per lane), then the four slice sums are
// added in wave order.
constexpr int GR_NT = 256;
__global__ __launch_bounds__(GR_NT) void k_gram_reduce(const double* __restrict__ part, int nwg, int a, int b, int sym,
                                                      double* __restrict__ out, int lda_out) {
  __shared__ double sl[GR_NT];
  const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + lane;
  const int ec = min(e, a * b - 1);
  const int64_t ab = (int64_t)a * b;
  const bool stored = !sym || (ec / b) / 16 <= (ec % b) / 16;
  double acc = 0.0;
  int w = stored ? q : nwg;
  for (; w + 28 < nwg; w += 32) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(w + 4 * u) * ab + ec];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += v[u];
  }
  for (; w < nwg; w += 4) acc += part[(int64_t)w * ab + ec];
  sl[threadIdx.x] = acc;
  __syncthreads();
  if (q != 0 || e >= a * b) return;
  const double sum = ((sl[lane] + sl[64 + lane]) + sl[128 + lane]) + sl[192 + lane];
  const int i = e / b, j = e % b;
  if (sym && (i / 16) > (j / 16)) return;   // lower tiles are not stored
  // sym = 2: a diagonal tile is not symmetric in rounding; its upper half is
  // mirrored too
  const bool dmirror = sym == 2 && (i / 16) == (j / 16);
  if (dmirror && i > j) return;
  out[(int64_t)i * lda_out + j] = sum;
  if (sym && ((i / 16) < (j / 16) || (dmirror && i < j))) out[(int64_t)j * lda_out + i] = sum;
}

// ------------------------------------------------- small dense, one WG
// Workgroup barrier for data exchanged between waves.  LDS needs only the
// barrier.  For global memory the stores must be complete and visible before
// other waves read them: __syncthreads() alone emits no wait for outstanding
// global stores on gfx950, so an agent-scope fence is added.
template <bool LDS>
NLSP_DEV void wg_sync() {
  if (!LDS) __threadfence();
  __syncthreads();
}

// Cyclic Jacobi eigensolver for a symmetric m x m matrix (Golub & Van Loan,
// Sec. 8.5), parallel ("round-robin") ordering: m/2 disjoint rotations per
// round, m-1 rounds per sweep.  A round forms its rotations from the current
// 2 x 2 diagonal blocks and applies G <- J^T G J as one pass over the 2 x 2
// blocks (rows of pair a, columns of pair b: J_b on the columns, then J_a on
// the rows), so each element is read and written once per round.  The
// rotations (c, s per pair, pairs in the order of the round-robin formula)
// are recorded in `rot` for k_jacobi_vecs; nsweeps[0] receives the number of
// sweeps recorded.  The working copy of G lives in LDS when LDS = true
// (m <= 128), else in Gg itself.  On exit Gg holds the rotated matrix (its
// diagonal converges to the eigenvalues).  m even.
NLSP_DEV void rr_pair(int rnd, int t, int m, int& p, int& q) {
  if (t == 0) {
    p = rnd;
    q = m - 1;
  } else {
    p = (rnd + t) % (m - 1);
    q = (rnd - t + (m - 1)) % (m - 1);
  }
  if (p > q) {
    const int tmp = p;
    p = q;
    q = tmp;
  }
}

// The rotation (c, s) that annihilates a_pq of the 2 x 2 block [a_pp a_pq;
// a_pq a_qq] (Golub & Van Loan, the symmetric Schur decomposition: the
// smaller root of t^2 + 2 tau t - 1 = 0, tau = (a_qq - a_pp) / (2 a_pq)).
NLSP_DEV void jacobi_rotation(double app, double aqq, double apq, double& c, double& s) {
  c = 1.0;
  s = 0.0;
  if (apq != 0.0 && fabs(apq) > 1e-300) {
    const double tau = (aqq - app) / (2.0 * apq);
    const double tt = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
    c = 1.0 / sqrt(1.0 + tt * tt);
    s = tt * c;
  }
}

// The 2 x 2 block of G at rows (pa, qa) and columns (pb, qb) after
// J_a^T (block) J_b: the column rotation (cb, sb), then the row rotation
// (ca, sa).
NLSP_DEV void rotate_block(double ca, double sa, double cb, double sb, double g11, double g12, double g21,
                           double g22, double& o11, double& o12, double& o21, double& o22) {
  const double h11 = cb * g11 - sb * g12, h12 = sb * g11 + cb * g12;   // columns: J_b
  const double h21 = cb * g21 - sb * g22, h22 = sb * g21 + cb * g22;
  o11 = ca * h11 - sa * h21;                                           // rows: J_a
  o21 = sa * h11 + ca * h21;
  o12 = ca * h12 - sa * h22;
  o22 = sa * h12 + ca * h22;
}

template <bool LDS>
__global__ __launch_bounds__(1024) void k_jacobi_eig(double* __restrict__ Gg, int m, int max_sweeps,
                                                     double* __restrict__ rot, int* __restrict__ nsweeps,
                                                     double* __restrict__ offnorm) {
  extern __shared__ double dyn[];
  __shared__ double cs[128], sn[128];
  __shared__ int pp[128], qq[128];
  __shared__ double red[16];
  const int t = threadIdx.x, nt = blockDim.x;
  double* G = LDS ? dyn : Gg;
  if (LDS)
    for (int idx = t; idx < m * m; idx += nt) G[idx] = Gg[idx];
  wg_sync<LDS>();
  const int half = m / 2;
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int idx = t; idx < m * m; idx += nt) {
      const double g = G[idx];
      tot += g * g;
      if (idx / m != idx % m) off += g * g;
    }
    off = block_sum(off, red);
    __syncthreads();
    tot = block_sum(tot, red);
    if (t == 0) offnorm[0] = sqrt(off / (tot > 0 ? tot : 1.0));
    if (off <= 1e-30 * tot) break;
    double* rs = rot + (int64_t)sweep * (m - 1) * half * 2;
    for (int rnd = 0; rnd < m - 1; ++rnd) {
      if (t < half) {
        int p, q;
        rr_pair(rnd, t, m, p, q);
        double c, s;
        jacobi_rotation(G[p * m + p], G[q * m + q], G[p * m + q], c, s);
        cs[t] = c;
        sn[t] = s;
        pp[t] = p;
        qq[t] = q;
        rs[((int64_t)rnd * half + t) * 2] = c;
        rs[((int64_t)rnd * half + t) * 2 + 1] = s;
      }
      __syncthreads();
      // the launch has a multiple of m/2 threads, so this thread's column
      // pair b is the same for every block it updates: its indices and
      // rotation are read once per round; row pairs a are wave-uniform
      const int b = t % half;
      const int pb = pp[b], qb = qq[b];
      const double cb = cs[b], sb = sn[b];
      for (int a = t / half; a < half; a += nt / half) {
        const int pa = pp[a], qa = qq[a];
        const double ca = cs[a], sa = sn[a];
        const double g11 = G[pa * m + pb], g12 = G[pa * m + qb], g21 = G[qa * m + pb], g22 = G[qa * m + qb];
        rotate_block(ca, sa, cb, sb, g11, g12, g21, g22, G[pa * m + pb], G[pa * m + qb], G[qa * m + pb],
                     G[qa * m + qb]);
      }
      wg_sync<LDS>();
    }
  }
  if (t == 0) nsweeps[0] = sweep;
  if (LDS)
    for (int idx = t; idx < m * m; idx += nt) Gg[idx] = G[idx];
}

// Multi-workgroup form for m > 128, where G does not fit in LDS: one launch
// per round, G_out = J^T G_in J between two buffers, one thread per 2 x 2
// block forming the two rotations it needs from G_in; k_jacobi_check opens
// each sweep.
// Same rotations, same block arithmetic and same stopping rule as
// k_jacobi_eig.  ctl: [sweeps recorded, converged].
constexpr int JR_THREADS = 256;
__global__ __launch_bounds__(1024) void k_jacobi_check(const double* __restrict__ G, int m, int sweep,
                                                       int* __restrict__ ctl, double* __restrict__ offnorm) {
  __shared__ double red[16];
  const int t = threadIdx.x;
  double off = 0.0, tot = 0.0;
  for (int idx = t; idx < m * m; idx += blockDim.x) {
    const double g = G[idx];
    tot += g * g;
    if (idx / m != idx % m) off += g * g;
  }
  off = block_sum(off, red);
  __syncthreads();
  tot = block_sum(tot, red);
  if (t == 0) {
    offnorm[0] = sqrt(off / (tot > 0 ? tot : 1.0));
    const int conv = off <= 1e-30 * tot;
    ctl[0] = conv ? sweep : sweep + 1;
    ctl[1] = conv;
  }
}

__global__ __launch_bounds__(JR_THREADS) void k_jacobi_round(const double* __restrict__ Gin,
                                                             double* __restrict__ Gout, int m, int rnd,
                                                             double* __restrict__ rs) {
  // each thread forms the two rotations its block needs itself (the pair
  // indices follow from the round), so every load of the round is issued at
  // once and no barrier is needed; workgroup 0 records the rotations
  const int half = m / 2;
  const int g = blockIdx.x * JR_THREADS + threadIdx.x;
  if (g >= half * half) return;
  const int a = g / half, b = g - a * half;
  int pa, qa, pb, qb;
  rr_pair(rnd, a, m, pa, qa);
  rr_pair(rnd, b, m, pb, qb);
  const double g11 = Gin[pa * m + pb], g12 = Gin[pa * m + qb], g21 = Gin[qa * m + pb], g22 = Gin[qa * m + qb];
  const double apa = Gin[pa * m + pa], aqa = Gin[qa * m + qa], apqa = Gin[pa * m + qa];
  const double apb = Gin[pb * m + pb], aqb = Gin[qb * m + qb], apqb = Gin[pb * m + qb];
  double ca, sa, cb, sb;
  jacobi_rotation(apa, aqa, apqa, ca, sa);
  jacobi_rotation(apb, aqb, apqb, cb, sb);
  if (g < half) {   // a = 0: thread b records rotation b
    rs[((int64_t)rnd * half + b) * 2] = cb;
    rs[((int64_t)rnd * half + b) * 2 + 1] = sb;
  }
  rotate_block(ca, sa, cb, sb, g11, g12, g21, g22, Gout[pa * m + pb], Gout[pa * m + qb], Gout[qa * m + pb],
               Gout[qa * m + qb]);
}

// V = J_1 J_2 ... from the recorded rotations.  Each row of V evolves on its
// own (row_i <- row_i J), so one wave keeps one row in LDS and applies every
// round's disjoint rotations, one pair per lane, in the recorded order.  The
// rotations are staged in LDS in chunks of JV_PAIRS pairs (whole rounds),
// loaded by the whole workgroup with 16-byte loads one chunk ahead; a lane's
// pair indices follow the round-robin formula incrementally (both move up by
// one per round, modulo m - 1).
constexpr int JV_PAIRS = 1024;              // pairs per staged chunk
constexpr int JV_CPT = JV_PAIRS / 256;      // (c, s) pairs per thread and chunk
__global__ __launch_bounds__(256) void k_jacobi_vecs(const double* __restrict__ rot,
                                                     const int* __restrict__ nsweeps, int m,
                                                     double* __restrict__ V) {
  extern __shared__ double vsh[];   // 4 rows of m, then two chunks of 2 JV_PAIRS
  const int t = threadIdx.x, w = t / 64, lane = t % 64;
  const int i = blockIdx.x * 4 + w;   // m is a multiple of 4
  double* row = vsh + w * m;
  double* cbuf[2] = {vsh + 4 * m, vsh + 4 * m + 2 * JV_PAIRS};
  const int half = m / 2, mm = m - 1;
  const int rpc = JV_PAIRS / half;    // whole rounds per chunk
  const int cpairs = rpc * half;      // pairs per chunk (<= JV_PAIRS)
  for (int j = lane; j < m; j += 64) row[j] = (j == i) ? 1.0 : 0.0;
  const int64_t nr = (int64_t)nsweeps[0] * mm;   // rounds recorded, in order
  const int64_t nch = (nr + rpc - 1) / rpc;
  const int64_t npairs = nr * half;
  const double2* rot2 = reinterpret_cast<const double2*>(rot);
  double2 reg[JV_CPT];
  auto fetch = [&](int64_t c) {
#pragma unroll
    for (int u = 0; u < JV_CPT; ++u) {
      const int64_t g = c * cpairs + min(t + u * 256, cpairs - 1);
      reg[u] = rot2[min(g, npairs - 1)];
    }
  };
  auto stage = [&](double* buf) {
#pragma unroll
    for (int u = 0; u < JV_CPT; ++u) {
      if (t + u * 256 < cpairs) {
        buf[2 * (t + u * 256)] = reg[u].x;
        buf[2 * (t + u * 256) + 1] = reg[u].y;
      }
    }
  };
  // round-robin state of this lane's pairs k = lane, lane + 64 at round 0
  int pr[2], qr[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int k = lane + 64 * u;
    pr[u] = k == 0 ? 0 : k % mm;
    qr[u] = k == 0 ? mm : (mm - k) % mm;
  }
  if (nch > 0) {
    fetch(0);
    stage(cbuf[0]);
  }
  __syncthreads();
  if (nch > 1) fetch(1);
  for (int64_t c = 0; c < nch; ++c) {
    const double* cur = cbuf[c & 1];
    const int nrc = (int)min<int64_t>(rpc, nr - c * rpc);
    for (int rl = 0; rl < nrc; ++rl) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int k = lane + 64 * u;
        if (k < half) {
          const int p = min(pr[u], qr[u]), q = max(pr[u], qr[u]);
          const double cc = cur[2 * (rl * half + k)], ss = cur[2 * (rl * half + k) + 1];
          const double vp = row[p], vq = row[q];
          row[p] = cc * vp - ss * vq;
          row[q] = ss * vp + cc * vq;
        }
        // next round: both indices move up by one modulo m - 1 (pair 0 keeps q = m - 1)
        pr[u] = pr[u] + 1 == mm ? 0 : pr[u] + 1;
        if (k != 0) qr[u] = qr[u] + 1 == mm ? 0 : qr[u] + 1;
      }
      __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();   // every wave is done with the buffer the next stage overwrites
    if (c + 1 < nch) stage(cbuf[(c + 1) & 1]);
    __syncthreads();
    if (c + 2 < nch) fetch(c + 2);
  }
  for (int j = lane; j < m; j += 64) V[(int64_t)i * m + j] = row[j];
}

// Sort eigenpairs descending; sigma = sqrt(max(lambda, 0)); T = V_k diag(lambda_k^-1/2)
// (m x k, padded columns zero; with `unscaled`, T = V_k); info[0] = 1 if
// lambda_k <= (1e-6 sigma_1)^2.
// The Gram route resolves singular values only down to about sqrt(eps) sigma_1
// (the eigenvalues of G = S^T S carry rounding of order m eps lambda_1), so a
// sigma_k below 1e-6 sigma_1 cannot be told apart from zero: S is then
// numerically of rank < k and P_0 = S V_k / sigma_k would amplify noise.
__global__ __launch_bounds__(256) void k_eig_finish(const double* __restrict__ G,
                                                    const double* __restrict__ V, int m, int mreal,
                                                    int k, int kpad, double* __restrict__ sigma,
                                                    double* __restrict__ T, int* info, int unscaled) {
  __shared__ int order[256];
  __shared__ double lam[256];
  const int t = threadIdx.x;
  for (int i = t; i < m; i += blockDim.x) lam[i] = G[i * m + i];
  __syncthreads();
  // descending order, ties by lower index: the rank of i counts the entries
  // that precede it
  for (int i = t; i < m; i += blockDim.x) {
    const double li = lam[i];
    int r = 0;
    for (int j = 0; j < m; ++j) {
      const double lj = lam[j];
      r += (lj > li || (lj == li && j < i)) ? 1 : 0;
    }
    order[r] = i;
  }
  __syncthreads();
  if (t == 0) {
    const double l1 = lam[order[0]] > 0 ? lam[order[0]] : 0.0;
    const double lk = lam[order[k - 1]];
    info[0] = (lk <= 1e-12 * l1 || !(lk > 0)) ? 1 : 0;
  }
  for (int i = t; i < mreal; i += blockDim.x) {
    const double l = lam[order[i]];
    sigma[i] = sqrt(l > 0 ? l : 0.0);
  }
  for (int idx = t; idx < m * kpad; idx += blockDim.x) {
    const int r = idx / kpad, j = idx % kpad;
    double v = 0.0;
    if (j < k) {
      const double l = lam[order[j]];
      v = unscaled ? V[r * m + order[j]] : ((l > 0) ? V[r * m + order[j]] / sqrt(l) : 0.0);
    }
    T[idx] = v;
  }
}

// Cholesky G = L L^T of an SPD k x k matrix (right-looking, one workgroup);
// L lower (upper part zero).  Working copy in LDS when LDS = true (k <= 128).
// info[0] = 1 if a pivot is not above rtol times its original diagonal entry
// (rtol = 0: not positive; for a Gram matrix X^T X, rtol > 0 flags a column
// of X that is numerically a combination of the earlier ones).
template <bool LDS>
__global__ __launch_bounds__(1024) void k_cholesky(const double* __restrict__ G, int ldg, int k,
                                                   double* __restrict__ Lg, int ldl, int* info, double rtol) {
  extern __shared__ double dyn[];
  __shared__ double piv;
  __shared__ int bad;
  const int t = threadIdx.x, nt = blockDim.x;
  double* L = LDS ? dyn : Lg;
  const int ld = LDS ? k : ldl;
  for (int idx = t; idx < k * k; idx += nt) {
    const int i = idx / k, j = idx % k;
    L[i * ld + j] = (j <= i) ? G[i * ldg + j] : 0.0;
  }
  if (t == 0) bad = 0;
  wg_sync<LDS>();
  for (int j = 0; j < k; ++j) {
    if (t == 0) {
      const double d = L[j * ld + j];
      if (!(d > 0.0) || !(d > rtol * G[j * ldg + j])) bad = 1;
      piv = (d > 0.0) ? sqrt(d) : 1.0;
      L[j * ld + j] = piv;
    }
    wg_sync<LDS>();
    for (int i = j + 1 + t; i < k; i += nt) L[i * ld + j] /= piv;
    wg_sync<LDS>();
    const int rem = k - j - 1;
    for (int idx = t; idx < rem * rem; idx += nt) {
      const int i = j + 1 + idx / rem, c = j + 1 + idx % rem;
      if (c <= i) L[i * ld + c] -= L[i * ld + j] * L[c * ld + j];
    }
    wg_sync<LDS>();
  }
  if (LDS)
    for (int idx = t; idx < k * k; idx += nt) Lg[(idx / k) * ldl + idx % k] = L[idx];
  if (t == 0) info[0] = bad;
}

// Inverse of a lower-triangular k x k matrix, 64 < k <= 128, row by row:
// row i of L^-1 is (e_i - L[i][0:i] L^-1[0:i][:]) / L[i][i].  L and the rows
// of L^-1 computed so far sit in LDS as packed lower triangles (2 x 66 KB at
// k = 128); 8 lanes share an entry's sum (strided over c, then a butterfly),
// one barrier per row.  Written zero-padded to (kp, kp).
constexpr int TRI_ROWS_MAX = 128;
inline size_t tri_rows_lds(int k) { return sizeof(double) * (size_t)k * (k + 1); }
__global__ __launch_bounds__(1024) void k_tri_inv_rows(const double* __restrict__ L, int ldl, int k,
                                                       double* __restrict__ Li, int kp) {
  extern __shared__ double tri[];
  const int tk = k * (k + 1) / 2;
  double* Lp = tri;          // L[i][c] at i (i + 1) / 2 + c
  double* Xp = tri + tk;     // (L^-1)[i][c] likewise
  const int t = threadIdx.x, j = t >> 3, p = t & 7;
  for (int e = t; e < tk; e += 1024) {
    int i = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
    while (i * (i + 1) / 2 > e) --i;
    while ((i + 1) * (i + 2) / 2 <= e) ++i;
    Lp[e] = L[(int64_t)i * ldl + (e - i * (i + 1) / 2)];
  }
  __syncthreads();
  for (int i = 0; i < k; ++i) {
    const double* Li_row = Lp + i * (i + 1) / 2;
    double s = 0.0;
    if (j < i)
      for (int c = j + p; c < i; c += 8) s += Li_row[c] * Xp[c * (c + 1) / 2 + j];
    s += __shfl_xor(s, 1, 8);
    s += __shfl_xor(s, 2, 8);
    s += __shfl_xor(s, 4, 8);
    if (p == 0 && j <= i) Xp[i * (i + 1) / 2 + j] = ((j == i ? 1.0 : 0.0) - s) / Li_row[i];
    __syncthreads();
  }
  for (int e = t; e < kp * kp; e += 1024) {
    const int r = e / kp, c = e % kp;
    Li[e] = (r < k && c <= r) ? Xp[r * (r + 1) / 2 + c] : 0.0;
  }
}

// Inverse of a lower-triangular k x k matrix L, written zero-padded to
// (kp, kp): column j of L^-1 solves L x = e_j by forward substitution.
__global__ __launch_bounds__(256) void k_tri_inv_lower(const double* __restrict__ L, int ldl, int k,
                                                       double* __restrict__ Li, int kp) {
  // thread j forms column j of L^-1 by forward substitution; for kp <= 64 the
  // columns and L itself sit in LDS (no round trip through memory per row)
  __shared__ double Ls[64 * 65];
  __shared__ double X[64 * 65];
  const int t = threadIdx.x;
  if (kp <= 64) {
    for (int e = t; e < kp * kp; e += blockDim.x) {
      const int i = e / kp, c = e % kp;
      Ls[i * 65 + c] = (i < k && c < k) ? L[i * ldl + c] : 0.0;
    }
    __syncthreads();
    const int j = t;
    if (j < kp) {
      for (int i = 0; i < kp; ++i) X[i * 65 + j] = 0.0;
      if (j < k)
        for (int i = j; i < k; ++i) {
          double s = (i == j) ? 1.0 : 0.0;
          for (int c = j; c < i; ++c) s -= Ls[i * 65 + c] * X[c * 65 + j];
          X[i * 65 + j] = s / Ls[i * 65 + i];
        }
    }
    __syncthreads();
    for (int e = t; e < kp * kp; e += blockDim.x) Li[e] = X[(e / kp) * 65 + e % kp];
    return;
  }
  const int j = blockIdx.x * blockDim.x + t;
  if (j >= kp) return;
  for (int i = 0; i < kp; ++i) Li[i * kp + j] = 0.0;
  if (j >= k) return;
  for (int i = j; i < k; ++i) {
    double s = (i == j) ? 1.0 : 0.0;
    for (int c = j; c < i; ++c) s -= L[i * ldl + c] * Li[c * kp + j];
    Li[i * kp + j] = s / L[i * ldl + i];
  }
}

// C (n, b) = X (n, a) * B (a, b) in float64 for a b beyond what one LDS copy
// of B holds (the setup's S V with a = m, CholeskyQR2's X R^-1 with a = k):
// the columns of B are split into slices of BC = 16 JW columns, and a
// persistent workgroup (one per CU) keeps its slice in LDS, rows padded by 4
// doubles so the four 4-row groups that one MFMA reads fall on different
// banks, then walks blocks of 128 rows, one 16-row tile per wave.  The
// workgroups of the slices of the same row blocks are consecutive logical
// blocks (xcd_remap), so they run on one XCD and the repeated reads of X hit
// its L2.  v_mfma_f64_16x16x4f64: a lane loads 4 consecutive k of its row
// (16 or 32 bytes) and feeds 4 products with them, the k index permuted the
// same way for B (MFMA u takes k = k0 + 4 (lane / 16) + u); the next 16 k of
// X are loaded before the products of the current ones.  a multiple of 16.
constexpr int TSW_NT = 512, TSW_ROWS = 128;
constexpr int TSW_LDS = 18432;   // doubles of the B slice in LDS (144 KB)

template <typename T>
NLSP_DEV void ld4(const T* p, T (&v)[4]) {
  if constexpr (sizeof(T) == 4) {
    const float4 x = *reinterpret_cast<const float4*>(p);
    v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
  } else {
    const double2 x = reinterpret_cast<const double2*>(p)[0], y = reinterpret_cast<const double2*>(p)[1];
    v[0] = x.x; v[1] = x.y; v[2] = y.x; v[3] = y.y;
  }
}

template <typename T, int JW>
__global__ __launch_bounds__(TSW_NT) void k_tsgemm_wide(const T* __restrict__ X, int64_t n, int a,
                                                        const double* __restrict__ B, int b, int nsplit,
                                                        double* __restrict__ C, int ldc, int bcols_out) {
  extern __shared__ double bsl[];   // a rows of LDB
  constexpr int BC = 16 * JW, LDB = BC + 4;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int slice = lb % nsplit, ngrp = gridDim.x / nsplit;
  const int grp = lb / nsplit, c0 = slice * BC;
  if (grp >= ngrp) return;   // a remainder block (uniform)
  for (int idx = threadIdx.x; idx < a * BC; idx += TSW_NT) {
    const int r = idx / BC, cc = idx - r * BC;
    bsl[r * LDB + cc] = B[(int64_t)r * b + c0 + cc];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
  const int64_t nblk = (n + TSW_ROWS - 1) / TSW_ROWS;
  for (int64_t blk = grp; blk < nblk; blk += ngrp) {
    const int64_t r0 = blk * TSW_ROWS + 16 * w;
    const T* xr = X + min(r0 + li, n - 1) * a + 4 * lk;   // rows past n: a clamped row, not stored
    d4_t acc[JW];
#pragma unroll
    for (int q = 0; q < JW; ++q) acc[q] = d4_t{0.0, 0.0, 0.0, 0.0};
    T xv[4], xn[4];
    ld4<T>(xr, xv);
    for (int k0 = 0; k0 < a; k0 += 16) {
      ld4<T>(xr + min(k0 + 16, a - 16), xn);
      const double* br = bsl + (k0 + 4 * lk) * LDB + li;
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int q = 0; q < JW; ++q)
          acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)xv[u], br[u * LDB + 16 * q], acc[q], 0, 0, 0);
#pragma unroll
      for (int u = 0; u < 4; ++u) xv[u] = xn[u];
    }
#pragma unroll
    for (int q = 0; q < JW; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = r0 + 4 * v + lk;   // float64 MFMA output row order
        const int col = c0 + 16 * q + li;
        if (row < n && col < bcols_out) C[row * ldc + col] = acc[q][v];
      }
  }
}

// The same product with B staged in LDS once per workgroup (a b <= 8192):
// the waves of a workgroup walk the 16-row tiles tile0 + w, tile0 + w + W, ...
// (W = waves in the grid), so B is read from HBM once per workgroup instead
// of once per MFMA.  Same operand layout and summation order as k_tsgemm.
constexpr int TSG_LDS = 8192;   // doubles of B in LDS
template <typename T, int MAXJ>
__global__ __launch_bounds__(256) void k_tsgemm_lds(const T* __restrict__ X, int64_t n, int a,
                                                    const double* __restrict__ B, int b,
                                                    double* __restrict__ C, int ldc, int bcols_out) {
  __shared__ double bs[TSG_LDS];
  for (int idx = threadIdx.x; idx < a * b; idx += blockDim.x) bs[idx] = B[idx];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int TB = b / 16;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t tiles = (n + 15) / 16;
  const int64_t step = (int64_t)gridDim.x * (blockDim.x / 64);
  for (int64_t tile = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64; tile < tiles; tile += step) {
    const int64_t r0 = tile * 16;
    d4_t acc[MAXJ];
#pragma unroll
    for (int q = 0; q < MAXJ; ++q) acc[q] = d4_t{0.0, 0.0, 0.0, 0.0};
    const int64_t ra = r0 + li;
#pragma unroll 8
    for (int k0 = 0; k0 < a; k0 += 4) {
      const double av = (ra < n) ? (double)X[ra * a + k0 + lk] : 0.0;
      const double* br = bs + (k0 + lk) * b + li;
#pragma unroll
      for (int q = 0; q < MAXJ; ++q) {
        if (q < TB) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, br[16 * q], acc[q], 0, 0, 0);
      }
    }
#pragma unroll
    for (int q = 0; q < MAXJ; ++q) {
      if (q < TB) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t row = r0 + 4 * v + lk;   // float64 MFMA output row order
          const int col = 16 * q + li;
          if (row < n && col < bcols_out) C[row * ldc + col] = acc[q][v];
        }
      }
    }
  }
}

// Inverse of the upper-triangular R = L^T given L lower: Ri = L^-T, (kp x kp)
// zero padded; reuses the lower inverse: (L^T)^-1 = (L^-1)^T.
__global__ void k_transpose_pad(const double* __restrict__ A, int kp, double* __restrict__ B) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= kp * kp) return;
  const int i = idx / kp, j = idx % kp;
  B[j * kp + i] = A[idx];
}

// Largest-magnitude entry of each column (lowest row on ties), in two
// passes: every workgroup scans a row range of the whole (n, ld) block with
// coalesced loads (lane t takes column t % ld) and keeps, per column, the
// first maximum of |P|; k_colsign_finish combines the workgroups in order and
// stores the column signs, which k_copy_cols_signed applies.
constexpr int CS_BLOCKS = 1024;

__global__ __launch_bounds__(256) void k_colmax_partial(const double* __restrict__ P, int64_t n, int ld,
                                                        int64_t rows_per, double* __restrict__ pv,
                                                        int64_t* __restrict__ pi) {
  __shared__ double bv[256];
  __shared__ int64_t bi[256];
  const int t = threadIdx.x;
  const int per = 256 / ld;                // rows per pass (ld <= 256, a power of two)
  const int c = t % ld, r = t / ld;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per, r1 = min(n, r0 + rows_per);
  double best = -1.0;
  int64_t bidx = r0;
  if (r < per) {
    // rows in increasing order, eight loads issued before the first compare
    int64_t i = r0 + r;
    for (; i + 7 * per < r1; i += 8 * per) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = fabs(P[(i + u * per) * ld + c]);
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (v[u] > best) {
          best = v[u];
          bidx = i + u * per;
        }
    }
    for (; i < r1; i += per) {
      const double v = fabs(P[i * ld + c]);
      if (v > best) {
        best = v;
        bidx = i;
      }
    }
  }
  bv[t] = best;
  bi[t] = bidx;
  __syncthreads();
  // combine the `per` threads of each column (rows r, r + per, ... interleave,
  // so ties go to the lower row index)
  if (t < ld) {
    double b = bv[t];
    int64_t bx = bi[t];
    for (int q = 1; q < per; ++q) {
      const double v = bv[q * ld + t];
      const int64_t x = bi[q * ld + t];
      if (v > b || (v == b && x < bx)) {
        b = v;
        bx = x;
      }
    }
    pv[(int64_t)blockIdx.x * ld + t] = b;
    pi[(int64_t)blockIdx.x * ld + t] = bx;
  }
}

__global__ __launch_bounds__(256) void k_colsign_finish(const double* __restrict__ P, int ld, int k, int nblk,
                                                        const double* __restrict__ pv,
                                                        const int64_t* __restrict__ pi,
                                                        double* __restrict__ sign) {
  const int c = threadIdx.x;
  if (c >= k) return;
  double b = -1.0;
  int64_t bx = 0;
  // partials in workgroup order, sixteen loaded before the first compare
  int w = 0;
  for (; w + 16 <= nblk; w += 16) {
    double v[16];
    int64_t x[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      v[u] = pv[(int64_t)(w + u) * ld + c];
      x[u] = pi[(int64_t)(w + u) * ld + c];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (v[u] > b || (v[u] == b && x[u] < bx)) {
        b = v[u];
        bx = x[u];
      }
  }
  for (; w < nblk; ++w) {
    const double v = pv[(int64_t)w * ld + c];
    const int64_t x = pi[(int64_t)w * ld + c];
    if (v > b || (v == b && x < bx)) {
      b = v;
      bx = x;
    }
  }
  sign[c] = (P[bx * ld + c] < 0.0) ? -1.0 : 1.0;
}

// Copy (n, k) with leading dimension lda into (n, kout) row-major, column j
// multiplied by sign[j].
__global__ void k_copy_cols_signed(const double* __restrict__ A, int lda, int64_t n, int k,
                                   const double* __restrict__ sign, double* __restrict__ B, int ldb) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * k) return;
  const int64_t i = idx / k;
  const int j = (int)(idx % k);
  B[i * ldb + j] = sign[j] * A[i * lda + j];
}

// Copy (n, k) with leading dimension lda into (n, kout) row-major.
__global__ void k_copy_cols(const double* __restrict__ A, int lda, int64_t n, int k,
                            double* __restrict__ B, int ldb) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * ldb) return;
  const int64_t i = idx / ldb;
  const int j = (int)(idx % ldb);
  B[idx] = (j < k) ? A[i * lda + j] : 0.0;
}

__global__ void k_pad_square(const double* __restrict__ A, int lda, int k, double* __restrict__ B,
                             int ldb, int kout) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= kout * kout) return;
  const int i = idx / kout, j = idx % kout;
  B[i * ldb + j] = (i < k && j < k) ? A[i * lda + j] : 0.0;
}

__global__ void k_to_f32(const double* __restrict__ A, float* __restrict__ B, int64_t cnt) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < cnt) B[idx] = (float)A[idx];
}

// ------------------------------------------------------------ host helpers
constexpr int LDS_DENSE_MAX = 128;   // m or k up to which the dense kernels work in LDS

constexpr int JACOBI_MAX_SWEEPS = 40;

inline size_t rot_doubles(int m) { return (size_t)JACOBI_MAX_SWEEPS * (m - 1) * (m / 2) * 2; }

// threads of the eigensolver: the largest multiple of lcm(m/2, 64) up to
// 1024 (whole waves, and a fixed column pair per thread)
inline int eig_threads(int m) {
  const int h = m / 2;
  int g = h, r = 64;
  while (r) { const int tmp = g % r; g = r; r = tmp; }
  const int l = h / g * 64;
  return (1024 / l) * l;
}

// Eigenpairs of the symmetric m x m matrix G: on return G holds the rotated
// matrix and V the accumulated rotations.  G2 (m x m doubles) is scratch for
// m > 128, whose rounds run as separate launches; there the host reads the
// convergence flag after each sweep (one stream synchronisation per sweep).
static int launch_eig(double* G, double* G2, double* V, int m, double* rot, int* nsweeps, double* off,
                      hipStream_t s) {
  // m is padded to a multiple of 16
  if (m < 16 || m % 16 != 0 || m > 256 || eig_threads(m) < 64) return NLSP_E_INVALID;
  if (m <= LDS_DENSE_MAX) {
    const size_t sh = sizeof(double) * m * m;
    NLSP_HIP(hipFuncSetAttribute((const void*)k_jacobi_eig<true>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh));
    hipLaunchKernelGGL(k_jacobi_eig<true>, dim3(1), dim3(eig_threads(m)), sh, s, G, m, JACOBI_MAX_SWEEPS, rot,
                       nsweeps, off);
  } else {
    // m - 1 rounds per sweep (odd), so the current matrix alternates between
    // the buffers from sweep to sweep
    const int half = m / 2, nwg = ceil_div(half * half, JR_THREADS);
    double* buf[2] = {G, G2};
    int sweep = 0;
    for (; sweep < JACOBI_MAX_SWEEPS; ++sweep) {
      const double* cur = buf[sweep & 1];
      hipLaunchKernelGGL(k_jacobi_check, dim3(1), dim3(1024), 0, s, cur, m, sweep, nsweeps, off);
      int ctl[2] = {0, 0};
      NLSP_HIP(hipMemcpyAsync(ctl, nsweeps, sizeof(ctl), hipMemcpyDeviceToHost, s));
      NLSP_HIP(hipStreamSynchronize(s));
      if (ctl[1]) break;
      double* rs = rot + (size_t)sweep * (m - 1) * half * 2;
      for (int rnd = 0; rnd < m - 1; ++rnd)
        hipLaunchKernelGGL(k_jacobi_round, dim3(nwg), dim3(JR_THREADS), 0, s, buf[(sweep + rnd) & 1],
                           buf[(sweep + rnd + 1) & 1], m, rnd, rs);
      NLSP_HIP(hipGetLastError());
    }
    if (sweep & 1) NLSP_HIP(hipMemcpyAsync(G, G2, sizeof(double) * m * m, hipMemcpyDeviceToDevice, s));
  }
  hipLaunchKernelGGL(k_jacobi_vecs, dim3(m / 4), dim3(256), sizeof(double) * (4 * m + 4 * JV_PAIRS), s, rot, nsweeps,
                     m, V);
  NLSP_HIP(hipGetLastError());
  return NLSP_OK;
}

// L^-1 (zero-padded to kp x kp) of the lower-triangular k x k matrix L
static int launch_tri_inv(const double* L, int ldl, int k, double* Li, int kp, hipStream_t s) {
  if (k > 64 && k <= TRI_ROWS_MAX) {
    NLSP_HIP(hipFuncSetAttribute((const void*)k_tri_inv_rows, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)tri_rows_lds(TRI_ROWS_MAX)));
    hipLaunchKernelGGL(k_tri_inv_rows, dim3(1), dim3(1024), tri_rows_lds(k), s, L, ldl, k, Li, kp);
  } else {
    hipLaunchKernelGGL(k_tri_inv_lower, dim3(1), dim3(256), 0, s, L, ldl, k, Li, kp);
  }
  NLSP_HIP(hipGetLastError());
  return NLSP_OK;
}

static int launch_chol(const double* G, int ldg, int k, double* L, int ldl, int* info,
                       hipStream_t s, double rtol = 0.0) {
  if (k <= LDS_DENSE_MAX) {
    const size_t sh = sizeof(double) * k * k;
    NLSP_HIP(hipFuncSetAttribute((const void*)k_cholesky<true>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh));
    hipLaunchKernelGGL(k_cholesky<true>, dim3(1), dim3(1024), sh, s, G, ldg, k, L, ldl, info, rtol);
  } else {
    hipLaunchKernelGGL(k_cholesky<false>, dim3(1), dim3(1024), 0, s, G, ldg, k, L, ldl, info, rtol);
  }
  NLSP_HIP(hipGetLastError());
  return NLSP_OK;
}
struct GramPlan {
  int nwg;
  int64_t rows_per_wg;
};

inline GramPlan gram_plan(int64_t n) {
  GramPlan g;
  g.nwg = (int)std::max<int64_t>(1, std::min<int64_t>(512, (n + 255) / 256));
  g.rows_per_wg = ((n + g.nwg - 1) / g.nwg + 3) / 4 * 4;
  g.nwg = (int)((n + g.rows_per_wg - 1) / g.rows_per_wg);
  return g;
}

// X^T Y (a x b, a, b multiples of 16) into out (leading dim ldo).  `part`
// holds nwg*a*b doubles.  sym = 1: Y = X; sym = 2: a product known to be
// symmetric (X^T A X as P^T (A P)); both form the upper triangle of 16 x 16
// tiles and mirror it.
template <typename T>
static int gram(const T* X, const T* Y, int64_t n, int a, int b, int sym, double* part,
                double* out, int ldo, hipStream_t s) {
  const GramPlan g = gram_plan(n);
  const int TA = a / 16, TB = b / 16;
  if (sym == 2 && a != b) return NLSP_E_INVALID;
  const int ntiles = sym ? TA * (TA + 1) / 2 : TA * TB;
  // up to 16 waves, tiles dealt round-robin: 3 slots per wave up to 48 tiles, 9 up to 144
  const int vecs = GS_ROWS * (a + (sym == 1 ? 0 : b)) / GsVec<T>::VE;
  const int waves = std::min(16, std::max({1, ntiles, (vecs + 64 * GS_MAXV - 1) / (64 * GS_MAXV)}));
  const int per_wave = (ntiles + waves - 1) / waves;
  if (per_wave > 9) return NLSP_E_INVALID;
  const int threads = 64 * waves;
  if (vecs > GS_MAXV * threads || gs_lds_bytes(a, b, sym) > 65536) return NLSP_E_INVALID;
  if (reinterpret_cast<uintptr_t>(X) % 16 != 0 || reinterpret_cast<uintptr_t>(Y) % 16 != 0) return NLSP_E_INVALID;
  if (per_wave <= 3)
    hipLaunchKernelGGL((k_gram_partial<T, 3>), dim3(g.nwg), dim3(threads), gs_lds_bytes(a, b, sym), s, X, Y, n,
                       a, b, sym, g.rows_per_wg, part);
  else
    hipLaunchKernelGGL((k_gram_partial<T, 9>), dim3(g.nwg), dim3(threads), gs_lds_bytes(a, b, sym), s, X, Y, n,
                       a, b, sym, g.rows_per_wg, part);
  hipLaunchKernelGGL(k_gram_reduce, dim3(ceil_div(a * b, 64)), dim3(GR_NT), 0, s, part, g.nwg, a, b,
                     sym, out, ldo);
  NLSP_HIP(hipGetLastError());
  return NLSP_OK;
}

template <typename T>
static void tsgemm(const T* X, int64_t n, int a, const double* B, int b, double* C, int ldc,
                   int bcols_out, hipStream_t s) {
  const int64_t tiles = (n + 15) / 16;
  if ((int64_t)a * b <= TSG_LDS) {
    // two workgroups per CU (LDS), four 16-row tiles per wave and more
    const unsigned wgs = (unsigned)std::max<int64_t>(1, std::min<int64_t>(512, ceil_div(tiles, 16)));
    if (b <= 64)
      hipLaunchKernelGGL((k_tsgemm_lds<T, 4>), dim3(wgs), dim3(256), 0, s, X, n, a, B, b, C, ldc, bcols_out);
    else if (b <= 128)
      hipLaunchKernelGGL((k_tsgemm_lds<T, 8>), dim3(wgs), dim3(256), 0, s, X, n, a, B, b, C, ldc, bcols_out);
    else
      hipLaunchKernelGGL((k_tsgemm_lds<T, 16>), dim3(wgs), dim3(256), 0, s, X, n, a, B, b, C, ldc, bcols_out);
    return;
  }
  // the widest slice of 16, 32, 64 or 128 columns that divides b and fits in LDS
  int jw = 8;
  while (jw > 1 && (b % (16 * jw) != 0 || (size_t)a * (16 * jw + 4) > (size_t)TSW_LDS)) jw /= 2;
  const int nsplit = b / (16 * jw);
  const size_t sh = sizeof(double) * a * (16 * jw + 4);
  // one workgroup per CU (LDS), a multiple of nsplit; no more row groups than row blocks
  const int64_t nblk = (n + TSW_ROWS - 1) / TSW_ROWS;
  const int ngrp = (int)std::max<int64_t>(1, std::min<int64_t>(256 / nsplit, nblk));
  const unsigned wgs = (unsigned)(ngrp * nsplit);
  auto go = [&](auto kern) {
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    hipLaunchKernelGGL(kern, dim3(wgs), dim3(TSW_NT), sh, s, X, n, a, B, b, nsplit, C, ldc, bcols_out);
  };
  switch (jw) {
    case 8: go(k_tsgemm_wide<T, 8>); break;
    case 4: go(k_tsgemm_wide<T, 4>); break;
    case 2: go(k_tsgemm_wide<T, 2>); break;
    default: go(k_tsgemm_wide<T, 1>);
  }
}

inline int pad16(int v) { return (v + 15) / 16 * 16; }

struct SetupLayout {
  void* S0buf;      // (n, mp) relaxation ping
  void* S1buf;      // (n, mp) relaxation pong
  double* P0;       // (n, kp16)
  double* P1;       // (n, kp16)
  double* part;     // Gram partials
  double* G;        // (mp, mp)
  double* V;        // (mp, mp)
  double* T;        // (mp, kp16)
  double* Rinv;     // (kp16, kp16)
  double* Lk;       // (kp16, kp16)
  double* off;      // 4
  int* info;        // 4
  double* rot;      // Jacobi rotations, rot_doubles(mp)
  int* nsweeps;     // 1
  double* cmax;     // column maxima per workgroup (CS_BLOCKS, kq)
  int64_t* cidx;    // their rows
  double* csign;    // (kq)
  size_t bytes;
};

inline SetupLayout carve_setup(void* ws, int64_t n, int m, int k, int prec) {
  const int mp = pad16(m) + (pad16(m) % 2), kq = pad16(k);
  const size_t es = (prec == NLSP_MIXED) ? 4 : 8;
  Carver cv(ws);
  SetupLayout L;
  L.S0buf = cv.take<char>(n * mp * es);
  L.S1buf = cv.take<char>(n * mp * es);
  L.P0 = cv.take<double>(n * kq);
  L.P1 = cv.take<double>(n * kq);
  const GramPlan g = gram_plan(n);
  L.part = cv.take<double>((size_t)g.nwg * mp * mp);
  L.G = cv.take<double>((size_t)mp * mp);
  L.V = cv.take<double>((size_t)mp * mp);
  L.T = cv.take<double>((size_t)mp * kq);
  L.Rinv = cv.take<double>((size_t)kq * kq);
  L.Lk = cv.take<double>((size_t)kq * kq);
  L.off = cv.take<double>(4);
  L.info = cv.take<int>(4);
  L.rot = cv.take<double>(rot_doubles(mp));
  L.nsweeps = cv.take<int>(4);
  L.cmax = cv.take<double>((size_t)CS_BLOCKS * kq);
  L.cidx = cv.take<int64_t>((size_t)CS_BLOCKS * kq);
  L.csign = cv.take<double>(kq);
  L.bytes = cv.bytes();
  return L;
}

// CholeskyQR2 in float64 of the (rows, cq) matrix in Pa whose columns past kr
// are zero: twice G = X^T X, G = L L^T, X <- X L^-T.  On return Pa holds the
// orthonormal factor (the two buffers are swapped as the passes alternate).
// info[0], info[1]: a Cholesky pivot of pass 1, 2 not above rtol times its
// diagonal entry (see k_cholesky).  Uses the layout's part, G, Lk, T and Rinv
// (sized for cq).
static int cholqr2(double*& Pa, double*& Pb, int64_t rows, int cq, int kr, const SetupLayout& L, int* info,
                   hipStream_t s, double rtol = 0.0) {
  for (int pass = 0; pass < 2; ++pass) {
    int rc = gram<double>(Pa, Pa, rows, cq, cq, 1, L.part, L.G, cq, s);
    if (rc) return rc;
    rc = launch_chol(L.G, cq, kr, L.Lk, cq, info + pass, s, rtol);
    if (rc) return rc;
    rc = launch_tri_inv(L.Lk, cq, kr, L.T, cq, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_transpose_pad, dim3(ceil_div(cq * cq, 256)), dim3(256), 0, s, L.T, cq, L.Rinv);
    tsgemm<double>(Pa, rows, cq, L.Rinv, cq, Pb, cq, cq, s);
    std::swap(Pa, Pb);
  }
  return NLSP_OK;
}

// Pout (n, k) = the first k columns of X (n, ld), each column signed so that
// its entry of largest magnitude is positive (lowest row on ties).
static void signed_columns(const double* X, int64_t n, int ld, int k, const SetupLayout& L, double* Pout,
                           hipStream_t s) {
  const int64_t rows_per = (n + CS_BLOCKS - 1) / CS_BLOCKS;
  const int nblk = (int)((n + rows_per - 1) / rows_per);
  hipLaunchKernelGGL(k_colmax_partial, dim3(nblk), dim3(256), 0, s, X, n, ld, rows_per, L.cmax, L.cidx);
  hipLaunchKernelGGL(k_colsign_finish, dim3(1), dim3(256), 0, s, X, ld, k, nblk, L.cmax, L.cidx, L.csign);
  hipLaunchKernelGGL(k_copy_cols_signed, dim3(ceil_div(n * k, 256)), dim3(256), 0, s, X, ld, n, k, L.csign,
                     Pout, k);
}

// Copies S0 (n, m) float64 into the padded (n, mp) buffer of element type T.
template <typename T>
__global__ void k_load_S0(const double* __restrict__ S0, int64_t n, int m, int mp, T* __restrict__ S) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * mp) return;
  const int64_t i = idx / mp;
  const int j = (int)(idx % mp);
  S[idx] = (T)((j < m) ? S0[i * m + j] : 0.0);
}

template <typename T>
static int setup_impl(const OpDev& op, const double* S0, int m, int k, double omega, int s1,
                      double* Pout, double* sigma, const SetupLayout& L, hipStream_t s) {
  const int64_t n = op.n;
  const int mp = pad16(m) + (pad16(m) % 2), kq = pad16(k);
  T* Sa = static_cast<T*>(L.S0buf);
  T* Sb = static_cast<T*>(L.S1buf);
  // the first sweep reads S0 itself when it needs no padding (float64; the
  // float32 z-march rounds each value as it loads it), else a padded copy
  int it0 = 0;
  if (s1 > 0 && m == mp && reinterpret_cast<uintptr_t>(S0) % 16 == 0) {
    if constexpr (std::is_same<T, double>::value) {
      launch_cols<double>(op, mp, omega, 0, S0, Sb, s);
      it0 = 1;
    } else {
      if (zmarch_cols_relax_f64in(op, omega, mp, S0, Sb, s)) it0 = 1;
    }
    if (it0) std::swap(Sa, Sb);
  }
  if (it0 == 0) hipLaunchKernelGGL(k_load_S0<T>, dim3(ceil_div(n * mp, 256)), dim3(256), 0, s, S0, n, m, mp, Sa);
  for (int it = it0; it < s1; ++it) {
    launch_cols<T>(op, mp, omega, 0, Sa, Sb, s);
    std::swap(Sa, Sb);
  }
  // Gram and eigenpairs
  int rc = gram<T>(Sa, Sa, n, mp, mp, 1, L.part, L.G, mp, s);
  if (rc) return rc;
  rc = launch_eig(L.G, L.part, L.V, mp, L.rot, L.nsweeps, L.off, s);
  if (rc) return rc;
  hipLaunchKernelGGL(k_eig_finish, dim3(1), dim3(256), 0, s, L.G, L.V, mp, m, k, kq, sigma, L.T,
                     L.info, 0);
  // P0 = S T
  tsgemm<T>(Sa, n, mp, L.T, kq, L.P0, kq, kq, s);
  // CholeskyQR2 in float64
  double* Pa = L.P0;
  double* Pb = L.P1;
  rc = cholqr2(Pa, Pb, n, kq, k, L, L.info + 1, s);
  if (rc) return rc;
  signed_columns(Pa, n, kq, k, L, Pout, s);
  NLSP_HIP(hipGetLastError());
  int hinfo[4] = {0, 0, 0, 0};
  NLSP_HIP(hipMemcpyAsync(hinfo, L.info, sizeof(hinfo), hipMemcpyDeviceToHost, s));
  NLSP_HIP(hipStreamSynchronize(s));
  if (hinfo[1] || hinfo[2]) return NLSP_E_NOT_SPD;
  if (hinfo[0]) return NLSP_E_RANK;
  return NLSP_OK;
}

// ------------------------------------------- randomized range finder
// Basis from a sketch of S (randomized subspace iteration followed by the
// direct SVD of the small projected matrix), with a caller-drawn test matrix
// Omega (m x l):
//   Y = S Omega, Q_Y = orth(Y);  q times: Q_Z = orth(S^T Q_Y), Q_Y = orth(S Q_Z)
//   C = S^T Q_Y (= B^T, B = Q_Y^T S);  C^T C = B B^T = U_B diag(sigma^2) U_B^T
//   P0 = Q_Y U_B[:, :k], P = CholeskyQR2(P0), column signs as setup_spectral_P.
// orth is CholeskyQR2 in float64.  The eigenproblem is l x l instead of m x m.
struct RandLayout {
  SetupLayout base;   // carved with k -> l: P0/P1 (n, lq), T (mp, lq), Rinv/Lk (lq, lq)
  double* Om;         // (mp, lq) padded test matrix
  double* C;          // (mp, lq) S^T Q_Y
  double* Cb;         // (mp, lq) its orthonormal factor's ping buffer
  float* QY32;        // (n, lq) float copy of Q_Y (mixed form)
  int* info;          // 64 Cholesky / rank flags
  size_t bytes;
};

inline RandLayout carve_rand(void* ws, int64_t n, int m, int l, int prec) {
  RandLayout R;
  R.base = carve_setup(ws, n, m, l, prec);
  const int mp = pad16(m) + (pad16(m) % 2), lq = pad16(l);
  Carver cv(ws);
  cv.off = R.base.bytes;
  R.Om = cv.take<double>((size_t)mp * lq);
  R.C = cv.take<double>((size_t)mp * lq);
  R.Cb = cv.take<double>((size_t)mp * lq);
  R.QY32 = cv.take<float>(prec == NLSP_MIXED ? (size_t)n * lq : 1);
  R.info = cv.take<int>(64);
  R.bytes = cv.bytes();
  return R;
}

// S^T Q_Y (mp x lq) into C; the float form multiplies a float copy of Q_Y.
template <typename T>
static int sketch_cross(const T* S, const double* QY, int64_t n, int mp, int lq, const RandLayout& R,
                        hipStream_t s) {
  if constexpr (sizeof(T) == 4) {
    hipLaunchKernelGGL(k_to_f32, dim3(ceil_div(n * lq, 256)), dim3(256), 0, s, QY, R.QY32, n * lq);
    return gram<float>(S, R.QY32, n, mp, lq, 0, R.base.part, R.C, lq, s);
  } else {
    return gram<double>(S, QY, n, mp, lq, 0, R.base.part, R.C, lq, s);
  }
}

// A sketch column whose residual after the earlier columns is below 1e-6 of
// its norm (pivot^2 <= 1e-12 times the diagonal of the Gram matrix) makes the
// sketch numerically rank-deficient, the same threshold as the rank test on
// sigma_k / sigma_1.
constexpr double kSketchRankTol = 1e-12;

template <typename T>
static int randomized_impl(const OpDev& op, const double* S0, int m, int k, double omega, int s1,
                           const double* Omega, int l, int q, double* Pout, double* sigma, const RandLayout& R,
                           hipStream_t s) {
  const SetupLayout& L = R.base;
  const int64_t n = op.n;
  const int mp = pad16(m) + (pad16(m) % 2), kq = pad16(k), lq = pad16(l);
  T* Sa = static_cast<T*>(L.S0buf);
  T* Sb = static_cast<T*>(L.S1buf);
  hipLaunchKernelGGL(k_load_S0<T>, dim3(ceil_div(n * mp, 256)), dim3(256), 0, s, S0, n, m, mp, Sa);
  for (int it = 0; it < s1; ++it) {
    launch_cols<T>(op, mp, omega, 0, Sa, Sb, s);
    std::swap(Sa, Sb);
  }
  NLSP_HIP(hipMemsetAsync(R.Om, 0, sizeof(double) * mp * lq, s));
  hipLaunchKernelGGL(k_copy_cols, dim3(ceil_div((int64_t)m * lq, 256)), dim3(256), 0, s, Omega, l, (int64_t)m, l,
                     R.Om, lq);
  // Y = S Omega, Q_Y = orth(Y)
  double* Ya = L.P0;
  double* Yb = L.P1;
  int slot = 1;
  tsgemm<T>(Sa, n, mp, R.Om, lq, Ya, lq, lq, s);
  int rc = cholqr2(Ya, Yb, n, lq, l, L, R.info + slot, s, kSketchRankTol);
  slot += 2;
  if (rc) return rc;
  for (int it = 0; it < q; ++it) {
    // Q_Z = orth(S^T Q_Y) (mp x lq, in C / Cb), then Q_Y = orth(S Q_Z)
    rc = sketch_cross<T>(Sa, Ya, n, mp, lq, R, s);
    if (rc) return rc;
    double* Ca = R.C;
    double* Cb = R.Cb;
    rc = cholqr2(Ca, Cb, mp, lq, l, L, R.info + slot, s, kSketchRankTol);
    slot += 2;
    if (rc) return rc;
    tsgemm<T>(Sa, n, mp, Ca, lq, Ya, lq, lq, s);
    rc = cholqr2(Ya, Yb, n, lq, l, L, R.info + slot, s, kSketchRankTol);
    slot += 2;
    if (rc) return rc;
  }
  // C = S^T Q_Y; C^T C = B B^T and its eigenpairs (l x l)
  rc = sketch_cross<T>(Sa, Ya, n, mp, lq, R, s);
  if (rc) return rc;
  rc = gram<double>(R.C, R.C, mp, lq, lq, 1, L.part, L.G, lq, s);
  if (rc) return rc;
  rc = launch_eig(L.G, L.part, L.V, lq, L.rot, L.nsweeps, L.off, s);
  if (rc) return rc;
  hipLaunchKernelGGL(k_eig_finish, dim3(1), dim3(256), 0, s, L.G, L.V, lq, l, k, kq, sigma, L.T, R.info, 1);
  // P0 = Q_Y U_B[:, :k] (into the free buffer), CholeskyQR2, signs
  tsgemm<double>(Ya, n, lq, L.T, kq, Yb, kq, kq, s);
  double* Pa = Yb;
  double* Pb = Ya;
  rc = cholqr2(Pa, Pb, n, kq, k, L, R.info + slot, s);
  if (rc) return rc;
  signed_columns(Pa, n, kq, k, L, Pout, s);
  NLSP_HIP(hipGetLastError());
  int hinfo[64] = {};
  NLSP_HIP(hipMemcpyAsync(hinfo, R.info, sizeof(hinfo), hipMemcpyDeviceToHost, s));
  NLSP_HIP(hipStreamSynchronize(s));
  if (hinfo[slot] || hinfo[slot + 1]) return NLSP_E_NOT_SPD;
  // a sketch that is not of full rank l, or sigma_k lost in rounding
  for (int i = 0; i < slot; ++i)
    if (hinfo[i]) return NLSP_E_RANK;
  return NLSP_OK;
}

// ------------------------------------------------------------ Galerkin
struct CoarseLayout {
  double* Pp;     // (n, kp) padded P
  double* Y;      // (n, kp) A P, then relaxation ping buffer
  double* Z;      // (n, kp) pong
  double* part;
  double* Acp;    // (kp, kp)
  double* Lp;     // (kp, kp)
  int* info;
  size_t bytes;
};

inline CoarseLayout carve_coarse(void* ws, int64_t n, int kp) {
  Carver cv(ws);
  CoarseLayout L;
  L.Pp = cv.take<double>(n * kp);
  L.Y = cv.take<double>(n * kp);
  L.Z = cv.take<double>(n * kp);
  const GramPlan g = gram_plan(n);
  L.part = cv.take<double>((size_t)g.nwg * kp * kp);
  L.Acp = cv.take<double>((size_t)kp * kp);
  L.Lp = cv.take<double>((size_t)kp * kp);
  L.info = cv.take<int>(4);
  L.bytes = cv.bytes();
  return L;
}

}  // namespace nlsp

using namespace nlsp;

extern "C" {

size_t setup_spectral_P_workspace_bytes(const nlsp_operator* A, int m, int k, int prec) {
  const int64_t n = op_size(A);
  if (n < 1 || k < 1 || m < k || m > 256 || (prec != NLSP_FP64 && prec != NLSP_MIXED)) return 0;
  return carve_setup(nullptr, n, m, k, prec).bytes;
}

int setup_spectral_P(const nlsp_operator* A, const double* S0, int m, int k, double omega, int s1,
                     int prec, double* P, double* sigma, void* ws, size_t ws_bytes, void* stream) {
  const int64_t n = op_size(A);
  if (n < 1 || !S0 || !P || !sigma) return NLSP_E_INVALID;
  if (k < 1 || m < k || m > 256 || (int64_t)m > n || s1 < 0 || !(omega > 0)) return NLSP_E_INVALID;
  if (prec != NLSP_FP64 && prec != NLSP_MIXED) return NLSP_E_INVALID;
  const size_t need = carve_setup(nullptr, n, m, k, prec).bytes;
  if (!ws_ok(ws, ws_bytes, need)) return NLSP_E_WORKSPACE;
  const SetupLayout L = carve_setup(ws, n, m, k, prec);
  const OpDev op = make_op(*A);
  hipStream_t s = as_stream(stream);
  NLSP_HIP(hipMemsetAsync(L.info, 0, sizeof(int) * 4, s));
  if (prec == NLSP_FP64) return setup_impl<double>(op, S0, m, k, omega, s1, P, sigma, L, s);
  return setup_impl<float>(op, S0, m, k, omega, s1, P, sigma, L, s);
}

size_t setup_randomized_P_workspace_bytes(const nlsp_operator* A, int m, int k, int l, int prec) {
  const int64_t n = op_size(A);
  if (n < 1 || k < 1 || l < k || m < l || m > 256 || (prec != NLSP_FP64 && prec != NLSP_MIXED)) return 0;
  return carve_rand(nullptr, n, m, l, prec).bytes;
}

int setup_randomized_P(const nlsp_operator* A, const double* S0, int m, int k, double omega, int s1,
                       const double* Omega, int l, int q, int prec, double* P, double* sigma, void* ws,
                       size_t ws_bytes, void* stream) {
  const int64_t n = op_size(A);
  if (n < 1 || !S0 || !Omega || !P || !sigma) return NLSP_E_INVALID;
  if (k < 1 || l < k || m < l || m > 256 || (int64_t)m > n || s1 < 0 || !(omega > 0)) return NLSP_E_INVALID;
  if (q < 0 || q > 8 || (prec != NLSP_FP64 && prec != NLSP_MIXED)) return NLSP_E_INVALID;
  const size_t need = carve_rand(nullptr, n, m, l, prec).bytes;
  if (!ws_ok(ws, ws_bytes, need)) return NLSP_E_WORKSPACE;
  const RandLayout R = carve_rand(ws, n, m, l, prec);
  const OpDev op = make_op(*A);
  hipStream_t s = as_stream(stream);
  NLSP_HIP(hipMemsetAsync(R.info, 0, sizeof(int) * 64, s));
  if (prec == NLSP_FP64) return randomized_impl<double>(op, S0, m, k, omega, s1, Omega, l, q, P, sigma, R, s);
  return randomized_impl<float>(op, S0, m, k, omega, s1, Omega, l, q, P, sigma, R, s);
}

size_t galerkin_coarse_workspace_bytes(const nlsp_operator* A, int k) {
  const int64_t n = op_size(A);
  const int kp = padded_rank(k);
  if (n < 1 || kp < 0) return 0;
  return carve_coarse(nullptr, n, kp).bytes;
}

int galerkin_coarse(const nlsp_operator* A, const double* P, int k, double omega, int nu,
                    double* Ac, double* Lout, double* Linv, double* Q64, float* Q32, void* ws,
                    size_t ws_bytes, void* stream) {
  const int64_t n = op_size(A);
  const int kp = padded_rank(k);
  if (n < 1 || kp < 0 || !P || !Ac || !Lout || !Linv || (!Q64 && !Q32)) return NLSP_E_INVALID;
  if ((int64_t)k > n || nu < 1 || !(omega > 0)) return NLSP_E_INVALID;
  const size_t need = carve_coarse(nullptr, n, kp).bytes;
  if (!ws_ok(ws, ws_bytes, need)) return NLSP_E_WORKSPACE;
  const CoarseLayout L = carve_coarse(ws, n, kp);
  const OpDev op = make_op(*A);
  hipStream_t s = as_stream(stream);
  NLSP_HIP(hipMemsetAsync(L.info, 0, sizeof(int) * 4, s));
  // padded P (P itself when k is a multiple of 16 and P is 16-byte aligned:
  // it is only read), Y = A P, A_c = P^T Y (symmetric: the upper tiles,
  // mirrored)
  const double* Pp = P;
  if (kp != k || reinterpret_cast<uintptr_t>(P) % 16 != 0) {
    hipLaunchKernelGGL(k_copy_cols, dim3(ceil_div(n * kp, 256)), dim3(256), 0, s, P, k, n, k, L.Pp, kp);
    Pp = L.Pp;
  }
  launch_cols<double>(op, kp, omega, 1, Pp, L.Y, s);
  int rc = gram<double>(Pp, L.Y, n, kp, kp, 2, L.part, L.Acp, kp, s);
  if (rc) return rc;
  hipLaunchKernelGGL(k_pad_square, dim3(ceil_div(k * k, 256)), dim3(256), 0, s, L.Acp, kp, k, Ac, k, k);
  rc = launch_chol(L.Acp, kp, k, L.Lp, kp, L.info, s);
  if (rc) return rc;
  hipLaunchKernelGGL(k_pad_square, dim3(ceil_div(k * k, 256)), dim3(256), 0, s, L.Lp, kp, k, Lout, k, k);
  {
    const int rc2 = launch_tri_inv(L.Lp, kp, k, Linv, kp, s);
    if (rc2) return rc2;
  }
  // Q = (I - w D^-1 A)^nu P
  const double* cur = Pp;
  double* bufs[2] = {L.Y, L.Z};
  bool q32_done = false;
  for (int it = 0; it < nu; ++it) {
    // only the float32 Q wanted: the last sweep stores it rounded (3-D FV7)
    if (it == nu - 1 && !Q64 && zmarch_cols_relax_f32out(op, omega, kp, cur, Q32, s)) {
      q32_done = true;
      break;
    }
    double* dst = bufs[it & 1];
    launch_cols<double>(op, kp, omega, 0, cur, dst, s);
    cur = dst;
  }
  if (Q64)
    NLSP_HIP(hipMemcpyAsync(Q64, cur, sizeof(double) * n * kp, hipMemcpyDeviceToDevice, s));
  if (Q32 && !q32_done)
    hipLaunchKernelGGL(k_to_f32, dim3(ceil_div(n * kp, 256)), dim3(256), 0, s, cur, Q32, n * kp);
  NLSP_HIP(hipGetLastError());
  int info = 0;
  NLSP_HIP(hipMemcpyAsync(&info, L.info, sizeof(int), hipMemcpyDeviceToHost, s));
  NLSP_HIP(hipStreamSynchronize(s));
  return info ? NLSP_E_NOT_SPD : NLSP_OK;
}

}  // extern "C"
