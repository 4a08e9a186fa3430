// Preconditioned conjugate gradients with the spectral two-level
// preconditioner (Sec. 4.1 two-grid solver evaluation; the algorithm's
// preconditioner application), gfx950.
//
// Preconditioner.  For nu1 = nu2 = nu sweeps of weighted Jacobi the two-grid
// operator of the algorithm is, exactly,
//     M^-1 r = J_{2nu} r + Q A_c^-1 Q^T r,     Q = (I - w D^-1 A)^nu P,
// (J_{2nu} r = 2nu Jacobi sweeps on A z = r from z = 0).  Q and the inverse
// Cholesky factor of A_c come from galerkin_coarse.  For nu = 1,
// J_2 r = 2w D^-1 r - w^2 D^-1 A D^-1 r needs one stencil pass, which is fused
// with the prolongation; the restriction Q^T r is fused with the r update.
//
// One iteration = three kernels, each ending in a grid reduction finished by
// the last workgroup to arrive (fixed summation order, so results are
// bitwise reproducible):
//   phase 1  p <- z + beta p (double-buffered), q = A p, partial p^T q
//            last WG: alpha = gamma / p^T q
//   phase 2  x += alpha p, r -= alpha q, partial ||r||^2, partial Q^T r
//            last WG: convergence test, e = L^-T L^-1 (Q^T r)
//   phase 3  w = J_2 r, z = w + Q e, partial r^T z (and r^T z_old)
//            last WG: beta
// Vectors and every reduction are float64; in the mixed form Q, the smoother
// and the prolongation products are float32.
#include <vector>

#include "device_common.hpp"
#include "host_common.hpp"

namespace nlsp {

constexpr int NT = 512;  // threads per workgroup of the solver kernels

struct RhsState {
  double gamma, alpha, beta, delta;
  double rr, ff, rzold, rr_true;
  int active, iters, status, conv;
  int par, pad0, pad1, pad2;
};

struct SysDev {
  OpDev op;
  int R, kp, nblk, blk0;
  int chunk_rows;          // rows per chunk: floor(NT / R); threads past chunk_rows*R idle in elementwise parts
  int64_t nchunks;
  const void* Q;           // (n, kp), float or double
  const double* Linv;      // (kp, kp)
  const double* f;
  double* x;
  double* r;
  double* p0;
  double* p1;
  double* q;
  double* z;
  void* w0;                // J_{2nu} r work buffers (nu > 1), element type of Q
  void* w1;
  const double* dinv;
  const float* dinv32;
  double* part;            // nblk * pstride partial sums
  int pstride;
  int nu;
  unsigned* ticket;
  RhsState* st;
  int* sys_active;
  double* e;               // (kp, R)
  double omega, tol2;
  int maxit, flexible;
};

// partial-sum slots inside one workgroup's record (doubles)
// [0, kp*R) restriction, then R each for: delta, rr, gamma', r^T z_old, ff
NLSP_DEV int slot_scalar(const SysDev& S, int which) { return S.kp * S.R + which * S.R; }
enum { SL_DELTA = 0, SL_RR = 1, SL_GAM = 2, SL_RZOLD = 3, SL_FF = 4, SL_COUNT = 5 };

// XCD-aware order: hardware places workgroup b on XCD b % 8; give each XCD a
// contiguous range of logical blocks so that stencil halos are served from
// that XCD's L2.
NLSP_DEV int xcd_remap(int b, int nb) {
  const int x = b & 7, q = nb >> 3, rem = nb & 7;
  const int start = x * q + (x < rem ? x : rem);
  return start + (b >> 3);
}

NLSP_DEV const SysDev& my_sys(const SysDev* sys, const int* blk2sys, int nsys) {
  return sys[nsys == 1 ? 0 : blk2sys[blockIdx.x]];
}

template <typename T>
struct Vec4;
template <>
struct Vec4<float> {
  using type = float4;
};
template <>
struct Vec4<double> {
  using type = double4;
};

template <typename QT>
NLSP_DEV void load4(const QT* p, QT (&v)[4]) {
  const typename Vec4<QT>::type t = *reinterpret_cast<const typename Vec4<QT>::type*>(p);
  v[0] = t.x;
  v[1] = t.y;
  v[2] = t.z;
  v[3] = t.w;
}

// Sum of per-thread values over the threads that share c = t % R; the totals
// land in red[c] (LDS) for c < R.  Deterministic.  All threads call.
NLSP_DEV void block_sum_rhs(double v, int R, double* red, double* sh /* NT doubles */) {
  const int t = threadIdx.x;
  __syncthreads();
  sh[t] = v;
  __syncthreads();
  if (t < R) {
    double s = 0.0;
    for (int k = t; k < NT; k += R) s += sh[k];
    red[t] = s;
  }
  __syncthreads();
}

// Last-workgroup reduction of `count` consecutive partial slots starting at
// `off` over all nblk records.  Result in out[0..count) (LDS).  All threads of
// the last workgroup call.
NLSP_DEV void reduce_partials(const SysDev& S, int off, int count, double* out, double* sh) {
  const int t = threadIdx.x;
  const double* P = S.part;
  for (int base = 0; base < count; base += NT) {
    const int cnt = min(NT, count - base);
    const int groups = NT / cnt;               // >= 1
    const int e = t % cnt, g = t / cnt;
    double s = 0.0;
    if (g < groups)
      for (int b = g; b < S.nblk; b += groups) s += P[(int64_t)b * S.pstride + off + base + e];
    __syncthreads();
    sh[t] = (g < groups) ? s : 0.0;
    __syncthreads();
    if (t < cnt) {
      double tot = 0.0;
      for (int gg = 0; gg < groups; ++gg) tot += sh[gg * cnt + t];
      out[base + t] = tot;
    }
    __syncthreads();
  }
}

NLSP_DEV void deactivate(const SysDev& S, int c, int status, int* n_active) {
  S.st[c].active = 0;
  S.st[c].status = status;
  atomicSub(S.sys_active, 1);
  atomicSub(n_active, 1);
}

// e = L^-T (L^-1 c) for every RHS, c in LDS (kp*R), result to S.e (global).
NLSP_DEV void coarse_solve(const SysDev& S, const double* cvec, double* tmp) {
  const int kp = S.kp, R = S.R, t = threadIdx.x;
  for (int idx = t; idx < kp * R; idx += NT) {
    const int i = idx / R, c = idx % R;
    double s = 0.0;
    for (int j = 0; j <= i; ++j) s += S.Linv[i * kp + j] * cvec[j * R + c];
    tmp[idx] = s;
  }
  __syncthreads();
  for (int idx = t; idx < kp * R; idx += NT) {
    const int i = idx / R, c = idx % R;
    double s = 0.0;
    for (int j = i; j < kp; ++j) s += S.Linv[j * kp + i] * tmp[j * R + c];
    S.e[idx] = s;
  }
}

// Restriction accumulators: thread t owns column chunk jc (4 columns) of RHS c
// for row group rg; the workgroup streams rows of Q with consecutive lanes on
// consecutive 4-column chunks of a row (coalesced).
struct RestrictMap {
  int lpr, pairs, rg, ngr, jc, c, npair_iter;
};

NLSP_DEV RestrictMap restrict_map(int kp, int R) {
  RestrictMap m;
  const int t = threadIdx.x;
  m.lpr = kp / 4;
  m.pairs = m.lpr * R;
  if (m.pairs <= NT) {
    m.ngr = NT / m.pairs;
    m.rg = t / m.pairs;
    const int pr = t % m.pairs;
    m.jc = pr % m.lpr;
    m.c = pr / m.lpr;
    m.npair_iter = 1;
  } else {
    m.ngr = 1;
    m.rg = 0;
    m.jc = 0;
    m.c = 0;
    m.npair_iter = (m.pairs + NT - 1) / NT;
  }
  return m;
}

template <typename QT>
NLSP_DEV double prod(QT q, double r) {
  return (double)(q * (QT)r);  // float32 products in the mixed form
}

// acc[pi][u] += sum over the chunk rows of Q[row][4 jc + u] * rv[row*R + c]
template <typename QT, int MAXP>
NLSP_DEV void restrict_chunk(const QT* __restrict__ Q, int64_t row0, int nrows, int kp, int R,
                             const RestrictMap& m, const double* rv, double (&acc)[MAXP][4]) {
  if (m.pairs <= NT) {
    if (m.rg >= m.ngr) return;
    const QT* qb = Q + (row0 + m.rg) * kp + 4 * m.jc;
    const int stride = m.ngr;
    int row = m.rg;
#pragma unroll 4
    for (; row < nrows; row += stride) {
      QT qv[4];
      load4(qb, qv);
      qb += (int64_t)stride * kp;
      const double rvv = rv[row * R + m.c];
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[0][u] += prod<QT>(qv[u], rvv);
    }
  } else {
    for (int pi = 0; pi < m.npair_iter && pi < MAXP; ++pi) {
      const int pr = threadIdx.x + pi * NT;
      if (pr >= m.pairs) break;
      const int jc = pr % m.lpr, c = pr / m.lpr;
      for (int row = 0; row < nrows; ++row) {
        QT qv[4];
        load4(Q + (row0 + row) * kp + 4 * jc, qv);
        const double rvv = rv[row * R + c];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[pi][u] += prod<QT>(qv[u], rvv);
      }
    }
  }
}

// Workgroup total of the restriction accumulators -> part[0 .. kp*R) of this
// workgroup's record (layout j*R + c).  red: LDS of 32*NT bytes.
template <int MAXP>
NLSP_DEV void restrict_finish(const RestrictMap& m, int kp, int R, double (&acc)[MAXP][4],
                              double* red, double* out) {
  const int t = threadIdx.x;
  if (m.pairs <= NT) {
    const int KR = kp * R;
    __syncthreads();
    if (m.rg < m.ngr) {
#pragma unroll
      for (int u = 0; u < 4; ++u) red[m.rg * KR + (4 * m.jc + u) * R + m.c] = acc[0][u];
    }
    __syncthreads();
    for (int idx = t; idx < KR; idx += NT) {
      double s = 0.0;
      for (int g = 0; g < m.ngr; ++g) s += red[g * KR + idx];
      out[idx] = s;
    }
  } else {
    for (int pi = 0; pi < m.npair_iter && pi < MAXP; ++pi) {
      const int pr = t + pi * NT;
      if (pr >= m.pairs) break;
      const int jc = pr % m.lpr, c = pr / m.lpr;
#pragma unroll
      for (int u = 0; u < 4; ++u) out[(4 * jc + u) * R + c] = acc[pi][u];
    }
  }
}

// ys[row*R + c] = sum_j Q[row][j] e[j][c] for the chunk rows (prolongation),
// arithmetic in QT; lanes of a row reduce with butterflies.
template <typename QT>
NLSP_DEV void prolong_chunk(const QT* __restrict__ Q, int64_t row0, int nrows, int kp, int R,
                            const QT* ev /* LDS (kp*R) */, QT* ys) {
  const int t = threadIdx.x;
  const int lpr = kp / 4, pairs = lpr * R;
  if (pairs <= NT) {
    const int ngr = NT / pairs, rg = t / pairs, pr = t % pairs;
    const int jc = pr % lpr, c = pr / lpr;
    QT e4[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) e4[u] = ev[(4 * jc + u) * R + c];
    // all lanes of a wave must take part in the butterflies: iterate a
    // uniform trip count and mask the rows past the end
    const int trips = (nrows + ngr - 1) / ngr;
#pragma unroll 4
    for (int it = 0; it < trips; ++it) {
      const int row = rg + it * ngr;
      QT s = QT(0);
      if (rg < ngr && row < nrows) {
        QT qv[4];
        load4(Q + (row0 + row) * kp + 4 * jc, qv);
        s = qv[0] * e4[0] + qv[1] * e4[1] + qv[2] * e4[2] + qv[3] * e4[3];
      }
      s = group_sum(s, lpr);
      if (jc == 0 && rg < ngr && row < nrows) ys[row * R + c] = s;
    }
  } else {
    for (int idx = t; idx < nrows * R; idx += NT) {
      const int row = idx / R, c = idx % R;
      QT s = QT(0);
      for (int j = 0; j < kp; ++j) s += Q[(row0 + row) * kp + j] * ev[j * R + c];
      ys[idx] = s;
    }
  }
}

struct ChunkRange {
  int64_t c0, c1;
};

NLSP_DEV ChunkRange my_chunks(const SysDev& S, int lb) {
  const int64_t per = (S.nchunks + S.nblk - 1) / S.nblk;
  ChunkRange cr;
  cr.c0 = (int64_t)lb * per;
  cr.c1 = min(S.nchunks, cr.c0 + per);
  return cr;
}

// ----------------------------------------------------------------- kernels
__global__ __launch_bounds__(NT) void k_dinv(OpDev op, double* dinv, float* dinv32) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= op.n) return;
  int x, y, z;
  decompose(op, i, x, y, z);
  const double d = 1.0 / op_diag<double>(op, i, x, y, z);
  dinv[i] = d;
  dinv32[i] = (float)d;
}

// r = f - A x for the RHS in `mask`; partial ||r||^2, Q^T r and (init) ||f||^2.
// Last workgroup: coarse solve, (re)activation.  Used at start-up (init = 1)
// and for residual replacement (init = 0).
template <typename QT>
__global__ __launch_bounds__(NT) void k_residual(const SysDev* __restrict__ sys,
                                                 const int* __restrict__ blk2sys, int nsys,
                                                 int* n_active, unsigned mask, int init) {
  __shared__ double rv[NT];
  __shared__ double sh[NT];
  __shared__ double red[4 * NT];
  __shared__ double outv[4 * NT];
  const SysDev& S = my_sys(sys, blk2sys, nsys);
  const int lb = xcd_remap(blockIdx.x - S.blk0, S.nblk);
  const int t = threadIdx.x, R = S.R, c = t % R;
  const bool on = (mask >> c) & 1u;
  const QT* Q = static_cast<const QT*>(S.Q);
  const RestrictMap m = restrict_map(S.kp, R);
  double acc[4][4] = {};
  double rr = 0.0, ff = 0.0;
  const ChunkRange cr = my_chunks(S, lb);
  for (int64_t ch = cr.c0; ch < cr.c1; ++ch) {
    const int64_t row0 = ch * S.chunk_rows;
    const int nrows = (int)min<int64_t>(S.chunk_rows, S.op.n - row0);
    const int64_t i = row0 + t / R;
    double rvv = 0.0;
    if (on && t / R < nrows) {
      int px, py, pz;
      decompose(S.op, i, px, py, pz);
      const double* X = S.x;
      const double ax = op_row<double>(S.op, i, px, py, pz, [&](int64_t j) { return X[j * R + c]; });
      const double fi = S.f[i * R + c];
      rvv = fi - ax;
      S.r[i * R + c] = rvv;
      rr += rvv * rvv;
      ff += fi * fi;
    }
    __syncthreads();
    rv[t] = rvv;
    __syncthreads();
    restrict_chunk<QT, 4>(Q, row0, nrows, S.kp, R, m, rv, acc);
  }
  double* mypart = S.part + (int64_t)lb * S.pstride;
  restrict_finish<4>(m, S.kp, R, acc, red, mypart);
  block_sum_rhs(rr, R, outv, sh);
  if (t < R) mypart[slot_scalar(S, SL_RR) + t] = outv[t];
  block_sum_rhs(ff, R, outv, sh);
  if (t < R) mypart[slot_scalar(S, SL_FF) + t] = outv[t];
  if (!arrive_last(S.ticket, S.nblk)) return;
  // ---- last workgroup
  reduce_partials(S, slot_scalar(S, SL_RR), R, outv, sh);
  if (t < R && ((mask >> t) & 1u)) {
    RhsState& st = S.st[t];
    st.rr = outv[t];
  }
  __syncthreads();
  if (init) {
    reduce_partials(S, slot_scalar(S, SL_FF), R, outv, sh);
    if (t < R && ((mask >> t) & 1u)) S.st[t].ff = outv[t];
  }
  __syncthreads();
  if (t < R && ((mask >> t) & 1u)) {
    RhsState& st = S.st[t];
    const double tol2 = S.tol2 * st.ff;
    int want;
    if (!(st.rr == st.rr) || st.rr > 1.7e308 || !(st.ff == st.ff) || st.ff > 1.7e308) {
      want = 0;
      st.status = NLSP_E_NONFINITE;
    } else if (st.ff == 0.0 || st.rr <= tol2) {
      want = 0;
      st.conv = 1;
      st.status = NLSP_OK;
    } else {
      want = 1;
      st.conv = 0;
      st.status = NLSP_NOT_CONVERGED;
    }
    if (want != st.active) {
      atomicAdd(S.sys_active, want - st.active);
      atomicAdd(n_active, want - st.active);
      st.active = want;
    }
  }
  reduce_partials(S, 0, S.kp * R, red, sh);
  coarse_solve(S, red, outv);
}

// phase 1: p_new = z + beta p_old (double buffer), q = A p_new, partial p^T q
__global__ __launch_bounds__(NT) void k_phase1(const SysDev* __restrict__ sys,
                                               const int* __restrict__ blk2sys, int nsys,
                                               int* n_active) {
  __shared__ double sh[NT];
  __shared__ double outv[NT];
  const SysDev& S = my_sys(sys, blk2sys, nsys);
  if (*S.sys_active == 0) return;
  const int lb = xcd_remap(blockIdx.x - S.blk0, S.nblk);
  const int t = threadIdx.x, R = S.R, c = t % R;
  const RhsState& st = S.st[c];
  const bool act = st.active != 0;
  const double beta = st.beta;
  const double* pold = st.par ? S.p1 : S.p0;
  double* pnew = st.par ? S.p0 : S.p1;
  const double* Z = S.z;
  double dp = 0.0;
  const ChunkRange cr = my_chunks(S, lb);
  if (act) {
    for (int64_t ch = cr.c0; ch < cr.c1; ++ch) {
      const int64_t row0 = ch * S.chunk_rows;
      const int64_t i = row0 + t / R;
      if (t / R >= S.chunk_rows || i >= S.op.n) continue;
      int px, py, pz;
      decompose(S.op, i, px, py, pz);
      auto pn = [&](int64_t j) { return Z[j * R + c] + beta * pold[j * R + c]; };
      const double pi = pn(i);
      const double qi = op_row<double>(S.op, i, px, py, pz, pn);
      pnew[i * R + c] = pi;
      S.q[i * R + c] = qi;
      dp += pi * qi;
    }
  }
  double* mypart = S.part + (int64_t)lb * S.pstride;
  block_sum_rhs(dp, R, outv, sh);
  if (t < R) mypart[slot_scalar(S, SL_DELTA) + t] = outv[t];
  if (!arrive_last(S.ticket, S.nblk)) return;
  reduce_partials(S, slot_scalar(S, SL_DELTA), R, outv, sh);
  if (t < R && S.st[t].active) {
    RhsState& s2 = S.st[t];
    const double d = outv[t];
    s2.delta = d;
    s2.par ^= 1;
    if (!(d == d) || d > 1.7e308 || d < -1.7e308) {
      deactivate(S, t, NLSP_E_NONFINITE, n_active);
    } else if (!(d > 0.0)) {
      deactivate(S, t, NLSP_E_BREAKDOWN, n_active);
    } else {
      s2.alpha = s2.gamma / d;
    }
  }
}

// phase 2: x += alpha p, r -= alpha q, partial ||r||^2 and Q^T r;
// last workgroup: convergence test and coarse solve
template <typename QT>
__global__ __launch_bounds__(NT) void k_phase2(const SysDev* __restrict__ sys,
                                               const int* __restrict__ blk2sys, int nsys,
                                               int* n_active) {
  __shared__ double rv[NT];
  __shared__ double sh[NT];
  __shared__ double red[4 * NT];
  __shared__ double outv[4 * NT];
  const SysDev& S = my_sys(sys, blk2sys, nsys);
  if (*S.sys_active == 0) return;
  const int lb = xcd_remap(blockIdx.x - S.blk0, S.nblk);
  const int t = threadIdx.x, R = S.R, c = t % R;
  const RhsState& st = S.st[c];
  const bool act = st.active != 0;
  const double alpha = st.alpha;
  const double* P = st.par ? S.p1 : S.p0;  // phase 1 flipped the parity
  const QT* Q = static_cast<const QT*>(S.Q);
  const RestrictMap m = restrict_map(S.kp, R);
  double acc[4][4] = {};
  double rr = 0.0;
  const ChunkRange cr = my_chunks(S, lb);
  for (int64_t ch = cr.c0; ch < cr.c1; ++ch) {
    const int64_t row0 = ch * S.chunk_rows;
    const int nrows = (int)min<int64_t>(S.chunk_rows, S.op.n - row0);
    double rvv = 0.0;
    if (act && t / R < nrows) {
      const int64_t g = (row0 + t / R) * R + c;
      S.x[g] += alpha * P[g];
      rvv = S.r[g] - alpha * S.q[g];
      S.r[g] = rvv;
      rr += rvv * rvv;
    }
    __syncthreads();
    rv[t] = rvv;
    __syncthreads();
    restrict_chunk<QT, 4>(Q, row0, nrows, S.kp, R, m, rv, acc);
  }
  double* mypart = S.part + (int64_t)lb * S.pstride;
  restrict_finish<4>(m, S.kp, R, acc, red, mypart);
  block_sum_rhs(rr, R, outv, sh);
  if (t < R) mypart[slot_scalar(S, SL_RR) + t] = outv[t];
  if (!arrive_last(S.ticket, S.nblk)) return;
  reduce_partials(S, slot_scalar(S, SL_RR), R, outv, sh);
  if (t < R && S.st[t].active) {
    RhsState& s2 = S.st[t];
    const double rrv = outv[t];
    s2.rr = rrv;
    s2.iters += 1;
    if (!(rrv == rrv) || rrv > 1.7e308) {
      deactivate(S, t, NLSP_E_NONFINITE, n_active);
    } else if (rrv <= S.tol2 * s2.ff) {
      s2.conv = 1;
      deactivate(S, t, NLSP_OK, n_active);
    } else if (s2.iters >= S.maxit) {
      deactivate(S, t, NLSP_NOT_CONVERGED, n_active);
    }
  }
  __syncthreads();
  reduce_partials(S, 0, S.kp * R, red, sh);
  coarse_solve(S, red, outv);
}

// J_{2nu} sweeps for nu > 1: first = 1 computes y2 = y1 + w D^-1 (r - A y1)
// with y1 = w D^-1 r; later sweeps y <- y + w D^-1 (r - A y).  PT arithmetic.
template <typename PT>
__global__ __launch_bounds__(NT) void k_sweep(const SysDev* __restrict__ sys,
                                              const int* __restrict__ blk2sys, int nsys, int first,
                                              int src) {
  const SysDev& S = my_sys(sys, blk2sys, nsys);
  if (*S.sys_active == 0) return;
  const int lb = xcd_remap(blockIdx.x - S.blk0, S.nblk);
  const int t = threadIdx.x, R = S.R, c = t % R;
  if (!S.st[c].active) return;
  const PT om = PT(S.omega);
  const PT* yin = static_cast<const PT*>(src ? S.w1 : S.w0);
  PT* yout = static_cast<PT*>(first ? S.w0 : (src ? S.w0 : S.w1));
  const double* Rv = S.r;
  const ChunkRange cr = my_chunks(S, lb);
  for (int64_t ch = cr.c0; ch < cr.c1; ++ch) {
    const int64_t row0 = ch * S.chunk_rows;
    const int64_t i = row0 + t / R;
    if (t / R >= S.chunk_rows || i >= S.op.n) continue;
    int px, py, pz;
    decompose(S.op, i, px, py, pz);
    const PT di = (sizeof(PT) == 4) ? PT(S.dinv32[i]) : PT(S.dinv[i]);
    const PT ri = PT(Rv[i * R + c]);
    PT yi, ay;
    if (first) {
      auto y1 = [&](int64_t j) {
        const PT dj = (sizeof(PT) == 4) ? PT(S.dinv32[j]) : PT(S.dinv[j]);
        return om * dj * PT(Rv[j * R + c]);
      };
      yi = y1(i);
      ay = op_row<PT>(S.op, i, px, py, pz, y1);
    } else {
      yi = yin[i * R + c];
      ay = op_row<PT>(S.op, i, px, py, pz, [&](int64_t j) { return yin[j * R + c]; });
    }
    yout[i * R + c] = yi + om * di * (ri - ay);
  }
}

// phase 3: z = J_{2nu} r + Q e, partial r^T z (and r^T z_old); last
// workgroup: beta.  wsrc < 0: J_2 inline (nu = 1); else read buffer w{wsrc}.
template <typename QT>
__global__ __launch_bounds__(NT) void k_phase3(const SysDev* __restrict__ sys,
                                               const int* __restrict__ blk2sys, int nsys,
                                               int* n_active, int wsrc) {
  __shared__ QT ws[NT];
  __shared__ QT ys[NT];
  __shared__ QT ev[2048];
  __shared__ double sh[NT];
  __shared__ double outv[NT];
  const SysDev& S = my_sys(sys, blk2sys, nsys);
  if (*S.sys_active == 0) return;
  const int lb = xcd_remap(blockIdx.x - S.blk0, S.nblk);
  const int t = threadIdx.x, R = S.R, c = t % R;
  const RhsState& st = S.st[c];
  const bool act = st.active != 0;
  const QT* Q = static_cast<const QT*>(S.Q);
  const QT om = QT(S.omega);
  for (int idx = t; idx < S.kp * R; idx += NT) ev[idx] = QT(S.e[idx]);
  const double* Rv = S.r;
  double gam = 0.0, rzo = 0.0;
  const ChunkRange cr = my_chunks(S, lb);
  for (int64_t ch = cr.c0; ch < cr.c1; ++ch) {
    const int64_t row0 = ch * S.chunk_rows;
    const int nrows = (int)min<int64_t>(S.chunk_rows, S.op.n - row0);
    const bool mine = act && t / R < nrows;
    const int64_t i = row0 + t / R;
    QT w = QT(0);
    if (mine) {
      if (wsrc < 0) {
        int px, py, pz;
        decompose(S.op, i, px, py, pz);
        auto dj = [&](int64_t j) -> QT {
          return (sizeof(QT) == 4) ? QT(S.dinv32[j]) : QT(S.dinv[j]);
        };
        auto y = [&](int64_t j) { return dj(j) * QT(Rv[j * R + c]); };
        const QT yi = y(i);
        const QT ay = op_row<QT>(S.op, i, px, py, pz, y);
        w = QT(2) * om * yi - om * om * dj(i) * ay;
      } else {
        const QT* wb = static_cast<const QT*>(wsrc ? S.w1 : S.w0);
        w = wb[i * R + c];
      }
    }
    __syncthreads();
    ws[t] = w;
    __syncthreads();
    prolong_chunk<QT>(Q, row0, nrows, S.kp, R, ev, ys);
    __syncthreads();
    if (mine) {
      const int64_t g = i * R + c;
      const double zn = (double)ws[t] + (double)ys[t];
      const double ri = Rv[g];
      if (S.flexible) rzo += ri * S.z[g];
      S.z[g] = zn;
      gam += ri * zn;
    }
  }
  double* mypart = S.part + (int64_t)lb * S.pstride;
  block_sum_rhs(gam, R, outv, sh);
  if (t < R) mypart[slot_scalar(S, SL_GAM) + t] = outv[t];
  block_sum_rhs(rzo, R, outv, sh);
  if (t < R) mypart[slot_scalar(S, SL_RZOLD) + t] = outv[t];
  if (!arrive_last(S.ticket, S.nblk)) return;
  reduce_partials(S, slot_scalar(S, SL_GAM), 2 * R, outv, sh);
  if (t < R && S.st[t].active) {
    RhsState& s2 = S.st[t];
    const double g = outv[t], rz = outv[R + t];
    if (!(g == g) || g > 1.7e308) {
      deactivate(S, t, NLSP_E_NONFINITE, n_active);
    } else if (!(g > 0.0)) {
      deactivate(S, t, NLSP_E_BREAKDOWN, n_active);
    } else {
      s2.beta = S.flexible ? (g - rz) / s2.gamma : g / s2.gamma;
      s2.gamma = g;
      s2.rzold = rz;
    }
  }
}

// ||f - A x||^2 per RHS (true residual) into st.rr_true
__global__ __launch_bounds__(NT) void k_true_residual(const SysDev* __restrict__ sys,
                                                      const int* __restrict__ blk2sys, int nsys) {
  __shared__ double sh[NT];
  __shared__ double outv[NT];
  const SysDev& S = my_sys(sys, blk2sys, nsys);
  const int lb = xcd_remap(blockIdx.x - S.blk0, S.nblk);
  const int t = threadIdx.x, R = S.R, c = t % R;
  double s = 0.0;
  const ChunkRange cr = my_chunks(S, lb);
  const double* X = S.x;
  for (int64_t ch = cr.c0; ch < cr.c1; ++ch) {
    const int64_t i = ch * S.chunk_rows + t / R;
    if (t / R >= S.chunk_rows || i >= S.op.n) continue;
    int px, py, pz;
    decompose(S.op, i, px, py, pz);
    const double ax = op_row<double>(S.op, i, px, py, pz, [&](int64_t j) { return X[j * R + c]; });
    const double d = S.f[i * R + c] - ax;
    s += d * d;
  }
  double* mypart = S.part + (int64_t)lb * S.pstride;
  block_sum_rhs(s, R, outv, sh);
  if (t < R) mypart[slot_scalar(S, SL_DELTA) + t] = outv[t];
  if (!arrive_last(S.ticket, S.nblk)) return;
  reduce_partials(S, slot_scalar(S, SL_DELTA), R, outv, sh);
  if (t < R) S.st[t].rr_true = outv[t];
}

__global__ void k_zero_cols(double* u, int64_t n, int R, unsigned mask) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n * R) return;
  if ((mask >> (g % R)) & 1u) u[g] = 0.0;
}

// ------------------------------------------------------------- host side
struct SolveLayout {
  double *r, *p0, *p1, *q, *z, *dinv, *part, *e;
  float* dinv32;
  void *w0, *w1;
  RhsState* st;
  SysDev* sysdev;
  unsigned* ticket;
  int* counters;  // [0] n_active, [1] sys_active
  size_t bytes;
};

inline int solver_blocks(int64_t nchunks) {
  const int cap = 512;
  return (int)std::min<int64_t>(nchunks, cap);
}

inline SolveLayout carve_solve(void* ws, int64_t n, int kp, int R, int nblk) {
  Carver cv(ws);
  SolveLayout L;
  L.r = cv.take<double>(n * R);
  L.p0 = cv.take<double>(n * R);
  L.p1 = cv.take<double>(n * R);
  L.q = cv.take<double>(n * R);
  L.z = cv.take<double>(n * R);
  L.w0 = cv.take<double>(n * R);
  L.w1 = cv.take<double>(n * R);
  L.dinv = cv.take<double>(n);
  L.dinv32 = cv.take<float>(n);
  const int pstride = kp * R + SL_COUNT * R;
  L.part = cv.take<double>((size_t)nblk * pstride);
  L.e = cv.take<double>((size_t)kp * R);
  L.st = cv.take<RhsState>(R);
  L.sysdev = cv.take<SysDev>(1);
  L.ticket = cv.take<unsigned>(4);
  L.counters = cv.take<int>(4);
  L.bytes = cv.bytes();
  return L;
}

template <typename QT>
static int run_pcg(const SysDev& hs, const SolveLayout& L, int R, const nlsp_pcg_opts* opts,
                   nlsp_rhs_info* info, hipStream_t stream) {
  const int nblk = hs.nblk;
  const SysDev* dsys = L.sysdev;
  int* n_active = L.counters;
  const unsigned all = (R >= 32) ? 0xffffffffu : ((1u << R) - 1u);
  const dim3 grid(nblk), block(NT);
  hipLaunchKernelGGL(k_dinv, dim3(ceil_div(hs.op.n, NT)), block, 0, stream, hs.op, L.dinv,
                     L.dinv32);
  hipLaunchKernelGGL(k_residual<QT>, grid, block, 0, stream, dsys, nullptr, 1, n_active, all, 1);
  auto launch_phase3 = [&]() {
    if (hs.nu == 1) {
      hipLaunchKernelGGL(k_phase3<QT>, grid, block, 0, stream, dsys, nullptr, 1, n_active, -1);
    } else {
      hipLaunchKernelGGL(k_sweep<QT>, grid, block, 0, stream, dsys, nullptr, 1, 1, 0);
      int src = 0;
      for (int s = 1; s < 2 * hs.nu - 1; ++s) {
        hipLaunchKernelGGL(k_sweep<QT>, grid, block, 0, stream, dsys, nullptr, 1, 0, src);
        src ^= 1;
      }
      hipLaunchKernelGGL(k_phase3<QT>, grid, block, 0, stream, dsys, nullptr, 1, n_active, src);
    }
  };
  launch_phase3();
  NLSP_HIP(hipGetLastError());
  std::vector<RhsState> hst(R);
  NLSP_HIP(hipMemcpyAsync(hst.data(), L.st, sizeof(RhsState) * R, hipMemcpyDeviceToHost, stream));
  NLSP_HIP(hipStreamSynchronize(stream));
  unsigned zero_mask = 0;
  for (int c = 0; c < R; ++c)
    if (hst[c].ff == 0.0) zero_mask |= 1u << c;
  if (zero_mask)
    hipLaunchKernelGGL(k_zero_cols, dim3(ceil_div(hs.op.n * R, 256)), dim3(256), 0, stream, hs.x,
                       hs.op.n, R, zero_mask);
  const int every = std::max(1, opts->check_every);
  int guard = 0;
  // every RHS stops by maxit iterations; the launch budget is a hard bound
  // on the host loop in case the device-side bookkeeping were ever wrong
  int64_t launched = 0;
  const int64_t launch_cap = (int64_t)hs.maxit + 2 * every + 64;
  for (;;) {
    int h_active = 0;
    NLSP_HIP(hipMemcpyAsync(&h_active, n_active, sizeof(int), hipMemcpyDeviceToHost, stream));
    NLSP_HIP(hipStreamSynchronize(stream));
    if (h_active > 0 && launched < launch_cap) {
      launched += every;
      for (int it = 0; it < every; ++it) {
        hipLaunchKernelGGL(k_phase1, grid, block, 0, stream, dsys, nullptr, 1, n_active);
        hipLaunchKernelGGL(k_phase2<QT>, grid, block, 0, stream, dsys, nullptr, 1, n_active);
        launch_phase3();
      }
      NLSP_HIP(hipGetLastError());
      continue;
    }
    // every RHS stopped: confirm the converged ones with the true residual
    hipLaunchKernelGGL(k_true_residual, grid, block, 0, stream, dsys, nullptr, 1);
    NLSP_HIP(hipGetLastError());
    NLSP_HIP(hipMemcpyAsync(hst.data(), L.st, sizeof(RhsState) * R, hipMemcpyDeviceToHost, stream));
    NLSP_HIP(hipStreamSynchronize(stream));
    unsigned redo = 0;
    for (int c = 0; c < R; ++c) {
      RhsState& s = hst[c];
      if (s.conv && s.ff > 0.0 && s.rr_true > hs.tol2 * s.ff && s.iters < hs.maxit) redo |= 1u << c;
    }
    if (!redo || ++guard > 16) break;
    // residual replacement: r = f - A x for `redo`, then continue iterating
    for (int c = 0; c < R; ++c)
      if ((redo >> c) & 1u) {
        hst[c].conv = 0;
      }
    NLSP_HIP(hipMemcpyAsync(L.st, hst.data(), sizeof(RhsState) * R, hipMemcpyHostToDevice, stream));
    hipLaunchKernelGGL(k_residual<QT>, grid, block, 0, stream, dsys, nullptr, 1, n_active, redo, 0);
    launch_phase3();
    NLSP_HIP(hipGetLastError());
  }
  int worst = NLSP_OK;
  for (int c = 0; c < R; ++c) {
    const RhsState& s = hst[c];
    info[c].iters = s.iters;
    info[c].status = s.status;
    info[c].relres = (s.ff > 0.0) ? std::sqrt(s.rr_true / s.ff) : 0.0;
    if (s.status < 0 && (worst >= 0 || s.status < worst)) worst = s.status;
    if (s.status == NLSP_NOT_CONVERGED && worst == NLSP_OK) worst = NLSP_NOT_CONVERGED;
  }
  return worst;
}

}  // namespace nlsp

using namespace nlsp;

extern "C" {

size_t pcg_solve_workspace_bytes(const nlsp_operator* A, int k, int R) {
  const int64_t n = op_size(A);
  const int kp = padded_rank(k);
  if (n < 1 || kp < 0 || R < 1 || R > 16 || kp * R > 2048) return 0;
  const int64_t nchunks = (n + NT / R - 1) / (NT / R);
  return carve_solve(nullptr, n, kp, R, solver_blocks(nchunks)).bytes;
}

int pcg_solve(const nlsp_operator* A, const nlsp_two_level* M, const double* f, double* u, int R,
              const nlsp_pcg_opts* opts, nlsp_rhs_info* info, void* ws, size_t ws_bytes,
              void* stream_) {
  const int64_t n = op_size(A);
  if (n < 1 || !M || !f || !u || !opts || !info) return NLSP_E_INVALID;
  if (R < 1 || R > 16) return NLSP_E_INVALID;
  const int kp = padded_rank(M->k);
  if (kp < 0 || M->nu < 1 || !(M->omega > 0) || !M->Linv) return NLSP_E_INVALID;
  if (kp * R > 2048) return NLSP_E_INVALID;  // LDS staging of the coarse vectors
  if (M->prec == NLSP_FP64 ? !M->Q64 : (M->prec == NLSP_MIXED ? !M->Q32 : true))
    return NLSP_E_INVALID;
  if (!(opts->rtol > 0) || opts->maxit < 1 || opts->check_every < 1) return NLSP_E_INVALID;
  if ((int64_t)M->k > n) return NLSP_E_INVALID;
  const int chunk_rows = NT / R;
  const int64_t nchunks = (n + chunk_rows - 1) / chunk_rows;
  const int nblk = solver_blocks(nchunks);
  const SolveLayout L0 = carve_solve(nullptr, n, kp, R, nblk);
  if (!ws_ok(ws, ws_bytes, L0.bytes)) return NLSP_E_WORKSPACE;
  const SolveLayout L = carve_solve(ws, n, kp, R, nblk);
  hipStream_t stream = as_stream(stream_);

  SysDev hs{};
  hs.op = make_op(*A);
  hs.R = R;
  hs.kp = kp;
  hs.nblk = nblk;
  hs.blk0 = 0;
  hs.chunk_rows = chunk_rows;
  hs.nchunks = nchunks;
  hs.Q = (M->prec == NLSP_FP64) ? (const void*)M->Q64 : (const void*)M->Q32;
  hs.Linv = M->Linv;
  hs.f = f;
  hs.x = u;
  hs.r = L.r;
  hs.p0 = L.p0;
  hs.p1 = L.p1;
  hs.q = L.q;
  hs.z = L.z;
  hs.w0 = L.w0;
  hs.w1 = L.w1;
  hs.dinv = L.dinv;
  hs.dinv32 = L.dinv32;
  hs.part = L.part;
  hs.pstride = kp * R + SL_COUNT * R;
  hs.nu = M->nu;
  hs.ticket = L.ticket;
  hs.st = L.st;
  hs.sys_active = L.counters + 1;
  hs.e = L.e;
  hs.omega = M->omega;
  hs.tol2 = opts->rtol * opts->rtol;
  hs.maxit = opts->maxit;
  hs.flexible = opts->flexible ? 1 : 0;

  std::vector<RhsState> st0(R);
  for (auto& s : st0) {
    s = RhsState{};
    s.gamma = 1.0;
    s.active = 0;
    s.status = NLSP_NOT_CONVERGED;
  }
  NLSP_HIP(hipMemsetAsync(L.p0, 0, sizeof(double) * n * R, stream));
  NLSP_HIP(hipMemsetAsync(L.p1, 0, sizeof(double) * n * R, stream));
  NLSP_HIP(hipMemsetAsync(L.z, 0, sizeof(double) * n * R, stream));
  NLSP_HIP(hipMemsetAsync(L.ticket, 0, sizeof(unsigned) * 4, stream));
  NLSP_HIP(hipMemsetAsync(L.counters, 0, sizeof(int) * 4, stream));
  NLSP_HIP(hipMemcpyAsync(L.st, st0.data(), sizeof(RhsState) * R, hipMemcpyHostToDevice, stream));
  NLSP_HIP(hipMemcpyAsync(L.sysdev, &hs, sizeof(SysDev), hipMemcpyHostToDevice, stream));
  if (M->prec == NLSP_FP64) return run_pcg<double>(hs, L, R, opts, info, stream);
  return run_pcg<float>(hs, L, R, opts, info, stream);
}

}  // extern "C"
