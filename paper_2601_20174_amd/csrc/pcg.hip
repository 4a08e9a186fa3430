// Preconditioned conjugate gradients with the spectral two-level
// preconditioner (Sec. 4.1 two-grid solver evaluation; the algorithm's
// preconditioner application), gfx950.
//
// Preconditioner.  For nu1 = nu2 = nu sweeps of weighted Jacobi the two-grid
// operator of the algorithm is, exactly,
//     M^-1 r = J_{2nu} r + Q A_c^-1 Q^T r,     Q = (I - w D^-1 A)^nu P,
// (J_{2nu} r = 2nu Jacobi sweeps on A z = r from z = 0).  Q and the inverse
// Cholesky factor of A_c come from galerkin_coarse.  For nu = 1,
// J_2 r = 2w D^-1 r - w^2 D^-1 A D^-1 r needs one stencil pass.
//
// One iteration = two kernels and two grid reductions.  The restriction is
// linear, so Q^T r_new = Q^T r - alpha Q^T q: kernel A restricts q instead of
// the new residual, and the residual update, smoother and prolongation share
// kernel B without a grid synchronisation between them.
//   kernel A  convergence test of r; beta; p <- z + beta p (double buffer);
//             q = A p; partials p^T q and Q^T q
//   kernel B  alpha; c <- c - alpha Q^T q; e = A_c^-1 c; x += alpha p;
//             r_new = r - alpha q (double buffer); z = J r_new + Q e;
//             partials r^T z, r^T z_old, ||r||^2
// Grid reductions are finished by the consumer: every workgroup of the next
// kernel sums the per-workgroup partials it needs in a fixed order (so all
// workgroups obtain bit-identical scalars and runs are reproducible), while its
// own loads are in flight.  Only Q^T q (k values per RHS) is pre-summed by the
// last workgroup of each group of 16 inside kernel A (and, for large k*R,
// once more by the last group).  The per-RHS state is double-buffered by
// iteration parity: iteration `it` reads stat[it & 1] and only workgroup 0 of
// kernel B writes stat[(it + 1) & 1].
// Vectors and every reduction are float64; in the mixed form Q, the smoother
// and the prolongation products are float32.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <vector>

#include <hip/hip_ext.h>

#include "device_common.hpp"
#include "host_common.hpp"

namespace nlsp {

constexpr int NT = 512;   // threads per workgroup of the solver kernels
constexpr int MAXR = 16;  // right-hand sides per solve

struct RhsStatus {
  double gamma_old;  // r^T z of the previous iteration (beta's denominator)
  double ff;         // ||f||^2
  int active;        // still iterating
  int iters;         // updates of x completed
  int status;        // nlsp_status of this RHS
  int par;           // p buffer holding the current direction
  int restart;       // next kernel A uses beta = 0
  int conv;          // stopped by the recursive residual test (true residual pending)
  int pad0, pad1;
};

struct SysDev {
  OpDev op;
  int R, kp, nblk, blk0;
  int chunk_rows;          // rows per chunk: floor(NT / R); threads past chunk_rows*R idle
  int64_t nchunks;
  int64_t cpb;             // chunks per workgroup: ceil(nchunks / nblk)
  int rw;                  // restriction record width: kp*R + 2R
  const void* Q;           // (n, kp), float or double
  const double* Linv;      // (kp, kp) inverse Cholesky factor of A_c
  const double* Ainv;      // (kp, kp) = L^-T L^-1
  const double* f;
  double* x;
  double* r[2];            // residual, by iteration parity
  double* p[2];            // search direction, by RhsStatus::par
  double* q;
  double* z;
  void* w[2];              // J_{2nu} r work buffers (nu > 1), element type of Q
  const double* dinv;
  const float* dinv32;
  double* bpart[2];        // [nblk][3R]  kernel-B partials [r^T z | r^T z_old | ||r||^2], by parity
  double* rpart;           // [nblk][rw]  restriction records [Q^T v | v-scalar | ||f||^2]
  double* rgrp;            // [ngrp][rw]  group records
  double* estate[2];       // [kp*R]      e = A_c^-1 Q^T r by parity
  double* dpart;           // [nblk][R]   true-residual partials
  unsigned* ticket;        // ticket_words(nblk)
  RhsStatus* stat[2];      // [R] each
  int* nact;               // [2] active RHS in the stat buffer of that parity
  int* n_active;           // host-visible copy
  double* rr_true;         // [R]
  double omega, tol2;
  int maxit, flexible, nu;
  unsigned rmask;          // RHS a restart launch applies to (ANDed with the launch mask)
};

// XCD-aware order: hardware places workgroup b on XCD b % 8; give each XCD a
// contiguous range of logical blocks so that stencil halos are served from
// that XCD's L2.
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

// ------------------------------------------------------------- reductions
// In-place tree sum over "rows" of an LDS array laid out as sh[row*W + col]
// (rows 0..nrows-1, W columns): on return sh[col] holds the column sums.
// Pairing is fixed (row r with row r + h), so the result is deterministic.
// All threads call; contains __syncthreads.
NLSP_DEV void lds_tree_rows(double* sh, int nrows, int W) {
  __syncthreads();
  while (nrows > 1) {
    const int h = (nrows + 1) / 2;
    for (int idx = threadIdx.x; idx < (nrows - h) * W; idx += NT) sh[idx] += sh[idx + h * W];
    __syncthreads();
    nrows = h;
  }
}

NLSP_DEV bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// R a power of two <= 64: butterflies inside each wave over the lanes that
// share c = lane % R, then the wave totals in wave order (one barrier round).
// K values per thread; totals to red[k*R + c].  `sh` holds >= 8 K R doubles.
template <int K>
NLSP_DEV void block_sum_waves(const double (&v0)[K], int R, double* red, double* sh) {
  constexpr int NW = NT / WAVE;
  double v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = v0[k];
  for (int o = WAVE / 2; o >= R; o >>= 1)
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += __shfl_xor(v[k], o, WAVE);
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  __syncthreads();
  if (lane < R)
#pragma unroll
    for (int k = 0; k < K; ++k) sh[(w * K + k) * R + lane] = v[k];
  __syncthreads();
  if (threadIdx.x < K * R) {
    const int k = threadIdx.x / R, c = threadIdx.x % R;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < NW; ++q) s += sh[(q * K + k) * R + c];
    red[threadIdx.x] = s;
  }
  __syncthreads();
}

// Sum of per-thread values over the threads that share c = t % R; the totals
// land in red[c] (LDS) for c < R.  Deterministic.  All threads call.
// `sh` holds NT + 16 doubles.
NLSP_DEV void block_sum_rhs(double v, int R, double* red, double* sh) {
  if (pow2(R) && R <= WAVE) {
    const double vv[1] = {v};
    block_sum_waves<1>(vv, R, red, sh);
    return;
  }
  const int t = threadIdx.x;
  const int nrows = (NT + R - 1) / R;
  __syncthreads();
  sh[t] = v;
  if (t < nrows * R - NT) sh[NT + t] = 0.0;   // pad the last partial row
  lds_tree_rows(sh, nrows, R);
  if (t < R) red[t] = sh[t];
  __syncthreads();
}

// Sum of `count` consecutive slots starting at `off` over `nrec` records of
// `stride` doubles at `base`, in ascending record order per thread and a fixed
// tree across threads; result in out[0..count) (LDS).  COHERENT selects
// device-coherent loads (records written earlier in the same kernel by other
// workgroups); plain loads serve records from a previous kernel.  Loads are
// issued in batches so their latencies overlap.  All threads call.
template <bool COHERENT>
NLSP_DEV void sum_records(const double* base, int nrec, int stride, int off, int count, double* out,
                          double* sh) {
  constexpr int B = 8;
  const int t = threadIdx.x;
  for (int c0 = 0; c0 < count; c0 += NT) {
    const int cnt = min(NT, count - c0);
    const int groups = NT / cnt;               // >= 1
    const int e = t % cnt, g = t / cnt;
    double s = 0.0;
    if (g < groups) {
      for (int r0 = g; r0 < nrec; r0 += B * groups) {
        double v[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
          const int r = r0 + u * groups;
          const double* a = &base[(int64_t)r * stride + off + c0 + e];
          v[u] = (r < nrec) ? (COHERENT ? load_partial(a) : *a) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < B; ++u) s += v[u];
      }
    }
    __syncthreads();
    sh[t] = (g < groups) ? s : 0.0;
    lds_tree_rows(sh, groups, cnt);
    if (t < cnt) out[c0 + t] = sh[t];
    __syncthreads();
  }
}

// Small reductions split in two so that their loads can be issued before a
// large prefetch (vector loads of a wave complete in issue order): rec_issue
// loads the records a thread sums (at most 8; the caller checks rec_fits),
// rec_finish adds them in ascending record order and across threads with a
// fixed tree.  Same result as sum_records.
NLSP_DEV bool rec_fits(int nrec, int count) { return count <= NT && nrec <= 8 * (NT / count); }

template <bool COHERENT>
NLSP_DEV void rec_issue(const double* base, int nrec, int stride, int off, int count, double (&v)[8]) {
  const int t = threadIdx.x;
  const int groups = NT / count, e = t % count, g = t / count;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int r = g + u * groups;
    const double* a = &base[(int64_t)r * stride + off + e];
    v[u] = (g < groups && r < nrec) ? (COHERENT ? load_partial(a) : *a) : 0.0;
  }
}

NLSP_DEV void rec_finish(const double (&v)[8], int count, double* out, double* sh) {
  const int t = threadIdx.x;
  const int groups = NT / count, g = t / count;
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < 8; ++u) s += v[u];
  __syncthreads();
  sh[t] = (g < groups) ? s : 0.0;
  lds_tree_rows(sh, groups, count);
  if (t < count) out[t] = sh[t];
  __syncthreads();
}

// e = A_c^-1 c for every RHS: c in LDS (kp*R, layout j*R + r), result to
// eout (LDS or global, same layout).  Thread t takes row i = t / SL of A_c^-1
// and the column slice js = t % SL (SL consecutive lanes), all R right-hand
// sides at once; the slices are added with butterflies.
// The first 8 entries of this thread's row slice of A_c^-1, loaded ahead of
// coarse_apply so that their latency overlaps other waits.
NLSP_DEV void coarse_prefetch(const double* __restrict__ Ainv, int kp, double (&a)[8]) {
  const int t = threadIdx.x;
  const int SL = min(NT / kp, kp);
  const int i = t / SL, js = t % SL;
  const int len = kp / SL;
  const double* row = Ainv + (int64_t)(i < kp ? i : 0) * kp + js * len;
#pragma unroll
  for (int u = 0; u < 8; ++u) a[u] = (u < len) ? row[u] : 0.0;
}

NLSP_DEV void coarse_apply(const double* __restrict__ Ainv, int kp, int R, const double* cvec,
                           double* eout, const double* pre = nullptr) {
  const int t = threadIdx.x;
  const int SL = min(NT / kp, kp);            // lanes per row (power of two, <= kp)
  const int i = t / SL, js = t % SL;
  const int len = kp / SL;                    // >= 1
  const bool on = i < kp;                     // threads past kp*SL are idle
  double acc[MAXR];
#pragma unroll
  for (int r = 0; r < MAXR; ++r) acc[r] = 0.0;
  const double* row = Ainv + (int64_t)(on ? i : 0) * kp + js * len;
  for (int j0 = 0; on && j0 < len; j0 += 8) {
    double a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = (pre && j0 == 0) ? pre[u] : ((j0 + u < len) ? row[j0 + u] : 0.0);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (j0 + u >= len) break;
      const int j = js * len + j0 + u;
#pragma unroll
      for (int r = 0; r < MAXR; ++r)
        if (r < R) acc[r] += a[u] * cvec[j * R + r];
    }
  }
#pragma unroll
  for (int r = 0; r < MAXR; ++r) {
    if (r < R) {
      const double v = group_sum(acc[r], SL);
      if (on && js == 0) eout[i * R + r] = v;
    }
  }
}

// A_c^-1 = Linv^T Linv (kp x kp), once per solve
__global__ void k_coarse_inverse(const double* __restrict__ Linv, int kp, double* __restrict__ Ainv) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= kp * kp) return;
  const int i = idx / kp, j = idx % kp;
  double s = 0.0;
  for (int l = (i > j ? i : j); l < kp; ++l) s += Linv[l * kp + i] * Linv[l * kp + j];
  Ainv[idx] = s;
}

// ------------------------------------------------------------------ Q passes
// Thread t owns the 4-column chunk jc of right-hand side c in row group rg:
// t = jc + lpr*(c + R*rg), lpr = kp/4 lanes per row, so consecutive lanes read
// consecutive 16-byte pieces of a row of Q (coalesced) and the lanes of one
// row form an aligned group for butterflies.  Row group rg handles the chunk
// rows rg, rg + ngr, rg + 2 ngr, ...  kp*R <= 2048 keeps lpr*R <= NT.
struct QMap {
  int lpr, ngr, rg, jc, c;
  bool on;
};

NLSP_DEV QMap q_map(int kp, int R) {
  QMap m;
  const int t = threadIdx.x;
  m.lpr = kp / 4;
  const int pairs = m.lpr * R;
  m.ngr = NT / pairs;
  m.rg = t / pairs;
  const int pr = t % pairs;
  m.jc = pr % m.lpr;
  m.c = pr / m.lpr;
  m.on = m.rg < m.ngr;
  return m;
}

// rows handled by a thread in a chunk of nrows rows (uniform over the workgroup)
NLSP_DEV int q_trips(const QMap& m, int nrows) { return (nrows + m.ngr - 1) / m.ngr; }

// NB rows of Q for one thread, issued together so their latencies overlap
template <typename QT, int NB>
struct QBatch {
  QT v[NB][4];
};

template <typename QT, int NB>
NLSP_DEV void q_fetch(const QT* __restrict__ Q, int64_t row0, int nrows, int kp, const QMap& m,
                      int w0, QBatch<QT, NB>& b) {
#pragma unroll
  for (int w = 0; w < NB; ++w) {
    const int row = m.rg + (w0 + w) * m.ngr;
    if (m.on && row < nrows) {
      load4(Q + (row0 + row) * kp + 4 * m.jc, b.v[w]);
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) b.v[w][u] = QT(0);
    }
  }
}

// Restriction products are formed in float64 also when Q is stored in float32:
// Q^T r is carried by the recurrence c <- c - alpha Q^T q, whose absolute
// error must stay far below |Q^T r| as r shrinks by 1e-8 (float32 products
// would leave an error near 1e-7 |Q^T r_0|).  Storage, and so traffic, stay
// float32.
template <typename QT>
NLSP_DEV double prod(QT q, double r) {
  return (double)q * r;
}

// acc[u] += sum over the thread's chunk rows of Q[row][4 jc + u] * rv[row*R + c];
// `b` holds the first batch (fetched by the caller), later batches are fetched
// here.
template <typename QT, int NB>
NLSP_DEV void restrict_rows(const QT* __restrict__ Q, int64_t row0, int nrows, int kp, int R,
                            const QMap& m, const double* rv, QBatch<QT, NB>& b, double (&acc)[4]) {
  const int trips = q_trips(m, nrows);
  for (int w0 = 0; w0 < trips; w0 += NB) {
    if (w0 > 0) q_fetch<QT, NB>(Q, row0, nrows, kp, m, w0, b);
#pragma unroll
    for (int w = 0; w < NB; ++w) {
      const int row = m.rg + (w0 + w) * m.ngr;
      if (m.on && row < nrows) {
        const double r = rv[row * R + m.c];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] += prod<QT>(b.v[w][u], r);
      }
    }
  }
}

// Workgroup total of the restriction accumulators -> out[0 .. kp*R) (layout
// j*R + c) with device-coherent stores.  red: LDS of >= 4*NT doubles.
NLSP_DEV void restrict_finish(const QMap& m, int kp, int R, const double (&acc)[4], double* red,
                              double* out) {
  const int KR = kp * R;
  const int pairs = m.lpr * R;                 // lanes of one row group
  if (pow2(pairs) && pairs <= WAVE && (NT / WAVE) * KR <= 4 * NT + 128) {
    // the row groups inside a wave add with butterflies (lanes xor pairs, ...),
    // then the 8 wave totals in wave order
    double v[4] = {acc[0], acc[1], acc[2], acc[3]};
    for (int o = WAVE / 2; o >= pairs; o >>= 1)
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] += __shfl_xor(v[u], o, WAVE);
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    __syncthreads();
    if (lane < pairs)
#pragma unroll
      for (int u = 0; u < 4; ++u) red[w * KR + (4 * m.jc + u) * R + m.c] = v[u];
    __syncthreads();
    for (int idx = threadIdx.x; idx < KR; idx += NT) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < NT / WAVE; ++q) s += red[q * KR + idx];
      store_partial(&out[idx], s);
    }
    return;
  }
  __syncthreads();
  if (m.on) {
#pragma unroll
    for (int u = 0; u < 4; ++u) red[m.rg * KR + (4 * m.jc + u) * R + m.c] = acc[u];
  }
  lds_tree_rows(red, m.ngr, KR);
  for (int idx = threadIdx.x; idx < KR; idx += NT) store_partial(&out[idx], red[idx]);
}

// ys[row*R + c] = sum_j Q[row][j] e[j][c] for the chunk rows (prolongation),
// arithmetic in QT; the lpr lanes of a row add with butterflies.  All lanes
// run the same trip count (shuffles need the whole wave).
template <typename QT, int NB>
NLSP_DEV void prolong_rows(const QT* __restrict__ Q, int64_t row0, int nrows, int kp, int R,
                           const QMap& m, const QT (&e4)[4], QBatch<QT, NB>& b, QT* ys) {
  const int trips = q_trips(m, nrows);
  for (int w0 = 0; w0 < trips; w0 += NB) {
    if (w0 > 0) q_fetch<QT, NB>(Q, row0, nrows, kp, m, w0, b);
#pragma unroll
    for (int w = 0; w < NB; ++w) {
      if (w0 + w >= trips) break;
      const int row = m.rg + (w0 + w) * m.ngr;
      QT sdot = b.v[w][0] * e4[0] + b.v[w][1] * e4[1] + b.v[w][2] * e4[2] + b.v[w][3] * e4[3];
      sdot = group_sum(sdot, m.lpr);
      if (m.jc == 0 && m.on && row < nrows) ys[row * R + m.c] = sdot;
    }
  }
}

template <typename QT>
struct QB {
  static constexpr int NB = (sizeof(QT) == 4) ? 6 : 4;  // no spills at 128 VGPRs
};

struct ChunkRange {
  int64_t c0, c1;
};

NLSP_DEV ChunkRange my_chunks(const SysDev& S, int lb) {
  ChunkRange cr;
  cr.c0 = (int64_t)lb * S.cpb;
  cr.c1 = min(S.nchunks, cr.c0 + S.cpb);
  return cr;
}

// Restriction epilogue (kernel A and k_residual): this workgroup's record
// [Q^T v | s1 | s2] (already in rpart) is summed per group of 16 by the
// group's last workgroup into rgrp.  The next kernel sums the group records
// in order and applies A_c^-1 itself, so this kernel ends one ticket level
// earlier.
NLSP_DEV void restriction_epilogue(const SysDev& S, int lb, double* red, double* sh) {
  if (!arrive_group(S.ticket, S.nblk, lb)) return;
  const int grp = lb / TICKET_GROUP;
  const int r0 = grp * TICKET_GROUP;
  const int nrec = min(TICKET_GROUP, S.nblk - r0);
  sum_records<true>(S.rpart + (int64_t)r0 * S.rw, nrec, S.rw, 0, S.rw, red, sh);
  double* grec = S.rgrp + (int64_t)grp * S.rw;
  for (int idx = threadIdx.x; idx < S.rw; idx += NT) store_partial(&grec[idx], red[idx]);
}

// ----------------------------------------------------- per-iteration scalars
// What every workgroup of kernels A and B derives from kernel B's partials of
// the previous iteration: r^T z, r^T z_old and ||r||^2 of the current residual,
// the convergence test and whether the direction is updated.
struct IterScalars {
  double gam[MAXR], rzo[MAXR], rr[MAXR], beta[MAXR];
  int conv[MAXR];       // ||r|| <= rtol ||f||
  int act[MAXR];        // direction and q computed this iteration
  int bad[MAXR];        // r^T z not positive / not finite, or ||r|| not finite
};

NLSP_DEV bool finite_pos(double v) { return v > 0.0 && v <= 1.7e308; }

// Loads of kernel B's partials [r^T z | r^T z_old | ||r||^2] of iteration it,
// issued early (see rec_issue); `fast` is false when they do not fit.
// With R <= 4 (3R <= 12) and at most NT records, thread t loads record t
// whole (`tiny`) and the records are added with butterflies; otherwise
// rec_issue/rec_finish, or sum_records when that does not fit either.  The
// per-RHS status is loaded here too, by threads t < R.
struct ScalarLoads {
  double v[12];
  bool fast, tiny;
  RhsStatus st;
};

NLSP_DEV void scalars_issue(const SysDev& S, int it, ScalarLoads& L) {
  const int R = S.R, t = threadIdx.x;
  L.tiny = (R <= 4 && pow2(R) && S.nblk <= NT);
  L.fast = !L.tiny && rec_fits(S.nblk, 3 * R);
  if (L.tiny) {
    const double* rec = S.bpart[it & 1] + (int64_t)min(t, S.nblk - 1) * 3 * R;
#pragma unroll
    for (int j = 0; j < 12; ++j) L.v[j] = (j < 3 * R && t < S.nblk) ? rec[j] : 0.0;
  } else if (L.fast) {
    double v8[8];
    rec_issue<false>(S.bpart[it & 1], S.nblk, 3 * R, 0, 3 * R, v8);
#pragma unroll
    for (int j = 0; j < 8; ++j) L.v[j] = v8[j];
  }
  if (t < R) L.st = S.stat[it & 1][t];
}

NLSP_DEV void scalars_finish(const SysDev& S, const RhsStatus* cur, const ScalarLoads& L,
                             IterScalars& sc, double* buf, double* sh, int it) {
  const int R = S.R;
  if (L.tiny) {
    // all 64 lanes of a wave hold different records: full butterflies per value
    constexpr int NW = NT / WAVE;
    double v[12];
#pragma unroll
    for (int j = 0; j < 12; ++j) v[j] = L.v[j];
#pragma unroll
    for (int j = 0; j < 12; ++j)
      if (j < 3 * R)   // uniform
#pragma unroll
        for (int o = WAVE / 2; o >= 1; o >>= 1) v[j] += __shfl_xor(v[j], o, WAVE);
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    __syncthreads();
    if (lane == 0)
#pragma unroll
      for (int j = 0; j < 12; ++j)
        if (j < 3 * R) sh[w * 3 * R + j] = v[j];
    __syncthreads();
    if (threadIdx.x < 3 * R) {
      double a = 0.0;
#pragma unroll
      for (int q = 0; q < NW; ++q) a += sh[q * 3 * R + threadIdx.x];
      buf[threadIdx.x] = a;
    }
    __syncthreads();
  } else if (L.fast) {
    double v8[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v8[j] = L.v[j];
    rec_finish(v8, 3 * R, buf, sh);
  } else {
    sum_records<false>(S.bpart[it & 1], S.nblk, 3 * R, 0, 3 * R, buf, sh);
  }
  if (threadIdx.x < R) {
    const int c = threadIdx.x;
    const RhsStatus& st = L.st;
    const double g = buf[c], rz = buf[R + c], rr = buf[2 * R + c];
    sc.gam[c] = g;
    sc.rzo[c] = rz;
    sc.rr[c] = rr;
    const int rr_ok = rr <= 1.7e308;                       // false for NaN / Inf
    sc.conv[c] = st.active && rr_ok && rr <= S.tol2 * st.ff;
    sc.bad[c] = st.active && !sc.conv[c] && (!rr_ok || !finite_pos(g));
    sc.act[c] = st.active && !sc.conv[c] && !sc.bad[c] && st.iters < S.maxit;
    double beta = 0.0;
    if (!st.restart && sc.act[c])
      beta = S.flexible ? (g - rz) / st.gamma_old : g / st.gamma_old;
    sc.beta[c] = beta;
  }
  __syncthreads();
}

// Sum over the threads sharing c = t % R of three values at once: the totals
// land in red[k*R + c], k < 3.  One tree instead of three.  `sh` holds
// 3*(NT + 16) doubles.
NLSP_DEV void block_sum_rhs3(double a, double b, double d, int R, double* red, double* sh) {
  if (pow2(R) && R <= WAVE) {
    const double vv[3] = {a, b, d};
    block_sum_waves<3>(vv, R, red, sh);
    return;
  }
  const int t = threadIdx.x;
  const int nrows = (NT + R - 1) / R;
  __syncthreads();
  // row-major [row][3R]: thread t = row*R + c
  const int row = t / R, c = t % R;
  sh[row * 3 * R + c] = a;
  sh[row * 3 * R + R + c] = b;
  sh[row * 3 * R + 2 * R + c] = d;
  if (t < nrows * R - NT) {   // pad the last partial row
    const int pr = (NT + t) / R, pc = (NT + t) % R;
    sh[pr * 3 * R + pc] = 0.0;
    sh[pr * 3 * R + R + pc] = 0.0;
    sh[pr * 3 * R + 2 * R + pc] = 0.0;
  }
  lds_tree_rows(sh, nrows, 3 * R);
  if (t < 3 * R) red[t] = sh[t];
  __syncthreads();
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

// r = f - A x into `rout` for the RHS in `mask` (others untouched);
// restriction records [Q^T r | ||r||^2 | ||f||^2], then the group (and top)
// epilogue.  Used at start-up and for residual replacement.
template <typename QT>
__global__ __launch_bounds__(NT, 4) void k_residual(const SysDev* __restrict__ sys,
                                                    const int* __restrict__ blk2sys, int nsys,
                                                    unsigned mask, int rout) {
  __shared__ double rv[NT];
  __shared__ double sh[NT + 16];
  __shared__ double red[4 * NT + 128];
  __shared__ double outv[MAXR];
  const SysDev& S = my_sys(sys, blk2sys, nsys);
  mask &= S.rmask;
  const int lb = xcd_remap(blockIdx.x - S.blk0, S.nblk);
  const int t = threadIdx.x, R = S.R, c = t % R;
  const bool on = (mask >> c) & 1u;
  const QT* Q = static_cast<const QT*>(S.Q);
  const QMap m = q_map(S.kp, R);
  constexpr int NB = QB<QT>::NB;
  QBatch<QT, NB> qb;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  double rr = 0.0, ff = 0.0;
  double* Rout = S.r[rout];
  const ChunkRange cr = my_chunks(S, lb);
  for (int64_t ch = cr.c0; ch < cr.c1; ++ch) {
    const int64_t row0 = ch * S.chunk_rows;
    const int nrows = (int)min<int64_t>(S.chunk_rows, S.op.n - row0);
    q_fetch<QT, NB>(Q, row0, nrows, S.kp, m, 0, qb);
    const int64_t i = row0 + t / R;
    double rvv = 0.0;
    if (on && t / R < nrows) {
      int px, py, pz;
      decompose(S.op, i, px, py, pz);
      const double* X = S.x;
      const double ax = op_row<double>(S.op, i, px, py, pz, [&](int64_t j) { return X[j * R + c]; });
      const double fi = S.f[i * R + c];
      rvv = fi - ax;
      Rout[i * R + c] = rvv;
      rr += rvv * rvv;
      ff += fi * fi;
    }
    __syncthreads();
    rv[t] = rvv;
    __syncthreads();
    restrict_rows<QT, NB>(Q, row0, nrows, S.kp, R, m, rv, qb, acc);
  }
  double* rec = S.rpart + (int64_t)lb * S.rw;
  restrict_finish(m, S.kp, R, acc, red, rec);
  const int KR = S.kp * R;
  block_sum_rhs(rr, R, outv, sh);
  if (t < R) store_partial(&rec[KR + t], outv[t]);
  block_sum_rhs(ff, R, outv, sh);
  if (t < R) store_partial(&rec[KR + R + t], outv[t]);
  restriction_epilogue(S, lb, red, sh);
}

// kernel A: convergence test; beta; p_new = z + beta p_old (double buffer);
// q = A p_new; restriction records [Q^T q | p^T q | 0], summed per group of 16
// workgroups by the epilogue
template <typename QT>
__global__ __launch_bounds__(NT, 4) void k_iter_a(const SysDev* __restrict__ sys,
                                                  const int* __restrict__ blk2sys, int nsys, int it) {
  __shared__ double qv[NT];
  __shared__ double sh[NT + 16];
  __shared__ double red[4 * NT + 128];
  __shared__ double buf[4 * MAXR];
  __shared__ IterScalars sc;
  const SysDev& S = my_sys(sys, blk2sys, nsys);
  const int lb = xcd_remap(blockIdx.x - S.blk0, S.nblk);
  const int t = threadIdx.x, R = S.R, c = t % R;
  const QT* Q = static_cast<const QT*>(S.Q);
  const QMap m = q_map(S.kp, R);
  constexpr int NB = QB<QT>::NB;
  QBatch<QT, NB> qb;
  const ChunkRange cr = my_chunks(S, lb);
  const RhsStatus* cur = S.stat[it & 1];
  ScalarLoads sl;
  scalars_issue(S, it, sl);                                   // small loads first,
  int64_t row0 = cr.c0 * S.chunk_rows;
  int nrows = (cr.c0 < cr.c1) ? (int)min<int64_t>(S.chunk_rows, S.op.n - row0) : 0;
  if (cr.c0 < cr.c1) q_fetch<QT, NB>(Q, row0, nrows, S.kp, m, 0, qb);  // then Q,
  if (S.nact[it & 1] == 0) return;                            // then the early exit
  scalars_finish(S, cur, sl, sc, buf, sh, it);
  const bool act = sc.act[c] != 0;
  const double beta = sc.beta[c];
  const int par = cur[c].par;
  const double* pold = S.p[par];
  double* pnew = S.p[par ^ 1];
  const double* Z = S.z;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  double dp = 0.0;
  for (int64_t ch = cr.c0; ch < cr.c1; ++ch) {
    if (ch > cr.c0) {
      row0 = ch * S.chunk_rows;
      nrows = (int)min<int64_t>(S.chunk_rows, S.op.n - row0);
      q_fetch<QT, NB>(Q, row0, nrows, S.kp, m, 0, qb);
    }
    double qval = 0.0;
    if (act && t / R < nrows) {
      const int64_t i = row0 + t / R;
      int px, py, pz;
      decompose(S.op, i, px, py, pz);
      auto pn = [&](int64_t j) { return Z[j * R + c] + beta * pold[j * R + c]; };
      const double pi = pn(i);
      qval = op_row<double>(S.op, i, px, py, pz, pn);
      pnew[i * R + c] = pi;
      S.q[i * R + c] = qval;
      dp += pi * qval;
    }
    __syncthreads();
    qv[t] = qval;
    __syncthreads();
    restrict_rows<QT, NB>(Q, row0, nrows, S.kp, R, m, qv, qb, acc);
  }
  double* rec = S.rpart + (int64_t)lb * S.rw;
  restrict_finish(m, S.kp, R, acc, red, rec);
  const int KR = S.kp * R;
  block_sum_rhs(dp, R, buf, sh);
  if (t < R) {
    store_partial(&rec[KR + t], buf[t]);
    store_partial(&rec[KR + R + t], 0.0);
  }
  restriction_epilogue(S, lb, red, sh);
}

// J_{2nu} sweeps for nu > 1 on the new residual r_new = r_in - a q (a = alpha,
// or 0 at a restart): first = 1 computes y2 = y1 + w D^-1 (r_new - A y1) with
// y1 = w D^-1 r_new; later sweeps y <- y + w D^-1 (r_new - A y).  Every RHS
// still marked active in stat[it & 1] is swept.
template <typename PT>
__global__ __launch_bounds__(NT) void k_sweep(const SysDev* __restrict__ sys,
                                              const int* __restrict__ blk2sys, int nsys, int it,
                                              int restart, int rin, int first, int src) {
  __shared__ double sh[NT + 16];
  __shared__ double buf[4 * MAXR];
  __shared__ double s_alpha[MAXR];
  __shared__ IterScalars sc;
  const SysDev& S = my_sys(sys, blk2sys, nsys);
  if (!restart && S.nact[it & 1] == 0) return;
  const int lb = xcd_remap(blockIdx.x - S.blk0, S.nblk);
  const int t = threadIdx.x, R = S.R, c = t % R;
  const RhsStatus* cur = S.stat[it & 1];
  if (!restart) {
    ScalarLoads sl;
    scalars_issue(S, it, sl);
    scalars_finish(S, cur, sl, sc, buf, sh, it);
    if (t < R) {
      double pq = 0.0;   // p^T q: entry kp R + t of the group records, in order
      for (int g = 0; g < ticket_groups(S.nblk); ++g) pq += S.rgrp[(int64_t)g * S.rw + S.kp * R + t];
      s_alpha[t] = sc.gam[t] / pq;
    }
  } else if (t < R) {
    s_alpha[t] = 0.0;
  }
  __syncthreads();
  if (!cur[c].active) return;
  const PT om = PT(S.omega);
  const double a = s_alpha[c];
  const double* Rin = S.r[rin];
  const double* Qv = S.q;
  auto rnew = [&](int64_t j) { return Rin[j * R + c] - a * Qv[j * R + c]; };
  const PT* yin = static_cast<const PT*>(S.w[src]);
  PT* yout = static_cast<PT*>(S.w[first ? 0 : (src ^ 1)]);
  const ChunkRange cr = my_chunks(S, lb);
  for (int64_t ch = cr.c0; ch < cr.c1; ++ch) {
    const int64_t i = ch * S.chunk_rows + t / R;
    if (t / R >= S.chunk_rows || i >= S.op.n) continue;
    int px, py, pz;
    decompose(S.op, i, px, py, pz);
    auto dj = [&](int64_t j) -> PT { return (sizeof(PT) == 4) ? PT(S.dinv32[j]) : PT(S.dinv[j]); };
    const PT ri = PT(rnew(i));
    PT yi, ay;
    if (first) {
      auto y1 = [&](int64_t j) { return om * dj(j) * PT(rnew(j)); };
      yi = y1(i);
      ay = op_row<PT>(S.op, i, px, py, pz, y1);
    } else {
      yi = yin[i * R + c];
      ay = op_row<PT>(S.op, i, px, py, pz, [&](int64_t j) { return yin[j * R + c]; });
    }
    yout[i * R + c] = yi + om * dj(i) * (ri - ay);
  }
}

// kernel B: status; alpha; e <- e - alpha A_c^-1 Q^T q (so e = A_c^-1 Q^T r_new);
// x += alpha p; r_new = r - alpha q into r[(it+1)&1]; z = J r_new + Q e;
// partials [r^T z | r^T z_old | ||r_new||^2] into bpart[(it+1)&1].
//   restart = 0: an iteration; group records [Q^T q | p^T q | 0] from kernel A
//   restart = 1: after k_residual (which wrote r into r[(it+1)&1] and group
//                records [Q^T r | ||r||^2 | ||f||^2]) for the RHS in
//                `mask`: no update, `init` also takes ||f||^2, and the next
//                kernel A uses beta = 0.
// wsrc < 0: J_2 inline (nu = 1); else J_{2nu} r_new is read from w[wsrc].
template <typename QT>
__global__ __launch_bounds__(NT, 4) void k_iter_b(const SysDev* __restrict__ sys,
                                                  const int* __restrict__ blk2sys, int nsys, int it,
                                                  int restart, unsigned mask, int init, int wsrc) {
  __shared__ QT ws[NT];
  __shared__ QT ys[NT];
  __shared__ double sh[3 * (NT + 16)];
  __shared__ double ebuf[2048];
  __shared__ double dq[2048];
  __shared__ double cg[2048 + 2 * MAXR];
  __shared__ double tscal[2 * MAXR];
  __shared__ double buf[4 * MAXR];
  __shared__ double s_alpha[MAXR];
  __shared__ int s_upd[MAXR], s_next[MAXR];
  __shared__ IterScalars sc;
  const SysDev& S = my_sys(sys, blk2sys, nsys);
  mask &= S.rmask;
  const int nxt = (it + 1) & 1;
  const int KR = S.kp * S.R;
  if (!restart && S.nact[it & 1] == 0) {
    // nothing iterates: carry the state over to the next parity
    if (blockIdx.x == S.blk0) {
      for (int idx = threadIdx.x; idx < KR; idx += NT) S.estate[nxt][idx] = S.estate[it & 1][idx];
      if (threadIdx.x < S.R) S.stat[nxt][threadIdx.x] = S.stat[it & 1][threadIdx.x];
      if (threadIdx.x == 0) {
        S.nact[nxt] = 0;
        *S.n_active = 0;
      }
    }
    return;
  }
  const int lb = xcd_remap(blockIdx.x - S.blk0, S.nblk);
  const int t = threadIdx.x, R = S.R, c = t % R;
  const QT* Q = static_cast<const QT*>(S.Q);
  const QMap m = q_map(S.kp, R);
  constexpr int NB = QB<QT>::NB;
  QBatch<QT, NB> qb;
  const ChunkRange cr = my_chunks(S, lb);
  const RhsStatus* cur = S.stat[it & 1];
  // small loads first (scalars, the restriction's group records, e), then Q
  ScalarLoads sl;
  sl.fast = sl.tiny = false;
  if (!restart) scalars_issue(S, it, sl);
  const int ngrp = ticket_groups(S.nblk);
  const bool gfast = rec_fits(ngrp, S.rw);
  double gv[8], av[8];
  if (gfast) rec_issue<false>(S.rgrp, ngrp, S.rw, 0, S.rw, gv);
  coarse_prefetch(S.Ainv, S.kp, av);
  for (int idx = t; idx < KR; idx += NT) ebuf[idx] = S.estate[it & 1][idx];
  int64_t row0 = cr.c0 * S.chunk_rows;
  int nrows = (cr.c0 < cr.c1) ? (int)min<int64_t>(S.chunk_rows, S.op.n - row0) : 0;
  if (cr.c0 < cr.c1) q_fetch<QT, NB>(Q, row0, nrows, S.kp, m, 0, qb);
  if (!restart) scalars_finish(S, cur, sl, sc, buf, sh, it);
  // c = [Q^T v | s1 | s2] summed over the groups in order (v = q, or r after
  // k_residual), then dq = A_c^-1 Q^T v
  if (gfast)
    rec_finish(gv, S.rw, cg, sh);
  else
    sum_records<false>(S.rgrp, ngrp, S.rw, 0, S.rw, cg, sh);
  coarse_apply(S.Ainv, S.kp, R, cg, dq, av);
  if (t < 2 * R) tscal[t] = cg[KR + t];
  __syncthreads();
  if (restart)
    for (int idx = t; idx < KR; idx += NT)
      if ((mask >> (idx % R)) & 1u) ebuf[idx] = dq[idx];
  __syncthreads();
  // ---- per-RHS decisions (identical in every workgroup) and the new state
  if (t < R) {
    RhsStatus nx = cur[t];
    int upd = 0, next = 0;
    double alpha = 0.0;
    if (restart) {
      if ((mask >> t) & 1u) {
        if (init) nx.ff = tscal[R + t];
        nx.restart = 1;
        nx.conv = 0;
        if (!(nx.ff <= 1.7e308)) {
          nx.status = NLSP_E_NONFINITE;
        } else {
          nx.status = NLSP_NOT_CONVERGED;
          next = 1;
        }
      } else {
        next = nx.active;
      }
      upd = next && ((mask >> t) & 1u);
    } else if (cur[t].active) {
      nx.restart = 0;
      if (sc.conv[t]) {
        nx.status = NLSP_OK;
        nx.conv = 1;
      } else if (sc.bad[t]) {
        // r^T z <= 0 with finite values is a breakdown; anything non-finite is not
        const bool gfin = sc.gam[t] == sc.gam[t] && fabs(sc.gam[t]) <= 1.7e308;
        const bool rfin = sc.rr[t] <= 1.7e308;
        nx.status = (gfin && rfin) ? NLSP_E_BREAKDOWN : NLSP_E_NONFINITE;
      } else if (!sc.act[t]) {
        nx.status = NLSP_NOT_CONVERGED;   // maxit reached
      } else {
        const double d = tscal[t];
        nx.par ^= 1;                      // kernel A wrote the new direction
        nx.gamma_old = sc.gam[t];
        if (!finite_pos(d)) {
          nx.status = (d == d && d <= 1.7e308) ? NLSP_E_BREAKDOWN : NLSP_E_NONFINITE;
        } else {
          alpha = sc.gam[t] / d;
          upd = 1;
          next = 1;
          nx.iters += 1;
        }
      }
    }
    nx.active = next;
    s_alpha[t] = alpha;
    s_upd[t] = upd;
    s_next[t] = next;
    if (lb == 0) S.stat[nxt][t] = nx;
  }
  __syncthreads();
  // ---- e = A_c^-1 Q^T r_new (workgroup 0 keeps it for the next iteration)
  if (!restart)
    for (int idx = t; idx < KR; idx += NT) ebuf[idx] -= s_alpha[idx % R] * dq[idx];
  __syncthreads();
  if (lb == 0) {
    for (int idx = t; idx < KR; idx += NT) S.estate[nxt][idx] = ebuf[idx];
    if (t == 0) {
      int cnt = 0;
      for (int k = 0; k < R; ++k) cnt += s_next[k];
      S.nact[nxt] = cnt;
      *S.n_active = cnt;
    }
  }
  // ---- x += alpha p; r_new = r - alpha q; z = J r_new + Q e
  const bool upd = s_upd[c] != 0;
  const double alpha = s_alpha[c];
  QT e4[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) e4[u] = QT(ebuf[(4 * m.jc + u) * R + m.c]);
  const QT om = QT(S.omega);
  const double* Rin = S.r[restart ? nxt : (it & 1)];
  double* Rout = S.r[nxt];
  const double* Qv = S.q;
  const double* P = S.p[cur[c].par ^ 1];
  auto rnew = [&](int64_t j) { return restart ? Rin[j * R + c] : Rin[j * R + c] - alpha * Qv[j * R + c]; };
  double gam = 0.0, rzo = 0.0, rr = 0.0;
  for (int64_t ch = cr.c0; ch < cr.c1; ++ch) {
    if (ch > cr.c0) {
      row0 = ch * S.chunk_rows;
      nrows = (int)min<int64_t>(S.chunk_rows, S.op.n - row0);
      q_fetch<QT, NB>(Q, row0, nrows, S.kp, m, 0, qb);
    }
    const bool mine = upd && t / R < nrows;
    const int64_t i = row0 + t / R;
    QT w = QT(0);
    double ri = 0.0;
    if (mine) {
      ri = rnew(i);
      if (wsrc < 0) {
        int px, py, pz;
        decompose(S.op, i, px, py, pz);
        auto dj = [&](int64_t j) -> QT {
          return (sizeof(QT) == 4) ? QT(S.dinv32[j]) : QT(S.dinv[j]);
        };
        auto y = [&](int64_t j) { return dj(j) * QT(rnew(j)); };
        const QT yi = y(i);
        const QT ay = op_row<QT>(S.op, i, px, py, pz, y);
        w = QT(2) * om * yi - om * om * dj(i) * ay;
      } else {
        w = static_cast<const QT*>(S.w[wsrc])[i * R + c];
      }
    }
    __syncthreads();
    ws[t] = w;
    prolong_rows<QT, NB>(Q, row0, nrows, S.kp, R, m, e4, qb, ys);
    __syncthreads();
    if (mine) {
      const int64_t g = i * R + c;
      if (!restart) {
        S.x[g] += alpha * P[g];
        Rout[g] = ri;
      }
      const double zn = (double)ws[t] + (double)ys[t];
      if (S.flexible) rzo += ri * S.z[g];
      S.z[g] = zn;
      gam += ri * zn;
      rr += ri * ri;
    }
  }
  block_sum_rhs3(gam, rzo, rr, R, buf, sh);
  if (t < 3 * R) S.bpart[nxt][(int64_t)lb * 3 * R + t] = buf[t];
}

// ||f - A x||^2 partials per RHS (true residual) into dpart
__global__ __launch_bounds__(NT) void k_true_residual(const SysDev* __restrict__ sys,
                                                      const int* __restrict__ blk2sys, int nsys) {
  __shared__ double sh[NT + 16];
  __shared__ double buf[MAXR];
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
  block_sum_rhs(s, R, buf, sh);
  if (t < R) S.dpart[(int64_t)lb * R + t] = buf[t];
}

// one workgroup per system: rr_true = sum of the true-residual partials
__global__ __launch_bounds__(NT) void k_true_finish(const SysDev* __restrict__ sys) {
  __shared__ double sh[NT + 16];
  __shared__ double buf[MAXR];
  const SysDev& S = sys[blockIdx.x];
  sum_records<false>(S.dpart, S.nblk, S.R, 0, S.R, buf, sh);
  if (threadIdx.x < S.R) S.rr_true[threadIdx.x] = buf[threadIdx.x];
}

__global__ void k_zero_cols(double* u, int64_t n, int R, unsigned mask) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n * R) return;
  if ((mask >> (g % R)) & 1u) u[g] = 0.0;
}

// ------------------------------------------------------------- host side
// ------------------------------------------------------------------ host side
// Per-system buffers.  The arrays that must start at zero come first and are
// carved for every system of a batch before anything else, so one fill clears
// them all.
struct SolveLayout {
  double *p0, *p1, *q, *z, *estate0, *estate1;
  unsigned* ticket;
  double *r0, *r1, *dinv, *bpart0, *bpart1, *rpart, *rgrp, *dpart, *Ainv;
  float* dinv32;
  void *w0, *w1;
};

// Arrays shared by the systems of a batch (contiguous, so the host reads or
// writes them with one copy): per-RHS status by parity, true residuals,
// counters [nact(0), nact(1), active, -] per system, descriptors, block map.
struct BatchLayout {
  RhsStatus *stat0, *stat1;
  double* rr_true;
  int* counters;
  SysDev* sysdev;
  int* blk2sys;
  char* zero_begin;
  size_t zero_bytes;
  size_t bytes;
};

struct SysShape {
  int64_t n;
  int kp, R, nblk;
  int64_t nchunks;
  int chunk_rows;
};

// Workgroups per system: one per chunk of NT / R rows up to a cap (512 for a
// single system, NLSP_SOLVER_BLOCKS overrides it for tuning), or, in a batch,
// one per `rows_per_block` rows.
inline int solver_blocks(int64_t nchunks) {
  int cap = 512;
  if (const char* e = std::getenv("NLSP_SOLVER_BLOCKS")) {
    const int v = std::atoi(e);
    if (v >= 1 && v <= 65536) cap = v;
  }
  return (int)std::min<int64_t>(nchunks, cap);
}

inline int restriction_width(int kp, int R) { return kp * R + 2 * R; }

inline SysShape shape_of(int64_t n, int kp, int R, int rows_per_block) {
  SysShape h;
  h.n = n;
  h.kp = kp;
  h.R = R;
  h.chunk_rows = NT / R;
  h.nchunks = (n + h.chunk_rows - 1) / h.chunk_rows;
  if (rows_per_block <= 0) {
    h.nblk = solver_blocks(h.nchunks);
  } else {
    const int64_t cpb = std::max<int64_t>(1, rows_per_block / h.chunk_rows);
    h.nblk = (int)std::min<int64_t>((h.nchunks + cpb - 1) / cpb, 65536);
  }
  return h;
}

inline void carve_zero(Carver& cv, const SysShape& h, SolveLayout& L) {
  const int64_t nR = h.n * h.R;
  L.p0 = cv.take<double>(nR);
  L.p1 = cv.take<double>(nR);
  L.q = cv.take<double>(nR);
  L.z = cv.take<double>(nR);
  L.estate0 = cv.take<double>((size_t)h.kp * h.R);
  L.estate1 = cv.take<double>((size_t)h.kp * h.R);
  L.ticket = cv.take<unsigned>(ticket_words(h.nblk));
}

inline void carve_rest(Carver& cv, const SysShape& h, SolveLayout& L) {
  const int64_t nR = h.n * h.R;
  const int rw = restriction_width(h.kp, h.R);
  L.r0 = cv.take<double>(nR);
  L.r1 = cv.take<double>(nR);
  L.w0 = cv.take<double>(nR);
  L.w1 = cv.take<double>(nR);
  L.dinv = cv.take<double>(h.n);
  L.dinv32 = cv.take<float>(h.n);
  L.bpart0 = cv.take<double>((size_t)h.nblk * 3 * h.R);
  L.bpart1 = cv.take<double>((size_t)h.nblk * 3 * h.R);
  L.rpart = cv.take<double>((size_t)h.nblk * rw);
  L.rgrp = cv.take<double>((size_t)ticket_groups(h.nblk) * rw);
  L.dpart = cv.take<double>((size_t)h.nblk * h.R);
  L.Ainv = cv.take<double>((size_t)h.kp * h.kp);
}

// Carves the whole workspace (base == nullptr: sizes only).  `Ls` receives the
// per-system layouts when non-null.
inline BatchLayout carve_batch(void* ws, const std::vector<SysShape>& sh, std::vector<SolveLayout>* Ls) {
  const int nsys = (int)sh.size();
  const int R = sh[0].R;
  int64_t blocks = 0;
  for (const auto& h : sh) blocks += h.nblk;
  Carver cv(ws);
  BatchLayout B;
  B.stat0 = cv.take<RhsStatus>((size_t)nsys * R);
  B.stat1 = cv.take<RhsStatus>((size_t)nsys * R);
  B.rr_true = cv.take<double>((size_t)nsys * R);
  B.counters = cv.take<int>((size_t)nsys * 4);
  B.sysdev = cv.take<SysDev>(nsys);
  B.blk2sys = cv.take<int>((size_t)std::max<int64_t>(1, blocks));
  std::vector<SolveLayout> tmp(nsys);
  const size_t z0 = align_up(cv.off);
  for (int i = 0; i < nsys; ++i) carve_zero(cv, sh[i], tmp[i]);
  const size_t z1 = align_up(cv.off);
  for (int i = 0; i < nsys; ++i) carve_rest(cv, sh[i], tmp[i]);
  B.zero_begin = cv.base ? cv.base + z0 : nullptr;
  B.zero_bytes = z1 - z0;
  B.bytes = cv.bytes();
  if (Ls) *Ls = tmp;
  return B;
}

// device descriptor of one system
inline SysDev make_sysdev(const nlsp_operator& A, const nlsp_two_level& M, const double* f, double* u,
                          const SysShape& h, const SolveLayout& L, const BatchLayout& B, int i, int blk0,
                          const nlsp_pcg_opts* opts) {
  SysDev hs{};
  const int R = h.R;
  hs.op = make_op(A);
  hs.R = R;
  hs.kp = h.kp;
  hs.nblk = h.nblk;
  hs.blk0 = blk0;
  hs.chunk_rows = h.chunk_rows;
  hs.nchunks = h.nchunks;
  hs.cpb = (h.nchunks + h.nblk - 1) / h.nblk;
  hs.rw = restriction_width(h.kp, R);
  hs.Q = (M.prec == NLSP_FP64) ? (const void*)M.Q64 : (const void*)M.Q32;
  hs.Linv = M.Linv;
  hs.Ainv = L.Ainv;
  hs.f = f;
  hs.x = u;
  hs.r[0] = L.r0;
  hs.r[1] = L.r1;
  hs.p[0] = L.p0;
  hs.p[1] = L.p1;
  hs.q = L.q;
  hs.z = L.z;
  hs.w[0] = L.w0;
  hs.w[1] = L.w1;
  hs.dinv = L.dinv;
  hs.dinv32 = L.dinv32;
  hs.bpart[0] = L.bpart0;
  hs.bpart[1] = L.bpart1;
  hs.rpart = L.rpart;
  hs.rgrp = L.rgrp;
  hs.estate[0] = L.estate0;
  hs.estate[1] = L.estate1;
  hs.dpart = L.dpart;
  hs.ticket = L.ticket;
  hs.stat[0] = B.stat0 + (size_t)i * R;
  hs.stat[1] = B.stat1 + (size_t)i * R;
  hs.nact = B.counters + 4 * i;
  hs.n_active = B.counters + 4 * i + 2;
  hs.rr_true = B.rr_true + (size_t)i * R;
  hs.nu = M.nu;
  hs.omega = M.omega;
  hs.tol2 = opts->rtol * opts->rtol;
  hs.maxit = opts->maxit;
  hs.flexible = opts->flexible ? 1 : 0;
  hs.rmask = 0xffffffffu;
  return hs;
}

// One solve of `nsys` systems (nsys = 1: pcg_solve).  Every system advances
// in the same launches; a system whose right-hand sides have all stopped
// exits its workgroups at their first instruction.  The host polls the
// per-system active counts every `check_every` iterations; with `graph` the
// check_every iterations are captured once in a hipGraph and replayed (their
// kernels read the iteration only through its parity, and check_every is
// even).
template <typename QT>
static int run_pcg(int nsys, std::vector<SysDev>& hs, const BatchLayout& B, const nlsp_pcg_opts* opts,
                   nlsp_rhs_info* info, bool graph, hipStream_t stream) {
  const int R = hs[0].R;
  int nblk = 0;
  for (const auto& h : hs) nblk += h.nblk;
  const SysDev* dsys = B.sysdev;
  const int* b2s = (nsys == 1) ? nullptr : B.blk2sys;
  const unsigned all = (1u << R) - 1u;
  const int nu = hs[0].nu;
  const dim3 grid(nblk), block(NT);
  nlsp_kernel_timing* tm = opts->timing;
  const int tphase = (tm && tm->phase >= 1 && tm->phase <= 2) ? tm->phase : 0;
  const int tevery = tm ? std::max(1, tm->every) : 1;
  std::vector<hipEvent_t> evs;
  int64_t phase_launch[3] = {0, 0, 0};
  // `launch(a, b)` enqueues one kernel with hipExtLaunchKernelGGL; a and b are
  // the start/stop events of a timed launch, null otherwise
  auto timed = [&](int ph, auto&& launch) {
    const bool on = (ph == tphase) && (phase_launch[ph]++ % tevery == 0);
    hipEvent_t a = nullptr, b = nullptr;
    if (on && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess) {
      launch(a, b);
      evs.push_back(a);
      evs.push_back(b);
    } else {
      if (a) (void)hipEventDestroy(a);
      launch(nullptr, nullptr);
    }
  };
  // J_{2nu} r_new (nu > 1) and kernel B of iteration `it`
  auto launch_b = [&](hipStream_t st, int it, int restart, unsigned mask, int init, bool can_time) {
    int wsrc = -1;
    if (nu > 1) {
      const int rin = restart ? ((it + 1) & 1) : (it & 1);
      hipLaunchKernelGGL(k_sweep<QT>, grid, block, 0, st, dsys, b2s, nsys, it, restart, rin, 1, 0);
      int src = 0;
      for (int s = 1; s < 2 * nu - 1; ++s) {
        hipLaunchKernelGGL(k_sweep<QT>, grid, block, 0, st, dsys, b2s, nsys, it, restart, rin, 0, src);
        src ^= 1;
      }
      wsrc = src;
    }
    if (can_time) {
      timed(2, [&](hipEvent_t a, hipEvent_t b) {
        hipExtLaunchKernelGGL(k_iter_b<QT>, grid, block, 0, st, a, b, 0, dsys, b2s, nsys, it, restart, mask,
                              init, wsrc);
      });
    } else {
      hipLaunchKernelGGL(k_iter_b<QT>, grid, block, 0, st, dsys, b2s, nsys, it, restart, mask, init, wsrc);
    }
  };
  hipGraphExec_t gexec = nullptr;
  hipGraph_t gph = nullptr;
  auto release = [&]() {
    if (tm) {
      double tot = 0.0;
      for (size_t i = 0; i + 1 < evs.size(); i += 2) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, evs[i], evs[i + 1]) == hipSuccess) tot += ms;
      }
      tm->total_ms = tot;
      tm->launches = (int)(evs.size() / 2);
    }
    for (hipEvent_t e : evs) (void)hipEventDestroy(e);
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (gph) (void)hipGraphDestroy(gph);
  };
  // stops with the HIP error, after releasing events and graphs
#define NLSP_RUN(call)                  \
  do {                                  \
    if ((call) != hipSuccess) {         \
      release();                        \
      return NLSP_E_HIP;                \
    }                                   \
  } while (0)
  for (int i = 0; i < nsys; ++i) {
    hipLaunchKernelGGL(k_dinv, dim3(ceil_div(hs[i].op.n, NT)), block, 0, stream, hs[i].op,
                       const_cast<double*>(hs[i].dinv), const_cast<float*>(hs[i].dinv32));
    hipLaunchKernelGGL(k_coarse_inverse, dim3(ceil_div(hs[i].kp * hs[i].kp, 256)), dim3(256), 0, stream,
                       hs[i].Linv, hs[i].kp, const_cast<double*>(hs[i].Ainv));
  }
  // start-up as iteration -1: r = f - A x into r[0], then kernel B in restart mode
  hipLaunchKernelGGL(k_residual<QT>, grid, block, 0, stream, dsys, b2s, nsys, all, 0);
  launch_b(stream, -1, 1, all, 1, true);
  NLSP_RUN(hipGetLastError());
  std::vector<RhsStatus> hst((size_t)nsys * R);
  NLSP_RUN(hipMemcpyAsync(hst.data(), B.stat0, sizeof(RhsStatus) * nsys * R, hipMemcpyDeviceToHost, stream));
  NLSP_RUN(hipStreamSynchronize(stream));
  for (int i = 0; i < nsys; ++i) {
    unsigned zero_mask = 0;
    for (int c = 0; c < R; ++c)
      if (hst[(size_t)i * R + c].ff == 0.0) zero_mask |= 1u << c;
    if (zero_mask)
      hipLaunchKernelGGL(k_zero_cols, dim3(ceil_div(hs[i].op.n * R, 256)), dim3(256), 0, stream, hs[i].x,
                         hs[i].op.n, R, zero_mask);
  }
  int every = std::max(1, opts->check_every);
  if (graph && (every & 1)) ++every;   // replayed bodies keep the iteration parity
  int guard = 0;
  int it = 0;  // next iteration index; stat[it & 1] is the current state
  // every RHS stops by maxit iterations; the launch budget is a hard bound on
  // the host loop in case the device-side bookkeeping were ever wrong
  int64_t launched = 0;
  const int64_t launch_cap = (int64_t)hs[0].maxit + 2 * every + 64;
  std::vector<int> cnt((size_t)nsys * 4);
  for (;;) {
    NLSP_RUN(hipMemcpyAsync(cnt.data(), B.counters, sizeof(int) * 4 * nsys, hipMemcpyDeviceToHost, stream));
    NLSP_RUN(hipStreamSynchronize(stream));
    int any = 0;
    for (int i = 0; i < nsys; ++i) any += cnt[(size_t)4 * i + 2] > 0;
    if (any && launched < launch_cap) {
      if (graph) {
        if (!gexec) {
          hipStream_t cs = nullptr;
          NLSP_RUN(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
          if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            (void)hipStreamDestroy(cs);
            release();
            return NLSP_E_HIP;
          }
          for (int k = 0; k < every; ++k) {
            hipLaunchKernelGGL(k_iter_a<QT>, grid, block, 0, cs, dsys, b2s, nsys, it + k);
            launch_b(cs, it + k, 0, 0u, 0, false);
          }
          const hipError_t ce = hipStreamEndCapture(cs, &gph);
          (void)hipStreamDestroy(cs);
          NLSP_RUN(ce);
          NLSP_RUN(hipGraphInstantiate(&gexec, gph, nullptr, nullptr, 0));
        }
        NLSP_RUN(hipGraphLaunch(gexec, stream));
        it += every;
      } else {
        for (int k = 0; k < every; ++k, ++it) {
          timed(1, [&](hipEvent_t a, hipEvent_t b) {
            hipExtLaunchKernelGGL(k_iter_a<QT>, grid, block, 0, stream, a, b, 0, dsys, b2s, nsys, it);
          });
          launch_b(stream, it, 0, 0u, 0, true);
        }
      }
      launched += every;
      NLSP_RUN(hipGetLastError());
      continue;
    }
    // every RHS stopped: confirm the converged ones with the true residual
    hipLaunchKernelGGL(k_true_residual, grid, block, 0, stream, dsys, b2s, nsys);
    hipLaunchKernelGGL(k_true_finish, dim3(nsys), block, 0, stream, dsys);
    NLSP_RUN(hipGetLastError());
    RhsStatus* cur_d = (it & 1) ? B.stat1 : B.stat0;
    std::vector<double> rrt((size_t)nsys * R);
    NLSP_RUN(hipMemcpyAsync(hst.data(), cur_d, sizeof(RhsStatus) * nsys * R, hipMemcpyDeviceToHost, stream));
    NLSP_RUN(hipMemcpyAsync(rrt.data(), B.rr_true, sizeof(double) * nsys * R, hipMemcpyDeviceToHost, stream));
    NLSP_RUN(hipStreamSynchronize(stream));
    std::vector<unsigned> redo(nsys, 0u);
    bool any_redo = false;
    for (int i = 0; i < nsys; ++i)
      for (int c = 0; c < R; ++c) {
        const RhsStatus& s = hst[(size_t)i * R + c];
        if (s.conv && s.ff > 0.0 && rrt[(size_t)i * R + c] > hs[i].tol2 * s.ff && s.iters < hs[i].maxit) {
          redo[i] |= 1u << c;
          any_redo = true;
        }
      }
    if (!any_redo || ++guard > 16) {
      int worst = NLSP_OK;
      for (size_t j = 0; j < (size_t)nsys * R; ++j) {
        const RhsStatus& s = hst[j];
        info[j].iters = s.iters;
        info[j].status = s.status;
        info[j].relres = (s.ff > 0.0) ? std::sqrt(rrt[j] / s.ff) : 0.0;
        if (s.status < 0 && (worst >= 0 || s.status < worst)) worst = s.status;
        if (s.status == NLSP_NOT_CONVERGED && worst == NLSP_OK) worst = NLSP_NOT_CONVERGED;
      }
      release();
      return worst;
    }
    // residual replacement: r = f - A x for the `redo` RHS into r[it & 1] and
    // those RHS restart from it (kernel B in restart mode as iteration it - 1,
    // reading stat[(it - 1) & 1], which receives the current state of every
    // system with the redo RHS made active)
    std::vector<SysDev> hr = hs;   // descriptors with the restart masks
    for (int i = 0; i < nsys; ++i) {
      for (int c = 0; c < R; ++c)
        if ((redo[i] >> c) & 1u) hst[(size_t)i * R + c].active = 1;
      cnt[(size_t)4 * i + ((it - 1) & 1)] = __builtin_popcount(redo[i]);
      hr[i].rmask = redo[i];
    }
    RhsStatus* prev_d = ((it - 1) & 1) ? B.stat1 : B.stat0;
    NLSP_RUN(hipMemcpyAsync(prev_d, hst.data(), sizeof(RhsStatus) * nsys * R, hipMemcpyHostToDevice, stream));
    NLSP_RUN(hipMemcpyAsync(B.counters, cnt.data(), sizeof(int) * 4 * nsys, hipMemcpyHostToDevice, stream));
    NLSP_RUN(hipMemcpyAsync(B.sysdev, hr.data(), sizeof(SysDev) * nsys, hipMemcpyHostToDevice, stream));
    hipLaunchKernelGGL(k_residual<QT>, grid, block, 0, stream, dsys, b2s, nsys, all, it & 1);
    launch_b(stream, it - 1, 1, all, 0, true);
    NLSP_RUN(hipMemcpyAsync(B.sysdev, hs.data(), sizeof(SysDev) * nsys, hipMemcpyHostToDevice, stream));
    NLSP_RUN(hipGetLastError());
    // the host arrays above are reused by the next pass: finish their copies
    NLSP_RUN(hipStreamSynchronize(stream));
  }
#undef NLSP_RUN
}

// Validation of one system against the batch's common settings; 0 if fine.
inline bool system_ok(const nlsp_operator* A, const nlsp_two_level* M, const double* f, const double* u, int R,
                      int64_t n) {
  if (n < 1 || !M || !f || !u) return false;
  if (R < 1 || R > MAXR || n * R >= (int64_t(1) << 31)) return false;
  const int kp = padded_rank(M->k);
  if (kp < 0 || M->nu < 1 || !(M->omega > 0) || !M->Linv) return false;
  if (kp * R > 2048) return false;  // LDS staging of the coarse vectors
  if (M->prec == NLSP_FP64 ? !M->Q64 : (M->prec == NLSP_MIXED ? !M->Q32 : true)) return false;
  if ((int64_t)M->k > n) return false;
  return true;
}

inline bool opts_ok(const nlsp_pcg_opts* o) {
  return o && o->rtol > 0 && o->maxit >= 1 && o->check_every >= 1;
}

// Sets up and runs a batch; nsys = 1 and rows_per_block = 0 is pcg_solve.
static int solve_batch(int nsys, const nlsp_operator* const* As, const nlsp_two_level* const* Ms,
                       const double* const* fs, double* const* us, int R, int rows_per_block,
                       const nlsp_pcg_opts* opts, nlsp_rhs_info* info, void* ws, size_t ws_bytes, bool graph,
                       hipStream_t stream) {
  std::vector<SysShape> sh(nsys);
  for (int i = 0; i < nsys; ++i) sh[i] = shape_of(op_size(As[i]), padded_rank(Ms[i]->k), R, rows_per_block);
  if (!ws_ok(ws, ws_bytes, carve_batch(nullptr, sh, nullptr).bytes)) return NLSP_E_WORKSPACE;
  std::vector<SolveLayout> Ls;
  const BatchLayout B = carve_batch(ws, sh, &Ls);
  std::vector<SysDev> hs(nsys);
  std::vector<int> b2s;
  int blk0 = 0;
  for (int i = 0; i < nsys; ++i) {
    hs[i] = make_sysdev(*As[i], *Ms[i], fs[i], us[i], sh[i], Ls[i], B, i, blk0, opts);
    for (int b = 0; b < sh[i].nblk; ++b) b2s.push_back(i);
    blk0 += sh[i].nblk;
  }
  // iteration -1 reads stat[1]: every RHS starts active with a fresh direction
  std::vector<RhsStatus> st0((size_t)nsys * R);
  for (auto& s : st0) {
    s = RhsStatus{};
    s.gamma_old = 1.0;
    s.active = 1;
    s.restart = 1;
    s.status = NLSP_NOT_CONVERGED;
  }
  // counters per system: nact(0) = 0, nact(1) = R (the iteration -1 state has
  // every RHS active), active = 0
  std::vector<int> counters0((size_t)nsys * 4, 0);
  for (int i = 0; i < nsys; ++i) counters0[(size_t)4 * i + 1] = R;
  NLSP_HIP(hipMemsetAsync(B.zero_begin, 0, B.zero_bytes, stream));
  NLSP_HIP(hipMemcpyAsync(B.counters, counters0.data(), sizeof(int) * 4 * nsys, hipMemcpyHostToDevice, stream));
  NLSP_HIP(hipMemcpyAsync(B.stat1, st0.data(), sizeof(RhsStatus) * nsys * R, hipMemcpyHostToDevice, stream));
  NLSP_HIP(hipMemcpyAsync(B.sysdev, hs.data(), sizeof(SysDev) * nsys, hipMemcpyHostToDevice, stream));
  if (nsys > 1)
    NLSP_HIP(hipMemcpyAsync(B.blk2sys, b2s.data(), sizeof(int) * b2s.size(), hipMemcpyHostToDevice, stream));
  // the host arrays above are locals: their copies must finish before return
  NLSP_HIP(hipStreamSynchronize(stream));
  if (Ms[0]->prec == NLSP_FP64) return run_pcg<double>(nsys, hs, B, opts, info, graph, stream);
  return run_pcg<float>(nsys, hs, B, opts, info, graph, stream);
}

}  // namespace nlsp

using namespace nlsp;

extern "C" {

size_t pcg_solve_workspace_bytes(const nlsp_operator* A, int k, int R) {
  const int64_t n = op_size(A);
  const int kp = padded_rank(k);
  if (n < 1 || kp < 0 || R < 1 || R > MAXR || kp * R > 2048 || n * R >= (int64_t(1) << 31)) return 0;
  return carve_batch(nullptr, {shape_of(n, kp, R, 0)}, nullptr).bytes;
}

int pcg_solve(const nlsp_operator* A, const nlsp_two_level* M, const double* f, double* u, int R,
              const nlsp_pcg_opts* opts, nlsp_rhs_info* info, void* ws, size_t ws_bytes,
              void* stream_) {
  const int64_t n = op_size(A);
  if (!info || !opts_ok(opts) || !system_ok(A, M, f, u, R, n)) return NLSP_E_INVALID;
  return solve_batch(1, &A, &M, &f, &u, R, 0, opts, info, ws, ws_bytes, false, as_stream(stream_));
}

size_t pcg_solve_batched_workspace_bytes(int nsys, const nlsp_system* sys, int R, int rows_per_block) {
  if (nsys < 1 || !sys || R < 1 || R > MAXR || rows_per_block < 0) return 0;
  std::vector<SysShape> sh(nsys);
  for (int i = 0; i < nsys; ++i) {
    const int64_t n = op_size(&sys[i].A);
    const int kp = padded_rank(sys[i].M.k);
    if (n < 1 || kp < 0 || kp * R > 2048 || n * R >= (int64_t(1) << 31)) return 0;
    sh[i] = shape_of(n, kp, R, rows_per_block);
  }
  return carve_batch(nullptr, sh, nullptr).bytes;
}

int pcg_solve_batched(int nsys, const nlsp_system* sys, int R, int rows_per_block, const nlsp_pcg_opts* opts,
                      nlsp_rhs_info* info, void* ws, size_t ws_bytes, void* stream_) {
  if (nsys < 1 || !sys || !info || !opts_ok(opts) || rows_per_block < 0) return NLSP_E_INVALID;
  std::vector<const nlsp_operator*> As(nsys);
  std::vector<const nlsp_two_level*> Ms(nsys);
  std::vector<const double*> fs(nsys);
  std::vector<double*> us(nsys);
  int64_t blocks = 0;
  for (int i = 0; i < nsys; ++i) {
    const nlsp_system& s = sys[i];
    const int64_t n = op_size(&s.A);
    if (!system_ok(&s.A, &s.M, s.f, s.u, R, n)) return NLSP_E_INVALID;
    // one precision, smoother and k for the whole batch (one kernel per step)
    if (s.M.prec != sys[0].M.prec || s.M.nu != sys[0].M.nu || s.M.k != sys[0].M.k) return NLSP_E_INVALID;
    As[i] = &s.A;
    Ms[i] = &s.M;
    fs[i] = s.f;
    us[i] = s.u;
    blocks += shape_of(n, padded_rank(s.M.k), R, rows_per_block).nblk;
  }
  if (blocks > (int64_t(1) << 30)) return NLSP_E_INVALID;
  const bool graph = opts->timing == nullptr;
  return solve_batch(nsys, As.data(), Ms.data(), fs.data(), us.data(), R, rows_per_block, opts, info, ws,
                     ws_bytes, graph, as_stream(stream_));
}

// ---------------------------------------------------------------- autotuner
// Candidate tile sizes (rows of a system per workgroup) tried by
// pcg_solve_batched_tune, as multiples of the NT / R rows of one chunk; 0 is
// the default one-workgroup-per-chunk plan.
static const int kTuneChunks[] = {0, 2, 4, 8, 16, 32};
static const int kTuneCount = sizeof(kTuneChunks) / sizeof(kTuneChunks[0]);

int pcg_solve_batched_tune_candidates(int R, int* rows_per_block) {
  if (R < 1 || R > MAXR) return 0;
  for (int c = 0; c < kTuneCount; ++c)
    if (rows_per_block) rows_per_block[c] = kTuneChunks[c] * (NT / R);
  return kTuneCount;
}

size_t pcg_solve_batched_tune_workspace_bytes(int nsys, const nlsp_system* sys, int R) {
  if (nsys < 1 || !sys || R < 1 || R > MAXR) return 0;
  size_t most = 0, us = 0;
  for (int c = 0; c < kTuneCount; ++c) {
    const size_t b = pcg_solve_batched_workspace_bytes(nsys, sys, R, kTuneChunks[c] * (NT / R));
    if (b == 0) return 0;
    most = std::max(most, b);
  }
  for (int i = 0; i < nsys; ++i) us += align_up((size_t)op_size(&sys[i].A) * R * sizeof(double));
  return align_up(most) + us;
}

int pcg_solve_batched_tune(int nsys, const nlsp_system* sys, int R, const nlsp_pcg_opts* opts, int iters,
                           int* best_rows_per_block, double* ms, void* ws, size_t ws_bytes, void* stream_) {
  if (nsys < 1 || !sys || !opts_ok(opts) || iters < 2 || !best_rows_per_block) return NLSP_E_INVALID;
  const size_t need = pcg_solve_batched_tune_workspace_bytes(nsys, sys, R);
  if (need == 0) return NLSP_E_INVALID;
  if (!ws_ok(ws, ws_bytes, need)) return NLSP_E_WORKSPACE;
  hipStream_t stream = as_stream(stream_);
  size_t solve_bytes = 0;
  for (int c = 0; c < kTuneCount; ++c)
    solve_bytes = std::max(solve_bytes, pcg_solve_batched_workspace_bytes(nsys, sys, R, kTuneChunks[c] * (NT / R)));
  char* base = static_cast<char*>(ws);
  // the trial solves iterate on copies of the initial guesses
  std::vector<nlsp_system> trial(sys, sys + nsys);
  size_t off = align_up(solve_bytes);
  for (int i = 0; i < nsys; ++i) {
    trial[i].u = reinterpret_cast<double*>(base + off);
    off += align_up((size_t)op_size(&sys[i].A) * R * sizeof(double));
  }
  nlsp_pcg_opts o = *opts;
  o.maxit = iters;
  o.check_every = iters + (iters & 1);
  o.timing = nullptr;
  std::vector<nlsp_rhs_info> info((size_t)nsys * R);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  NLSP_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return NLSP_E_HIP;
  }
  double best = 1e300;
  int best_c = 0, rc = NLSP_OK;
  for (int c = 0; c < kTuneCount && rc == NLSP_OK; ++c) {
    const int rpb = kTuneChunks[c] * (NT / R);
    for (int i = 0; i < nsys && rc == NLSP_OK; ++i)
      if (hipMemcpyAsync(trial[i].u, sys[i].u, (size_t)op_size(&sys[i].A) * R * sizeof(double),
                         hipMemcpyDeviceToDevice, stream) != hipSuccess)
        rc = NLSP_E_HIP;
    if (rc != NLSP_OK) break;
    if (hipEventRecord(e0, stream) != hipSuccess) { rc = NLSP_E_HIP; break; }
    const int r = pcg_solve_batched(nsys, trial.data(), R, rpb, &o, info.data(), ws, solve_bytes, stream);
    if (r < 0) { rc = r; break; }
    float t = 0.f;
    if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&t, e0, e1) != hipSuccess) { rc = NLSP_E_HIP; break; }
    if (ms) ms[c] = t;
    if (t < best) {
      best = t;
      best_c = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != NLSP_OK) return rc;
  *best_rows_per_block = kTuneChunks[best_c] * (NT / R);
  return NLSP_OK;
}

}  // extern "C"
