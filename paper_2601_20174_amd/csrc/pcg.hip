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
// One iteration = two kernels and one grid reduction point per kernel, in the
// single-reduction arrangement of CG (the scalars of both inner products are
// gathered where z and w = A z are formed):
//   update  (reads the partials of the previous update and the matvec's
//            records) beta; p^T q = z^T w + beta (z^T q_old + p_old^T w)
//            + beta^2 p_old^T q_old; alpha; p = z + beta p_old;
//            q = w + beta q_old; x += alpha p; r_new = r - alpha q;
//            c_new = c - alpha g, g = A_c^-1 Q^T q = Qt^T w + beta g_old;
//            z = J r_new + Q c_new; partials r^T z, r^T z_old, ||r||^2, p^T q
//   matvec  w = A z; records [Qt^T w | z^T w | z^T q + p^T w]
// with Qt = Q A_c^-1 formed once per solve, so the coarse coefficients
// c = A_c^-1 Q^T r are carried by recurrences and never need a coarse solve
// inside the iteration.  In exact arithmetic p, q, x, r, z are those of
// standard PCG (q = A p by induction, p^T q by expanding both recurrences);
// p^T q uses the dot product of the stored vectors, not a scalar recurrence.
// The matvec kernel waits for no scalar, so it streams from its first
// instruction; the update kernel needs no coarse solve before its stream.
// Grid reductions are finished by the consumer: every workgroup of the next
// kernel sums the per-workgroup partials it needs in a fixed order (so all
// workgroups obtain bit-identical scalars and runs are reproducible), while its
// own loads are in flight.  Only the restriction records (k values per RHS)
// are pre-summed by the last workgroup of each group of 16.  The per-RHS state
// is double-buffered by iteration parity: iteration `it` reads stat[it & 1]
// and only workgroup 0 of the update kernel writes stat[(it + 1) & 1].
// Vectors and every reduction are float64; in the mixed form Q, Qt, the
// smoother and the prolongation products are float32.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include <hip/hip_ext.h>

#include "device_common.hpp"
#include "host_common.hpp"

namespace nlsp {

constexpr int NT = 512;   // threads per workgroup of the solver kernels
constexpr int MAXR = 16;  // right-hand sides per solve
constexpr int BW = 4;     // update-kernel partials per RHS: r^T z, r^T z_old, ||r||^2, p^T q

struct RhsStatus {
  double gamma_old;  // r^T z of the previous iteration (beta's denominator)
  double ff;         // ||f||^2
  int active;        // still iterating
  int iters;         // updates of x completed
  int status;        // nlsp_status of this RHS
  int restart;       // the next update uses beta = 0
  int conv;          // stopped by the recursive residual test (true residual pending)
  int pad0, pad1, pad2;
};

struct SysDev {
  OpDev op;
  int R, kp, nblk, blk0;
  int chunk_rows;          // rows per chunk: floor(NT / R); threads past chunk_rows*R idle
  int64_t nchunks;
  int64_t cpb;             // chunks per workgroup: ceil(nchunks / nblk)
  int rw;                  // restriction record width: kp*R + 2R
  int gw;                  // group record width: rw + 4R (the update partials ride along)
  // device pointers (global address space in the device pass)
  Glob<const void>* Q;     // (n, kp), float, double or float16: prolongation
  Glob<const void>* Qt;    // (n, kp) Q A_c^-1, same type: restriction to coarse coefficients
  // float16 basis (Q and Qt both point to W s, W = Q L^-T, see run_pcg):
  // [1 / s, 1 / s], the inverse power-of-two scale folded into c before the
  // prolongation and into the restriction sums; the float32 Q that W is
  // formed from (host use only)
  Glob<const double>* qscale;
  const void* qsrc;
  Glob<const double>* Linv;  // (kp, kp) inverse Cholesky factor of A_c
  Glob<double>* Ainv;      // (kp, kp) = L^-T L^-1
  Glob<const double>* f;
  Glob<double>* x;
  Glob<double>* r[2];      // residual, by iteration parity
  Glob<double>* p;         // search direction (updated in place)
  Glob<double>* q[2];      // A p, by iteration parity
  Glob<double>* z;         // preconditioned residual (updated in place)
  Glob<double>* w;         // A z
  Glob<void>* wj[2];       // J_{2nu} r work buffers (nu > 1), arithmetic type of Q
  Glob<double>* dinv;
  Glob<float>* dinv32;
  Glob<double>* bpart[2];  // [nblk][4R]  update partials [r^T z | r^T z_old | ||r||^2 | p^T q], by parity
  Glob<double>* rpart;     // [nblk][rw]  restriction records [Qt^T v | s1 | s2]
  Glob<double>* rgrp;      // [ngrp][gw]  group records [restriction record | update partials]
  Glob<double>* cstate[2]; // [kp*R]      c = A_c^-1 Q^T r, by parity
  Glob<double>* gstate[2]; // [kp*R]      g = A_c^-1 Q^T q, by parity
  Glob<double>* dpart;     // [nblk][R]   true-residual partials
  Glob<unsigned>* ticket;  // ticket_words(nblk)
  Glob<RhsStatus>* stat[2];  // [R] each
  Glob<int>* nact;         // [2] active RHS in the stat buffer of that parity
  Glob<int>* n_active;     // host-visible copy
  Glob<double>* rr_true;   // [R]
  double omega, tol2;
  int maxit, flexible, nu;
  unsigned rmask;          // RHS a restart launch applies to (ANDed with the launch mask)
  int ylines;              // 2-D line march of the matrix-core kernels (chunks ordered y fastest)
  int zorder;              // 3-D chunks ordered z fastest (the x-lines split into whole chunks)
  int nxq;                 // chunks per x-line when zorder or ylines
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

template <>
struct Vec4<_Float16> {
  using type = _Float16 __attribute__((ext_vector_type(4)));
};

// Arithmetic type of a stored basis element: a float16 basis is used in float.
template <typename QS>
struct Arith {
  using type = QS;
};
template <>
struct Arith<_Float16> {
  using type = float;
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
// unconditionally from clamped addresses and without touching the values, so
// that no wait follows the loads; rec_finish masks the surplus, adds them in
// ascending record order and across threads with a fixed tree.  Same result as
// sum_records.
NLSP_DEV bool rec_fits(int nrec, int count) { return count <= NT && nrec <= 8 * (NT / count); }

template <bool COHERENT>
NLSP_DEV void rec_issue(const double* base, int nrec, int stride, int off, int count, double (&v)[8]) {
  const int t = threadIdx.x;
  const int groups = NT / count, e = t % count, g = t / count;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const auto a = &base[(int64_t)min(g + u * groups, nrec - 1) * stride + off + e];
    v[u] = COHERENT ? load_partial(a) : *a;
  }
}

NLSP_DEV void rec_finish(const double (&v)[8], int nrec, int count, double* out, double* sh) {
  const int t = threadIdx.x;
  const int groups = NT / count, g = t / count;
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < 8; ++u) s += (g < groups && g + u * groups < nrec) ? v[u] : 0.0;
  __syncthreads();
  sh[t] = (g < groups) ? s : 0.0;
  lds_tree_rows(sh, groups, count);
  if (t < count) out[t] = sh[t];
  __syncthreads();
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

// NB rows of Q for one thread, issued together so their latencies overlap.
// get() converts an element to the arithmetic type where it is used, so a
// float16 row stays packed (two registers) until then.
template <typename QT, int NB>
struct QBatch {
  QT v[NB][4];
  NLSP_DEV void load(int w, const QT* p) { load4(p, v[w]); }
  NLSP_DEV QT get(int w, int u) const { return v[w][u]; }
};
template <int NB>
struct QBatch<_Float16, NB> {
  typename Vec4<_Float16>::type v[NB];
  NLSP_DEV void load(int w, const _Float16* p) { v[w] = *reinterpret_cast<const typename Vec4<_Float16>::type*>(p); }
  NLSP_DEV float get(int w, int u) const { return (float)v[w][u]; }
};

// Rows past the chunk (and idle row groups) load a clamped row instead of
// branching around the load: the consumers only use rows < nrows of active row
// groups, and an unconditional load is never waited for before the next one.
template <typename QT, int NB>
NLSP_DEV void q_fetch(const QT* __restrict__ Q, int64_t row0, int nrows, int kp, const QMap& m,
                      int w0, QBatch<QT, NB>& b) {
#pragma unroll
  for (int w = 0; w < NB; ++w) {
    const int row = min(m.rg + (w0 + w) * m.ngr, nrows - 1);
    b.load(w, Q + (row0 + row) * kp + 4 * m.jc);
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
        for (int u = 0; u < 4; ++u) acc[u] += prod<typename Arith<QT>::type>(b.get(w, u), r);
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

// restrict_finish plus the workgroup sums of two per-thread values per RHS
// (t % R) in one barrier round: out[KR + k*R + c] for k < 2.  Both use wave
// butterflies; needs R a power of two (the caller falls back otherwise).
NLSP_DEV void restrict_finish_x2(const QMap& m, int kp, int R, const double (&acc)[4], const double (&x)[2],
                                 double* red, double* out) {
  const int KR = kp * R;
  const int pairs = m.lpr * R;
  constexpr int NW = NT / WAVE;
  double v[4] = {acc[0], acc[1], acc[2], acc[3]};
  for (int o = WAVE / 2; o >= pairs; o >>= 1)
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] += __shfl_xor(v[u], o, WAVE);
  double y[2] = {x[0], x[1]};
  for (int o = WAVE / 2; o >= R; o >>= 1)
#pragma unroll
    for (int k = 0; k < 2; ++k) y[k] += __shfl_xor(y[k], o, WAVE);
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  double* red2 = red + NW * KR;
  __syncthreads();
  if (lane < pairs)
#pragma unroll
    for (int u = 0; u < 4; ++u) red[w * KR + (4 * m.jc + u) * R + m.c] = v[u];
  if (lane < R)
#pragma unroll
    for (int k = 0; k < 2; ++k) red2[(w * 2 + k) * R + lane] = y[k];
  __syncthreads();
  for (int idx = threadIdx.x; idx < KR + 2 * R; idx += NT) {
    double s = 0.0;
    if (idx < KR) {
#pragma unroll
      for (int q = 0; q < NW; ++q) s += red[q * KR + idx];
    } else {
      const int j = idx - KR;   // k*R + c
#pragma unroll
      for (int q = 0; q < NW; ++q) s += red2[q * 2 * R + j];
    }
    store_partial(&out[idx], s);
  }
}

// ys[row*R + c] = sum_j Q[row][j] e[j][c] for the chunk rows (prolongation),
// arithmetic in QA (the basis's arithmetic type); the lpr lanes of a row add
// with butterflies.  All lanes run the same trip count (shuffles need the
// whole wave).
template <typename QS, int NB, typename QA = typename Arith<QS>::type>
NLSP_DEV void prolong_rows(const QS* __restrict__ Q, int64_t row0, int nrows, int kp, int R,
                           const QMap& m, const QA (&e4)[4], QBatch<QS, NB>& b, QA* ys) {
  const int trips = q_trips(m, nrows);
  for (int w0 = 0; w0 < trips; w0 += NB) {
    if (w0 > 0) q_fetch<QS, NB>(Q, row0, nrows, kp, m, w0, b);
#pragma unroll
    for (int w = 0; w < NB; ++w) {
      if (w0 + w >= trips) break;
      const int row = m.rg + (w0 + w) * m.ngr;
      QA sdot = b.get(w, 0) * e4[0] + b.get(w, 1) * e4[1] + b.get(w, 2) * e4[2] + b.get(w, 3) * e4[3];
      sdot = group_sum(sdot, m.lpr);
      if (m.jc == 0 && m.on && row < nrows) ys[row * R + m.c] = sdot;
    }
  }
}

template <typename QT>
struct QB {
  // update kernel: 4 rows of Q per thread in flight (float; measured against
  // 2, 3, 5, 6 and 8 on the 2-D workload); 2 keeps the float64 kernel at 128
  // VGPRs without spills; float16 rows are half as long, so twice as many
  // keep the same bytes in flight
  static constexpr int NB = sizeof(QT) == 8 ? 2 : (sizeof(QT) == 4 ? 4 : 8);
  // matvec and residual kernels (measured against 2, 3, 5 and 6)
  static constexpr int NBR = sizeof(QT) == 2 ? 8 : 4;
};

// ---------------------------------------------- MFMA form of the basis passes
// For R = 16 right-hand sides (kp = 64 or 128) and R = 8 (kp = 32 or 64) the
// passes are 16 x 16 x 4 matrix products on the matrix cores, the right-hand
// sides forming the 16 columns of one tile (with R = 8 the upper 8 columns
// are zero and their results dropped), so every element of Q / Qt is loaded
// once per pass instead of once per right-hand side.  Operands: lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16]; the accumulator element v
// of lane l is D[4 (l / 16) + v][l % 16] for the float32 product and
// D[4 v + l / 16][l % 16] for the float64 one.
//   matvec: (Qt^T w) tile I = sum over rows of Qt[row][16 I + i] w[row][c],
//     float64 products (as restrict_rows); kp / 16 column tiles, each over
//     8 / (kp / 16) waves with a slice of the chunk's rows each.
//   update: (Q c) for the NT / R rows of a chunk in QT, waves = (NT / R) / 16
//     row tiles x R / 4 slices of 4 kp / R columns (one or two blocks of 16),
//     the slices added in order through LDS.
constexpr int MF_T = 16;   // columns of a tile
// one line of the update kernel's 2-D march: (NT / R + 2) cells x R, at most
// (64 + 2) x 8 and (32 + 2) x 16
constexpr int YM_SLOT = 34 * 16;
inline bool mf_ok(int R, int kp) {
  return (R == 16 && (kp == 64 || kp == 128)) || (R == 8 && (kp == 32 || kp == 64));
}

template <typename QT>
struct MfAcc;
template <>
struct MfAcc<float> {
  typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct MfAcc<double> {
  typedef double type __attribute__((ext_vector_type(4)));
};
NLSP_DEV MfAcc<float>::type mf_mma(float a, float b, MfAcc<float>::type c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
NLSP_DEV MfAcc<double>::type mf_mma(double a, double b, MfAcc<double>::type c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// accumulator slot (v, lane) holding D[i][c] of a 16 x 16 tile: v * 64 + lane
template <typename QT>
NLSP_DEV int mf_slot(int i, int c) {
  return sizeof(QT) == 4 ? (i & 3) * 64 + (i >> 2) * 16 + c : (i >> 2) * 64 + (i & 3) * 16 + c;
}

struct ChunkRange {
  int64_t c0, c1;
};

// First row of logical chunk ch.  For 3-D operators whose x-lines split into
// whole chunks, chunks are enumerated z fastest: logical chunk ch is plane
// ch % nz of the column (y, x-segment) ch / nz, so the consecutive chunks of
// a workgroup march through z (a row's z-neighbours are the workgroup's own
// previous and next chunk) and the workgroups of one XCD hold neighbouring
// columns.  Otherwise chunks are consecutive row ranges.
NLSP_DEV int64_t chunk_row0(const SysDev& S, int64_t ch) {
  const int cr = S.chunk_rows;
  // chunk counts fit 32 bits (n R < 2^31 is checked at entry): 32-bit divisions
  const uint32_t c32 = (uint32_t)ch;
  if (S.zorder) {
    const uint32_t nz = (uint32_t)S.op.nz, nxq = (uint32_t)S.nxq;
    const uint32_t col = c32 / nz, z = c32 - col * nz;
    const uint32_t y = col / nxq, xq = col - y * nxq;
    return ((int64_t)z * S.op.ny + y) * S.op.nx + (int64_t)xq * cr;
  }
  if (S.ylines) {
    // 2-D 9-point operators with the matrix-core kernels march through y the
    // same way (logical chunk ch is line ch % ny of the x-segment ch / ny),
    // which their line rings rely on
    const uint32_t ny = (uint32_t)S.op.ny;
    const uint32_t xq = c32 / ny, y = c32 - xq * ny;
    return (int64_t)y * S.op.nx + (int64_t)xq * cr;
  }
  return ch * cr;
}

NLSP_DEV ChunkRange my_chunks(const SysDev& S, int lb) {
  ChunkRange cr;
  cr.c0 = (int64_t)lb * S.cpb;
  cr.c1 = min(S.nchunks, cr.c0 + S.cpb);
  return cr;
}

// Restriction epilogue (matvec kernel and k_residual): this workgroup's
// record [Qt^T v | s1 | s2] (already in rpart) is summed per group of 16 by
// the group's last workgroup into rgrp, together with the group's partials of
// the preceding update kernel (bpart[bpar]; zeros for bpar < 0), so the next
// update kernel reads one short list of group records and sums it in order
// itself.  This kernel ends one ticket level early.
NLSP_DEV void restriction_epilogue(const SysDev& S, int lb, double* red, double* sh, int bpar) {
  if (!arrive_group(S.ticket, S.nblk, lb)) return;
  const int grp = lb / TICKET_GROUP;
  const int r0 = grp * TICKET_GROUP;
  const int nrec = min(TICKET_GROUP, S.nblk - r0);
  const int bw = BW * S.R;
  const auto ra = S.rpart + (int64_t)r0 * S.rw;
  const auto rb = S.bpart[bpar < 0 ? 0 : bpar] + (int64_t)r0 * bw;
  if (S.gw <= NT && nrec <= 4 * (NT / S.gw)) {
    // one pass over [record | partials]: at most 4 records per thread, all
    // loads issued before the first add
    const int t = threadIdx.x, cnt = S.gw, groups = NT / cnt, e = t % cnt, g = t / cnt;
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = min(g + u * groups, nrec - 1);
      const double x = load_partial(&ra[(int64_t)r * S.rw + min(e, S.rw - 1)]);
      const double y = rb[(int64_t)r * bw + max(e - S.rw, 0)];
      v[u] = (e < S.rw) ? x : y;
    }
    double sum = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      sum += (g < groups && g + u * groups < nrec && (e < S.rw || bpar >= 0)) ? v[u] : 0.0;
    __syncthreads();
    sh[t] = (g < groups) ? sum : 0.0;
    lds_tree_rows(sh, groups, cnt);
    if (t < cnt) red[t] = sh[t];
    __syncthreads();
  } else {
    sum_records<true>(ra, nrec, S.rw, 0, S.rw, red, sh);
    if (bpar >= 0) {
      sum_records<false>(rb, nrec, bw, 0, bw, red + S.rw, sh);
    } else {
      for (int idx = threadIdx.x; idx < bw; idx += NT) red[S.rw + idx] = 0.0;
      __syncthreads();
    }
  }
  double* grec = S.rgrp + (int64_t)grp * S.gw;
  for (int idx = threadIdx.x; idx < S.gw; idx += NT) store_partial(&grec[idx], red[idx]);
}

NLSP_DEV bool finite_pos(double v) { return v > 0.0 && v <= 1.7e308; }

// Sum over the threads sharing c = t % R of K values at once: the totals land
// in red[k*R + c].  One tree instead of K.  `sh` holds K*(NT + 16) doubles.
template <int K>
NLSP_DEV void block_sum_rhsk(const double (&v)[K], int R, double* red, double* sh) {
  if (pow2(R) && R <= WAVE) {
    block_sum_waves<K>(v, R, red, sh);
    return;
  }
  const int t = threadIdx.x;
  const int nrows = (NT + R - 1) / R;
  __syncthreads();
  // row-major [row][K R]: thread t = row*R + c
  const int row = t / R, c = t % R;
#pragma unroll
  for (int k = 0; k < K; ++k) sh[row * K * R + k * R + c] = v[k];
  if (t < nrows * R - NT) {   // pad the last partial row
    const int pr = (NT + t) / R, pc = (NT + t) % R;
#pragma unroll
    for (int k = 0; k < K; ++k) sh[pr * K * R + k * R + pc] = 0.0;
  }
  lds_tree_rows(sh, nrows, K * R);
  if (t < K * R) red[t] = sh[t];
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

// Face weights of a finite-volume operator, once per solve: for each cell i
// and axis a, the weight of the face to the next cell along a (0 where there
// is none), in float64 and formed in float32 from the rounded coefficients,
// the same expressions op_row evaluates.
__global__ __launch_bounds__(NT) void k_faces(OpDev op, double* fw64, float* fw32) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= op.n) return;
  int x, y, z;
  decompose(op, i, x, y, z);
  const int64_t sxy = (int64_t)op.nx * op.ny;
  const bool up[3] = {x < op.nx - 1, y < op.ny - 1, z < op.nz - 1};
  const int64_t jn[3] = {i + 1, i + op.nx, i + sxy};
  const double ai = op.coef[i];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double aj = op.coef[up[a] ? jn[a] : i];
    fw64[a * op.n + i] = up[a] ? harmonic<double>(ai, aj) : 0.0;
    fw32[a * op.n + i] = up[a] ? harmonic<float>((float)ai, (float)aj) : 0.0f;
  }
}

// Qt = Q A_c^-1 (n x kp), once per solve: restricting with Qt gives the
// coarse coefficients A_c^-1 Q^T v directly.  64 rows per workgroup and
// column tiles of 64; thread t forms the 4 x 4 block of rows 4 (t / 16) ..
// and columns 4 (t % 16) .. of the tile.  The rows of Q are staged
// transposed (and in Q's own type) and the tile of A_c^-1 as is, so each
// step l reads 4 consecutive values of each with two 16-byte LDS reads and
// feeds 16 fused multiply-adds.  float64 arithmetic, sums over l ascending.
template <typename QT>
__global__ __launch_bounds__(256) void k_qtilde(const QT* __restrict__ Q, const double* __restrict__ Ainv,
                                                int64_t n, int kp, QT* __restrict__ Qt) {
  constexpr int QW = 64 + 16 / (int)sizeof(QT);   // padded row of the transposed tile
  __shared__ __align__(16) QT qs[64][QW];         // qs[l][row]
  __shared__ __align__(16) double as[64][64];     // as[l][column]
  const int t = threadIdx.x;
  const int64_t row0 = (int64_t)blockIdx.x * 64;
  const int rg = t / 16, cg = t % 16;
  for (int ct = 0; ct < kp; ct += 64) {
    const int TW = min(64, kp - ct);   // kp is a multiple of 16
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    for (int l0 = 0; l0 < kp; l0 += 64) {
      const int LW = min(64, kp - l0);
      __syncthreads();
      for (int idx = t; idx < 64 * LW; idx += 256) {
        const int rr = idx / LW, l = idx % LW;
        const int64_t row = row0 + rr;
        qs[l][rr] = (row < n) ? Q[row * kp + l0 + l] : QT(0);
      }
      for (int idx = t; idx < LW * 64; idx += 256) {
        const int l = idx / 64, j = idx % 64;
        as[l][j] = (j < TW) ? Ainv[(int64_t)(l0 + l) * kp + ct + j] : 0.0;
      }
      __syncthreads();
#pragma unroll 4
      for (int l = 0; l < LW; ++l) {
        double a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = (double)qs[l][4 * rg + i];
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = as[l][4 * cg + j];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t row = row0 + 4 * rg + i;
      if (row < n)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (4 * cg + j < TW) Qt[row * kp + ct + 4 * cg + j] = QT(acc[i][j]);
    }
  }
}

// A float16 Qt is stored as Qt s_Qt: its restriction sums are multiplied by
// 1 / s_Qt (a power of two, so exactly as if Qt were stored unscaled).
template <typename QS, int K>
NLSP_DEV void unscale_restriction(const SysDev& S, double (&acc)[K]) {
  if constexpr (sizeof(QS) == 2) {
    const double is = S.qscale[1];
#pragma unroll
    for (int u = 0; u < K; ++u) acc[u] *= is;
  }
}

// r = f - A x into `rout` for the RHS in `mask` (others untouched);
// restriction records [Qt^T r | ||r||^2 | ||f||^2] (Qt^T r = A_c^-1 Q^T r),
// then the group epilogue.  Used at start-up and for residual replacement.
template <typename QS>
__global__ __launch_bounds__(NT, 4) void k_residual(const SysDev* __restrict__ sys,
                                                    const int* __restrict__ blk2sys, int nsys,
                                                    unsigned mask, int rout) {
  __shared__ double rv[NT];
  __shared__ double sh[2 * (NT + 16)];
  __shared__ double red[4 * NT + 128];
  __shared__ double outv[2 * MAXR];
  const SysDev& S = my_sys(sys, blk2sys, nsys);
  mask &= S.rmask;
  const int lb = xcd_remap(blockIdx.x - S.blk0, S.nblk);
  const int t = threadIdx.x, R = S.R, c = t % R;
  const bool on = (mask >> c) & 1u;
  const QS* Qt = static_cast<const QS*>(S.Qt);
  const QMap m = q_map(S.kp, R);
  constexpr int NB = QB<QS>::NBR;
  QBatch<QS, NB> qb;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  double rr = 0.0, ff = 0.0;
  double* Rout = S.r[rout];
  const ChunkRange cr = my_chunks(S, lb);
  for (int64_t ch = cr.c0; ch < cr.c1; ++ch) {
    const int64_t row0 = chunk_row0(S, ch);
    const int nrows = (int)min<int64_t>(S.chunk_rows, S.op.n - row0);
    q_fetch<QS, NB>(Qt, row0, nrows, S.kp, m, 0, qb);
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
    restrict_rows<QS, NB>(Qt, row0, nrows, S.kp, R, m, rv, qb, acc);
  }
  unscale_restriction<QS>(S, acc);
  double* rec = S.rpart + (int64_t)lb * S.rw;
  restrict_finish(m, S.kp, R, acc, red, rec);
  const int KR = S.kp * R;
  const double v2[2] = {rr, ff};
  block_sum_rhsk<2>(v2, R, outv, sh);
  if (t < 2 * R) store_partial(&rec[KR + t], outv[t]);
  restriction_epilogue(S, lb, red, sh, -1);
}

// Matvec kernel of iteration `it` (after the update kernel of `it`):
// w = A z for the new z; restriction records [Qt^T w | z^T w | z^T q + p^T w]
// (q, p: this iteration's direction pair), summed per group of 16 workgroups
// by the epilogue.  Nothing here waits for a scalar: every workgroup streams
// from its first instruction.  In a batch, a system whose right-hand sides
// have all stopped exits at once.
template <typename QS, bool MF, bool YM = false, bool ZM = false>
__global__ __launch_bounds__(NT, 4) void k_matvec(const SysDev* __restrict__ sys,
                                                  const int* __restrict__ blk2sys, int nsys, int it) {
  __shared__ double wv[NT];
  // line ring of the 2-D 9-point march: 4 lines of (segment + 2 halo cells) x R
  // values of z
  __shared__ double zring[((YM || ZM) && MF) ? 4 * YM_SLOT : 1];
  __shared__ double sh[2 * (NT + 16)];
  __shared__ double red[4 * NT + 128];
  __shared__ double buf[2 * MAXR];
  const SysDev& S = my_sys(sys, blk2sys, nsys);
  // a system whose right-hand sides have all stopped skips the pass; the
  // count is loaded first and tested after the row loads are issued, so the
  // test costs no extra round trip
  const int na = S.nact[(it + 1) & 1];
  const int lb = xcd_remap(blockIdx.x - S.blk0, S.nblk);
  const int t = threadIdx.x, R = S.R, c = t % R;
  const QS* Qt = static_cast<const QS*>(S.Qt);
  const QMap m = q_map(S.kp, R);
  constexpr int NB = QB<QS>::NBR;
  QBatch<QS, NB> qb;
  const ChunkRange cr = my_chunks(S, lb);
  const double* Z = S.z;
  const double* Pv = S.p;
  const double* Qv = S.q[(it + 1) & 1];
  if constexpr (MF) {
    // wave: column tile I of Qt and row slice sl of each chunk (kp = 128: the
    // whole chunk; kp = 64: two waves per tile, half the rows each)
    const int wave = t / WAVE, lane = t % WAVE, lr = lane & 15, lg = lane >> 4;
    const int TI = S.kp / 16, WPT = (NT / WAVE) / TI;
    const int I = wave % TI, sl = wave / TI, rps = S.chunk_rows / WPT, ksteps = rps / 4;
    typename MfAcc<double>::type acc = {0.0, 0.0, 0.0, 0.0};
    double zw = 0.0, e1 = 0.0;
    // 2-D 9-point systems marched through y (chunk_row0): z of line y + 1 is
    // loaded one chunk ahead into an LDS ring and the stencil of line y reads
    // its 9 operands there (the gather below sums the same terms in the same
    // order; the two may contract them into FMAs differently); the basis
    // operands and q, p of the next chunk are loaded ahead too
    bool ym = false;
    if constexpr (YM) {
      // (chunk indices fit 32 bits)
      const uint32_t ny32 = (uint32_t)S.op.ny;
      ym = S.ylines && cr.c0 < cr.c1 && (uint32_t)cr.c0 / ny32 == (uint32_t)(cr.c1 - 1) / ny32;
      if (ym) {
        // descriptor fields and the stencil in registers: the loop's stores
        // would otherwise make the compiler load them again
        const int nx = S.op.nx, ny = S.op.ny, crw = S.chunk_rows, kpq = S.kp;
        double* const Wout = S.w;
        double cf[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) cf[k] = S.op.coef[k];
        const int seg = (int)((uint32_t)cr.c0 / ny32);
        const int x0 = seg * crw;
        const int ly0 = (int)(cr.c0 - (int64_t)seg * ny), ly1 = ly0 + (int)(cr.c1 - cr.c0);
        const int xl = t / R;   // this lane's cell of the segment (chunk_rows = NT / R)
        // lanes t < 2 R also carry the cell just left (t < R) or right of the segment
        const int hs = t / R, xh = hs ? x0 + crw : x0 - 1;
        const bool hl = t < 2 * R && xh >= 0 && xh < nx;
        auto slot = [&](int ly) { return zring + (ly & 3) * YM_SLOT; };
        auto row_of = [&](int ly) { return (int64_t)ly * nx + x0; };   // first row of line ly's segment
        double zc = 0.0, zh = 0.0;   // line in flight: this lane's cell and halo cell
        auto zload = [&](int ly) {
          if (ly >= 0 && ly < ny) {
            zc = Z[(row_of(ly) + xl) * R + c];
            if (hl) zh = Z[((int64_t)ly * nx + xh) * R + c];
          }
        };
        auto zput = [&](int ly) {
          if (ly >= 0 && ly < ny) {
            slot(ly)[(xl + 1) * R + c] = zc;
            if (hl) slot(ly)[(hs ? crw + 1 : 0) * R + c] = zh;
          }
        };
        QS an[8];
        double qn = 0.0, pn = 0.0;
        auto rload = [&](int ly) {
          const int64_t row0 = row_of(ly);
#pragma unroll
          for (int s = 0; s < 8; ++s)
            an[s] = Qt[(row0 + sl * rps + 4 * min(s, ksteps - 1) + lg) * kpq + 16 * I + lr];
          const int64_t g = (row0 + xl) * R + c;
          qn = Qv[g];
          pn = Pv[g];
        };
        zload(ly0 - 1);
        zput(ly0 - 1);
        zload(ly0);
        zput(ly0);
        zload(ly0 + 1);
        rload(ly0);
        if (na == 0) return;   // uniform over the workgroup (one system), before any barrier
        for (int ly = ly0; ly < ly1; ++ly) {
          zput(ly + 1);
          QS a[8];
#pragma unroll
          for (int s = 0; s < 8; ++s) a[s] = an[s];
          const double qi = qn, pi = pn;
          if (ly + 1 < ly1) {
            zload(ly + 2);
            rload(ly + 1);
          }
          __syncthreads();
          double wval = 0.0;
#pragma unroll
          for (int dy = -1; dy <= 1; ++dy) {
            const double* sv = slot(ly + dy);
            const bool oky = ly + dy >= 0 && ly + dy < ny;
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
              const int xx = x0 + xl + dx;
              const bool ok = oky && xx >= 0 && xx < nx;
              const double vj = sv[(xl + dx + 1) * R + c];
              wval += ok ? cf[(dy + 1) * 3 + (dx + 1)] * vj : 0.0;
            }
          }
          const double zi = slot(ly)[(xl + 1) * R + c];
          store_partial(&Wout[(row_of(ly) + xl) * R + c], wval);
          zw += zi * wval;
          e1 += zi * qi + pi * wval;
          wv[t] = wval;
          __syncthreads();
#pragma unroll
          for (int s = 0; s < 8; ++s)
            if (s < ksteps) acc = mf_mma((double)a[s], lr < R ? wv[(sl * rps + 4 * s + lg) * R + lr] : 0.0, acc);
        }
      }
    }
    // 3-D finite-volume systems marched through z (chunk_row0): a
    // workgroup's run of chunks is the planes of one (y, x-segment) column.
    // z of plane z + 1 (and the two cells beside the segment) is loaded one
    // plane ahead into an LDS ring; the -y and +y neighbours, the cell's face
    // weights (one per lane, exchanged with lane shuffles) and coefficient
    // are loaded one plane ahead into registers, so the stencil of op_row
    // (the same terms in the same order) waits for no load.
    bool zm = false;
    if constexpr (ZM) {
      const uint32_t nz32 = (uint32_t)S.op.nz;
      zm = S.zorder && S.op.kind == NLSP_OP_FV7 && cr.c0 < cr.c1 &&
           (uint32_t)cr.c0 / nz32 == (uint32_t)(cr.c1 - 1) / nz32;
      if (zm) {
        const int nx = S.op.nx, ny = S.op.ny, nz = S.op.nz, crw = S.chunk_rows, kpq = S.kp;
        const int64_t n = S.op.n, sxy = (int64_t)nx * ny;
        double* const Wout = S.w;
        const double* const FW = S.op.fw64;
        const double* const AC = S.op.coef;
        const uint32_t col = (uint32_t)cr.c0 / nz32;
        const int yq = (int)(col / (uint32_t)S.nxq), x0 = (int)(col - (uint32_t)yq * (uint32_t)S.nxq) * crw;
        const int z0 = (int)(cr.c0 - (int64_t)col * nz), z1 = z0 + (int)(cr.c1 - cr.c0);
        const int xl = t / R, px = x0 + xl;   // this lane's cell of the segment (chunk_rows = NT / R)
        const int hs = t / R, xh = hs ? x0 + crw : x0 - 1;
        const bool hl = t < 2 * R && xh >= 0 && xh < nx;
        const bool inx0 = px > 0, inx1 = px < nx - 1, iny0 = yq > 0, iny1 = yq < ny - 1;
        auto slot = [&](int pz) { return zring + (pz & 3) * YM_SLOT; };
        auto row_of = [&](int pz) { return ((int64_t)pz * ny + yq) * nx + x0; };   // first row of plane pz's segment
        // loads take a workgroup-uniform base (the plane's segment) and a
        // 32-bit lane offset
        const int lo = xl * R + c, lh = (xh - x0) * R + c, ny_r = nx * R;
        double zc = 0.0, zh = 0.0;   // plane in flight: this lane's cell and halo cell
        auto zload = [&](int pz) {
          if (pz >= 0 && pz < nz) {
            const double* Zp = Z + row_of(pz) * R;
            zc = Zp[lo];
            if (hl) zh = Zp[lh];
          }
        };
        auto zput = [&](int pz) {
          if (pz >= 0 && pz < nz) {
            slot(pz)[(xl + 1) * R + c] = zc;
            if (hl) slot(pz)[(hs ? crw + 1 : 0) * R + c] = zh;
          }
        };
        // per plane: -y and +y neighbours (a missing one reads the cell
        // itself), the face weight of face c of the cell (lanes c < 6, in
        // op_row's order and indexing) and the cell's coefficient
        double ymv = 0.0, ypv = 0.0, fwv = 0.0, apv = 0.0;
        const int fc = min(c, 5);
        auto sload = [&](int pz) {
          const int64_t r0 = row_of(pz);
          const double* Zp = Z + r0 * R;
          ymv = Zp[iny0 ? lo - ny_r : lo];
          ypv = Zp[iny1 ? lo + ny_r : lo];
          const bool inf = fc == 0 ? inx0 : fc == 2 ? iny0 : fc == 4 ? pz > 0 : true;
          const int step = fc == 0 ? 1 : fc == 2 ? nx : (int)sxy;
          fwv = (FW + (int64_t)(fc / 2) * n + r0)[((fc & 1) == 0 && inf) ? xl - step : xl];
          apv = (AC + r0)[xl];
        };
        zload(z0 - 1);
        zput(z0 - 1);
        zload(z0);
        zput(z0);
        zload(z0 + 1);
        sload(z0);
        if (na == 0) return;   // uniform over the workgroup (one system), before any barrier
        const int sbase = (t & (WAVE - 1)) - c;   // lane of the cell's first right-hand side
        for (int pz = z0; pz < z1; ++pz) {
          zput(pz + 1);
          if (pz + 1 < z1) zload(pz + 2);
          // this plane's basis operands and q, p: used after the stencil
          // and the barrier that follows it (a float64 basis is loaded after
          // the stencil instead: its operands take twice the registers)
          const int64_t row0 = row_of(pz);
          const QS* Qp = Qt + row0 * kpq;
          QS a[8];
          auto aload = [&]() {
#pragma unroll
            for (int s = 0; s < 8; ++s) a[s] = Qp[(sl * rps + 4 * min(s, ksteps - 1) + lg) * kpq + 16 * I + lr];
          };
          if constexpr (sizeof(QS) != 8) aload();
          const double qi = (Qv + row0 * R)[lo], pi = (Pv + row0 * R)[lo];
          __syncthreads();
          // op_row's face loop: faces -x, +x, -y, +y, -z, +z
          const bool in[6] = {inx0, inx1, iny0, iny1, pz > 0, pz < nz - 1};
          const double aP = apv;
          const double own = slot(pz)[(xl + 1) * R + c];
          const double vn[6] = {slot(pz)[xl * R + c], slot(pz)[(xl + 2) * R + c], ymv, ypv,
                                slot(pz - 1)[(xl + 1) * R + c], slot(pz + 1)[(xl + 1) * R + c]};
          double d = 0.0, sum = 0.0;
#pragma unroll
          for (int f = 0; f < 6; ++f) {
            const double tf = __shfl(fwv, sbase + f);
            d += in[f] ? tf : 2.0 * aP;
            sum += in[f] ? tf * vn[f] : 0.0;
          }
          const double wval = d * own - sum;
          if (pz + 1 < z1) sload(pz + 1);
          if constexpr (sizeof(QS) == 8) aload();
          store_partial(&(Wout + row0 * R)[lo], wval);
          zw += own * wval;
          wv[t] = wval;
          __syncthreads();
#pragma unroll
          for (int s = 0; s < 8; ++s)
            if (s < ksteps) acc = mf_mma((double)a[s], lr < R ? wv[(sl * rps + 4 * s + lg) * R + lr] : 0.0, acc);
          e1 += own * qi + pi * wval;
        }
      }
    }
    if (!ym && !zm)
    for (int64_t ch = cr.c0; ch < cr.c1; ++ch) {
      const int64_t row0 = chunk_row0(S, ch);
      const int nrows = (int)min<int64_t>(S.chunk_rows, S.op.n - row0);
      QS a[8];   // A operands of this chunk, loaded before the stencil (rows past the chunk: a clamped row)
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int rr = min(sl * rps + 4 * min(s, ksteps - 1) + lg, nrows - 1);
        a[s] = Qt[(row0 + rr) * S.kp + 16 * I + lr];
      }
      double wval = 0.0;
      if (t / R < nrows) {
        const int64_t i = row0 + t / R;
        const int64_t g = i * R + c;
        int px, py, pz;
        decompose(S.op, i, px, py, pz);
        const double zi = Z[g], qi = Qv[g], pi = Pv[g];
        wval = op_row<double, MF>(S.op, i, px, py, pz, [&](int64_t j) { return Z[j * R + c]; });
        if (na != 0) {
          store_partial(&S.w[g], wval);
          zw += zi * wval;
          e1 += zi * qi + pi * wval;
        }
      }
      if (na == 0) return;   // uniform over the workgroup (one system), before any barrier
      __syncthreads();
      wv[t] = wval;   // rows past the chunk hold 0
      __syncthreads();
#pragma unroll
      for (int s = 0; s < 8; ++s)
        if (s < ksteps) acc = mf_mma((double)a[s], lr < R ? wv[(sl * rps + 4 * s + lg) * R + lr] : 0.0, acc);
    }
    if constexpr (sizeof(QS) == 2) {
      const double is = S.qscale[1];
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[v] *= is;
    }
    double* rec = S.rpart + (int64_t)lb * S.rw;
    const int KR = S.kp * R;
    if (WPT == 1) {
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (lr < R) store_partial(&rec[(16 * I + 4 * v + lg) * R + lr], acc[v]);
    } else {
      __syncthreads();
#pragma unroll
      for (int v = 0; v < 4; ++v) red[wave * 256 + v * 64 + lane] = acc[v];
      __syncthreads();
      for (int idx = t; idx < KR; idx += NT) {
        const int j = idx / R, cc = idx % R;
        double sum = 0.0;
        for (int q = 0; q < WPT; ++q) sum += red[(q * TI + j / 16) * 256 + mf_slot<double>(j % 16, cc)];
        store_partial(&rec[idx], sum);
      }
    }
    const double v2[2] = {zw, e1};
    block_sum_rhsk<2>(v2, R, buf, sh);
    if (t < 2 * R) store_partial(&rec[KR + t], buf[t]);
    restriction_epilogue(S, lb, red, sh, (it + 1) & 1);
    return;
  }
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  double zw = 0.0, e1 = 0.0;
  for (int64_t ch = cr.c0; ch < cr.c1; ++ch) {
    const int64_t row0 = chunk_row0(S, ch);
    const int nrows = (int)min<int64_t>(S.chunk_rows, S.op.n - row0);
    q_fetch<QS, NB>(Qt, row0, nrows, S.kp, m, 0, qb);
    double wval = 0.0;
    if (t / R < nrows) {
      const int64_t i = row0 + t / R;
      const int64_t g = i * R + c;
      int px, py, pz;
      decompose(S.op, i, px, py, pz);
      const double zi = Z[g], qi = Qv[g], pi = Pv[g];
      wval = op_row<double, MF>(S.op, i, px, py, pz, [&](int64_t j) { return Z[j * R + c]; });
      if (na != 0) {
        store_partial(&S.w[g], wval);
        zw += zi * wval;
        e1 += zi * qi + pi * wval;
      }
    }
    if (na == 0) return;   // uniform over the workgroup (one system), before any barrier
    __syncthreads();
    wv[t] = wval;
    __syncthreads();
    restrict_rows<QS, NB>(Qt, row0, nrows, S.kp, R, m, wv, qb, acc);
  }
  unscale_restriction<QS>(S, acc);
  double* rec = S.rpart + (int64_t)lb * S.rw;
  const int KR = S.kp * R;
  const double v2[2] = {zw, e1};
  if (pow2(R) && m.lpr * R <= WAVE && (NT / WAVE) * (KR + 2 * R) <= 4 * NT + 128) {
    restrict_finish_x2(m, S.kp, R, acc, v2, red, rec);
  } else {
    restrict_finish(m, S.kp, R, acc, red, rec);
    block_sum_rhsk<2>(v2, R, buf, sh);
    if (t < 2 * R) store_partial(&rec[KR + t], buf[t]);
  }
  restriction_epilogue(S, lb, red, sh, (it + 1) & 1);
}

// J_{2nu} sweeps for nu > 1 on the new residual r[rin] (written by the update
// phase, or by k_residual): first = 1 computes y2 = y1 + w D^-1 (r - A y1)
// with y1 = w D^-1 r; later sweeps y <- y + w D^-1 (r - A y).  Every RHS
// marked active in stat[spar] is swept.
template <typename PT>
__global__ __launch_bounds__(NT) void k_sweep(const SysDev* __restrict__ sys,
                                              const int* __restrict__ blk2sys, int nsys, int spar, int rin,
                                              int first, int src) {
  const SysDev& S = my_sys(sys, blk2sys, nsys);
  if (S.nact[spar] == 0) return;
  const int lb = xcd_remap(blockIdx.x - S.blk0, S.nblk);
  const int t = threadIdx.x, R = S.R, c = t % R;
  if (!S.stat[spar][c].active) return;
  const PT om = PT(S.omega);
  const double* Rin = S.r[rin];
  const PT* yin = static_cast<const PT*>(S.wj[src]);
  PT* yout = static_cast<PT*>(S.wj[first ? 0 : (src ^ 1)]);
  const ChunkRange cr = my_chunks(S, lb);
  auto dj = [&](int64_t j) -> PT { return (sizeof(PT) == 4) ? PT(S.dinv32[j]) : PT(S.dinv[j]); };
  for (int64_t ch = cr.c0; ch < cr.c1; ++ch) {
    const int64_t i = chunk_row0(S, ch) + t / R;
    if (t / R >= S.chunk_rows || i >= S.op.n) continue;
    int px, py, pz;
    decompose(S.op, i, px, py, pz);
    const PT ri = PT(Rin[i * R + c]);
    PT yi, ay;
    if (first) {
      auto y1 = [&](int64_t j) { return om * dj(j) * PT(Rin[j * R + c]); };
      yi = y1(i);
      ay = op_row<PT>(S.op, i, px, py, pz, y1);
    } else {
      yi = yin[i * R + c];
      ay = op_row<PT>(S.op, i, px, py, pz, [&](int64_t j) { return yin[j * R + c]; });
    }
    yout[i * R + c] = yi + om * dj(i) * (ri - ay);
  }
}

// Phases of the update kernel.
constexpr int PH_UPD = 1;   // decisions; p, q, x and the new residual
constexpr int PH_Z = 2;     // z = J r_new + Q c_new; partials r^T z, r^T z_old, ||r||^2

// Update kernel of iteration `it`.  Every workgroup sums the partials of the
// previous update kernel [r^T z | r^T z_old | ||r||^2 | p^T q] and the group
// records of the matvec kernel [Qt^T w | z^T w | z^T q_old + p_old^T w] in a
// fixed order and takes, per RHS, the same decisions:
//   convergence test on ||r||; beta; p^T q of the new pair from
//   z^T w + beta (z^T q_old + p_old^T w) + beta^2 p_old^T q_old; alpha;
//   g = A_c^-1 Q^T q = Qt^T w + beta g_old;  c_new = c - alpha g.
// Then per row: p = z + beta p_old; q = w + beta q_old (q double-buffered by
// parity); x += alpha p; r_new = r - alpha q (double-buffered); and, with
// PH_Z, z = J_2 r_new + Q c_new with J_2 formed from the neighbours' r_new
// (nu = 1; for nu > 1 J_{2nu} r_new comes from wj[wsrc]).  Partials of
// [r^T z | r^T z_old | ||r||^2 | p^T q] into bpart[(it+1)&1].
//   restart = 1: after k_residual (r in r[(it+1)&1], group records
//     [Qt^T r | ||r||^2 | ||f||^2]) for the RHS in `mask`: c = Qt^T r, no
//     update, `init` also takes ||f||^2, and the next iteration uses beta = 0.
//   phase = PH_UPD only (nu > 1): stops after r_new; phase = PH_Z only, not a
//     restart: z for the RHS the update phase advanced (stat[(it+1)&1]).
template <typename QS, bool MF, bool YM = false>
__global__ __launch_bounds__(NT, 4) void k_update(const SysDev* __restrict__ sys,
                                                  const int* __restrict__ blk2sys, int nsys, int it,
                                                  int restart, unsigned mask, int init, int phase, int wsrc) {
  using QT = typename Arith<QS>::type;   // arithmetic of the smoother and the prolongation
  __shared__ QT ws[NT];
  __shared__ QT ys[NT];
  __shared__ QT mfpart[MF ? (NT / WAVE) * 256 : 1];   // MFMA prolongation: per-wave partial tiles
  // line ring of the 2-D 9-point march: 4 lines of (segment + 2 halo cells) x R
  // smoother operands
  __shared__ QT yring[(YM && MF && sizeof(QT) == 4) ? 4 * YM_SLOT : 1];
  __shared__ double sh[NT + 16];
  // cvec: c_new = A_c^-1 Q^T r_new; gvec: g = A_c^-1 Q^T q; cg: the matvec (or
  // k_residual) group records, summed.  The region serves the final partial
  // sums once they are dead.
  __shared__ double big[3 * 2048 + 6 * MAXR];
  double* cvec = big;
  double* gvec = big + 2048;
  double* cg = big + 2 * 2048;   // [Qt^T w | z^T w | e1 | r^T z | r^T z_old | ||r||^2 | p^T q]
  __shared__ double buf[BW * MAXR];          // final partial sums
  __shared__ double s_alpha[MAXR], s_beta[MAXR];
  __shared__ int s_upd[MAXR], s_rs[MAXR], s_next[MAXR];
  const SysDev& S = my_sys(sys, blk2sys, nsys);
  mask &= S.rmask;
  const int cp = it & 1, nxt = (it + 1) & 1;
  const int KR = S.kp * S.R;
  const bool decide = restart || (phase & PH_UPD);
  const bool normal = decide && !restart;
  const int lb = xcd_remap(blockIdx.x - S.blk0, S.nblk);
  const int t = threadIdx.x, R = S.R, c = t % R;
  const Glob<const QS>* Q = (Glob<const QS>*)S.Q;
  const QMap m = q_map(S.kp, R);
  constexpr int NB = QB<QS>::NB;
  QBatch<QS, NB> qb;
  const ChunkRange cr = my_chunks(S, lb);
  // every load of the prologue is issued before the first wait, and the same
  // number of them on every path (waits complete in issue order, and a count
  // that depends on a branch makes the compiler wait for everything): status,
  // active counts, group records, coarse state (into registers), then the
  // first batch of Q
  // status of RHS t (threads t < R use it), loaded unconditionally
  const RhsStatus st0 = S.stat[cp][min(t, R - 1)];
  const int nact_cp = S.nact[cp], nact_nxt = S.nact[nxt];
  const int act_nxt = S.stat[nxt][min(t, R - 1)].active;
  const int ngrp = ticket_groups(S.nblk);
  const bool gfast = decide && rec_fits(ngrp, S.gw);
  double gv[8];
  {
    const int cnt = gfast ? S.gw : 1;
    const int groups = NT / cnt, e = t % cnt, g = t / cnt;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      gv[u] = S.rgrp[gfast ? (int64_t)min(g + u * groups, ngrp - 1) * S.gw + e : 0];
  }
  double cin_r[4], gin_r[4];   // kp*R <= 2048 = 4 NT
  {
    const auto cin = decide ? S.cstate[cp] : S.cstate[nxt];
    const auto gin = S.gstate[cp];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = min(t + u * NT, KR - 1);
      cin_r[u] = cin[idx];
      gin_r[u] = gin[idx];
    }
  }
  // a workgroup without a chunk issues the same loads on row 0
  const bool has = cr.c0 < cr.c1;
  int64_t row0 = has ? chunk_row0(S, cr.c0) : 0;
  int nrows = has ? (int)min<int64_t>(S.chunk_rows, S.op.n - row0) : 1;
  // MFMA prolongation: wave = row tile RT (of RTN) x column slice ks (of KS)
  // of kp / KS columns (nbk blocks of 16); a lane loads 4 consecutive columns
  // of one row per block, feeding 4 products
  const int mwave = t / WAVE, mlane = t % WAVE, mlr = mlane & 15, mlg = mlane >> 4;
  const int mRTN = S.chunk_rows / 16, mKS = (NT / WAVE) / mRTN;
  const int mRT = mwave % mRTN, mks = mwave / mRTN, mcols = S.kp / mKS, mnbk = mcols / 16;
  QBatch<QS, 2> q4;
  auto mf_fetch = [&](int64_t r0, int nr) {
#pragma unroll
    for (int blk = 0; blk < 2; ++blk)
      q4.load(blk, Q + (r0 + min(16 * mRT + mlr, nr - 1)) * S.kp + mks * mcols + 16 * min(blk, mnbk - 1) + 4 * mlg);
  };
  if constexpr (MF)
    mf_fetch(row0, nrows);
  else
    q_fetch<QS, NB>(Q, row0, nrows, S.kp, m, 0, qb);
  // float16 basis: c is multiplied by 1 / s_Q before the prolongation
  double isq = 1.0;
  if constexpr (sizeof(QS) == 2) isq = S.qscale[0];
  if (normal && nact_cp == 0) {
    // nothing iterates: carry the state over to the next parity
    if (blockIdx.x == S.blk0) {
      for (int idx = threadIdx.x; idx < KR; idx += NT) {
        S.cstate[nxt][idx] = S.cstate[cp][idx];
        S.gstate[nxt][idx] = S.gstate[cp][idx];
      }
      if (threadIdx.x < S.R) S.stat[nxt][threadIdx.x] = S.stat[cp][threadIdx.x];
      if (threadIdx.x == 0) {
        S.nact[nxt] = 0;
        *S.n_active = 0;
      }
    }
    return;
  }
  if (!decide && nact_nxt == 0) return;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int idx = t + u * NT;
    if (idx < KR) {
      cvec[idx] = cin_r[u];
      gvec[idx] = gin_r[u];
    }
  }
  if (decide) {
    if (gfast)
      rec_finish(gv, ngrp, S.gw, cg, sh);
    else
      sum_records<false>(S.rgrp, ngrp, S.gw, 0, S.gw, cg, sh);
    // ---- per-RHS decisions (identical in every workgroup) and the new state
    if (t < R) {
      // the status fields as scalars (a local struct would be placed in LDS)
      double gamma_old = st0.gamma_old, ff = st0.ff;
      int active = st0.active, iters = st0.iters, status = st0.status, rflag = st0.restart, conv = st0.conv;
      int upd = 0, next = 0, rs = 0;
      double alpha = 0.0, beta = 0.0;
      if (restart) {
        if ((mask >> t) & 1u) {
          if (init) ff = cg[KR + R + t];
          rflag = 1;
          conv = 0;
          if (!(ff <= 1.7e308)) {
            status = NLSP_E_NONFINITE;
          } else if (init && ff == 0.0) {
            // f = 0: the solution is u = 0 whatever the initial guess (the
            // host clears those columns of u); no iteration
            status = NLSP_OK;
          } else {
            status = NLSP_NOT_CONVERGED;
            next = 1;
          }
        } else {
          next = active;
        }
        upd = next && ((mask >> t) & 1u);
      } else if (active) {
        const double* up = cg + S.rw;   // the previous update's partials
        const double g = up[t], rz = up[R + t], rr = up[2 * R + t], pqo = up[3 * R + t];
        const double zw = cg[KR + t], e1 = cg[KR + R + t];
        const bool rr_ok = rr <= 1.7e308;                   // false for NaN / Inf
        const bool cv = rr_ok && rr <= S.tol2 * ff;
        rs = rflag;
        rflag = 0;
        if (cv) {
          status = NLSP_OK;
          conv = 1;
        } else if (!rr_ok || !finite_pos(g)) {
          // r^T z <= 0 with finite values is a breakdown; anything non-finite is not
          const bool gfin = g == g && fabs(g) <= 1.7e308;
          status = (gfin && rr_ok) ? NLSP_E_BREAKDOWN : NLSP_E_NONFINITE;
        } else if (iters >= S.maxit) {
          status = NLSP_NOT_CONVERGED;
        } else {
          beta = rs ? 0.0 : (S.flexible ? (g - rz) / gamma_old : g / gamma_old);
          const double pq = rs ? zw : zw + beta * e1 + beta * beta * pqo;
          gamma_old = g;
          if (!finite_pos(pq)) {
            status = (pq == pq && pq <= 1.7e308) ? NLSP_E_BREAKDOWN : NLSP_E_NONFINITE;
          } else {
            alpha = g / pq;
            upd = 1;
            next = 1;
            iters += 1;
          }
        }
      }
      s_alpha[t] = alpha;
      s_beta[t] = beta;
      s_upd[t] = upd;
      s_rs[t] = rs;
      s_next[t] = next;
      if (lb == 0) {
        RhsStatus nx{};
        nx.gamma_old = gamma_old;
        nx.ff = ff;
        nx.active = next;
        nx.iters = iters;
        nx.status = status;
        nx.restart = rflag;
        nx.conv = conv;
        S.stat[nxt][t] = nx;
      }
    }
    __syncthreads();
    // ---- coarse state: g = Qt^T q, c_new = c - alpha g (restart: c = Qt^T r)
    for (int idx = t; idx < KR; idx += NT) {
      const int r = idx % R;
      if (!s_upd[r]) continue;
      if (restart) {
        cvec[idx] = cg[idx];
        gvec[idx] = 0.0;
      } else {
        const double g = s_rs[r] ? cg[idx] : cg[idx] + s_beta[r] * gvec[idx];
        gvec[idx] = g;
        cvec[idx] -= s_alpha[r] * g;
      }
    }
    __syncthreads();
    if (lb == 0) {
      for (int idx = t; idx < KR; idx += NT) {
        S.cstate[nxt][idx] = cvec[idx];
        S.gstate[nxt][idx] = gvec[idx];
      }
      if (t == 0) {
        int cnt = 0;
        for (int k = 0; k < R; ++k) cnt += s_next[k];
        S.nact[nxt] = cnt;
        *S.n_active = cnt;
      }
    }
  } else {
    if (t < R) {
      s_upd[t] = act_nxt;   // advanced by the update phase
      s_alpha[t] = s_beta[t] = 0.0;
      s_rs[t] = 0;
    }
    __syncthreads();
  }
  // ---- the rows
  const bool upd = s_upd[c] != 0;
  const bool full = normal && (phase & PH_UPD);   // p, q, x, r_new formed here
  const double alpha = s_alpha[c], beta = s_beta[c];
  const bool rs = s_rs[c] != 0;
  const double* Rin = S.r[full ? cp : nxt];
  double* Rout = S.r[nxt];
  const double* Wv = S.w;
  const double* Qo = S.q[cp];
  double* Qn = S.q[nxt];
  // MFMA form: a workgroup marches through many chunks; the thread's own
  // entries of the row vectors of a later chunk are loaded at the end of the
  // current one.  They are the first loads a chunk waits for, so the order of
  // issue stays the order of use (waits complete in issue order; the basis
  // tile fetched ahead instead was measured slower).  With a float basis they
  // are loaded two chunks ahead: on z-ordered 3-D grids the next chunk is the
  // +z plane, whose r, w, q_old the stencil gathers, so that gather then hits
  // the cache (the float64 kernel has no registers left for the second set).
  // 3-D workload: mixed solve 1.43 -> 1.32 s (one ahead) -> 1.28 s (two
  // ahead), float64 1.71 -> 1.68 s.  The vector-lane float kernel loads them
  // one chunk ahead too (batched anisotropic leg, 16 chunks per workgroup:
  // 2.26 -> 2.12 s; 2-D solve 45.8 -> 45.55 ms).  There the smoother's centre
  // term is then formed from its own loads rather than shared with r_new, so
  // results move at float32 rounding level (same iteration counts).
  constexpr bool PF = MF || sizeof(QT) == 4;
  constexpr bool PF2 = MF && sizeof(QT) == 4;
  struct RowVals {
    double z, r, p, w, qo, x;
    float d;   // float inverse diagonal (two-ahead form only)
  } rv{}, rvn{};
  auto row_fetch_at = [&](RowVals& o, int64_t r1) {   // the chunk whose first row is r1
    const int nr = (int)min<int64_t>(S.chunk_rows, S.op.n - r1);
    const int64_t row = r1 + min(t / R, nr - 1);
    const int64_t gg = row * R + c;
    o.z = S.z[gg];
    o.r = Rin[gg];
    o.p = S.p[gg];
    o.w = Wv[gg];
    o.qo = Qo[gg];
    o.x = S.x[gg];
    if constexpr (PF2) o.d = S.dinv32[row];
  };
  auto row_fetch = [&](RowVals& o, int64_t ch1) { row_fetch_at(o, chunk_row0(S, ch1)); };
  // The chunk after the last of this workgroup belongs to the next workgroup;
  // on z-ordered grids it is still the +z plane of that last chunk (rvn is
  // read for r, w, q_old only, which this kernel does not write).
  const int64_t last_ch = S.nchunks - 1;
  if constexpr (PF)
    if (cr.c0 < cr.c1) {
      row_fetch(rv, cr.c0);
      if constexpr (PF2) row_fetch(rvn, min(cr.c0 + 1, last_ch));
    }
  auto qnew = [&](int64_t j) { return rs ? Wv[j * R + c] : Wv[j * R + c] + beta * Qo[j * R + c]; };
  auto rnew = [&](int64_t j) { return full ? Rin[j * R + c] - alpha * qnew(j) : Rin[j * R + c]; };
  auto dj = [&](int64_t j) -> QT { return (sizeof(QT) == 4) ? QT(S.dinv32[j]) : QT(S.dinv[j]); };
  // Two-ahead form on a z-ordered 3-D grid: the smoother's operand y = D^-1
  // r_new at the -z neighbour is this thread's own y of the previous chunk,
  // and at the +z neighbour it is formed from rvn, so neither plane is
  // gathered again (same expressions, same results).  For the first chunk the
  // -z value is gathered once here.  (3-D workload: mixed solve 1.28 ->
  // 1.23 s.)
  const bool zc = PF2 && S.op.kind == NLSP_OP_FV7 && S.op.nz > 1 && S.op.nx % S.chunk_rows == 0;
  QT yprev = QT(0);
  if constexpr (PF2) {
    if (zc && cr.c0 < cr.c1) {
      const int64_t r0c = chunk_row0(S, cr.c0);
      const int64_t i0 = r0c + min(t / R, (int)min<int64_t>(S.chunk_rows, S.op.n - r0c) - 1);
      const int64_t sxy = (int64_t)S.op.nx * S.op.ny;
      const int64_t j0 = i0 >= sxy ? i0 - sxy : i0;
      yprev = dj(j0) * QT(rnew(j0));
    }
  }
  QT e4[4];
  QT eb[2][4];   // MFMA: B operands c_new[k][lane % 16] for this lane's columns k
  if constexpr (MF) {
#pragma unroll
    for (int blk = 0; blk < 2; ++blk)
#pragma unroll
      for (int u = 0; u < 4; ++u)
        eb[blk][u] = mlr < R ? QT(cvec[(mks * mcols + 16 * min(blk, mnbk - 1) + 4 * mlg + u) * R + mlr] * isq)
                             : QT(0);
  } else {
#pragma unroll
    for (int u = 0; u < 4; ++u) e4[u] = QT(cvec[(4 * m.jc + u) * R + m.c] * isq);
  }
  const QT om = QT(S.omega);
  double gam = 0.0, rzo = 0.0, rr = 0.0, pq = 0.0;
  // 2-D 9-point operators, float basis: a march through y with the smoother
  // operands of three lines in an LDS ring.  The workgroup's chunks are
  // consecutive lines of one x-segment (chunk_row0), so the rows phase of line
  // y + 1 runs one chunk ahead of the stencil of line y and leaves each cell's
  // D^-1 r_new in the ring; only the cells just outside the segment and the
  // lines before the first and after the last chunk come from the global
  // vectors.  The gather path reads 27 float64 and 9 float32 values per lane
  // and chunk through the texture units instead (the same terms in the same
  // order; the two may contract them into FMAs differently).
  bool ym = false;
  if constexpr (PF2 && YM) {
    // (chunk indices fit 32 bits)
    const uint32_t ny32 = (uint32_t)S.op.ny;
    ym = (phase & PH_Z) && wsrc < 0 && S.ylines && cr.c0 < cr.c1 &&
         (uint32_t)cr.c0 / ny32 == (uint32_t)(cr.c1 - 1) / ny32;
    if (ym) {
      // descriptor fields in registers: the loop's stores would otherwise
      // make the compiler load them again
      const int nx = S.op.nx, ny = S.op.ny, crw = S.chunk_rows;
      double* const Pw = S.p;
      double* const Xw = S.x;
      double* const Zw = S.z;
      const bool flex = S.flexible != 0;
      const double* const cf = S.op.coef;   // the stencil (uniform loads)
      const int seg = (int)((uint32_t)cr.c0 / ny32);
      const int x0 = seg * crw;
      const int ly0 = (int)(cr.c0 - (int64_t)seg * ny), ly1 = ly0 + (int)(cr.c1 - cr.c0);
      auto row_of = [&](int ly) { return (int64_t)ly * nx + x0; };   // first row of line ly's segment
      const int xl = t / R;   // this lane's cell of the segment (every chunk is a whole line segment)
      auto slot = [&](int ly) { return yring + (ly & 3) * YM_SLOT; };
      auto yglob = [&](int64_t j) { return dj(j) * QT(rnew(j)); };
      // a line that no lane of this workgroup updates (the one before its
      // first line, the one after its last)
      auto line_glob = [&](int ly) {
        if (ly >= 0 && ly < ny && upd) slot(ly)[(xl + 1) * R + c] = yglob((int64_t)ly * nx + x0 + xl);
      };
      // the two cells of a line just outside the segment, lanes t < 2 R
      auto halo = [&](int ly) {
        if (ly < 0 || ly >= ny || t >= 2 * R || !upd) return;
        const int side = t / R, xh = side ? x0 + crw : x0 - 1;
        if (xh >= 0 && xh < nx) slot(ly)[(side ? crw + 1 : 0) * R + c] = yglob((int64_t)ly * nx + xh);
      };
      struct Cur {
        double ri, zo;
        QT d;
      };
      // the rows of line lyn from the row vectors in rv: p, q, x, r_new, and
      // the cell's D^-1 r_new into the ring
      auto rows_of = [&](int lyn, Cur& o) {
        const int64_t gg = (row_of(lyn) + xl) * R + c;
        o.ri = 0.0;
        o.zo = 0.0;
        o.d = QT(rv.d);
        if (!upd) return;
        o.zo = rv.z;
        if (full) {
          const double pi = rs ? o.zo : o.zo + beta * rv.p;
          const double qi = rs ? rv.w : rv.w + beta * rv.qo;
          store_partial(&Pw[gg], pi);
          store_partial(&Qn[gg], qi);
          store_partial(&Xw[gg], rv.x + alpha * pi);
          o.ri = rv.r - alpha * qi;
          pq += pi * qi;
        } else {
          o.ri = rv.r;
        }
        slot(lyn)[(xl + 1) * R + c] = o.d * QT(o.ri);
      };
      Cur cur, nxc;
      {
        line_glob(ly0 - 1);
        halo(ly0 - 1);
        rows_of(ly0, cur);
        halo(ly0);
        rv = rvn;
        // a line past the run is never used: its loads go to row 0, whose
        // lines every finishing workgroup reads and so stay in the L2
        row_fetch_at(rvn, ly0 + 2 < ly1 ? row_of(ly0 + 2) : 0);
      }
      for (int ly = ly0; ly < ly1; ++ly) {
        if (ly > ly0) {
          row0 = row_of(ly);
          nrows = crw;
          mf_fetch(row0, nrows);
        }
        if (ly + 1 < ly1)
          rows_of(ly + 1, nxc);
        else
          line_glob(ly + 1);
        halo(ly + 1);
        __syncthreads();
        const int64_t g = (row0 + xl) * R + c;
        QT wjv = QT(0);
        if (upd) {
          // the stencil of op_row (dy outer, dx inner, a term outside the
          // grid dropped by a select), operands from the ring
          QT ay = QT(0);
#pragma unroll
          for (int dy = -1; dy <= 1; ++dy) {
            const QT* sl = slot(ly + dy);
            const bool oky = ly + dy >= 0 && ly + dy < ny;
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
              const int xx = x0 + xl + dx;
              const bool ok = oky && xx >= 0 && xx < nx;
              const QT vj = sl[(xl + dx + 1) * R + c];
              ay += ok ? QT(cf[(dy + 1) * 3 + (dx + 1)]) * vj : QT(0);
            }
          }
          const QT yi = slot(ly)[(xl + 1) * R + c];   // this cell's own operand
          wjv = QT(2) * om * yi - om * om * cur.d * ay;
        }
        __syncthreads();
        ws[t] = wjv;
        {
          typename MfAcc<QT>::type pacc = {QT(0), QT(0), QT(0), QT(0)};
#pragma unroll
          for (int blk = 0; blk < 2; ++blk)
            if (blk < mnbk)
#pragma unroll
              for (int u = 0; u < 4; ++u) pacc = mf_mma(q4.get(blk, u), eb[blk][u], pacc);
#pragma unroll
          for (int v = 0; v < 4; ++v) mfpart[mwave * 256 + v * 64 + mlane] = pacc[v];
          __syncthreads();
          const int row = t / R, cc = t % R, sl2 = mf_slot<QT>(row % 16, cc);
          QT sum = QT(0);
#pragma unroll
          for (int k2 = 0; k2 < 4; ++k2)
            if (k2 < mKS) sum += mfpart[(k2 * mRTN + row / 16) * 256 + sl2];
          ys[t] = sum;
        }
        __syncthreads();
        if (upd) {
          const double zn = (double)ws[t] + (double)ys[t];
          if (full) store_partial(&Rout[g], cur.ri);
          store_partial(&Zw[g], zn);
          gam += cur.ri * zn;
          if (flex) rzo += cur.ri * cur.zo;
          rr += cur.ri * cur.ri;
        }
        cur = nxc;
        rv = rvn;
        row_fetch_at(rvn, ly + 3 < ly1 ? row_of(ly + 3) : 0);
      }
    }
  }
  if (!ym)
  for (int64_t ch = cr.c0; ch < cr.c1; ++ch) {
    if (ch > cr.c0) {
      row0 = chunk_row0(S, ch);
      nrows = (int)min<int64_t>(S.chunk_rows, S.op.n - row0);
      if (phase & PH_Z) {
        if constexpr (MF)
          mf_fetch(row0, nrows);
        else
          q_fetch<QS, NB>(Q, row0, nrows, S.kp, m, 0, qb);
      }
    }
    const bool mine = upd && t / R < nrows;
    const int64_t i = row0 + t / R;
    const int64_t g = i * R + c;
    double ri = 0.0, zo = 0.0;
    QT wjv = QT(0);
    if (mine) {
      zo = PF ? rv.z : S.z[g];
      if (full) {
        const double pi = rs ? zo : zo + beta * (PF ? rv.p : S.p[g]);
        const double qi = PF ? (rs ? rv.w : rv.w + beta * rv.qo) : qnew(i);
        // the vectors are written with device-coherent stores (store_partial):
        // they go to the coherence point shared by the XCDs, so the end of
        // the kernel has no dirty L2 lines of them to write back (measured on
        // the 2-D workload: 46.9 -> 45.9 ms per solve, against 46.3 ms with
        // nontemporal stores)
        store_partial(&S.p[g], pi);
        store_partial(&Qn[g], qi);
        store_partial(&S.x[g], (PF ? rv.x : S.x[g]) + alpha * pi);
        ri = (PF ? rv.r : Rin[g]) - alpha * qi;
        pq += pi * qi;
        if (!(phase & PH_Z)) store_partial(&Rout[g], ri);
      } else {
        ri = PF ? rv.r : Rin[g];
      }
      if (phase & PH_Z) {
        if (wsrc < 0) {
          int px, py, pz;
          decompose(S.op, i, px, py, pz);
          auto y = [&](int64_t j) { return dj(j) * QT(rnew(j)); };
          const QT yi = dj(i) * QT(ri);
          QT ay;
          if constexpr (PF2) {
            if (zc) {
              const double rz = full ? rvn.r - alpha * (rs ? rvn.w : rvn.w + beta * rvn.qo) : rvn.r;
              const QT yzp = QT(rvn.d) * QT(rz);
              ay = op_row<QT, MF, true>(S.op, i, px, py, pz, y, yprev, yzp);
            } else {
              ay = op_row<QT, MF>(S.op, i, px, py, pz, y);
            }
            yprev = yi;
          } else {
            ay = op_row<QT, MF>(S.op, i, px, py, pz, y);
          }
          wjv = QT(2) * om * yi - om * om * dj(i) * ay;
        } else {
          wjv = static_cast<const QT*>(S.wj[wsrc])[g];
        }
      }
    }
    if (phase & PH_Z) {
      __syncthreads();
      ws[t] = wjv;
      if constexpr (MF) {
        typename MfAcc<QT>::type pacc = {QT(0), QT(0), QT(0), QT(0)};
#pragma unroll
        for (int blk = 0; blk < 2; ++blk)
          if (blk < mnbk)
#pragma unroll
            for (int u = 0; u < 4; ++u) pacc = mf_mma(q4.get(blk, u), eb[blk][u], pacc);
#pragma unroll
        for (int v = 0; v < 4; ++v) mfpart[mwave * 256 + v * 64 + mlane] = pacc[v];
        __syncthreads();
        // ys[row * R + c]: the column slices of row tile row / 16, in order
        {
          const int row = t / R, cc = t % R, slot = mf_slot<QT>(row % 16, cc);
          QT sum = QT(0);
#pragma unroll
          for (int k2 = 0; k2 < 4; ++k2)
            if (k2 < mKS) sum += mfpart[(k2 * mRTN + row / 16) * 256 + slot];
          ys[t] = sum;
        }
      } else {
        prolong_rows<QS, NB>(Q, row0, nrows, S.kp, R, m, e4, qb, ys);
      }
      __syncthreads();
      if (mine) {
        const double zn = (double)ws[t] + (double)ys[t];
        if (full) store_partial(&Rout[g], ri);
        store_partial(&S.z[g], zn);
        gam += ri * zn;
        if (S.flexible) rzo += ri * zo;
        rr += ri * ri;
      }
    }
    if constexpr (PF2) {
      rv = rvn;
      row_fetch(rvn, min(ch + 2, last_ch));
    } else if constexpr (PF) {
      row_fetch(rv, min(ch + 1, cr.c1 - 1));
    }
  }
  double* bp = S.bpart[nxt] + (int64_t)lb * BW * R;
  static_assert(3 * 2048 + 6 * MAXR >= BW * (NT + 16), "partial-sum scratch");
  if (phase & PH_Z) {
    const double v4[4] = {gam, rzo, rr, pq};
    block_sum_rhsk<4>(v4, R, buf, big);   // cvec, gvec, cg are dead here
    // p^T q: this kernel's (full), none at a restart, the update phase's otherwise
    const int nw = (full || restart) ? BW * R : 3 * R;
    if (t < nw) bp[t] = buf[t];
  } else {
    const double v1[1] = {pq};
    block_sum_rhsk<1>(v1, R, buf, sh);
    if (t < R) bp[3 * R + t] = buf[t];
  }
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
    const int64_t i = chunk_row0(S, ch) + t / R;
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

// Largest |X| over cnt floats, as the bits of a non-negative float (ordered
// as unsigned integers): one atomic max per wave into *out (zeroed before).
// The maximum does not depend on the order, so the result is deterministic.
__global__ __launch_bounds__(256) void k_absmax(const float* __restrict__ X, int64_t cnt, unsigned* out) {
  float mx = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x)
    mx = fmaxf(mx, fabsf(X[i]));
  for (int o = WAVE / 2; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, WAVE));
  if ((threadIdx.x & (WAVE - 1)) == 0) atomicMax(out, __float_as_uint(mx));
}

// Y = float16(X s) with s = 2^-e, e the binary exponent of max |X| (so that
// |X s| < 1 and the large entries keep float16's 11 significant bits);
// inv[0] and inv[1] receive 1 / s = 2^e.  s = 1 for an all-zero X.
__global__ __launch_bounds__(256) void k_to_half(const float* __restrict__ X, int64_t cnt,
                                                 const unsigned* __restrict__ maxbits, _Float16* __restrict__ Y,
                                                 double* inv) {
  const float mx = __uint_as_float(*maxbits);
  int e = 0;
  if (mx > 0.f) (void)frexpf(mx, &e);
  const float sc = ldexpf(1.f, -e);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x)
    Y[i] = (_Float16)(X[i] * sc);
  if (blockIdx.x == 0 && threadIdx.x < 2) inv[threadIdx.x] = ldexp(1.0, e);
}

// B = A^T for a (kp, kp) matrix
__global__ void k_transpose_sq(const double* __restrict__ A, int kp, double* __restrict__ B) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= kp * kp) return;
  B[(idx % kp) * kp + idx / kp] = A[idx];
}

__global__ void k_zero_cols(double* u, int64_t n, int R, unsigned mask) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n * R) return;
  if ((mask >> (g % R)) & 1u) u[g] = 0.0;
}

// ----------------------------------------- the capturable (device-loop) form
// Everything the host-polled solve does with copies, fills and reads from the
// host is done here by kernels whose data travel as kernel arguments, so the
// whole solve can be enqueued without synchronising (and captured in a graph).

// the columns of u whose right-hand side is zero (||f||^2 = 0 in the status
// the start-up wrote) are cleared: u = 0 solves them whatever the guess
__global__ void k_zero_cols_dev(double* u, int64_t n, int R, const RhsStatus* __restrict__ st) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n * R) return;
  if (st[g % R].ff == 0.0) u[g] = 0.0;
}

__global__ void k_fill_zero(uint32_t* p, int64_t words) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// start state: every RHS active with a fresh direction (iteration -1 reads
// stat[1]); counters nact(0) = 0, nact(1) = R, active = 0
__global__ void k_init_batch(int nsys, int R, RhsStatus* __restrict__ stat1, int* __restrict__ counters) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < nsys * R) {
    RhsStatus s{};
    s.gamma_old = 1.0;
    s.active = 1;
    s.restart = 1;
    s.status = NLSP_NOT_CONVERGED;
    stat1[g] = s;
  }
  if (g < nsys * 4) counters[g] = (g % 4 == 1) ? R : 0;
}

// a host block (descriptors, block map) carried to device memory as a kernel
// argument
constexpr int PUT_BYTES = 2048;
struct PutChunk {
  unsigned char b[PUT_BYTES];
};
__global__ void k_put_bytes(unsigned char* __restrict__ dst, PutChunk c, int nbytes) {
  for (int i = threadIdx.x; i < nbytes; i += blockDim.x) dst[i] = c.b[i];
}

// per RHS: iterations, status and the true relative residual; a RHS whose
// recursive residual passed but whose true residual did not is reported
// NOT_CONVERGED (this form has no residual replacement)
__global__ void k_finalize(const SysDev* __restrict__ sys, int nsys, int R, const RhsStatus* __restrict__ stat,
                           const double* __restrict__ rr_true, nlsp_rhs_info* __restrict__ info) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nsys * R) return;
  const RhsStatus s = stat[g];
  const double rrt = rr_true[g];
  nlsp_rhs_info o;
  o.iters = s.iters;
  o.status = s.status;
  o.relres = (s.ff > 0.0) ? sqrt(rrt / s.ff) : 0.0;
  if (s.status == NLSP_OK && s.ff > 0.0 && !(rrt <= sys[g / R].tol2 * s.ff)) o.status = NLSP_NOT_CONVERGED;
  info[g] = o;
}

// ------------------------------------------------------------- host side
// ------------------------------------------------------------------ host side
// Per-system buffers.  The arrays that must start at zero come first and are
// carved for every system of a batch before anything else, so one fill clears
// them all.
struct SolveLayout {
  double *p, *q0, *q1, *z, *w, *cstate0, *cstate1, *gstate0, *gstate1;
  unsigned* ticket;
  unsigned* qmax;   // [2] max |W| as float bits (float16 basis; one used)
  double* qscale;   // [2] 1 / s for the restriction and the prolongation (float16 basis)
  double *r0, *r1, *dinv, *bpart0, *bpart1, *rpart, *rgrp, *dpart, *Ainv, *Qt;
  float* dinv32;
  void *wj0, *wj1;
  double* fw64;   // face weights (null unless SysShape::faces)
  float* fw32;
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
  bool faces;   // face weights of a finite-volume operator formed once per solve
};

// In the matrix-core form (16 right-hand sides) every lane of a row would form
// the row's harmonic face means itself (float64 divisions in the matvec
// kernel); there they are formed once per solve into the workspace (3 n
// float64 + 3 n float32) and read instead (3-D workload: mixed solve 1.49 ->
// 1.43 s, float64 1.87 -> 1.71 s, bit-identical results).  The other forms
// keep forming them: a run-time switch between the two in those kernels cost
// the one-RHS 2-D solve 3 %.
inline bool use_faces(const nlsp_operator* A, int R, int kp) {
  return mf_ok(R, kp) && (A->kind == NLSP_OP_FV5 || A->kind == NLSP_OP_FV7);
}

// Workgroups per system: one per chunk of NT / R rows up to 512 (two per CU)
// for a single system, or, in a batch, one per `rows_per_block` rows.
inline int solver_blocks(int64_t nchunks) { return (int)std::min<int64_t>(nchunks, 512); }

inline int restriction_width(int kp, int R) { return kp * R + 2 * R; }

inline SysShape shape_of(int64_t n, int kp, int R, int rows_per_block, bool faces) {
  SysShape h;
  h.n = n;
  h.faces = faces;
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
  L.p = cv.take<double>(nR);
  L.q0 = cv.take<double>(nR);
  L.q1 = cv.take<double>(nR);
  L.z = cv.take<double>(nR);
  L.w = cv.take<double>(nR);
  L.cstate0 = cv.take<double>((size_t)h.kp * h.R);
  L.cstate1 = cv.take<double>((size_t)h.kp * h.R);
  L.gstate0 = cv.take<double>((size_t)h.kp * h.R);
  L.gstate1 = cv.take<double>((size_t)h.kp * h.R);
  L.ticket = cv.take<unsigned>(ticket_words(h.nblk));
  L.qmax = cv.take<unsigned>(2);
}

inline void carve_rest(Carver& cv, const SysShape& h, SolveLayout& L) {
  const int64_t nR = h.n * h.R;
  const int rw = restriction_width(h.kp, h.R);
  L.r0 = cv.take<double>(nR);
  L.r1 = cv.take<double>(nR);
  L.wj0 = cv.take<double>(nR);
  L.wj1 = cv.take<double>(nR);
  L.dinv = cv.take<double>(h.n);
  L.dinv32 = cv.take<float>(h.n);
  L.fw64 = h.faces ? cv.take<double>((size_t)3 * h.n) : nullptr;
  L.fw32 = h.faces ? cv.take<float>((size_t)3 * h.n) : nullptr;
  L.bpart0 = cv.take<double>((size_t)h.nblk * BW * h.R);
  L.bpart1 = cv.take<double>((size_t)h.nblk * BW * h.R);
  L.rpart = cv.take<double>((size_t)h.nblk * rw);
  L.rgrp = cv.take<double>((size_t)ticket_groups(h.nblk) * (rw + BW * h.R));
  L.dpart = cv.take<double>((size_t)h.nblk * h.R);
  L.Ainv = cv.take<double>((size_t)h.kp * h.kp);
  // sized for float64 and used as the type of Q; a float16 basis carves it
  // into W s (float16, n kp) and W (float32, formed first, at 4 n kp bytes)
  L.Qt = cv.take<double>((size_t)h.n * h.kp);
  L.qscale = cv.take<double>(2);
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
  hs.op.fw64 = as_glob((const double*)L.fw64);
  hs.op.fw32 = as_glob((const float*)L.fw32);
  hs.R = R;
  hs.kp = h.kp;
  hs.nblk = h.nblk;
  hs.blk0 = blk0;
  hs.chunk_rows = h.chunk_rows;
  hs.nchunks = h.nchunks;
  hs.cpb = (h.nchunks + h.nblk - 1) / h.nblk;
  hs.rw = restriction_width(h.kp, R);
  hs.gw = hs.rw + BW * R;
  hs.Q = as_glob((M.prec == NLSP_FP64) ? (const void*)M.Q64 : (const void*)M.Q32);
  hs.Qt = as_glob((const void*)L.Qt);
  hs.qscale = as_glob((const double*)L.qscale);
  hs.qsrc = M.Q32;
  if (M.prec == NLSP_MIXED_F16) {
    // one float16 matrix W s serves the restriction and the prolongation
    hs.Q = as_glob((const void*)L.Qt);
    hs.Qt = as_glob((const void*)L.Qt);
  }
  hs.Linv = as_glob((const double*)M.Linv);
  hs.Ainv = as_glob(L.Ainv);
  hs.f = as_glob(f);
  hs.x = as_glob(u);
  hs.r[0] = as_glob(L.r0);
  hs.r[1] = as_glob(L.r1);
  hs.p = as_glob(L.p);
  hs.q[0] = as_glob(L.q0);
  hs.q[1] = as_glob(L.q1);
  hs.z = as_glob(L.z);
  hs.w = as_glob(L.w);
  hs.wj[0] = as_glob((void*)L.wj0);
  hs.wj[1] = as_glob((void*)L.wj1);
  hs.dinv = as_glob(L.dinv);
  hs.dinv32 = as_glob(L.dinv32);
  hs.bpart[0] = as_glob(L.bpart0);
  hs.bpart[1] = as_glob(L.bpart1);
  hs.rpart = as_glob(L.rpart);
  hs.rgrp = as_glob(L.rgrp);
  hs.cstate[0] = as_glob(L.cstate0);
  hs.cstate[1] = as_glob(L.cstate1);
  hs.gstate[0] = as_glob(L.gstate0);
  hs.gstate[1] = as_glob(L.gstate1);
  hs.dpart = as_glob(L.dpart);
  hs.ticket = as_glob(L.ticket);
  hs.stat[0] = as_glob(B.stat0 + (size_t)i * R);
  hs.stat[1] = as_glob(B.stat1 + (size_t)i * R);
  hs.nact = as_glob(B.counters + 4 * i);
  hs.n_active = as_glob(B.counters + 4 * i + 2);
  hs.rr_true = as_glob(B.rr_true + (size_t)i * R);
  hs.nu = M.nu;
  hs.omega = M.omega;
  hs.tol2 = opts->rtol * opts->rtol;
  hs.maxit = opts->maxit;
  hs.flexible = opts->flexible ? 1 : 0;
  hs.rmask = 0xffffffffu;
  hs.zorder = (A.nz > 1 && A.nx % h.chunk_rows == 0) ? 1 : 0;
  hs.ylines = (A.kind == NLSP_OP_STENCIL9 && A.nz <= 1 && A.ny > 1 && A.nx % h.chunk_rows == 0 &&
               mf_ok(R, h.kp) && h.chunk_rows == NT / R)
                  ? 1
                  : 0;
  hs.nxq = A.nx / h.chunk_rows;
  return hs;
}

// One solve of `nsys` systems (nsys = 1: pcg_solve).  Every system advances
// in the same launches; a system whose right-hand sides have all stopped
// exits its workgroups at their first instruction.  The host polls the
// per-system active counts every `check_every` iterations; with `graph` the
// check_every iterations are captured once in a hipGraph and replayed (their
// kernels read the iteration only through its parity, and check_every is
// even).
template <typename QS>
static int run_pcg(int nsys, std::vector<SysDev>& hs, const BatchLayout& B, const std::vector<SolveLayout>& Ls,
                   const nlsp_pcg_opts* opts, nlsp_rhs_info* info, bool graph, hipStream_t stream,
                   nlsp_rhs_info* info_dev = nullptr) {
  using QT = typename Arith<QS>::type;
  const int R = hs[0].R;
  int nblk = 0;
  bool mf = true;   // MFMA basis passes when every system's (R, kp) has the matrix-core form
  bool ym = false;  // some system has the 2-D line march
  bool zmk = false; // some system has the 3-D plane march of the matvec kernel
  for (const auto& h : hs) {
    zmk = zmk || (h.zorder && h.op.kind == NLSP_OP_FV7);
    nblk += h.nblk;
    mf = mf && mf_ok(h.R, h.kp) && h.chunk_rows == NT / h.R;
    ym = ym || h.ylines;
  }
  // the marching kernels are separate instantiations, so that the others
  // keep their registers; the float64 update kernel has none left for a ring
  constexpr bool YMK = sizeof(QT) == 4;
  ym = ym && mf;
  // the matrix-core kernels read the face weights of finite-volume operators
  for (const auto& h : hs)
    if (mf && (h.op.kind == NLSP_OP_FV5 || h.op.kind == NLSP_OP_FV7) && h.op.fw64 == nullptr) return NLSP_E_INVALID;
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
  // the update kernel(s) of iteration `it`: one launch for nu = 1; for
  // nu > 1 the update phase, the J_{2nu} sweeps on r_new and the z phase
  auto launch_update = [&](hipStream_t st, int it, int restart, unsigned mask, int init, bool can_time) {
    auto upd = [&](int phase, int wsrc, bool timed_one) {
      if (timed_one) {
        timed(1, [&](hipEvent_t a, hipEvent_t b) {
          if (ym && YMK)
            hipExtLaunchKernelGGL((k_update<QS, true, YMK>), grid, block, 0, st, a, b, 0, dsys, b2s, nsys, it,
                                  restart, mask, init, phase, wsrc);
          else if (mf)
            hipExtLaunchKernelGGL((k_update<QS, true>), grid, block, 0, st, a, b, 0, dsys, b2s, nsys, it, restart,
                                  mask, init, phase, wsrc);
          else
            hipExtLaunchKernelGGL((k_update<QS, false>), grid, block, 0, st, a, b, 0, dsys, b2s, nsys, it, restart,
                                  mask, init, phase, wsrc);
        });
      } else {
        if (ym && YMK)
          hipLaunchKernelGGL((k_update<QS, true, YMK>), grid, block, 0, st, dsys, b2s, nsys, it, restart, mask,
                             init, phase, wsrc);
        else if (mf)
          hipLaunchKernelGGL((k_update<QS, true>), grid, block, 0, st, dsys, b2s, nsys, it, restart, mask, init,
                             phase, wsrc);
        else
          hipLaunchKernelGGL((k_update<QS, false>), grid, block, 0, st, dsys, b2s, nsys, it, restart, mask, init,
                             phase, wsrc);
      }
    };
    if (nu == 1) {
      upd(restart ? PH_Z : (PH_UPD | PH_Z), -1, can_time);
      return;
    }
    int spar = it & 1;
    if (!restart) {
      upd(PH_UPD, -1, can_time);
      spar = (it + 1) & 1;
    }
    const int rin = (it + 1) & 1;
    hipLaunchKernelGGL(k_sweep<QT>, grid, block, 0, st, dsys, b2s, nsys, spar, rin, 1, 0);
    int src = 0;
    for (int s = 1; s < 2 * nu - 1; ++s) {
      hipLaunchKernelGGL(k_sweep<QT>, grid, block, 0, st, dsys, b2s, nsys, spar, rin, 0, src);
      src ^= 1;
    }
    upd(PH_Z, src, false);
  };
  auto launch_matvec = [&](hipStream_t st, int it, bool can_time) {
    if (can_time) {
      timed(2, [&](hipEvent_t a, hipEvent_t b) {
        if (ym)
          hipExtLaunchKernelGGL((k_matvec<QS, true, true>), grid, block, 0, st, a, b, 0, dsys, b2s, nsys, it);
        else if (mf && zmk)
          hipExtLaunchKernelGGL((k_matvec<QS, true, false, true>), grid, block, 0, st, a, b, 0, dsys, b2s, nsys, it);
        else if (mf)
          hipExtLaunchKernelGGL((k_matvec<QS, true>), grid, block, 0, st, a, b, 0, dsys, b2s, nsys, it);
        else
          hipExtLaunchKernelGGL((k_matvec<QS, false>), grid, block, 0, st, a, b, 0, dsys, b2s, nsys, it);
      });
    } else {
      if (ym)
        hipLaunchKernelGGL((k_matvec<QS, true, true>), grid, block, 0, st, dsys, b2s, nsys, it);
      else if (mf && zmk)
        hipLaunchKernelGGL((k_matvec<QS, true, false, true>), grid, block, 0, st, dsys, b2s, nsys, it);
      else if (mf)
        hipLaunchKernelGGL((k_matvec<QS, true>), grid, block, 0, st, dsys, b2s, nsys, it);
      else
        hipLaunchKernelGGL((k_matvec<QS, false>), grid, block, 0, st, dsys, b2s, nsys, it);
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
    // (C casts: the descriptor's pointers carry the device's address space)
    hipLaunchKernelGGL(k_dinv, dim3(ceil_div(hs[i].op.n, NT)), block, 0, stream, hs[i].op, (double*)hs[i].dinv,
                       (float*)hs[i].dinv32);
    if (hs[i].op.fw64 != nullptr) {
      // formed from a copy of the descriptor without them (op_row is not used here)
      OpDev o = hs[i].op;
      double* f64 = (double*)o.fw64;
      float* f32 = (float*)o.fw32;
      o.fw64 = nullptr;
      o.fw32 = nullptr;
      hipLaunchKernelGGL(k_faces, dim3(ceil_div(o.n, NT)), block, 0, stream, o, f64, f32);
    }
    if constexpr (sizeof(QS) != 2)
      hipLaunchKernelGGL(k_coarse_inverse, dim3(ceil_div(hs[i].kp * hs[i].kp, 256)), dim3(256), 0, stream,
                         (const double*)hs[i].Linv, hs[i].kp, (double*)hs[i].Ainv);
    if constexpr (sizeof(QS) == 2) {
      // float16 basis: the coarse term Q A_c^-1 Q^T = W W^T, W = Q L^-T,
      // formed in float32 (float64 sums), then stored once as W s in
      // float16 and used by both the restriction (c = W^T r) and the
      // prolongation (W c).  With one rounded matrix on both sides the
      // preconditioner stays exactly symmetric; rounding Q and Q A_c^-1
      // separately made it slightly nonsymmetric, which cost up to 10 % more
      // iterations on small anisotropic systems.
      const int64_t cnt = hs[i].op.n * hs[i].kp;
      const float* q32 = static_cast<const float*>(hs[i].qsrc);
      _Float16* w16 = reinterpret_cast<_Float16*>(Ls[i].Qt);
      float* w32 = reinterpret_cast<float*>(w16 + 2 * cnt);
      double* linvT = Ls[i].Ainv;
      const dim3 cg((unsigned)std::min<int64_t>(1024, ceil_div(cnt, 256)));
      hipLaunchKernelGGL(k_transpose_sq, dim3(ceil_div(hs[i].kp * hs[i].kp, 256)), dim3(256), 0, stream,
                         (const double*)hs[i].Linv, hs[i].kp, linvT);
      hipLaunchKernelGGL(k_qtilde<float>, dim3(ceil_div(hs[i].op.n, 64)), dim3(256), 0, stream, q32,
                         (const double*)linvT, hs[i].op.n, hs[i].kp, w32);
      hipLaunchKernelGGL(k_absmax, cg, dim3(256), 0, stream, (const float*)w32, cnt, Ls[i].qmax);
      hipLaunchKernelGGL(k_to_half, cg, dim3(256), 0, stream, (const float*)w32, cnt, (const unsigned*)Ls[i].qmax,
                         w16, Ls[i].qscale);
    } else {
      hipLaunchKernelGGL(k_qtilde<QS>, dim3(ceil_div(hs[i].op.n, 64)), dim3(256), 0, stream, (const QS*)hs[i].Q,
                         (const double*)hs[i].Ainv, hs[i].op.n, hs[i].kp, (QS*)hs[i].Qt);
    }
  }
  // start-up as iteration -1: r = f - A x into r[0], the update kernel in
  // restart mode (c = Qt^T r, z = M^-1 r), then w = A z
  hipLaunchKernelGGL(k_residual<QS>, grid, block, 0, stream, dsys, b2s, nsys, all, 0);
  launch_update(stream, -1, 1, all, 1, true);
  launch_matvec(stream, -1, true);
  NLSP_RUN(hipGetLastError());
  if (info_dev) {
    // device loop: zero right-hand sides cleared on the device, then a fixed
    // budget of maxit iterations (the decisions of update kernel maxit stop
    // whatever still iterates), the true residuals and the per-RHS results,
    // all enqueued without waiting; a system whose right-hand sides have all
    // stopped leaves the remaining launches at their first instructions
    for (int i = 0; i < nsys; ++i)
      hipLaunchKernelGGL(k_zero_cols_dev, dim3(ceil_div(hs[i].op.n * R, 256)), dim3(256), 0, stream, hs[i].x,
                         hs[i].op.n, R, B.stat0 + (size_t)i * R);
    const int maxit = hs[0].maxit;
    for (int it = 0; it <= maxit; ++it) {
      launch_update(stream, it, 0, 0u, 0, false);
      if (it < maxit) launch_matvec(stream, it, false);
    }
    hipLaunchKernelGGL(k_true_residual, grid, block, 0, stream, dsys, b2s, nsys);
    hipLaunchKernelGGL(k_true_finish, dim3(nsys), block, 0, stream, dsys);
    hipLaunchKernelGGL(k_finalize, dim3(ceil_div(nsys * R, 256)), dim3(256), 0, stream, dsys, nsys, R,
                       ((maxit + 1) & 1) ? (const RhsStatus*)B.stat1 : (const RhsStatus*)B.stat0,
                       (const double*)B.rr_true, info_dev);
    NLSP_RUN(hipGetLastError());
    release();
    return NLSP_OK;
  }
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
            launch_update(cs, it + k, 0, 0u, 0, false);
            launch_matvec(cs, it + k, false);
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
          launch_update(stream, it, 0, 0u, 0, true);
          launch_matvec(stream, it, true);
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
        // the recursive residual passed but the true one did not and no
        // replacement is left (maxit reached or the replacement guard spent)
        if (s.status == NLSP_OK && s.ff > 0.0 && !(rrt[j] <= hs[j / R].tol2 * s.ff))
          info[j].status = NLSP_NOT_CONVERGED;
        const int st = info[j].status;
        if (st < 0 && (worst >= 0 || st < worst)) worst = st;
        if (st == NLSP_NOT_CONVERGED && worst == NLSP_OK) worst = NLSP_NOT_CONVERGED;
      }
      release();
      return worst;
    }
    // residual replacement: r = f - A x for the `redo` RHS into r[it & 1] and
    // those RHS restart from it (the update kernel in restart mode as iteration it - 1,
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
    hipLaunchKernelGGL(k_residual<QS>, grid, block, 0, stream, dsys, b2s, nsys, all, it & 1);
    launch_update(stream, it - 1, 1, all, 0, true);
    launch_matvec(stream, it - 1, true);
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
  if (M->prec == NLSP_FP64 ? !M->Q64 : ((M->prec == NLSP_MIXED || M->prec == NLSP_MIXED_F16) ? !M->Q32 : true))
    return false;
  if ((int64_t)M->k > n) return false;
  return true;
}

inline bool opts_ok(const nlsp_pcg_opts* o) {
  return o && o->rtol > 0 && o->maxit >= 1 && o->check_every >= 1;
}

// Tiles chosen by pcg_solve_batched_tune, per batch shape: the device, the
// basis precision, R, k, nu and every system's operator kind and size, in
// order.  rows_per_block = -1 in the batched entry points looks the shape up.
struct TuneKey {
  int dev, prec, R, k, nu;
  std::vector<int64_t> sys;   // kind, n for each system
  bool operator<(const TuneKey& o) const {
    return std::tie(dev, prec, R, k, nu, sys) < std::tie(o.dev, o.prec, o.R, o.k, o.nu, o.sys);
  }
};
static std::mutex g_tune_mu;
static std::map<TuneKey, int> g_tuned;

static bool tune_key(int nsys, const nlsp_system* sys, int R, TuneKey& key) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  key.dev = dev;
  key.prec = sys[0].M.prec;
  key.R = R;
  key.k = sys[0].M.k;
  key.nu = sys[0].M.nu;
  key.sys.resize(2 * (size_t)nsys);
  for (int i = 0; i < nsys; ++i) {
    key.sys[2 * (size_t)i] = sys[i].A.kind;
    key.sys[2 * (size_t)i + 1] = op_size(&sys[i].A);
  }
  return true;
}

// rows_per_block -1: the tile recorded for this batch shape on the current
// device, or 0 (the default plan) when none was; other values unchanged
static bool tuned_tile(int nsys, const nlsp_system* sys, int R, int* rpb) {
  TuneKey key;
  if (!tune_key(nsys, sys, R, key)) return false;
  std::lock_guard<std::mutex> g(g_tune_mu);
  const auto it = g_tuned.find(key);
  if (it == g_tuned.end()) return false;
  *rpb = it->second;
  return true;
}
static int resolve_tile(int nsys, const nlsp_system* sys, int R, int rows_per_block) {
  int rpb = 0;
  if (rows_per_block != -1) return rows_per_block;
  return tuned_tile(nsys, sys, R, &rpb) ? rpb : 0;
}

// Sets up and runs a batch; nsys = 1 and rows_per_block = 0 is pcg_solve.
static int solve_batch(int nsys, const nlsp_operator* const* As, const nlsp_two_level* const* Ms,
                       const double* const* fs, double* const* us, int R, int rows_per_block,
                       const nlsp_pcg_opts* opts, nlsp_rhs_info* info, void* ws, size_t ws_bytes, bool graph,
                       hipStream_t stream, nlsp_rhs_info* info_dev = nullptr) {
  std::vector<SysShape> sh(nsys);
  for (int i = 0; i < nsys; ++i)
    sh[i] = shape_of(op_size(As[i]), padded_rank(Ms[i]->k), R, rows_per_block,
                     use_faces(As[i], R, padded_rank(Ms[i]->k)));
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
  if (info_dev) {
    // device loop: the same start state, written by kernels (no host copy,
    // no fill, no wait)
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(1024, ceil_div(
                                             (int64_t)(B.zero_bytes / 4), 256)))),
                       dim3(256), 0, stream, reinterpret_cast<uint32_t*>(B.zero_begin), (int64_t)(B.zero_bytes / 4));
    hipLaunchKernelGGL(k_init_batch, dim3(ceil_div(std::max(nsys * R, nsys * 4), 256)), dim3(256), 0, stream, nsys,
                       R, B.stat1, B.counters);
    auto put = [&](void* dst, const void* src, size_t bytes) {
      for (size_t off = 0; off < bytes; off += PUT_BYTES) {
        PutChunk c;
        const int nb = (int)std::min<size_t>(PUT_BYTES, bytes - off);
        std::memcpy(c.b, static_cast<const unsigned char*>(src) + off, nb);
        hipLaunchKernelGGL(k_put_bytes, dim3(1), dim3(256), 0, stream, static_cast<unsigned char*>(dst) + off, c, nb);
      }
    };
    put(B.sysdev, hs.data(), sizeof(SysDev) * nsys);
    if (nsys > 1) put(B.blk2sys, b2s.data(), sizeof(int) * b2s.size());
    NLSP_HIP(hipGetLastError());
    if (Ms[0]->prec == NLSP_FP64) return run_pcg<double>(nsys, hs, B, Ls, opts, info, false, stream, info_dev);
    if (Ms[0]->prec == NLSP_MIXED_F16) return run_pcg<_Float16>(nsys, hs, B, Ls, opts, info, false, stream, info_dev);
    return run_pcg<float>(nsys, hs, B, Ls, opts, info, false, stream, info_dev);
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
  if (Ms[0]->prec == NLSP_FP64) return run_pcg<double>(nsys, hs, B, Ls, opts, info, graph, stream);
  if (Ms[0]->prec == NLSP_MIXED_F16) return run_pcg<_Float16>(nsys, hs, B, Ls, opts, info, graph, stream);
  return run_pcg<float>(nsys, hs, B, Ls, opts, info, graph, stream);
}

// ------------------------------------------------ non-allocating solve
// Scratch memory of pcg_solve_noalloc: a file-scope device array, so a caller
// that cannot allocate (graph capture elsewhere in its loop, a serving loop
// that forbids allocation) still gets the solver's workspace.  Every GPU the
// library runs on holds its own copy until the process ends.  Host code never
// passes the array's name to a kernel or a copy (on the host it is only a
// stand-in symbol): the device address comes from hipGetSymbolAddress, taken
// once per device with that device current.
static __device__ __align__(256) unsigned char scratch[NLSP_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (NLSP_E_HIP if the
// runtime cannot give it).
static int scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return NLSP_E_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return NLSP_E_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return NLSP_OK;
}

}  // namespace nlsp

using namespace nlsp;

extern "C" {

size_t pcg_solve_workspace_bytes(const nlsp_operator* A, int k, int R) {
  const int64_t n = op_size(A);
  const int kp = padded_rank(k);
  if (n < 1 || kp < 0 || R < 1 || R > MAXR || kp * R > 2048 || n * R >= (int64_t(1) << 31)) return 0;
  return carve_batch(nullptr, {shape_of(n, kp, R, 0, use_faces(A, R, kp))}, nullptr).bytes;
}

int pcg_solve(const nlsp_operator* A, const nlsp_two_level* M, const double* f, double* u, int R,
              const nlsp_pcg_opts* opts, nlsp_rhs_info* info, void* ws, size_t ws_bytes,
              void* stream_) {
  const int64_t n = op_size(A);
  if (!info || !opts_ok(opts) || !system_ok(A, M, f, u, R, n)) return NLSP_E_INVALID;
  // iterations are replayed from a hipGraph unless per-kernel event timing is
  // asked for (events attach to single dispatches)
  const bool graph = opts->timing == nullptr;
  return solve_batch(1, &A, &M, &f, &u, R, 0, opts, info, ws, ws_bytes, graph, as_stream(stream_));
}

int pcg_solve_noalloc(const nlsp_operator* A, const nlsp_two_level* M, const double* f, double* u, int R,
                      const nlsp_pcg_opts* opts, nlsp_rhs_info* info, void* stream_) {
  const int64_t n = op_size(A);
  if (!info || !opts_ok(opts) || opts->timing != nullptr || !system_ok(A, M, f, u, R, n)) return NLSP_E_INVALID;
  const size_t need = pcg_solve_workspace_bytes(A, M->k, R);
  if (need == 0) return NLSP_E_INVALID;
  if (need > NLSP_NOALLOC_SCRATCH_BYTES) return NLSP_E_WORKSPACE;
  void* ws = nullptr;
  const int rc = scratch_address(&ws);
  if (rc != NLSP_OK) return rc;
  // direct launches: no graph is instantiated, so nothing is allocated
  return solve_batch(1, &A, &M, &f, &u, R, 0, opts, info, ws, need, false, as_stream(stream_));
}

size_t pcg_solve_batched_workspace_bytes(int nsys, const nlsp_system* sys, int R, int rows_per_block) {
  if (nsys < 1 || !sys || R < 1 || R > MAXR || rows_per_block < -1) return 0;
  rows_per_block = resolve_tile(nsys, sys, R, rows_per_block);
  std::vector<SysShape> sh(nsys);
  for (int i = 0; i < nsys; ++i) {
    const int64_t n = op_size(&sys[i].A);
    const int kp = padded_rank(sys[i].M.k);
    if (n < 1 || kp < 0 || kp * R > 2048 || n * R >= (int64_t(1) << 31)) return 0;
    sh[i] = shape_of(n, kp, R, rows_per_block, use_faces(&sys[i].A, R, kp));
  }
  return carve_batch(nullptr, sh, nullptr).bytes;
}

int pcg_solve_batched(int nsys, const nlsp_system* sys, int R, int rows_per_block, const nlsp_pcg_opts* opts,
                      nlsp_rhs_info* info, void* ws, size_t ws_bytes, void* stream_) {
  if (nsys < 1 || !sys || !info || !opts_ok(opts) || rows_per_block < -1) return NLSP_E_INVALID;
  rows_per_block = resolve_tile(nsys, sys, R, rows_per_block);
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
    blocks += shape_of(n, padded_rank(s.M.k), R, rows_per_block, false).nblk;
  }
  if (blocks > (int64_t(1) << 30)) return NLSP_E_INVALID;
  const bool graph = opts->timing == nullptr;
  return solve_batch(nsys, As.data(), Ms.data(), fs.data(), us.data(), R, rows_per_block, opts, info, ws,
                     ws_bytes, graph, as_stream(stream_));
}

int pcg_solve_batched_async(int nsys, const nlsp_system* sys, int R, int rows_per_block, const nlsp_pcg_opts* opts,
                            nlsp_rhs_info* info_dev, void* ws, size_t ws_bytes, void* stream_) {
  if (nsys < 1 || !sys || !info_dev || !opts_ok(opts) || opts->timing || rows_per_block < -1)
    return NLSP_E_INVALID;
  rows_per_block = resolve_tile(nsys, sys, R, rows_per_block);
  std::vector<const nlsp_operator*> As(nsys);
  std::vector<const nlsp_two_level*> Ms(nsys);
  std::vector<const double*> fs(nsys);
  std::vector<double*> us(nsys);
  int64_t blocks = 0;
  for (int i = 0; i < nsys; ++i) {
    const nlsp_system& s = sys[i];
    const int64_t n = op_size(&s.A);
    if (!system_ok(&s.A, &s.M, s.f, s.u, R, n)) return NLSP_E_INVALID;
    if (s.M.prec != sys[0].M.prec || s.M.nu != sys[0].M.nu || s.M.k != sys[0].M.k) return NLSP_E_INVALID;
    As[i] = &s.A;
    Ms[i] = &s.M;
    fs[i] = s.f;
    us[i] = s.u;
    blocks += shape_of(n, padded_rank(s.M.k), R, rows_per_block, false).nblk;
  }
  if (blocks > (int64_t(1) << 30)) return NLSP_E_INVALID;
  return solve_batch(nsys, As.data(), Ms.data(), fs.data(), us.data(), R, rows_per_block, opts, nullptr, ws,
                     ws_bytes, false, as_stream(stream_), info_dev);
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
  TuneKey key;
  if (tune_key(nsys, sys, R, key)) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tuned[key] = *best_rows_per_block;
  }
  return NLSP_OK;
}

int pcg_solve_batched_tuned(int nsys, const nlsp_system* sys, int R, int* rows_per_block) {
  if (nsys < 1 || !sys || R < 1 || R > MAXR || !rows_per_block) return NLSP_E_INVALID;
  return tuned_tile(nsys, sys, R, rows_per_block) ? 1 : 0;
}

}  // extern "C"
