// Subspace-loss forward and backward for a batch of bases (float32 data,
// float32 MFMA products, float64 cross-workgroup sums in a fixed order).
//
//   plain     L_b = ||B_b - P_b P_b^T B_b||_F^2 / ||B_b||_F^2
//               = (||B||^2 - 2 tr(C C^T) + tr(C^T G C)) / ||B||^2,
//             C = P^T B, G = P^T P (valid for any P, orthonormal or not)
//             dL/dP = B M1 + P M2,  M1 = -(2/||B||^2) C^T (2I - G),
//                                    M2 =  (2/||B||^2) C C^T
//   weighted  L_b = 1 - sum_j w_j ||p_j^T B_b||^2 / ||B_b||^2; with
//             w_j = (k - j + 1)/k this is the NLSS loss (eq. nlss_loss)
//             dL/dP = B M1,  M1 = -(2/||B||^2) C^T diag(w)
//
// The forward pass forms T = P^T [B | P] (k x (m + k)) per row slab with
// v_mfma_f32_16x16x4f32, a second kernel adds the slabs in float64, takes the
// loss and stores the backward's small matrix M = [M1; M2] (per unit upstream
// gradient) in `saved`; the backward streams [B | P] once more and forms
// dL/dP = [B | P] M with the same MFMA.
#include <algorithm>
#include <type_traits>

#include "device_common.hpp"
#include "host_common.hpp"

namespace nlsp {

namespace sub {

constexpr int NT = 256;            // 4 waves
constexpr int NTF = 1024;          // the finishing kernel
constexpr int RB = 64;             // rows staged per block
constexpr int MAX_TILES = 64;      // 16 x 16 output tiles of P^T [B | P] (upper G only)
constexpr size_t LDS_MAX = 160 * 1024;

typedef float f4 __attribute__((ext_vector_type(4)));

NLSP_DEV f4 mfma4(float a, float b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

// Shapes of one batched product.  The staged block is [B | P] (P omitted when
// ks = 0); the forward forms P^T [B | P] over the tiles of P^T B and, when
// gt = 1, the upper tiles of G = P^T P.
struct Dims {
  int n, k, m, kp, mp, cols, KT, MT, ntiles;  // kp, mp: k, m rounded up to 16; cols = mp + (ks ? kp : 0)
  int gt, ks;                                 // G tiles included; P columns staged (k or 0)
  int rows_per_slab, nslab;
  int vec;                                    // 16-byte loads of B and P rows allowed
  FastDiv fm, fk;                             // division by m and by k
};

inline int round16(int v) { return (v + 15) / 16 * 16; }

inline int count_tiles(int KT, int MT, int gt) {
  int c = 0;
  for (int ti = 0; ti < KT; ++ti)
    for (int tj = 0; tj < MT + (gt ? KT : 0); ++tj)
      if (tj < MT || tj - MT >= ti) ++c;
  return c;
}

inline Dims make_dims(int batch, int n, int k, int m, bool gt = true, bool stage_p = true) {
  Dims d;
  d.n = n;
  d.k = k;
  d.m = m;
  d.kp = round16(k);
  d.mp = round16(m);
  d.gt = gt ? 1 : 0;
  d.ks = stage_p ? k : 0;
  d.cols = d.mp + (stage_p ? d.kp : 0);
  d.KT = d.kp / 16;
  d.MT = d.mp / 16;
  d.ntiles = count_tiles(d.KT, d.MT, d.gt);
  // about 2048 workgroups over the batch, slabs a multiple of RB rows
  const int64_t blocks = (n + RB - 1) / RB;
  int64_t want = (2048 + batch - 1) / batch;
  want = std::max<int64_t>(1, std::min<int64_t>(want, blocks));
  const int64_t per = (blocks + want - 1) / want;
  d.rows_per_slab = (int)(per * RB);
  d.nslab = (int)((n + d.rows_per_slab - 1) / d.rows_per_slab);
  d.vec = (m % 4 == 0 && d.ks % 4 == 0) ? 1 : 0;
  d.fm = make_fastdiv((uint32_t)m);
  d.fk = make_fastdiv((uint32_t)k);
  return d;
}

// linear tile id -> (ti, tj): row-major over ti, tj, without the tiles of G
// below its diagonal (or without G at all when gt = 0)
NLSP_DEV void tile_of(int id, int KT, int MT, int gt, int& ti, int& tj) {
  if (!gt) {
    ti = id / MT;
    tj = id - ti * MT;
    return;
  }
  ti = 0;
  int rowlen = MT + KT;
  while (id >= rowlen) {
    id -= rowlen;
    ++ti;
    rowlen = MT + KT - ti;
  }
  tj = (id < MT) ? id : MT + ti + (id - MT);
}

// Staging of [B | P] rows r0 .. r0 + RB of one sample into LDS: B in columns
// [0, m), P in [mp, mp + k), zero in the padding columns and in rows beyond n.
// The block's B rows and P rows are each one contiguous range in memory;
// every thread issues its share of 16-byte (or 4-byte) loads, up to NV of
// them, before it writes any, so the loads of a pass are in flight together
// (each load is clamped to a valid address and masked afterwards, which keeps
// the code free of branches around the loads).
//   TRANS = true   column-major X^T[c][r], stride xs (>= RB, multiple of 4)
//   TRANS = false  row-major X[r][c], stride xs (>= cols, multiple of 4)
// Optionally adds the squares of the B entries to *bsq.
constexpr int NV = 8;

template <bool VEC, bool TRANS>
NLSP_DEV void stage_rows(const float* __restrict__ Bs, const float* __restrict__ Ps, const Dims& d,
                         int64_t r0, float* X, int xs, float* bsq) {
  constexpr int W = VEC ? 4 : 1;                   // floats per load
  const int t = threadIdx.x;
  const int nb = RB * d.m / W, np = RB * d.ks / W;  // loads of the B and P ranges
  const int rmax = (int)min((int64_t)RB, (int64_t)d.n - r0);  // rows of this block that exist (>= 1)
  const float* Bb = Bs + r0 * d.m;
  const float* Pb = Ps + r0 * d.ks;
  const int lastb = rmax * d.m - W, lastp = rmax * d.ks - W;  // last valid load offsets
  float acc = 0.f;
  for (int base = 0; base < nb + np; base += NT * NV) {
    float v[NV][W];
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const int q = base + t + NT * j;
      const bool isb = q < nb;
      const int e = (isb ? q : q - nb) * W;
      const float* src = isb ? Bb + min(e, lastb) : Pb + max(0, min(e, lastp));
      if constexpr (VEC) {
        const float4 x = *reinterpret_cast<const float4*>(src);
        v[j][0] = x.x;
        v[j][1] = x.y;
        v[j][2] = x.z;
        v[j][3] = x.w;
      } else {
        v[j][0] = *src;
      }
    }
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const int q = base + t + NT * j;
      if (q < nb + np) {
        const bool isb = q < nb;
        const int e = (isb ? q : q - nb) * W;
        const int row = (int)fdiv((uint32_t)e, isb ? d.fm : d.fk);
        const int col = e - row * (isb ? d.m : d.k) + (isb ? 0 : d.mp);
        const bool live = row < rmax;
        float x[W];
#pragma unroll
        for (int u = 0; u < W; ++u) {
          x[u] = live ? v[j][u] : 0.f;
          if (isb) acc += x[u] * x[u];
        }
        if constexpr (TRANS) {
#pragma unroll
          for (int u = 0; u < W; ++u) X[(col + u) * xs + row] = x[u];
        } else if constexpr (VEC) {
          *reinterpret_cast<float4*>(X + row * xs + col) = float4{x[0], x[W > 1 ? 1 : 0], x[W > 2 ? 2 : 0],
                                                                  x[W > 3 ? 3 : 0]};
        } else {
          X[row * xs + col] = x[0];
        }
      }
    }
  }
  if (bsq) *bsq += acc;
}

// zero the padding columns [m, mp) and [mp + k, cols) of a staging buffer
template <bool TRANS>
NLSP_DEV void zero_padding(const Dims& d, float* X, int xs) {
  const int padb = d.mp - d.m, padp = d.ks ? d.kp - d.k : 0, pw = padb + padp;
  if (pw == 0) return;
  for (int e = threadIdx.x; e < RB * pw; e += NT) {
    const int r = e / pw, c0 = e % pw;
    const int c = (c0 < padb) ? d.m + c0 : d.mp + d.k + (c0 - padb);
    if (TRANS)
      X[c * xs + r] = 0.f;
    else
      X[r * xs + c] = 0.f;
  }
}

typedef float f4v __attribute__((ext_vector_type(4)));

NLSP_DEV f4v lds4(const float* p) { return *reinterpret_cast<const f4v*>(p); }

// partial T = P^T [B | P] over one row slab; per tile 256 floats in the MFMA
// output order (lane, v), then the slab's ||B||^2 in float64.  Wave w owns
// tiles w, w + 4, ..., w + 4 (TPW - 1); ids past the last tile repeat tile 0
// and are not stored.  The MFMA's contraction index kk = lane / 16 is mapped
// to the block rows 16 kk .. 16 kk + 15 over 16 steps, so a lane's operands
// for four consecutive steps are four consecutive floats of a column of X^T:
// one 16-byte LDS read feeds four MFMAs.
template <int TPW, bool VEC>
__global__ __launch_bounds__(NT) void k_fwd_partial(Dims d, const float* __restrict__ P,
                                                    const float* __restrict__ B, float* __restrict__ part,
                                                    double* __restrict__ bbpart) {
  extern __shared__ float X[];               // X^T: cols x xs
  __shared__ double red[NT / 64];
  const int slab = blockIdx.x, b = blockIdx.y;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  constexpr int xs = RB + 4;
  const float* Bs = B + (int64_t)b * d.n * d.m;
  const float* Ps = P + (int64_t)b * d.n * d.k;
  zero_padding<true>(d, X, xs);
  const int lc = lane & 15, lg = lane >> 4;
  const float* pa[TPW];
  const float* pb[TPW];
  f4 acc[TPW];
#pragma unroll
  for (int s = 0; s < TPW; ++s) {
    int id = w + 4 * s, ti, tj;
    if (id >= d.ntiles) id = 0;
    tile_of(id, d.KT, d.MT, d.gt, ti, tj);
    pa[s] = X + (d.mp + 16 * ti + lc) * xs + 16 * lg;
    pb[s] = X + (16 * tj + lc) * xs + 16 * lg;
    acc[s] = f4{0.f, 0.f, 0.f, 0.f};
  }
  float bsq = 0.f;
  const int64_t s0 = (int64_t)slab * d.rows_per_slab;
  const int64_t s1 = min((int64_t)(s0 + d.rows_per_slab), (int64_t)d.n);
  for (int64_t r0 = s0; r0 < s1; r0 += RB) {
    __syncthreads();
    stage_rows<VEC, true>(Bs, Ps, d, r0, X, xs, &bsq);
    __syncthreads();
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      f4v a[TPW], bv[TPW];
#pragma unroll
      for (int s = 0; s < TPW; ++s) {
        a[s] = lds4(pa[s] + 4 * s4);
        bv[s] = lds4(pb[s] + 4 * s4);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int s = 0; s < TPW; ++s) acc[s] = mfma4(a[s][u], bv[s][u], acc[s]);
    }
  }
  float* out = part + ((int64_t)b * d.nslab + slab) * d.ntiles * 256;
#pragma unroll
  for (int s = 0; s < TPW; ++s) {
    const int id = w + 4 * s;
    if (id < d.ntiles) {
#pragma unroll
      for (int v = 0; v < 4; ++v) out[(int64_t)id * 256 + v * 64 + lane] = acc[s][v];
    }
  }
  double bs = wave_sum((double)bsq);
  if (lane == 0) red[w] = bs;
  __syncthreads();
  if (threadIdx.x == 0) bbpart[(int64_t)b * d.nslab + slab] = ((red[0] + red[1]) + red[2]) + red[3];
}

// T summed over the slabs in slab order, float64: grid (ceil(nel / NT), batch),
// one element per thread, loads issued eight at a time
__global__ __launch_bounds__(NT) void k_fwd_reduce(Dims d, const float* __restrict__ part,
                                                   double* __restrict__ T64) {
  const int b = blockIdx.y;
  const int nel = d.ntiles * 256;
  const int e = blockIdx.x * NT + threadIdx.x;
  if (e >= nel) return;
  const float* pb = part + (int64_t)b * d.nslab * nel + e;
  double s = 0.0;
  for (int sl = 0; sl < d.nslab; sl += 8) {
    float v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = (sl + j < d.nslab) ? pb[(int64_t)(sl + j) * nel] : 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += (double)v[j];
  }
  T64[(int64_t)b * nel + e] = s;
}

// per sample: T (from the slab sums) and ||B||^2, the loss, and M = [M1; M2]
// for a unit upstream gradient; 16 waves share the small float64 products
__global__ __launch_bounds__(NTF) void k_fwd_finish(Dims d, const double* __restrict__ T64,
                                                   const double* __restrict__ bbpart,
                                                   const float* __restrict__ colw, float* __restrict__ loss,
                                                   double* __restrict__ loss64, float* __restrict__ Msave) {
  extern __shared__ double T[];     // k_p x cols
  __shared__ double H[64 * 64];     // C C^T (k x k)
  __shared__ double sh[NTF / 64];
  __shared__ double s_bb;
  const int b = blockIdx.x, t = threadIdx.x;
  const int cols = d.cols;
  const int tcs = cols + 1;         // odd row stride (doubles): rows fall in different banks
  const int nel = d.ntiles * 256;
  const double* tb = T64 + (int64_t)b * nel;
  for (int e = t; e < nel; e += NTF) {
    const int id = e >> 8, v = (e >> 6) & 3, lane = e & 63;
    int ti, tj;
    tile_of(id, d.KT, d.MT, d.gt, ti, tj);
    T[(16 * ti + 4 * (lane >> 4) + v) * tcs + 16 * tj + (lane & 15)] = tb[e];
  }
  if (t == 0) {
    double s = 0.0;
    for (int sl = 0; sl < d.nslab; ++sl) s += bbpart[(int64_t)b * d.nslab + sl];
    s_bb = s;
  }
  __syncthreads();
  // G below its diagonal tiles from the transposed upper part
  for (int e = t; e < d.kp * d.kp; e += NTF) {
    const int i = e / d.kp, j = e % d.kp;
    if (j / 16 < i / 16) T[i * tcs + d.mp + j] = T[j * tcs + d.mp + i];
  }
  __syncthreads();
  const int k = d.k, m = d.m;
  // H = C C^T, C = T[:, :m]
  for (int e = t; e < k * k; e += NTF) {
    const int i = e / k, j = e % k;
    double s = 0.0;
#pragma unroll 8
    for (int c = 0; c < m; ++c) s += T[i * tcs + c] * T[j * tcs + c];
    H[i * 64 + j] = s;
  }
  __syncthreads();
  const double bb = s_bb;
  const double inv = (bb > 0.0) ? 1.0 / bb : 0.0;
  // loss terms
  double part_l = 0.0;
  for (int e = t; e < k * k; e += NTF) {
    const int i = e / k, j = e % k;
    if (colw) {
      if (i == j) part_l += (double)colw[i] * H[i * 64 + i];
    } else {
      part_l += T[i * tcs + d.mp + j] * H[i * 64 + j] - ((i == j) ? 2.0 * H[i * 64 + i] : 0.0);
    }
  }
  part_l = wave_sum(part_l);
  if ((t & 63) == 0) sh[t >> 6] = part_l;
  __syncthreads();
  double lt = 0.0;
  for (int q = 0; q < NTF / 64; ++q) lt += sh[q];
  if (t == 0) {
    const double L = colw ? 1.0 - lt * inv : (bb + lt) * inv;
    loss64[b] = L;
    loss[b] = (float)L;
  }
  // M (cols x kp), float32, for a unit upstream gradient
  float* M = Msave + (int64_t)b * cols * d.kp;
  for (int e = t; e < cols * d.kp; e += NTF) {
    const int c = e / d.kp, j = e % d.kp;
    double v = 0.0;
    if (j < k) {
      if (c < m) {
        if (colw) {
          v = -2.0 * inv * (double)colw[j] * T[j * tcs + c];
        } else {
          double s = 0.0;
#pragma unroll 8
          for (int i = 0; i < k; ++i) s += T[i * tcs + c] * (((i == j) ? 2.0 : 0.0) - T[i * tcs + d.mp + j]);
          v = -2.0 * inv * s;
        }
      } else if (c >= d.mp && c - d.mp < k && !colw) {
        v = 2.0 * inv * H[(c - d.mp) * 64 + j];
      }
    }
    M[e] = (float)v;
  }
}

// dL/dP = g_b [B | P] M over one row slab; wave w forms rows 16 w .. 16 w + 15
// of each staged block, all KT column tiles at once.  The contraction runs
// over the cols = 4 cq columns of [B | P]; the MFMA's kk = lane / 16 takes
// columns kk cq .. kk cq + cq - 1 over cq steps, so four consecutive steps are
// four consecutive floats of a row of X and of a row of M^T (16-byte reads).
template <int KT, bool VEC>
__global__ __launch_bounds__(NT) void k_bwd(Dims d, const float* __restrict__ P, const float* __restrict__ B,
                                            const float* __restrict__ Msave, const float* __restrict__ gloss,
                                            float* __restrict__ gP) {
  extern __shared__ float lds[];
  const int slab = blockIdx.x, b = blockIdx.y;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int xs = d.cols + 4;             // X: RB x xs, row-major
  const int mts = d.cols + 4;            // M^T: kp x mts
  float* X = lds;
  float* MT = lds + RB * xs;
  zero_padding<false>(d, X, xs);
  const float g = gloss ? gloss[b] : 1.f;
  const float* Mb = Msave + (int64_t)b * d.cols * d.kp;
  for (int e = threadIdx.x; e < d.cols * d.kp; e += NT) MT[(e % d.kp) * mts + e / d.kp] = g * Mb[e];
  const float* Bs = B + (int64_t)b * d.n * d.m;
  const float* Ps = P + (int64_t)b * d.n * d.k;
  float* G = gP + (int64_t)b * d.n * d.k;
  const int64_t s0 = (int64_t)slab * d.rows_per_slab;
  const int64_t s1 = min((int64_t)(s0 + d.rows_per_slab), (int64_t)d.n);
  const int lr = lane & 15, lg = lane >> 4;
  const int cq = d.cols / 4;             // multiple of 4
  const float* xa = X + (16 * w + lr) * xs + lg * cq;
  const float* mb = MT + lr * mts + lg * cq;
  for (int64_t r0 = s0; r0 < s1; r0 += RB) {
    __syncthreads();
    stage_rows<VEC, false>(Bs, Ps, d, r0, X, xs, nullptr);
    __syncthreads();
    f4 acc[KT];
#pragma unroll
    for (int tj = 0; tj < KT; ++tj) acc[tj] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int c = 0; c < cq; c += 4) {
      const f4v a = lds4(xa + c);
      f4v bm[KT];
#pragma unroll
      for (int tj = 0; tj < KT; ++tj) bm[tj] = lds4(mb + 16 * tj * mts + c);
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int tj = 0; tj < KT; ++tj) acc[tj] = mfma4(a[u], bm[tj][u], acc[tj]);
    }
#pragma unroll
    for (int tj = 0; tj < KT; ++tj) {
      const int col = 16 * tj + lr;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = r0 + 16 * w + 4 * lg + v;
        if (row < s1 && col < d.k) G[row * d.k + col] = acc[tj][v];
      }
    }
  }
}

// ---------------------------------------------------- Galerkin product
// Y = A_b P_b for a batch of operators that share kind and grid: sample b uses
// coefficients coef + b * cstride (float32 products of the float64 stencil).
__global__ __launch_bounds__(NT) void k_gal_apply(OpDev op, int64_t cstride, int k, FastDiv fk,
                                                  const float* __restrict__ P, float* __restrict__ Y) {
  const int b = blockIdx.y;
  const uint32_t g = blockIdx.x * NT + threadIdx.x;
  if ((int64_t)g >= op.n * k) return;
  OpDev ob = op;
  if (ob.coef) ob.coef += (int64_t)b * cstride;
  const uint32_t i = fdiv(g, fk);
  const int c = (int)(g - i * (uint32_t)k);
  int px, py, pz;
  decompose(ob, i, px, py, pz);
  const float* Pb = P + (int64_t)b * op.n * k;
  Y[(int64_t)b * op.n * k + g] = op_row<float>(ob, i, px, py, pz, [&](int64_t j) { return Pb[j * k + c]; });
}

// A_c = (T + T^T) / 2 from the slab sums of T = P^T Y (tiles row-major, no G)
__global__ __launch_bounds__(NT) void k_gal_finish(Dims d, const double* __restrict__ T64, float* __restrict__ Ac) {
  const int b = blockIdx.x;
  const double* tb = T64 + (int64_t)b * d.ntiles * 256;
  auto at = [&](int i, int j) {
    const int id = (i >> 4) * d.MT + (j >> 4), r = i & 15;
    return tb[id * 256 + (r & 3) * 64 + (r >> 2) * 16 + (j & 15)];
  };
  for (int e = threadIdx.x; e < d.k * d.k; e += NT) {
    const int i = e / d.k, j = e % d.k;
    Ac[(int64_t)b * d.k * d.k + e] = (float)(0.5 * (at(i, j) + at(j, i)));
  }
}

// M = G + G^T (kp x kp, zero padded) for the Galerkin backward
__global__ __launch_bounds__(NT) void k_gal_bwd_prep(int k, int kp, const float* __restrict__ gAc,
                                                     float* __restrict__ M) {
  const int b = blockIdx.x;
  const float* G = gAc + (int64_t)b * k * k;
  for (int e = threadIdx.x; e < kp * kp; e += NT) {
    const int i = e / kp, j = e % kp;
    M[(int64_t)b * kp * kp + e] = (i < k && j < k) ? G[i * k + j] + G[j * k + i] : 0.f;
  }
}

// ------------------------------------------------------------- thin QR
// A = Q R (A: n x k per sample, R upper with positive diagonal) by
// CholeskyQR2: G = A^T A = R1^T R1, Q1 = A R1^-1, then once more on Q1, and
// R = R2 R1.  The backward (only Q is used downstream) is
//   dA = [dQ + Q copyltu(M)] R^-T,   M = -dQ^T Q,
// copyltu(M) the symmetric matrix with M's lower triangle, evaluated as
// [dQ | Q] [R^-T ; copyltu(M) R^-T] with the product kernels.
constexpr int QRK = 64;

// G (k x k) from the slab sums of T = P^T B (tiles row-major, no G tiles),
// symmetrised
NLSP_DEV void load_gram(const Dims& d, const double* tb, double* G) {
  for (int e = threadIdx.x; e < d.k * d.k; e += NT) {
    const int i = e / d.k, j = e % d.k;
    auto at = [&](int a, int c) {
      const int id = (a >> 4) * d.MT + (c >> 4), r = a & 15;
      return tb[id * 256 + (r & 3) * 64 + (r >> 2) * 16 + (c & 15)];
    };
    G[i * QRK + j] = 0.5 * (at(i, j) + at(j, i));
  }
}

// upper Cholesky factor R of G (G = R^T R) in place, and X = R^-1 (upper);
// returns false (in every thread) if a pivot is not positive
NLSP_DEV bool chol_inv(int k, double* G, double* X) {
  __shared__ int s_bad;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  for (int i = 0; i < k; ++i) {
    if (threadIdx.x == 0) {
      double d = G[i * QRK + i];
      for (int p = 0; p < i; ++p) d -= G[p * QRK + i] * G[p * QRK + i];
      if (!(d > 0.0)) {
        s_bad = 1;
        d = 1.0;
      }
      G[i * QRK + i] = sqrt(d);
    }
    __syncthreads();
    for (int j = i + 1 + threadIdx.x; j < k; j += NT) {
      double v = G[i * QRK + j];
      for (int p = 0; p < i; ++p) v -= G[p * QRK + i] * G[p * QRK + j];
      G[i * QRK + j] = v / G[i * QRK + i];
    }
    __syncthreads();
  }
  // R^-1 by columns (upper triangular back substitution), one thread per column
  for (int j = threadIdx.x; j < k; j += NT) {
    for (int i = 0; i < k; ++i) X[i * QRK + j] = 0.0;
    X[j * QRK + j] = 1.0 / G[j * QRK + j];
    for (int i = j - 1; i >= 0; --i) {
      double v = 0.0;
      for (int p = i + 1; p <= j; ++p) v += G[i * QRK + p] * X[p * QRK + j];
      X[i * QRK + j] = -v / G[i * QRK + i];
    }
  }
  __syncthreads();
  return s_bad == 0;
}

// pass 1 (first = 1): R1 from G = A^T A, M = R1^-1, Rprev = R1
// pass 2 (first = 0): R2 from G = Q1^T Q1, M = R2^-1, R = R2 Rprev
// M is (kp x kp) float32 row-major; R (k x k) float64; bad[b] |= 1 if a pivot
// was not positive
__global__ __launch_bounds__(NT) void k_qr_small(Dims d, const double* __restrict__ T64, int first,
                                                 double* __restrict__ Rprev, double* __restrict__ Rout,
                                                 float* __restrict__ M, int* __restrict__ bad) {
  __shared__ double G[QRK * QRK];
  __shared__ double X[QRK * QRK];
  const int b = blockIdx.x, k = d.k, kp = d.kp;
  load_gram(d, T64 + (int64_t)b * d.ntiles * 256, G);
  __syncthreads();
  const bool ok = chol_inv(k, G, X);
  if (threadIdx.x == 0 && !ok) bad[b] = 1;
  for (int e = threadIdx.x; e < kp * kp; e += NT) {
    const int i = e / kp, j = e % kp;
    M[(int64_t)b * kp * kp + e] = (i < k && j < k) ? (float)X[i * QRK + j] : 0.f;
  }
  double* Rp = Rprev + (int64_t)b * k * k;
  for (int e = threadIdx.x; e < k * k; e += NT) {
    const int i = e / k, j = e % k;
    if (first) {
      Rp[e] = (j >= i) ? G[i * QRK + j] : 0.0;
    } else {
      double v = 0.0;   // (R2 R1)_ij = sum_{i <= p <= j} R2_ip R1_pj
      for (int p = i; p <= j; ++p) v += G[i * QRK + p] * Rp[p * k + j];
      Rout[(int64_t)b * k * k + e] = (j >= i) ? v : 0.0;
    }
  }
}

// backward: from T = Q^T dQ (slab sums) and R, the stacked (2 kp x kp) matrix
// [R^-T ; C R^-T] with C_ij = -T[min(i,j)][max(i,j)] (= copyltu(-dQ^T Q))
__global__ __launch_bounds__(NT) void k_qr_bwd_small(Dims d, const double* __restrict__ T64,
                                                     const double* __restrict__ R, float* __restrict__ M) {
  __shared__ double G[QRK * QRK];   // R, then reused
  __shared__ double X[QRK * QRK];   // R^-1
  __shared__ double C[QRK * QRK];
  const int b = blockIdx.x, k = d.k, kp = d.kp;
  const double* Rb = R + (int64_t)b * k * k;
  const double* tb = T64 + (int64_t)b * d.ntiles * 256;
  auto at = [&](int a, int c) {
    const int id = (a >> 4) * d.MT + (c >> 4), r = a & 15;
    return tb[id * 256 + (r & 3) * 64 + (r >> 2) * 16 + (c & 15)];
  };
  for (int e = threadIdx.x; e < k * k; e += NT) {
    const int i = e / k, j = e % k;
    G[i * QRK + j] = Rb[e];
    C[i * QRK + j] = -at(min(i, j), max(i, j));
  }
  __syncthreads();
  for (int j = threadIdx.x; j < k; j += NT) {
    for (int i = 0; i < k; ++i) X[i * QRK + j] = 0.0;
    X[j * QRK + j] = 1.0 / G[j * QRK + j];
    for (int i = j - 1; i >= 0; --i) {
      double v = 0.0;
      for (int p = i + 1; p <= j; ++p) v += G[i * QRK + p] * X[p * QRK + j];
      X[i * QRK + j] = -v / G[i * QRK + i];
    }
  }
  __syncthreads();
  float* Mb = M + (int64_t)b * 2 * kp * kp;
  for (int e = threadIdx.x; e < 2 * kp * kp; e += NT) {
    const int r = e / kp, j = e % kp;
    double v = 0.0;
    if (j < k) {
      if (r < kp) {
        if (r < k) v = X[j * QRK + r];                       // (R^-T)_rj = (R^-1)_jr
      } else if (r - kp < k) {
        const int i = r - kp;                                // (C R^-T)_ij = sum_p C_ip (R^-1)_jp
        for (int p = j; p < k; ++p) v += C[i * QRK + p] * X[j * QRK + p];
      }
    }
    Mb[e] = (float)v;
  }
}

struct SubLayout {
  float* part;
  double* bbpart;
  double* T64;
  size_t bytes;
};

inline SubLayout carve_sub(void* ws, int batch, const Dims& d) {
  Carver c(ws);
  SubLayout L;
  L.part = c.take<float>((size_t)batch * d.nslab * d.ntiles * 256);
  L.bbpart = c.take<double>((size_t)batch * d.nslab);
  L.T64 = c.take<double>((size_t)batch * d.ntiles * 256);
  L.bytes = c.bytes();
  return L;
}

// saved: per sample loss in float64, then M (cols x kp float32)
inline size_t saved_bytes(int batch, const Dims& d) {
  return align_up((size_t)batch * sizeof(double)) + (size_t)batch * d.cols * d.kp * sizeof(float);
}

inline size_t fwd_lds(const Dims& d) { return (size_t)d.cols * (RB + 4) * sizeof(float); }
inline size_t fin_lds(const Dims& d) { return (size_t)d.kp * (d.cols + 1) * sizeof(double); }
inline size_t bwd_lds(const Dims& d) {
  return ((size_t)RB * (d.cols + 4) + (size_t)d.kp * (d.cols + 4)) * sizeof(float);
}

// k <= 64, m <= 256, at most 64 output tiles, and every kernel's LDS within a CU's
inline bool dims_ok(int batch, int n, int k, int m) {
  if (batch < 1 || n < 1 || k < 1 || m < 1 || k > 64 || m > 256) return false;
  if ((int64_t)batch * n * std::max(k, m) >= (int64_t(1) << 40)) return false;
  const Dims d = make_dims(batch, n, k, m);
  return d.ntiles <= MAX_TILES && fwd_lds(d) <= LDS_MAX && fin_lds(d) + 64 * 64 * 8 + 256 <= LDS_MAX &&
         bwd_lds(d) <= LDS_MAX;
}

// Galerkin product: forward T = P^T [Y | P] over the tiles of P^T Y only,
// backward [Y] (G + G^T); k <= 64, n k < 2^31 per sample
inline Dims gal_fwd_dims(int batch, int n, int k) { return make_dims(batch, n, k, k, false, true); }
inline Dims gal_bwd_dims(int batch, int n, int k) { return make_dims(batch, n, k, k, false, false); }
inline bool gal_ok(int batch, int64_t n, int k) {
  if (batch < 1 || n < 1 || k < 1 || k > 64 || n * k >= (int64_t(1) << 31)) return false;
  const Dims d = gal_fwd_dims(batch, (int)n, k);
  return d.ntiles <= MAX_TILES && fwd_lds(d) <= LDS_MAX && bwd_lds(gal_bwd_dims(batch, (int)n, k)) <= LDS_MAX;
}

// Size of a batched operator: the training kernels take structured grids
// only (a compressed-row operator is rejected).
inline int64_t batched_op_size(const nlsp_operator* A) { return (A && A->kind == NLSP_OP_CSR) ? -1 : op_size(A); }

// coefficient values per sample of a batched operator
inline int64_t coef_stride(const nlsp_operator& a, int64_t n) {
  switch (a.kind) {
    case NLSP_OP_FV5:
    case NLSP_OP_FV7: return n;
    case NLSP_OP_STENCIL9: return 9;
    default: return 0;
  }
}

template <typename K>
inline hipError_t allow_lds(K kernel, size_t bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

// ------------------------------------------------ Galerkin-convergence term
// J_b(P) = tr(S^T A S) - tr(W^T A_c^-1 W), W = P^T A S, A_c = P^T A P (the
// projected-energy objective of the appendix, in the projector identity's
// form).  With A_c = R^T R (R upper), V = R^-T W and Z = R^-1 V = A_c^-1 W:
//   J = tr(S^T A S) - ||V||_F^2,
//   dJ/dP = 2 [A P Z Z^T - A S Z^T] = [A S | A P] M,
//   M = [-2 Z^T ; 2 Z Z^T]   ((m + k) x k).
// The forward stores X = [A S | A P] (n x (m + k), float32) and M; the
// backward is one product pass over X.

// X[i][c] = (A S)_ic for c < m, (A P)_i(c-m) otherwise (float32 products of
// the float64 stencil), and per-workgroup partials of tr(S^T A S) in float64
__global__ __launch_bounds__(NT) void k_gterm_apply(OpDev op, int64_t cstride, int k, int m, FastDiv fw,
                                                    const float* __restrict__ P, const float* __restrict__ S,
                                                    float* __restrict__ X, double* __restrict__ spart) {
  __shared__ double sh[NT / 64];
  const int b = blockIdx.y;
  const int w = m + k;
  const uint32_t g = blockIdx.x * NT + threadIdx.x;
  OpDev ob = op;
  if (ob.coef) ob.coef += (int64_t)b * cstride;
  double ss = 0.0;
  if ((int64_t)g < op.n * w) {
    const uint32_t i = fdiv(g, fw);
    const int c = (int)(g - i * (uint32_t)w);
    int px, py, pz;
    decompose(ob, i, px, py, pz);
    const float* Sb = S + (int64_t)b * op.n * m;
    const float* Pb = P + (int64_t)b * op.n * k;
    float v;
    if (c < m) {
      v = op_row<float>(ob, i, px, py, pz, [&](int64_t j) { return Sb[j * m + c]; });
      ss = (double)Sb[(int64_t)i * m + c] * (double)v;
    } else {
      v = op_row<float>(ob, i, px, py, pz, [&](int64_t j) { return Pb[j * k + (c - m)]; });
    }
    X[(int64_t)b * op.n * w + g] = v;
  }
  ss = block_sum(ss, sh);
  if (threadIdx.x == 0) spart[(int64_t)b * gridDim.x + blockIdx.x] = ss;
}

// The same product row-blocked, for FV5 / FV7 / Poisson operators and m, k
// multiples of 4: a workgroup owns GT_TR consecutive rows of one sample, forms
// each row's face weights once into LDS (in float, as op_row<float>: the
// diagonal d and the face means t_f, a boundary face adding 2 a_P to d), then
// streams the (row, 4-column) items of [S | P] with 16-byte loads:
// (A v)_i = d v_i - sum_f [f inside] t_f v_j, faces in op_row's order.
constexpr int GT_TR = 64;
template <int NF>
__global__ __launch_bounds__(NT) void k_gterm_rows(OpDev op, int64_t cstride, int k, int m, FastDiv fcv,
                                                   const float* __restrict__ P, const float* __restrict__ S,
                                                   float* __restrict__ X, double* __restrict__ spart) {
  __shared__ float sw[GT_TR][NF + 1];   // d, t_f (0 for a boundary face)
  __shared__ int sj[GT_TR][NF];         // neighbour row minus the row (0 for a boundary face)
  __shared__ double sh[NT / 64];
  const int b = blockIdx.y;
  OpDev ob = op;
  if (ob.coef) ob.coef += (int64_t)b * cstride;
  const int64_t n = op.n;
  const int64_t r0 = (int64_t)blockIdx.x * GT_TR;
  const int nrows = (int)min((int64_t)GT_TR, n - r0);
  for (int t = threadIdx.x; t < nrows; t += NT) {
    const int64_t i = r0 + t;
    int x, y, z;
    decompose(ob, i, x, y, z);
    const int nx = ob.nx, ny = ob.ny;
    const int64_t sxy = (int64_t)nx * ny;
    const int64_t jn[6] = {-1, 1, -(int64_t)nx, (int64_t)nx, -sxy, sxy};
    const bool in[6] = {x > 0, x < nx - 1, y > 0, y < ny - 1, z > 0, z < ob.nz - 1};
    if (ob.kind == NLSP_OP_POISSON5) {
      sw[t][0] = 4.0f;
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        sw[t][1 + f] = in[f] ? 1.0f : 0.0f;
        sj[t][f] = in[f] ? (int)jn[f] : 0;
      }
    } else {
      const auto a = ob.coef;
      const float aP = float(a[i]);
      float d = 0.0f;
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const float tf = harmonic<float>(aP, float(a[in[f] ? i + jn[f] : i]));
        d += in[f] ? tf : 2.0f * aP;
        sw[t][1 + f] = in[f] ? tf : 0.0f;
        sj[t][f] = in[f] ? (int)jn[f] : 0;
      }
      sw[t][0] = d;
    }
  }
  __syncthreads();
  const int m4 = m / 4, CV = (int)fcv.d, total = nrows * CV;
  const float* Sb = S + (int64_t)b * n * m;
  const float* Pb = P + (int64_t)b * n * k;
  float* Xb = X + (int64_t)b * n * (m + k);
  double ss = 0.0;
  for (int idx = threadIdx.x; idx < total; idx += NT) {
    const int rl = (int)fdiv((uint32_t)idx, fcv), c4 = idx - rl * CV;
    const int64_t i = r0 + rl;
    const bool fromS = c4 < m4;
    const float* src = fromS ? Sb : Pb;
    const int w = fromS ? m : k;
    const int col = 4 * (fromS ? c4 : c4 - m4);
    const float4 vi = *reinterpret_cast<const float4*>(src + i * w + col);
    float4 vj[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) vj[f] = *reinterpret_cast<const float4*>(src + (i + sj[rl][f]) * w + col);
    const float d = sw[rl][0];
    float o[4];
    const float* vip = reinterpret_cast<const float*>(&vi);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      float sacc = 0.0f;
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const float tf = sw[rl][1 + f];
        sacc += sj[rl][f] != 0 ? tf * reinterpret_cast<const float*>(&vj[f])[e] : 0.0f;
      }
      o[e] = d * vip[e] - sacc;
      if (fromS) ss += (double)vip[e] * (double)o[e];
    }
    *reinterpret_cast<float4*>(Xb + i * (m + k) + 4 * c4) = make_float4(o[0], o[1], o[2], o[3]);
  }
  if (spart) {   // (m = 0, no partials: the plain Galerkin product Y = A P)
    ss = block_sum(ss, sh);
    if (threadIdx.x == 0) spart[(int64_t)b * gridDim.x + blockIdx.x] = ss;
  }
}

// per sample: T = P^T X from the slab sums, A_c = sym(T[:, m:]), W = T[:, :m],
// Cholesky, V = R^-T W, Z = R^-1 V, J, and M for a unit upstream gradient.
// LDS (dynamic): R and R^-1 (QRK x QRK each), V and Z (k x m each).
__global__ __launch_bounds__(NT) void k_gterm_finish(Dims d, int m, const double* __restrict__ T64,
                                                     const double* __restrict__ spart, int nspart,
                                                     float* __restrict__ J, float* __restrict__ E,
                                                     int* __restrict__ bad, float* __restrict__ Msave) {
  extern __shared__ double glds[];
  double* G = glds;                 // R (upper), then H = Z Z^T
  double* Xi = G + QRK * QRK;       // R^-1 (upper)
  double* V = Xi + QRK * QRK;       // W, then V = R^-T W   (k x m)
  double* Z = V + d.k * m;          // Z = R^-1 V           (k x m)
  __shared__ double sh[NT / 64];
  const int b = blockIdx.x, k = d.k, t = threadIdx.x;
  const double* tb = T64 + (int64_t)b * d.ntiles * 256;
  auto at = [&](int a, int c) {   // T[a][c], c < m + k
    const int id = (a >> 4) * d.MT + (c >> 4), r = a & 15;
    return tb[id * 256 + (r & 3) * 64 + (r >> 2) * 16 + (c & 15)];
  };
  for (int e = t; e < k * k; e += NT) {
    const int i = e / k, j = e % k;
    G[i * QRK + j] = 0.5 * (at(i, m + j) + at(j, m + i));
  }
  for (int e = t; e < k * m; e += NT) Z[e] = at(e / m, e % m);   // W, parked in Z
  // tr(S^T A S) from the apply kernel's partials, in order
  double tr = 0.0;
  if (t == 0)
    for (int q = 0; q < nspart; ++q) tr += spart[(int64_t)b * nspart + q];
  __syncthreads();
  const bool ok = chol_inv(k, G, Xi);
  if (t == 0) bad[b] = ok ? 0 : 1;
  // V = R^-T W: V_ic = sum_{p <= i} (R^-1)_pi W_pc
  for (int e = t; e < k * m; e += NT) {
    const int i = e / m, c = e % m;
    double v = 0.0;
    for (int p = 0; p <= i; ++p) v += Xi[p * QRK + i] * Z[p * m + c];
    V[e] = v;
  }
  __syncthreads();
  // Z = R^-1 V: Z_ic = sum_{p >= i} (R^-1)_ip V_pc;  ||V||^2
  double vv = 0.0;
  for (int e = t; e < k * m; e += NT) {
    const int i = e / m, c = e % m;
    double z = 0.0;
    for (int p = i; p < k; ++p) z += Xi[i * QRK + p] * V[p * m + c];
    Z[e] = z;
    vv += V[e] * V[e];
  }
  vv = block_sum(vv, sh);
  if (t == 0) {
    J[b] = (float)(tr - vv);
    if (E) E[b] = (float)tr;
  }
  // H = Z Z^T (k x k) into G
  for (int e = t; e < k * k; e += NT) {
    const int i = e / k, j = e % k;
    double h = 0.0;
    for (int c = 0; c < m; ++c) h += Z[i * m + c] * Z[j * m + c];
    G[i * QRK + j] = h;
  }
  __syncthreads();
  // M ((cols x kp), rows = columns of X): -2 Z^T over the A S columns, 2 Z Z^T
  // over the A P columns, zero padding
  float* Mb = Msave + (int64_t)b * d.cols * d.kp;
  for (int e = t; e < d.cols * d.kp; e += NT) {
    const int c = e / d.kp, j = e % d.kp;
    double v = 0.0;
    if (j < k) {
      if (c < m)
        v = -2.0 * Z[j * m + c];
      else if (c < m + k)
        v = 2.0 * G[(c - m) * QRK + j];
    }
    Mb[e] = (float)v;
  }
}

}  // namespace sub
}  // namespace nlsp

using namespace nlsp;
using namespace nlsp::sub;

// forward product partials + slab sums (shared by both forward passes)
inline int launch_products(const Dims& d, int batch, const float* P, const float* B, const SubLayout& L,
                           hipStream_t s) {
  const dim3 grid(d.nslab, batch);
  const size_t lds = fwd_lds(d);
  const int tpw = (d.ntiles + 3) / 4;
  int rc = NLSP_OK;
  auto go = [&](auto kern) {
    if (allow_lds(kern, lds) != hipSuccess) { rc = NLSP_E_HIP; return; }
    hipLaunchKernelGGL(kern, grid, dim3(NT), lds, s, d, P, B, L.part, L.bbpart);
  };
  auto pick = [&](auto vec) {
    constexpr bool V = decltype(vec)::value;
    switch (tpw) {
      case 1: go(k_fwd_partial<1, V>); break;
      case 2: go(k_fwd_partial<2, V>); break;
      case 3: go(k_fwd_partial<3, V>); break;
      case 4: go(k_fwd_partial<4, V>); break;
      case 5: case 6: go(k_fwd_partial<6, V>); break;
      case 7: case 8: go(k_fwd_partial<8, V>); break;
      case 9: case 10: case 11: case 12: go(k_fwd_partial<12, V>); break;
      default: go(k_fwd_partial<16, V>); break;
    }
  };
  if (d.vec) pick(std::true_type{}); else pick(std::false_type{});
  if (rc != NLSP_OK) return rc;
  hipLaunchKernelGGL(k_fwd_reduce, dim3(ceil_div((int64_t)d.ntiles * 256, NT), batch), dim3(NT), 0, s, d, L.part,
                     L.T64);
  return NLSP_OK;
}

// [B | P] M per row slab (shared by both backward passes); gloss may be null
inline int launch_bwd(const Dims& d, int batch, const float* P, const float* B, const float* M,
                      const float* gloss, float* gP, hipStream_t s) {
  const size_t lds = bwd_lds(d);
  int rc = NLSP_OK;
  auto go = [&](auto kern) {
    if (allow_lds(kern, lds) != hipSuccess) { rc = NLSP_E_HIP; return; }
    hipLaunchKernelGGL(kern, dim3(d.nslab, batch), dim3(NT), lds, s, d, P, B, M, gloss, gP);
  };
  auto pick = [&](auto vec) {
    constexpr bool V = decltype(vec)::value;
    switch (d.KT) {
      case 1: go(k_bwd<1, V>); break;
      case 2: go(k_bwd<2, V>); break;
      case 3: go(k_bwd<3, V>); break;
      default: go(k_bwd<4, V>); break;
    }
  };
  if (d.vec) pick(std::true_type{}); else pick(std::false_type{});
  return rc;
}

inline bool aligned16(const void* p) { return reinterpret_cast<uintptr_t>(p) % 16 == 0; }

namespace nlsp {
namespace sub {
// Captured energy per sample from the slab sums of C = P^T S (tiles of the
// forward product with P staged and no G tiles): e_j = sum_c C[j][c]^2 for rows j < k, each
// row by one thread over c in order, then the prefix sums
//   energy[b][r - 1] = (e_0 + ... + e_{r-1}) / ||S_b||_F^2   (r = 1 .. k)
// in order by one thread.  Float64 throughout.
__global__ __launch_bounds__(64) void k_energy_finish(Dims d, const double* __restrict__ T64,
                                                     const double* __restrict__ bbpart,
                                                     double* __restrict__ energy) {
  __shared__ double e[64];
  const int b = blockIdx.x, j = threadIdx.x;
  const double* tb = T64 + (int64_t)b * d.ntiles * 256;
  if (j < d.k) {
    const int ti = j / 16, r = j % 16;
    double s = 0.0;
    for (int c = 0; c < d.m; ++c) {
      const int id = ti * d.MT + c / 16;   // tiles row-major, no G tiles
      const double v = tb[id * 256 + (r & 3) * 64 + (r >> 2) * 16 + (c & 15)];
      s += v * v;
    }
    e[j] = s;
  }
  __syncthreads();
  if (j == 0) {
    double bb = 0.0;
    for (int sl = 0; sl < d.nslab; ++sl) bb += bbpart[(int64_t)b * d.nslab + sl];
    double acc = 0.0;
    for (int r = 0; r < d.k; ++r) {
      acc += e[r];
      energy[(int64_t)b * d.k + r] = acc / bb;
    }
  }
}
}  // namespace sub
}  // namespace nlsp

extern "C" {

// thin QR dims: products P^T B with B an n x k block (tiles of P^T B only)
inline Dims qr_dims(int batch, int n, int k, bool stage_p) { return make_dims(batch, n, k, k, false, stage_p); }
inline bool qr_ok(int batch, int64_t n, int k) {
  if (batch < 1 || n < k || k < 1 || k > QRK || n * k >= (int64_t(1) << 31)) return false;
  const Dims d = qr_dims(batch, (int)n, k, true);
  return d.ntiles <= MAX_TILES && fwd_lds(d) <= LDS_MAX && bwd_lds(d) <= LDS_MAX;
}

struct QrLayout {
  SubLayout prod;
  float* Q1;        // (batch, n, k)
  float* M;         // (batch, 2 kp, kp)
  double* R1;       // (batch, k, k)
  size_t bytes;
};

inline QrLayout carve_qr(void* ws, int batch, int n, int k) {
  const Dims d = qr_dims(batch, n, k, true);
  QrLayout L;
  L.prod = carve_sub(ws, batch, d);
  Carver c(ws ? static_cast<char*>(ws) + L.prod.bytes : nullptr);
  L.Q1 = c.take<float>((size_t)batch * n * k);
  L.M = c.take<float>((size_t)batch * 2 * d.kp * d.kp);
  L.R1 = c.take<double>((size_t)batch * k * k);
  L.bytes = L.prod.bytes + c.bytes();
  return L;
}

size_t subspace_loss_saved_bytes(int batch, int n, int k, int m) {
  if (!dims_ok(batch, n, k, m)) return 0;
  return saved_bytes(batch, make_dims(batch, n, k, m));
}

size_t subspace_loss_workspace_bytes(int batch, int n, int k, int m) {
  if (!dims_ok(batch, n, k, m)) return 0;
  return carve_sub(nullptr, batch, make_dims(batch, n, k, m)).bytes;
}

int subspace_loss_fwd(int batch, int n, int k, int m, const float* P, const float* B, const float* colw,
                      float* loss, void* saved, size_t saved_nbytes, void* ws, size_t ws_bytes, void* stream) {
  if (!dims_ok(batch, n, k, m) || !P || !B || !loss || !saved) return NLSP_E_INVALID;
  Dims d = make_dims(batch, n, k, m);
  if (!aligned16(P) || !aligned16(B)) d.vec = 0;
  if (saved_nbytes < saved_bytes(batch, d) || reinterpret_cast<uintptr_t>(saved) % WS_ALIGN)
    return NLSP_E_WORKSPACE;
  const size_t need = carve_sub(nullptr, batch, d).bytes;
  if (!ws_ok(ws, ws_bytes, need)) return NLSP_E_WORKSPACE;
  const SubLayout L = carve_sub(ws, batch, d);
  hipStream_t s = as_stream(stream);
  double* loss64 = static_cast<double*>(saved);
  float* Msave = reinterpret_cast<float*>(static_cast<char*>(saved) + align_up((size_t)batch * sizeof(double)));
  const int rc = launch_products(d, batch, P, B, L, s);
  if (rc != NLSP_OK) return rc;
  NLSP_HIP(allow_lds(k_fwd_finish, fin_lds(d)));
  hipLaunchKernelGGL(k_fwd_finish, dim3(batch), dim3(NTF), fin_lds(d), s, d, L.T64, L.bbpart, colw, loss, loss64,
                     Msave);
  NLSP_HIP(hipGetLastError());
  return NLSP_OK;
}

int subspace_loss_bwd(int batch, int n, int k, int m, const float* P, const float* B, const void* saved,
                      size_t saved_nbytes, const float* gloss, float* gP, void* stream) {
  if (!dims_ok(batch, n, k, m) || !P || !B || !saved || !gloss || !gP) return NLSP_E_INVALID;
  Dims d = make_dims(batch, n, k, m);
  if (!aligned16(P) || !aligned16(B)) d.vec = 0;
  if (saved_nbytes < saved_bytes(batch, d)) return NLSP_E_WORKSPACE;
  const float* Msave =
      reinterpret_cast<const float*>(static_cast<const char*>(saved) + align_up((size_t)batch * sizeof(double)));
  const int rc = launch_bwd(d, batch, P, B, Msave, gloss, gP, as_stream(stream));
  if (rc != NLSP_OK) return rc;
  NLSP_HIP(hipGetLastError());
  return NLSP_OK;
}

size_t captured_energy_workspace_bytes(int batch, int n, int k, int m) {
  if (!dims_ok(batch, n, k, m)) return 0;
  return carve_sub(nullptr, batch, make_dims(batch, n, k, m, false, true)).bytes;
}

int captured_energy(int batch, int n, int k, int m, const float* P, const float* S, double* energy, void* ws,
                    size_t ws_bytes, void* stream) {
  if (!dims_ok(batch, n, k, m) || !P || !S || !energy) return NLSP_E_INVALID;
  Dims d = make_dims(batch, n, k, m, false, true);   // P staged (the A operand), no G tiles
  if (!aligned16(P) || !aligned16(S)) d.vec = 0;
  if (d.ntiles > MAX_TILES || fwd_lds(d) > LDS_MAX) return NLSP_E_INVALID;
  if (!ws_ok(ws, ws_bytes, carve_sub(nullptr, batch, d).bytes)) return NLSP_E_WORKSPACE;
  const SubLayout L = carve_sub(ws, batch, d);
  hipStream_t s = as_stream(stream);
  const int rc = launch_products(d, batch, P, S, L, s);
  if (rc != NLSP_OK) return rc;
  hipLaunchKernelGGL(k_energy_finish, dim3(batch), dim3(64), 0, s, d, L.T64, L.bbpart, energy);
  NLSP_HIP(hipGetLastError());
  return NLSP_OK;
}

size_t galerkin_fwd_workspace_bytes(int batch, const nlsp_operator* A, int k) {
  const int64_t n = batched_op_size(A);
  if (n < 1 || !gal_ok(batch, n, k)) return 0;
  return carve_sub(nullptr, batch, gal_fwd_dims(batch, (int)n, k)).bytes;
}

int galerkin_fwd(int batch, const nlsp_operator* A, const float* P, int k, float* Ac, float* Y, void* ws,
                 size_t ws_bytes, void* stream) {
  const int64_t n = batched_op_size(A);
  if (n < 1 || !gal_ok(batch, n, k) || !P || !Ac || !Y || P == Y) return NLSP_E_INVALID;
  Dims d = gal_fwd_dims(batch, (int)n, k);
  if (!aligned16(P) || !aligned16(Y)) d.vec = 0;
  const size_t need = carve_sub(nullptr, batch, d).bytes;
  if (!ws_ok(ws, ws_bytes, need)) return NLSP_E_WORKSPACE;
  const SubLayout L = carve_sub(ws, batch, d);
  hipStream_t s = as_stream(stream);
  const OpDev op = make_op(*A);
  if ((A->kind == NLSP_OP_FV5 || A->kind == NLSP_OP_FV7 || A->kind == NLSP_OP_POISSON5) && k % 4 == 0 &&
      aligned16(P) && aligned16(Y)) {
    // row-blocked: the Galerkin-term product with no S block
    const FastDiv fcv = make_fastdiv((uint32_t)(k / 4));
    const unsigned nb = (unsigned)ceil_div(n, GT_TR);
    if (A->kind == NLSP_OP_FV7)
      hipLaunchKernelGGL(k_gterm_rows<6>, dim3(nb, batch), dim3(NT), 0, s, op, coef_stride(*A, n), k, 0, fcv, P,
                         nullptr, Y, nullptr);
    else
      hipLaunchKernelGGL(k_gterm_rows<4>, dim3(nb, batch), dim3(NT), 0, s, op, coef_stride(*A, n), k, 0, fcv, P,
                         nullptr, Y, nullptr);
  } else {
    hipLaunchKernelGGL(k_gal_apply, dim3(ceil_div(n * k, NT), batch), dim3(NT), 0, s, op, coef_stride(*A, n), k,
                       make_fastdiv((uint32_t)k), P, Y);
  }
  // T = P^T [Y | P], tiles of P^T Y only: Y is the "B" block, P the "P" block
  const int rc = launch_products(d, batch, P, Y, L, s);
  if (rc != NLSP_OK) return rc;
  hipLaunchKernelGGL(k_gal_finish, dim3(batch), dim3(NT), 0, s, d, L.T64, Ac);
  NLSP_HIP(hipGetLastError());
  return NLSP_OK;
}

size_t galerkin_bwd_workspace_bytes(int batch, int n, int k) {
  if (!gal_ok(batch, n, k)) return 0;
  return align_up((size_t)batch * round16(k) * round16(k) * sizeof(float));
}

int galerkin_bwd(int batch, int n, int k, const float* Y, const float* gAc, float* gP, void* ws, size_t ws_bytes,
                 void* stream) {
  if (!gal_ok(batch, n, k) || !Y || !gAc || !gP || Y == gP) return NLSP_E_INVALID;
  Dims d = gal_bwd_dims(batch, n, k);
  if (!aligned16(Y)) d.vec = 0;
  const size_t need = galerkin_bwd_workspace_bytes(batch, n, k);
  if (!ws_ok(ws, ws_bytes, need)) return NLSP_E_WORKSPACE;
  float* M = static_cast<float*>(ws);
  hipStream_t s = as_stream(stream);
  hipLaunchKernelGGL(k_gal_bwd_prep, dim3(batch), dim3(NT), 0, s, k, d.kp, gAc, M);
  // gP = [Y] (G + G^T): Y is the "B" block, no P block
  const int rc = launch_bwd(d, batch, Y, Y, M, nullptr, gP, s);
  if (rc != NLSP_OK) return rc;
  NLSP_HIP(hipGetLastError());
  return NLSP_OK;
}

size_t qr_thin_workspace_bytes(int batch, int n, int k) {
  if (!qr_ok(batch, n, k)) return 0;
  return carve_qr(nullptr, batch, n, k).bytes;
}

int qr_thin_fwd(int batch, int n, int k, const float* A, float* Q, double* R, int* bad, void* ws, size_t ws_bytes,
                void* stream) {
  if (!qr_ok(batch, n, k) || !A || !Q || !R || !bad || A == Q) return NLSP_E_INVALID;
  if (!ws_ok(ws, ws_bytes, carve_qr(nullptr, batch, n, k).bytes)) return NLSP_E_WORKSPACE;
  const QrLayout L = carve_qr(ws, batch, n, k);
  hipStream_t s = as_stream(stream);
  Dims dp = qr_dims(batch, n, k, true);       // P^T B
  Dims db = qr_dims(batch, n, k, false);      // B M
  if (!aligned16(A) || !aligned16(Q)) dp.vec = db.vec = 0;
  NLSP_HIP(hipMemsetAsync(bad, 0, sizeof(int) * batch, s));
  // pass 1: G = A^T A, R1, Q1 = A R1^-1
  int rc = launch_products(dp, batch, A, A, L.prod, s);
  if (rc != NLSP_OK) return rc;
  hipLaunchKernelGGL(k_qr_small, dim3(batch), dim3(NT), 0, s, dp, L.prod.T64, 1, L.R1, R, L.M, bad);
  rc = launch_bwd(db, batch, A, A, L.M, nullptr, L.Q1, s);
  if (rc != NLSP_OK) return rc;
  // pass 2: G = Q1^T Q1, R2, Q = Q1 R2^-1, R = R2 R1
  rc = launch_products(dp, batch, L.Q1, L.Q1, L.prod, s);
  if (rc != NLSP_OK) return rc;
  hipLaunchKernelGGL(k_qr_small, dim3(batch), dim3(NT), 0, s, dp, L.prod.T64, 0, L.R1, R, L.M, bad);
  rc = launch_bwd(db, batch, L.Q1, L.Q1, L.M, nullptr, Q, s);
  if (rc != NLSP_OK) return rc;
  NLSP_HIP(hipGetLastError());
  return NLSP_OK;
}

int qr_thin_bwd(int batch, int n, int k, const float* Q, const double* R, const float* gQ, float* gA, void* ws,
                size_t ws_bytes, void* stream) {
  if (!qr_ok(batch, n, k) || !Q || !R || !gQ || !gA || gA == Q || gA == gQ) return NLSP_E_INVALID;
  if (!ws_ok(ws, ws_bytes, carve_qr(nullptr, batch, n, k).bytes)) return NLSP_E_WORKSPACE;
  const QrLayout L = carve_qr(ws, batch, n, k);
  hipStream_t s = as_stream(stream);
  Dims dp = qr_dims(batch, n, k, true);
  if (!aligned16(Q) || !aligned16(gQ) || !aligned16(gA)) dp.vec = 0;
  // T = Q^T dQ (A operand Q, B block dQ)
  int rc = launch_products(dp, batch, Q, gQ, L.prod, s);
  if (rc != NLSP_OK) return rc;
  hipLaunchKernelGGL(k_qr_bwd_small, dim3(batch), dim3(NT), 0, s, dp, L.prod.T64, R, L.M);
  // dA = [dQ | Q] [R^-T ; C R^-T]
  rc = launch_bwd(dp, batch, Q, gQ, L.M, nullptr, gA, s);
  if (rc != NLSP_OK) return rc;
  NLSP_HIP(hipGetLastError());
  return NLSP_OK;
}

// ---------------------------------------------------------------- J(P)
// forward dims: products P^T X over the tiles of P^T X (X = [A S | A P] is
// the "B" block, P the "P" block); backward dims: X M, no P block
inline Dims gterm_fwd_dims(int batch, int n, int k, int m) { return make_dims(batch, n, k, m + k, false, true); }
inline Dims gterm_bwd_dims(int batch, int n, int k, int m) { return make_dims(batch, n, k, m + k, false, false); }
inline bool gterm_ok(int batch, int64_t n, int k, int m) {
  if (batch < 1 || n < 1 || k < 1 || m < 1 || k > QRK || m + k > 256 || k * m > 4096) return false;
  if (n * (m + k) >= (int64_t(1) << 31)) return false;
  const Dims d = gterm_fwd_dims(batch, (int)n, k, m);
  return d.ntiles <= MAX_TILES && fwd_lds(d) <= LDS_MAX && bwd_lds(gterm_bwd_dims(batch, (int)n, k, m)) <= LDS_MAX;
}
inline int gterm_apply_blocks(int64_t n, int k, int m) { return (int)ceil_div(n * (m + k), NT); }
inline size_t gterm_finish_lds(int k, int m) { return (2 * (size_t)QRK * QRK + 2 * (size_t)k * m) * sizeof(double); }

struct GtermSaved {
  float* X;   // (batch, n, m + k)
  float* M;   // (batch, cols, kp)
  size_t bytes;
};
inline GtermSaved carve_gterm(void* saved, int batch, int64_t n, int k, int m) {
  const Dims db = gterm_bwd_dims(batch, (int)n, k, m);
  Carver c(saved);
  GtermSaved G;
  G.X = c.take<float>((size_t)batch * n * (m + k));
  G.M = c.take<float>((size_t)batch * db.cols * db.kp);
  G.bytes = c.bytes();
  return G;
}

size_t galerkin_term_saved_bytes(int batch, const nlsp_operator* A, int k, int m) {
  const int64_t n = batched_op_size(A);
  if (n < 1 || !gterm_ok(batch, n, k, m)) return 0;
  return carve_gterm(nullptr, batch, n, k, m).bytes;
}

size_t galerkin_term_workspace_bytes(int batch, const nlsp_operator* A, int k, int m) {
  const int64_t n = batched_op_size(A);
  if (n < 1 || !gterm_ok(batch, n, k, m)) return 0;
  const SubLayout L = carve_sub(nullptr, batch, gterm_fwd_dims(batch, (int)n, k, m));
  return align_up(L.bytes) + align_up((size_t)batch * gterm_apply_blocks(n, k, m) * sizeof(double));
}

int galerkin_term_fwd(int batch, const nlsp_operator* A, const float* P, const float* S, int k, int m, float* J,
                      float* E, int* bad, void* saved, size_t saved_nbytes, void* ws, size_t ws_bytes,
                      void* stream) {
  const int64_t n = batched_op_size(A);
  if (n < 1 || !gterm_ok(batch, n, k, m) || !P || !S || !J || !bad || !saved) return NLSP_E_INVALID;
  const GtermSaved G = carve_gterm(nullptr, batch, n, k, m);
  if (saved_nbytes < G.bytes || reinterpret_cast<uintptr_t>(saved) % WS_ALIGN) return NLSP_E_WORKSPACE;
  const size_t need = galerkin_term_workspace_bytes(batch, A, k, m);
  if (!ws_ok(ws, ws_bytes, need)) return NLSP_E_WORKSPACE;
  const GtermSaved Gs = carve_gterm(saved, batch, n, k, m);
  Dims d = gterm_fwd_dims(batch, (int)n, k, m);
  if (!aligned16(P)) d.vec = 0;
  const SubLayout L = carve_sub(ws, batch, d);
  double* spart = reinterpret_cast<double*>(static_cast<char*>(ws) + align_up(L.bytes));
  hipStream_t s = as_stream(stream);
  const OpDev op = make_op(*A);
  // row-blocked product for face operators with 16-byte rows, else one element per thread
  const bool rows = (A->kind == NLSP_OP_FV5 || A->kind == NLSP_OP_FV7 || A->kind == NLSP_OP_POISSON5) &&
                    m % 4 == 0 && k % 4 == 0 && aligned16(P) && aligned16(S) && aligned16(Gs.X);
  int nb;
  if (rows) {
    nb = (int)ceil_div(n, GT_TR);
    const FastDiv fcv = make_fastdiv((uint32_t)((m + k) / 4));
    if (A->kind == NLSP_OP_FV7)
      hipLaunchKernelGGL(k_gterm_rows<6>, dim3(nb, batch), dim3(NT), 0, s, op, coef_stride(*A, n), k, m, fcv, P,
                         S, Gs.X, spart);
    else
      hipLaunchKernelGGL(k_gterm_rows<4>, dim3(nb, batch), dim3(NT), 0, s, op, coef_stride(*A, n), k, m, fcv, P,
                         S, Gs.X, spart);
  } else {
    nb = gterm_apply_blocks(n, k, m);
    hipLaunchKernelGGL(k_gterm_apply, dim3(nb, batch), dim3(NT), 0, s, op, coef_stride(*A, n), k, m,
                       make_fastdiv((uint32_t)(m + k)), P, S, Gs.X, spart);
  }
  // T = P^T X: X is the "B" block, P the "P" block
  int rc = launch_products(d, batch, P, Gs.X, L, s);
  if (rc != NLSP_OK) return rc;
  const size_t lds = gterm_finish_lds(k, m);
  if (allow_lds(k_gterm_finish, lds) != hipSuccess) return NLSP_E_HIP;
  const Dims db = gterm_bwd_dims(batch, (int)n, k, m);
  Dims df = d;
  df.cols = db.cols;   // the finishing kernel writes M with the backward's row count
  hipLaunchKernelGGL(k_gterm_finish, dim3(batch), dim3(NT), lds, s, df, m, L.T64, spart, nb, J, E, bad, Gs.M);
  NLSP_HIP(hipGetLastError());
  return NLSP_OK;
}

int galerkin_term_bwd(int batch, const nlsp_operator* A, int k, int m, const void* saved, const float* gJ,
                      float* gP, void* stream) {
  const int64_t n = batched_op_size(A);
  if (n < 1 || !gterm_ok(batch, n, k, m) || !saved || !gJ || !gP) return NLSP_E_INVALID;
  if (reinterpret_cast<uintptr_t>(saved) % WS_ALIGN) return NLSP_E_WORKSPACE;
  const GtermSaved Gs = carve_gterm(const_cast<void*>(saved), batch, n, k, m);
  const Dims d = gterm_bwd_dims(batch, (int)n, k, m);
  // dJ/dP = g_b X M: X is the "B" block, no P block
  const int rc = launch_bwd(d, batch, Gs.X, Gs.X, Gs.M, gJ, gP, as_stream(stream));
  if (rc != NLSP_OK) return rc;
  NLSP_HIP(hipGetLastError());
  return NLSP_OK;
}

}  // extern "C"
