// Device-side building blocks shared by the gfx950 kernels of the library:
// matrix-free stencil rows for the four operator kinds, deterministic wave64 /
// workgroup reductions and the "last workgroup to arrive" ticket used to
// finish a grid-wide reduction inside the producing kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nlsp.h"

#define NLSP_DEV __device__ __forceinline__

// Pointers that the device reads out of descriptors in memory are generic
// (flat) to the compiler, and flat accesses count against both the vector and
// the LDS/scalar wait counters, so every scalar or LDS wait would also drain
// the loads in flight.  Descriptor pointers are therefore declared in the
// global address space for the device pass (same layout and bits as on the
// host, where the qualifier is empty).
#if defined(__HIP_DEVICE_COMPILE__)
#define NLSP_GAS __attribute__((address_space(1)))
#else
#define NLSP_GAS
#endif

namespace nlsp {

template <typename T>
using Glob = NLSP_GAS T;

template <typename T>
__host__ __device__ inline Glob<T>* as_glob(T* p) {
  return (Glob<T>*)p;
}

constexpr int WAVE = 64;

// ------------------------------------------------------------------ indices
// Unsigned 32-bit division by a run-time constant d >= 1 with a precomputed
// multiplier ("round-up" method, Granlund & Montgomery 1994):
//   s = ceil(log2 d), m = floor(2^32 (2^s - d) / d) + 1,
//   n / d = (mulhi(n, m) + n) >> s      exact for every 32-bit n.
struct FastDiv {
  uint32_t d, m, s;
};

inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  f.s = 0;
  while ((1ull << f.s) < d) ++f.s;
  f.m = (uint32_t)((((1ull << 32) * ((1ull << f.s) - d)) / d) + 1);
  return f;
}

NLSP_DEV uint32_t fdiv(uint32_t n, const FastDiv& f) {
  return (uint32_t)(((uint64_t)__umulhi(n, f.m) + n) >> f.s);
}

// ------------------------------------------------------------------ operator
struct OpDev {
  int kind, nx, ny, nz;
  int64_t n;
  Glob<const double>* coef;
  FastDiv fx, fxy;   // division by nx and by nx*ny
  // Optional face weights of the finite-volume operators (null: formed on the
  // fly): fw64[a*n + i] = harmonic(a_i, a_j) in float64 and fw32 the same
  // formed in float32 from the rounded coefficients, for the face between i
  // and its neighbour j = i + 1, i + nx, i + nx*ny (axis a = 0, 1, 2).  Both
  // are what op_row would form, bit for bit (the mean is commutative).
  Glob<const double>* fw64;
  Glob<const float>* fw32;
  // compressed rows (NLSP_OP_CSR): entries rp[i] .. rp[i+1] - 1 of row i
  Glob<const int>* rp;
  Glob<const int>* ci;
};

inline OpDev make_op(const nlsp_operator& a) {
  OpDev o;
  o.kind = a.kind;
  o.nx = a.nx;
  o.ny = a.ny;
  o.nz = (a.kind == NLSP_OP_FV7) ? a.nz : 1;
  o.n = (int64_t)o.nx * o.ny * o.nz;
  o.coef = as_glob(a.coef);
  o.fx = make_fastdiv((uint32_t)o.nx);
  o.fxy = make_fastdiv((uint32_t)o.nx * (uint32_t)o.ny);
  o.fw64 = nullptr;
  o.fw32 = nullptr;
  o.rp = (a.kind == NLSP_OP_CSR) ? as_glob(a.row_ptr) : nullptr;
  o.ci = (a.kind == NLSP_OP_CSR) ? as_glob(a.col_idx) : nullptr;
  return o;
}

template <typename T>
NLSP_DEV T harmonic(T a, T b) {
  // 2ab/(a+b): commutative in IEEE arithmetic, so A stays exactly symmetric
  return (T(2) * a * b) / (a + b);
}

// (A v)_i for the unknown i at grid position (x, y, z).  `v(j)` returns the
// value of the operand at unknown j.  Arithmetic in T (double or float).
// FW: a finite-volume operator reads its face weights from op.fw64 / op.fw32
// (which must then be set) instead of forming the harmonic means.
// ZC (with FW): the operand at the -z and +z neighbours is given as vzm, vzp
// instead of being read through v (used only where those faces exist).
// Branch-free: a neighbour outside the grid reads row i itself and its term
// is discarded by a select, so every load of the row is issued before the
// first use (a load under a branch would be waited for inside the branch).
template <typename T, bool FW = false, bool ZC = false, typename V>
NLSP_DEV T op_row(const OpDev& op, int64_t i, int x, int y, int z, V v, T vzm = T(0), T vzp = T(0)) {
  const int nx = op.nx, ny = op.ny;
  switch (op.kind) {
    case NLSP_OP_POISSON5: {
      const int64_t jn[4] = {i - 1, i + 1, i - nx, i + nx};
      const bool in[4] = {x > 0, x < nx - 1, y > 0, y < ny - 1};
      T s = T(0);
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        const T vj = v(in[f] ? jn[f] : i);
        s += in[f] ? vj : T(0);
      }
      return T(4) * v(i) - s;
    }
    case NLSP_OP_FV5:
    case NLSP_OP_FV7: {
      // faces -x, +x, -y, +y (, -z, +z); a boundary face puts its Dirichlet
      // weight 2 a_P on the diagonal only
      const auto a = op.coef;
      const int64_t sxy = (int64_t)nx * ny;
      const int nf = (op.kind == NLSP_OP_FV7) ? 6 : 4;
      const int64_t jn[6] = {i - 1, i + 1, i - nx, i + nx, i - sxy, i + sxy};
      const bool in[6] = {x > 0, x < nx - 1, y > 0, y < ny - 1, z > 0, z < op.nz - 1};
      const T aP = T(a[i]);
      T d = T(0), s = T(0);
      if constexpr (FW) {
        const auto fw = [&] {
          if constexpr (sizeof(T) == 8)
            return op.fw64;
          else
            return op.fw32;
        }();
        // face f of axis f/2: the lower face (-) is stored at the lower
        // neighbour, the upper one at i; a boundary face reads i's own
        const int64_t n = op.n;
#pragma unroll
        for (int f = 0; f < 6; ++f) {
          if (f >= nf) break;
          const int64_t j = in[f] ? jn[f] : i;
          const int64_t fi = (f / 2) * n + ((in[f] && (f & 1) == 0) ? j : i);
          const T t = T(fw[fi]);
          const T vj = (ZC && f == 4) ? vzm : ((ZC && f == 5) ? vzp : v(j));
          d += in[f] ? t : T(2) * aP;
          s += in[f] ? t * vj : T(0);
        }
        return d * v(i) - s;
      }
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        if (f >= nf) break;
        const int64_t j = in[f] ? jn[f] : i;
        const T aj = T(a[j]), vj = v(j);
        const T t = harmonic<T>(aP, aj);
        d += in[f] ? t : T(2) * aP;
        s += in[f] ? t * vj : T(0);
      }
      return d * v(i) - s;
    }
    case NLSP_OP_CSR: {
      // the row's entries in stored order (a data-dependent trip count)
      const int e0 = op.rp[i], e1 = op.rp[i + 1];
      T s = T(0);
      for (int e = e0; e < e1; ++e) s += T(op.coef[e]) * v(op.ci[e]);
      return s;
    }
    default: {  // NLSP_OP_STENCIL9
      const auto c = op.coef;
      T s = T(0);
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          const bool ok = y + dy >= 0 && y + dy < ny && x + dx >= 0 && x + dx < nx;
          const T vj = v(ok ? i + dx + (int64_t)dy * nx : i);
          s += ok ? T(c[(dy + 1) * 3 + (dx + 1)]) * vj : T(0);
        }
      }
      return s;
    }
  }
}

// diag(A)_i
template <typename T>
NLSP_DEV T op_diag(const OpDev& op, int64_t i, int x, int y, int z) {
  switch (op.kind) {
    case NLSP_OP_POISSON5:
      return T(4);
    case NLSP_OP_FV5:
    case NLSP_OP_FV7: {
      const auto a = op.coef;
      const int nx = op.nx, ny = op.ny;
      const int64_t sxy = (int64_t)nx * ny;
      const T aP = T(a[i]);
      T d = T(0);
      auto face = [&](bool inside, int64_t j) {
        const T h = harmonic<T>(aP, T(a[inside ? j : i]));
        d += inside ? h : T(2) * aP;
      };
      face(x > 0, i - 1);
      face(x < nx - 1, i + 1);
      face(y > 0, i - nx);
      face(y < ny - 1, i + nx);
      if (op.kind == NLSP_OP_FV7) {
        face(z > 0, i - sxy);
        face(z < op.nz - 1, i + sxy);
      }
      return d;
    }
    case NLSP_OP_CSR: {
      const int e0 = op.rp[i], e1 = op.rp[i + 1];
      T d = T(0);
      for (int e = e0; e < e1; ++e)
        if (op.ci[e] == (int)i) d = T(op.coef[e]);
      return d;
    }
    default:
      return T(op.coef[4]);
  }
}

// grid position of unknown i (n < 2^31 is enforced by the host checks)
NLSP_DEV void decompose(const OpDev& op, int64_t i, int& x, int& y, int& z) {
  const uint32_t ui = (uint32_t)i;
  const uint32_t zz = fdiv(ui, op.fxy);
  const uint32_t rem = ui - zz * op.fxy.d;
  const uint32_t yy = fdiv(rem, op.fx);
  z = (int)zz;
  y = (int)yy;
  x = (int)(rem - yy * op.fx.d);
}

// Logical block index for a launch of nb blocks so that consecutive logical
// blocks run on the same XCD: the hardware deals blocks round-robin over the
// 8 XCDs (block b on XCD b % 8), so XCD x receives the contiguous logical range
// [start_x, start_x + count_x).  Keeps stencil neighbours in one L2.
NLSP_DEV int xcd_remap(int b, int nb) {
  const int x = b & 7, q = nb >> 3, rem = nb & 7;
  const int start = x * q + (x < rem ? x : rem);
  return start + (b >> 3);
}

// ---------------------------------------------------------------- reductions
template <typename T>
NLSP_DEV T wave_sum(T v) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

// Sum over the lanes of aligned groups of G lanes (G a power of two <= 64);
// every lane of a group receives the group sum.
template <typename T>
NLSP_DEV T group_sum(T v, int G) {
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

// Deterministic workgroup sum of one double per thread: wave butterflies, then
// the wave totals added in wave order by every thread.  `sh` holds
// blockDim.x/64 doubles.  Contains __syncthreads; all threads must call.
NLSP_DEV double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
  __syncthreads();
  if ((threadIdx.x & (WAVE - 1)) == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int k = 0; k < nw; ++k) s += sh[k];
  return s;
}

// Cross-workgroup partial sums.  Partials are written and read with
// agent-scope relaxed atomics, which compile to device-coherent stores and
// loads (sc1) that go to the coherence point shared by all XCDs instead of
// requiring a write-back of the whole L2 (what __threadfence() costs here).
template <typename P>
NLSP_DEV void store_partial(P p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename P>
NLSP_DEV double load_partial(P p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid-wide reductions finish inside the producing kernel in two levels.
// Workgroups are grouped by TICKET_GROUP consecutive logical indices.  Every
// workgroup writes its partial record with store_partial and calls
// arrive_group; the last workgroup of a group (arrive_group == true) sums the
// group's records, publishes a group record and calls arrive_top; the last of
// those (arrive_top == true) sums the group records.  Before each ticket
// every thread waits until its own device-coherent stores have completed.
// Counters are 64 bytes apart and are reset by the workgroup completing them.
// `tickets` holds ticket_words(nblocks) unsigned ints, zero before first use.
constexpr int TICKET_GROUP = 16;
constexpr int TICKET_STRIDE = 16;

__host__ __device__ inline int ticket_groups(int nblocks) { return (nblocks + TICKET_GROUP - 1) / TICKET_GROUP; }
__host__ __device__ inline int ticket_words(int nblocks) { return TICKET_STRIDE * (1 + ticket_groups(nblocks)); }

NLSP_DEV void wait_own_stores() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);  // all of this thread's memory operations done
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

template <typename P>
NLSP_DEV bool arrive_group(P tickets, unsigned nblocks, unsigned lb) {
  __shared__ int s_last;
  wait_own_stores();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned grp = lb / TICKET_GROUP;
    const unsigned gsize = min((unsigned)TICKET_GROUP, nblocks - grp * TICKET_GROUP);
    auto gt = tickets + TICKET_STRIDE * (1 + grp);
    const unsigned t1 = __hip_atomic_fetch_add(gt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_last = (t1 == gsize - 1) ? 1 : 0;
    if (s_last) __hip_atomic_store(gt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  return s_last != 0;
}

template <typename P>
NLSP_DEV bool arrive_top(P tickets, unsigned ngroups) {
  __shared__ int s_last;
  wait_own_stores();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned t2 = __hip_atomic_fetch_add(tickets, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_last = (t2 == ngroups - 1) ? 1 : 0;
    if (s_last) __hip_atomic_store(tickets, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  return s_last != 0;
}

}  // namespace nlsp
