// Device-side building blocks shared by the gfx950 kernels of the library:
// matrix-free stencil rows for the four operator kinds, deterministic wave64 /
// workgroup reductions and the "last workgroup to arrive" ticket used to
// finish a grid-wide reduction inside the producing kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nlsp.h"

#define NLSP_DEV __device__ __forceinline__

namespace nlsp {

constexpr int WAVE = 64;

// ------------------------------------------------------------------ operator
struct OpDev {
  int kind, nx, ny, nz;
  int64_t n;
  const double* coef;
};

inline OpDev make_op(const nlsp_operator& a) {
  OpDev o;
  o.kind = a.kind;
  o.nx = a.nx;
  o.ny = a.ny;
  o.nz = (a.kind == NLSP_OP_FV7) ? a.nz : 1;
  o.n = (int64_t)o.nx * o.ny * o.nz;
  o.coef = a.coef;
  return o;
}

template <typename T>
NLSP_DEV T harmonic(T a, T b) {
  // 2ab/(a+b): commutative in IEEE arithmetic, so A stays exactly symmetric
  return (T(2) * a * b) / (a + b);
}

// (A v)_i for the unknown i at grid position (x, y, z).  `v(j)` returns the
// value of the operand at unknown j.  Arithmetic in T (double or float).
template <typename T, typename V>
NLSP_DEV T op_row(const OpDev& op, int64_t i, int x, int y, int z, V v) {
  const int nx = op.nx, ny = op.ny;
  switch (op.kind) {
    case NLSP_OP_POISSON5: {
      T s = T(0);
      if (x > 0) s += v(i - 1);
      if (x < nx - 1) s += v(i + 1);
      if (y > 0) s += v(i - nx);
      if (y < ny - 1) s += v(i + nx);
      return T(4) * v(i) - s;
    }
    case NLSP_OP_FV5: {
      const double* a = op.coef;
      const T aP = T(a[i]);
      T d = T(0), s = T(0);
      auto face = [&](bool inside, int64_t j) {
        if (inside) {
          const T t = harmonic<T>(aP, T(a[j]));
          d += t;
          s += t * v(j);
        } else {
          d += T(2) * aP;
        }
      };
      face(x > 0, i - 1);
      face(x < nx - 1, i + 1);
      face(y > 0, i - nx);
      face(y < ny - 1, i + nx);
      return d * v(i) - s;
    }
    case NLSP_OP_FV7: {
      const double* a = op.coef;
      const int64_t sxy = (int64_t)nx * ny;
      const T aP = T(a[i]);
      T d = T(0), s = T(0);
      auto face = [&](bool inside, int64_t j) {
        if (inside) {
          const T t = harmonic<T>(aP, T(a[j]));
          d += t;
          s += t * v(j);
        } else {
          d += T(2) * aP;
        }
      };
      face(x > 0, i - 1);
      face(x < nx - 1, i + 1);
      face(y > 0, i - nx);
      face(y < ny - 1, i + nx);
      face(z > 0, i - sxy);
      face(z < op.nz - 1, i + sxy);
      return d * v(i) - s;
    }
    default: {  // NLSP_OP_STENCIL9
      const double* c = op.coef;
      T s = T(0);
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy) {
        if (y + dy < 0 || y + dy >= ny) continue;
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          if (x + dx < 0 || x + dx >= nx) continue;
          s += T(c[(dy + 1) * 3 + (dx + 1)]) * v(i + dx + (int64_t)dy * nx);
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
      const double* a = op.coef;
      const int nx = op.nx, ny = op.ny;
      const int64_t sxy = (int64_t)nx * ny;
      const T aP = T(a[i]);
      T d = T(0);
      auto face = [&](bool inside, int64_t j) { d += inside ? harmonic<T>(aP, T(a[j])) : T(2) * aP; };
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
    default:
      return T(op.coef[4]);
  }
}

NLSP_DEV void decompose(const OpDev& op, int64_t i, int& x, int& y, int& z) {
  const int64_t sxy = (int64_t)op.nx * op.ny;
  z = (int)(i / sxy);
  const int64_t rem = i - (int64_t)z * sxy;
  y = (int)(rem / op.nx);
  x = (int)(rem - (int64_t)y * op.nx);
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

// Every workgroup of a grid-wide reduction calls this after writing its
// partials.  Returns true (in all threads) in the workgroup that arrives
// last; that workgroup may then read every partial.  The ticket is reset by
// the last workgroup so the next launch can reuse it.
NLSP_DEV bool arrive_last(unsigned* ticket, unsigned nblocks) {
  __shared__ int s_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned t = atomicAdd(ticket, 1u);
    s_last = (t == nblocks - 1) ? 1 : 0;
    if (s_last) *ticket = 0u;
  }
  __syncthreads();
  const bool last = s_last != 0;
  if (last) __threadfence();
  return last;
}

}  // namespace nlsp
