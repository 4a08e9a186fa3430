// Matrix-free operator entry points: Q1 anisotropic stencil build, float64
// operator application and the float32 weighted-Jacobi sweep.
#include <algorithm>
#include <type_traits>

#include "device_common.hpp"
#include "host_common.hpp"

namespace nlsp {

// Q1 element stiffness for a constant tensor K on a square element, closed
// form: Ke = K11*Mxx + K22*Myy + K12*(Mxy + Mxy^T) with the bilinear
// reference integrals Mxx, Myy (entries in sixths) and Mxy = a b^T / 4,
// a = (-1, 1, 1, -1), b = (-1, -1, 1, 1) (local nodes (0,0),(1,0),(1,1),(0,1)).
// The 9-point stencil of an interior node sums the four elements around it.
__global__ void k_q1_stencil(int nsys, const double* __restrict__ et, double* __restrict__ out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsys) return;
  const double eps = et[2 * s], th = et[2 * s + 1];
  const double c = cos(th), sn = sin(th);
  const double k11 = c * c + eps * sn * sn, k22 = sn * sn + eps * c * c, k12 = (1.0 - eps) * c * sn;
  const double mxx[4][4] = {{2, -2, -1, 1}, {-2, 2, 1, -1}, {-1, 1, 2, -2}, {1, -1, -2, 2}};
  const double myy[4][4] = {{2, 1, -1, -2}, {1, 2, -2, -1}, {-1, -2, 2, 1}, {-2, -1, 1, 2}};
  const double av[4] = {-1, 1, 1, -1}, bv[4] = {-1, -1, 1, 1};
  const int ox[4] = {0, 1, 1, 0}, oy[4] = {0, 0, 1, 1};
  double ke[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j)
      ke[i][j] = (k11 * mxx[i][j] + k22 * myy[i][j]) / 6.0 +
                 k12 * 0.25 * (av[i] * bv[j] + av[j] * bv[i]);
  double st[9];
  for (int q = 0; q < 9; ++q) st[q] = 0.0;
  // node at the origin; elements with lower-left corner (ex, ey), ex, ey in {-1, 0}
  for (int ey = -1; ey <= 0; ++ey)
    for (int ex = -1; ex <= 0; ++ex) {
      int a = -1;
      for (int l = 0; l < 4; ++l)
        if (ex + ox[l] == 0 && ey + oy[l] == 0) a = l;
      for (int b = 0; b < 4; ++b) {
        const int dx = ex + ox[b], dy = ey + oy[b];
        st[(dy + 1) * 3 + (dx + 1)] += ke[a][b];
      }
    }
  for (int q = 0; q < 9; ++q) out[9 * s + q] = st[q];
}

// Row-blocked operator kernels for R right-hand sides.  A block owns TR
// consecutive rows (consecutive blocks on one XCD): its first threads form
// each row's stencil weights once (harmonic face means for FV5/FV7, in T)
// into LDS, then all threads stream the (row, rhs) pairs with the RHS index
// fastest, so every neighbour read is one coalesced run.
//   MODE 0: y = A x                                   (T = double)
//   MODE 1: y = x + omega D^-1 (b - A x)              (T = float)
constexpr int RNT = 256;
constexpr int TRMAX = 256;

NLSP_DEV int stencil_slots(const OpDev& op) {
  return op.kind == NLSP_OP_STENCIL9 ? 8 : (op.kind == NLSP_OP_FV7 ? 6 : 4);
}

NLSP_DEV int64_t slot_offset(const OpDev& op, int s) {
  if (op.kind == NLSP_OP_STENCIL9) {
    const int q = s < 4 ? s : s + 1;           // 3x3 positions without the centre
    return (int64_t)(q % 3 - 1) + (int64_t)(q / 3 - 1) * op.nx;
  }
  const int64_t sxy = (int64_t)op.nx * op.ny;
  switch (s) {
    case 0: return -1;
    case 1: return 1;
    case 2: return -(int64_t)op.nx;
    case 3: return op.nx;
    case 4: return -sxy;
    default: return sxy;
  }
}

// diagonal and off-diagonal entries of row i (w[0] = A_ii, w[1 + s] = A_ij for
// slot s) and the mask of the slots whose neighbour exists
template <typename T>
NLSP_DEV unsigned row_weights(const OpDev& op, int64_t i, int x, int y, int z, T* w) {
  const int nx = op.nx, ny = op.ny;
  unsigned mask = 0;
  if (op.kind == NLSP_OP_STENCIL9) {
    const double* c = op.coef;
    w[0] = T(c[4]);
    for (int s = 0; s < 8; ++s) {
      const int q = s < 4 ? s : s + 1;
      const int dx = q % 3 - 1, dy = q / 3 - 1;
      const bool in = x + dx >= 0 && x + dx < nx && y + dy >= 0 && y + dy < ny;
      w[1 + s] = in ? T(c[q]) : T(0);
      mask |= in ? (1u << s) : 0u;
    }
    return mask;
  }
  const bool in[6] = {x > 0, x < nx - 1, y > 0, y < ny - 1, z > 0, z < op.nz - 1};
  const int ns = (op.kind == NLSP_OP_FV7) ? 6 : 4;
  if (op.kind == NLSP_OP_POISSON5) {
    w[0] = T(4);
    for (int s = 0; s < 4; ++s) {
      w[1 + s] = in[s] ? T(-1) : T(0);
      mask |= in[s] ? (1u << s) : 0u;
    }
    return mask;
  }
  const double* a = op.coef;
  const T aP = T(a[i]);
  T d = T(0);
  for (int s = 0; s < ns; ++s) {
    if (in[s]) {
      const T t = harmonic<T>(aP, T(a[i + slot_offset(op, s)]));
      d += t;
      w[1 + s] = -t;
      mask |= 1u << s;
    } else {
      d += T(2) * aP;
      w[1 + s] = T(0);
    }
  }
  w[0] = d;
  return mask;
}

// Block order.  Each XCD receives a contiguous range of logical blocks
// (xcd_remap).  When a block holds part of one x-line (TR <= nx), logical
// blocks enumerate 8 y-slabs, then z, then the y-lines of the slab, then the
// pieces of the line, so an XCD sweeps its own y-slab plane by plane: the
// z-neighbours of a plane were read one slab-plane earlier (ny nx / 8 rows,
// well inside the XCD's L2) and the y-neighbours one line earlier.
struct BlockMap {
  int slab_lines;      // y-lines per slab (0: plain contiguous blocks)
  int bpl;             // blocks per x-line
};

NLSP_DEV void block_rows(const OpDev& op, const BlockMap& bm, int TR, int lb, int64_t& r0, int& nrows) {
  if (bm.slab_lines == 0) {
    r0 = (int64_t)lb * TR;
    nrows = (int)min((int64_t)TR, op.n - r0);
    return;
  }
  const int per_slab = bm.slab_lines * op.nz * bm.bpl;
  const int s = lb / per_slab;
  const int ylo = s * bm.slab_lines;
  const int ylen = min(bm.slab_lines, op.ny - ylo);
  int rem = lb - s * per_slab;
  const int z = rem / (ylen * bm.bpl);
  rem -= z * ylen * bm.bpl;
  const int yy = rem / bm.bpl, h = rem - yy * bm.bpl;
  r0 = ((int64_t)z * op.ny + ylo + yy) * op.nx + (int64_t)h * TR;
  nrows = min(TR, op.nx - h * TR);
}

template <typename T, int VW>
struct VecOf;
template <> struct VecOf<double, 1> { using type = double; };
template <> struct VecOf<double, 2> { using type = double2; };
template <> struct VecOf<float, 1> { using type = float; };
template <> struct VecOf<float, 4> { using type = float4; };

template <typename T, int VW>
NLSP_DEV void vload(const T* p, T (&v)[VW]) {
  using V = typename VecOf<T, VW>::type;
  const V x = *reinterpret_cast<const V*>(p);
  const T* e = reinterpret_cast<const T*>(&x);
#pragma unroll
  for (int u = 0; u < VW; ++u) v[u] = e[u];
}

template <typename T, int VW>
NLSP_DEV void vstore(T* p, const T (&v)[VW]) {
  using V = typename VecOf<T, VW>::type;
  V x;
  T* e = reinterpret_cast<T*>(&x);
#pragma unroll
  for (int u = 0; u < VW; ++u) e[u] = v[u];
  *reinterpret_cast<V*>(p) = x;
}

// VW consecutive right-hand sides per lane (16-byte accesses when VW > 1)
template <typename T, int MODE, int NS, int VW>
__global__ __launch_bounds__(RNT) void k_rows(OpDev op, BlockMap bm, int R, int TR, FastDiv fRV, T omega,
                                              const T* __restrict__ b, const T* __restrict__ x,
                                              T* __restrict__ y) {
  __shared__ T sw[TRMAX][9];
  __shared__ unsigned smask[TRMAX];
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  int64_t r0;
  int nrows;
  block_rows(op, bm, TR, lb, r0, nrows);
  for (int t = threadIdx.x; t < nrows; t += RNT) {
    int px, py, pz;
    decompose(op, r0 + t, px, py, pz);
    smask[t] = row_weights<T>(op, r0 + t, px, py, pz, sw[t]);
  }
  __syncthreads();
  int64_t off[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) off[s] = slot_offset(op, s) * R;
  const int RV = R / VW;
  // every neighbour load is issued; a missing neighbour reads the centre
  // value with weight 0, so the loads need no branches (the centre term is
  // always present, so non-finite inputs propagate exactly as before)
  constexpr int UNR = sizeof(T) == 8 ? 4 : 2;   // measured best per type on 16 right-hand sides
#pragma unroll UNR
  for (int idx = threadIdx.x; idx < nrows * RV; idx += RNT) {
    const int rl = (int)fdiv((uint32_t)idx, fRV);
    const int64_t g = r0 * R + (int64_t)idx * VW;     // row r0 + rl, right-hand sides from (idx - rl RV) VW
    const unsigned mk = smask[rl];
    const T* wr = sw[rl];
    T v[NS + 1][VW];
    vload<T, VW>(x + g, v[0]);
#pragma unroll
    for (int s = 0; s < NS; ++s) vload<T, VW>(x + g + (((mk >> s) & 1u) ? off[s] : 0), v[1 + s]);
    T out[VW];
#pragma unroll
    for (int u = 0; u < VW; ++u) {
      T acc = wr[0] * v[0][u];
#pragma unroll
      for (int s = 0; s < NS; ++s) acc += wr[1 + s] * v[1 + s][u];
      out[u] = acc;
    }
    if (MODE == 1) {
      T bb[VW];
      vload<T, VW>(b + g, bb);
#pragma unroll
      for (int u = 0; u < VW; ++u) out[u] = v[0][u] + omega * (bb[u] - out[u]) / wr[0];
    }
    vstore<T, VW>(y + g, out);
  }
}

// rows per block: 2048 (row, rhs) pairs, at most TRMAX rows
inline int rows_per_block(int R) { return R >= 4 ? std::max(16, std::min(TRMAX, 2048 / R)) : TRMAX; }

// launch shape: number of blocks and their order (see block_rows)
inline unsigned plan_rows(const OpDev& op, int TR, BlockMap& bm) {
  if (TR > op.nx || op.ny < 8) {
    bm.slab_lines = 0;
    bm.bpl = 0;
    return ceil_div(op.n, TR);
  }
  bm.bpl = (op.nx + TR - 1) / TR;
  bm.slab_lines = (op.ny + 7) / 8;
  return (unsigned)((int64_t)op.ny * op.nz * bm.bpl);
}

// launches k_rows for the operator kind with the widest vector the right-hand
// side count and the pointers allow
template <typename T, int MODE>
inline void launch_rows(const OpDev& op, int R, T omega, const T* b, const T* x, T* y, hipStream_t s) {
  constexpr int VMAX = 16 / sizeof(T);
  const bool vec = (R % VMAX == 0) && reinterpret_cast<uintptr_t>(x) % 16 == 0 &&
                   reinterpret_cast<uintptr_t>(y) % 16 == 0 && (!b || reinterpret_cast<uintptr_t>(b) % 16 == 0);
  const int TR = rows_per_block(R);
  BlockMap bm;
  const unsigned nb = plan_rows(op, TR, bm);
  auto go = [&](auto ns, auto vw) {
    constexpr int NS = decltype(ns)::value, VW = decltype(vw)::value;
    hipLaunchKernelGGL((k_rows<T, MODE, NS, VW>), dim3(nb), dim3(RNT), 0, s, op, bm, R, TR,
                       make_fastdiv((uint32_t)(R / VW)), omega, b, x, y);
  };
  auto pick = [&](auto vw) {
    switch (op.kind) {
      case NLSP_OP_FV7: go(std::integral_constant<int, 6>{}, vw); break;
      case NLSP_OP_STENCIL9: go(std::integral_constant<int, 8>{}, vw); break;
      default: go(std::integral_constant<int, 4>{}, vw);
    }
  };
  if (vec) pick(std::integral_constant<int, VMAX>{}); else pick(std::integral_constant<int, 1>{});
}

}  // namespace nlsp

using namespace nlsp;

extern "C" {

const char* nlsp_status_string(int s) {
  switch (s) {
    case NLSP_OK: return "NLSP_OK";
    case NLSP_NOT_CONVERGED: return "NLSP_NOT_CONVERGED";
    case NLSP_E_INVALID: return "NLSP_E_INVALID";
    case NLSP_E_NOT_SPD: return "NLSP_E_NOT_SPD";
    case NLSP_E_BREAKDOWN: return "NLSP_E_BREAKDOWN";
    case NLSP_E_NONFINITE: return "NLSP_E_NONFINITE";
    case NLSP_E_WORKSPACE: return "NLSP_E_WORKSPACE";
    case NLSP_E_HIP: return "NLSP_E_HIP";
    case NLSP_E_RANK: return "NLSP_E_RANK";
    default: return "NLSP_UNKNOWN_STATUS";
  }
}

int64_t nlsp_operator_size(const nlsp_operator* A) { return op_size(A); }

int nlsp_padded_rank(int k) { return padded_rank(k); }

int q1_aniso_stencil(int nsys, const double* eps_theta, double* stencil, void* stream) {
  if (nsys < 1 || !eps_theta || !stencil) return NLSP_E_INVALID;
  hipLaunchKernelGGL(k_q1_stencil, dim3(ceil_div(nsys, 64)), dim3(64), 0, as_stream(stream), nsys,
                     eps_theta, stencil);
  NLSP_HIP(hipGetLastError());
  return NLSP_OK;
}

int apply_operator(const nlsp_operator* A, const double* x, double* y, int R, void* stream) {
  const int64_t n = op_size(A);
  if (n < 1 || !x || !y || R < 1 || x == y || n * R >= (int64_t(1) << 31)) return NLSP_E_INVALID;
  const OpDev op = make_op(*A);
  launch_rows<double, 0>(op, R, 0.0, nullptr, x, y, as_stream(stream));
  NLSP_HIP(hipGetLastError());
  return NLSP_OK;
}

int jacobi_sweep_f32(const nlsp_operator* A, double omega, const float* b, const float* x,
                     float* y, int R, void* stream) {
  const int64_t n = op_size(A);
  if (n < 1 || !b || !x || !y || R < 1 || x == y || !(omega > 0) || n * R >= (int64_t(1) << 31))
    return NLSP_E_INVALID;
  const OpDev op = make_op(*A);
  launch_rows<float, 1>(op, R, (float)omega, b, x, y, as_stream(stream));
  NLSP_HIP(hipGetLastError());
  return NLSP_OK;
}

}  // extern "C"
