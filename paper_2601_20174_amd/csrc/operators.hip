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

// VW values of type TI at p, as T (float64 rows read into float32: two
// 16-byte loads, each value rounded once)
template <typename TI, typename T, int VW>
NLSP_DEV void vload_as(const TI* p, T (&v)[VW]) {
  if constexpr (std::is_same<TI, T>::value) {
    vload<T, VW>(p, v);
  } else {
    static_assert(std::is_same<TI, double>::value && std::is_same<T, float>::value && VW == 4, "row types");
    const double2 a = *reinterpret_cast<const double2*>(p);
    const double2 b = *reinterpret_cast<const double2*>(p + 2);
    v[0] = T(a.x);
    v[1] = T(a.y);
    v[2] = T(b.x);
    v[3] = T(b.y);
  }
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

// ------------------------------------------------------------ 3-D z-march
// For 3-D FV7 operators with R = LPR * VW right-hand sides (LPR = 2, 4 or 8
// lanes per row, VW values per lane).  A block owns a TX x TY tile of the x-y
// plane and marches over a range of planes z.  Every row is read from HBM once:
// planes z-1, z, z+1 sit in registers (plane z+2 is already in flight), the x
// and y neighbours come from an LDS copy of plane z with a one-cell halo, and
// the halo cells, neighbours' coefficients and (Jacobi) right-hand sides of
// plane z+1 are loaded one step ahead.  The row kernel instead reads each
// neighbour row through the cache hierarchy; here only the halo is re-read.
//
// Each step issues its loads for later steps before it consumes anything, and
// consumes only data loaded in earlier steps (the vector memory counter
// retires in issue order, so a wait for a fresh load would drain the
// prefetches too).  The register rings are indexed by constants (the z loop is
// unrolled by the ring length, 4), so no register that is still being loaded
// is ever copied.  The LDS plane is double-buffered: one barrier per step, and
// the barrier orders LDS only, leaving global loads in flight.
//
// Face weights as in row_weights: lane j of a row forms the harmonic means of
// faces j, j + LPR, ... (ceil(6 / LPR) of them) and the row's lanes exchange
// them with wave shuffles, so the coefficient divisions are not repeated per
// lane.  Arithmetic and summation order per output equal the row kernel's up
// to the compiler's choice of fused multiply-adds.
template <int LPR, int TX, int TY>
struct ZTile {
  static constexpr int NT = 64 * LPR;                    // threads
  static constexpr int CPP = NT / LPR, TYS = CPP / TX;   // cells per pass, y rows per pass
  static constexpr int IPT = TY / TYS;                   // cells per thread
  static constexpr int HC = 2 * TX + 2 * TY;             // halo cells of a plane
  static constexpr int HI = (HC * LPR + NT - 1) / NT;    // halo items per thread
  static constexpr int FF = (6 + LPR - 1) / LPR;         // faces per lane
  static_assert(CPP % TX == 0 && TY % TYS == 0 && IPT >= 1, "tile shape");
};

// workgroup barrier that orders LDS accesses only
NLSP_DEV void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// base + a byte offset (a scalar base and a 32-bit lane offset map onto the
// scalar-base form of the global load)
template <typename P>
NLSP_DEV P* at_b(P* base, uint32_t off) {
  using C = std::conditional_t<std::is_const<P>::value, const char, char>;
  return reinterpret_cast<P*>(reinterpret_cast<C*>(base) + off);
}

//   MODE 0: y = A x;  MODE 1: y = x + omega D^-1 (b - A x)  (as k_rows);
//   MODE 2: y = x - (omega / a_ii) (A x)  (the setup's relaxation, b = 0, in
//   the form of the multi-column setup pass)
// Storage T, arithmetic AT.  The R = LPR VW values of a row are columns
// blockIdx.y R .. of rows with stride ld (ld = R for the right-hand-side
// blocks of the operator entry points; wider for the setup's column blocks).
// x may be stored as TI (float64 rows relaxed as float32 rows: the setup's
// first sweep reads its float64 input directly), y as TO (float64 sums stored
// as float32: the float32 copy of the smoothed basis formed in the pass).
template <typename T, int MODE, int VW, int LPR, int TX, int TY, typename AT = T, bool SLAB = false,
          typename TI = T, typename TO = T>
__global__ __launch_bounds__(64 * LPR) void k_zmarch(OpDev op, int ntx, int nty, int zc, int ld_slab, AT omega,
                                                                   const T* __restrict__ b,
                                                                   const TI* __restrict__ x, TO* __restrict__ y) {
  using Z = ZTile<LPR, TX, TY>;
  static_assert(Z::NT == 64 * LPR, "launch bound");
  static_assert(!(SLAB && MODE == 1), "column slabs carry no right-hand side");
  constexpr int NT = Z::NT, R = LPR * VW, IPT = Z::IPT, TYS = Z::TYS, HI = Z::HI, FF = Z::FF;
  constexpr int LW = TX + 2, LSZ = (TY + 2) * LW * R;
  __shared__ T lds[2 * LSZ];
  // the row stride: R for the right-hand-side blocks (a constant there),
  // ld_slab for column slabs
  const int ld = SLAB ? ld_slab : R;
  if (SLAB) {
    x += (int64_t)blockIdx.y * R;
    y += (int64_t)blockIdx.y * R;
  }
  const int nx = op.nx, ny = op.ny, nz = op.nz;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);   // z-chunk major: an XCD sweeps whole planes
  const int tiles = ntx * nty;
  const int zb0 = lb / tiles, tt = lb - zb0 * tiles, ty = tt / ntx, tx = tt - ty * ntx;
  const int x0 = tx * TX, y0 = ty * TY, z0 = zb0 * zc, z1 = min(nz, z0 + zc);
  const int t = threadIdx.x, j = t % LPR, cl = t / LPR, cx = cl % TX, cy0 = cl / TX;
  const int gbase = (t & (WAVE - 1)) - j;
  const uint32_t sxy = (uint32_t)nx * ny;
  const int gx = min(x0 + cx, nx - 1);   // cells outside the grid compute on a clamped copy, store nothing
  uint32_t vo[IPT], co[IPT];             // byte offsets within a plane: values (lane's RHS), coefficient
  bool ok[IPT], inxy[IPT][4];
  int gyv[IPT];
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    const int yy = y0 + cy0 + u * TYS;
    ok[u] = x0 + cx < nx && yy < ny;
    const int gy = min(yy, ny - 1);
    gyv[u] = gy;
    const uint32_t ci = (uint32_t)gy * nx + gx;
    vo[u] = (ci * (uint32_t)ld + j * VW) * (uint32_t)sizeof(T);
    co[u] = ci * 8u;
    inxy[u][0] = gx > 0;
    inxy[u][1] = gx < nx - 1;
    inxy[u][2] = gy > 0;
    inxy[u][3] = gy < ny - 1;
  }
  // halo items: cells (lx, -1), (lx, TY), (-1, ly), (TX, ly) of the tile
  uint32_t ho[HI];   // byte offset within a plane
  int hl[HI];        // LDS element offset, -1: outside the grid (never read)
#pragma unroll
  for (int q = 0; q < HI; ++q) {
    const int h = t + q * NT, hc = h / LPR, hj = h % LPR;
    int lx, ly;
    if (hc < TX) { lx = hc; ly = -1; }
    else if (hc < 2 * TX) { lx = hc - TX; ly = TY; }
    else if (hc < 2 * TX + TY) { lx = -1; ly = hc - 2 * TX; }
    else { lx = TX; ly = hc - 2 * TX - TY; }
    const int hx = x0 + lx, hy = y0 + ly;
    const bool in = h < Z::HC * LPR && hx >= 0 && hx < nx && hy >= 0 && hy < ny;
    ho[q] = in ? (((uint32_t)hy * nx + hx) * (uint32_t)ld + hj * VW) * (uint32_t)sizeof(T) : 0u;
    hl[q] = in ? ((ly + 1) * LW + lx + 1) * R + hj * VW : -1;
  }
  // this lane's faces: z step and the in-plane byte offset of the neighbour's
  // coefficient (clamped into the grid: a missing face reads the cell itself)
  int fdz[FF];
  uint32_t fco[IPT][FF];
#pragma unroll
  for (int f = 0; f < FF; ++f) {
    const int s = min(j + f * LPR, 5);
    const int dx = s == 0 ? -1 : (s == 1 ? 1 : 0), dy = s == 2 ? -1 : (s == 3 ? 1 : 0);
    fdz[f] = s == 4 ? -1 : (s == 5 ? 1 : 0);
#pragma unroll
    for (int u = 0; u < IPT; ++u)
      fco[u][f] = ((uint32_t)min(max(gyv[u] + dy, 0), ny - 1) * nx + min(max(gx + dx, 0), nx - 1)) * 8u;
  }
  const double* a = op.coef;   // generic pointer of a global buffer: the loads stay global
  T pl[4][IPT][VW], hb[2][HI][VW], bq[2][IPT][VW];
  AT ac[2][IPT], af[2][IPT][FF];
  const int64_t pstride = (int64_t)sxy * ld;
  auto plane = [&](auto base, int z) { return base + (int64_t)min(max(z, 0), nz - 1) * pstride; };
  // byte offsets are formed for T; an input of a wider type scales them
  auto ld_plane = [&](T (&v)[IPT][VW], auto base, int z) {
    const auto p = plane(base, z);
    constexpr uint32_t XS = sizeof(*p) / sizeof(T);
#pragma unroll
    for (int u = 0; u < IPT; ++u) vload_as(at_b(p, vo[u] * XS), v[u]);
  };
  auto ld_halo = [&](T (&v)[HI][VW], int z) {
    const TI* p = plane(x, z);
    constexpr uint32_t XS = sizeof(TI) / sizeof(T);
#pragma unroll
    for (int q = 0; q < HI; ++q) vload_as(at_b(p, ho[q] * XS), v[q]);
  };
  auto ld_coef = [&](AT (&ap)[IPT], AT (&fp)[IPT][FF], int z) {
    const int zz = min(z, nz - 1), zlo = max(zz - 1, 0);
    const double* pa = a + (int64_t)zz * sxy;
    const double* pb = a + (int64_t)zlo * sxy;
#pragma unroll
    for (int f = 0; f < FF; ++f) {
      const uint32_t zo = (uint32_t)(min(max(zz + fdz[f], 0), nz - 1) - zlo) * sxy * 8u;
#pragma unroll
      for (int u = 0; u < IPT; ++u) fp[u][f] = AT(*at_b(pb, zo + fco[u][f]));
    }
#pragma unroll
    for (int u = 0; u < IPT; ++u) ap[u] = AT(*at_b(pa, co[u]));
  };
  auto step = [&](auto ph, int z) {
    constexpr int PH = decltype(ph)::value;
    // plane ring: z-1, z, z+1, and the slot that receives z+2; two-slot rings
    // for the halo, coefficients and right-hand sides of planes z and z+1
    constexpr int IP = (PH + 3) & 3, IC = PH, IN = (PH + 1) & 3, IF = (PH + 2) & 3;
    constexpr int H0 = PH & 1, H1 = (PH + 1) & 1;
    T* const buf = lds + H0 * LSZ;
    ld_coef(ac[H1], af[H1], z + 1);
    ld_plane(pl[IF], x, z + 2);
    ld_halo(hb[H1], z + 1);
    if (MODE == 1) ld_plane(bq[H1], b, z + 1);
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
      T* d = buf + ((cy0 + u * TYS + 1) * LW + cx + 1) * R + j * VW;
#pragma unroll
      for (int e = 0; e < VW; ++e) d[e] = pl[IC][u][e];
    }
#pragma unroll
    for (int q = 0; q < HI; ++q)
      if (hl[q] >= 0) {
#pragma unroll
        for (int e = 0; e < VW; ++e) buf[hl[q] + e] = hb[H0][q][e];
      }
    lds_barrier();
    TO* const yp = y + (int64_t)z * pstride;
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
      const bool in[6] = {inxy[u][0], inxy[u][1], inxy[u][2], inxy[u][3], z > 0, z < nz - 1};
      const AT aP = ac[H0][u];
      AT tf[FF];
#pragma unroll
      for (int f = 0; f < FF; ++f) tf[f] = harmonic<AT>(aP, af[H0][u][f]);
      AT w[7];
      AT d = AT(0);
#pragma unroll
      for (int s = 0; s < 6; ++s) {
        const AT th = __shfl(tf[s / LPR], gbase + s % LPR);
        d += in[s] ? th : AT(2) * aP;
        w[1 + s] = in[s] ? -th : AT(0);
      }
      w[0] = d;
      // a missing neighbour reads the centre value with weight 0 (as k_rows)
      const int ly = cy0 + u * TYS + 1, lx = cx + 1;
      const T* L = buf + j * VW;
      T v[7][VW];
#pragma unroll
      for (int e = 0; e < VW; ++e) v[0][e] = pl[IC][u][e];
      vload<T, VW>(L + (ly * LW + lx - (in[0] ? 1 : 0)) * R, v[1]);
      vload<T, VW>(L + (ly * LW + lx + (in[1] ? 1 : 0)) * R, v[2]);
      vload<T, VW>(L + ((ly - (in[2] ? 1 : 0)) * LW + lx) * R, v[3]);
      vload<T, VW>(L + ((ly + (in[3] ? 1 : 0)) * LW + lx) * R, v[4]);
#pragma unroll
      for (int e = 0; e < VW; ++e) {
        v[5][e] = in[4] ? pl[IP][u][e] : pl[IC][u][e];
        v[6][e] = in[5] ? pl[IN][u][e] : pl[IC][u][e];
      }
      T out[VW];
      const AT sc = (MODE == 2) ? omega / w[0] : AT(0);
#pragma unroll
      for (int e = 0; e < VW; ++e) {
        AT acc = w[0] * AT(v[0][e]);
#pragma unroll
        for (int s = 0; s < 6; ++s) acc += w[1 + s] * AT(v[1 + s][e]);
        if (MODE == 1) acc = AT(v[0][e]) + omega * (AT(bq[H0][u][e]) - acc) / w[0];
        if (MODE == 2) acc = AT(v[0][e]) - sc * acc;
        out[e] = T(acc);
      }
      // non-temporal: y is not read again by this pass, so its lines do not
      // displace the planes and halos that neighbouring tiles still read from
      // L2 (FV7 128^3, R = 16: float32 sweep 0.079 -> 0.075 ms)
      if (ok[u]) {
        typedef TO EV __attribute__((ext_vector_type(VW)));
        EV ev;
#pragma unroll
        for (int e = 0; e < VW; ++e) ev[e] = TO(out[e]);
        // byte offsets are formed for T; an output of another width scales them
        const uint32_t yo = (uint32_t)(((uint64_t)vo[u] * sizeof(TO)) / sizeof(T));
        __builtin_nontemporal_store(ev, reinterpret_cast<EV*>(at_b(yp, yo)));
      }
    }
  };
  ld_plane(pl[3], x, z0 - 1);
  ld_plane(pl[0], x, z0);
  ld_plane(pl[1], x, z0 + 1);
  ld_halo(hb[0], z0);
  ld_coef(ac[0], af[0], z0);
  if (MODE == 1) ld_plane(bq[0], b, z0);
  for (int z = z0; z < z1; z += 4) {   // z1 - z0 and the conditions below are uniform per block
    step(std::integral_constant<int, 0>{}, z);
    if (z + 1 < z1) step(std::integral_constant<int, 1>{}, z + 1);
    if (z + 2 < z1) step(std::integral_constant<int, 2>{}, z + 2);
    if (z + 3 < z1) step(std::integral_constant<int, 3>{}, z + 3);
  }
}

// tile 16 x 8 cells, 64 LPR threads; z-chunks of 32 planes for 256 threads
// or more, 16 otherwise, fewer while the grid gives under 512 blocks.  The
// planes at a chunk's ends are read again by the neighbouring chunk (2 of
// zc + 2 planes: 12.5 % extra at 16, 6 % at 32).  Measured on FV7 128^3,
// R = 16 with non-temporal stores: 32 planes against 16 (float64 apply
// 0.1155 -> 0.1143 ms, float32 sweep 0.0746 -> 0.0722 ms) and 64 (0.132 /
// 0.083 ms: too few blocks); a 16 x 16 tile measured slower for float64.
template <typename T, int MODE, int VW, int LPR, typename AT = T, bool SLAB = false, typename TI = T,
          typename TO = T>
inline void launch_zmarch(const OpDev& op, AT omega, const T* b, const TI* x, TO* y, hipStream_t s, int ld = LPR * VW,
                          int nslab = 1) {
  constexpr int TX = 16, TY = 8;
  using Z = ZTile<LPR, TX, TY>;
  const int ntx = (op.nx + TX - 1) / TX, nty = (op.ny + TY - 1) / TY;
  int zc = Z::NT >= 256 ? 32 : 16;
  while (zc > 4 && (int64_t)ntx * nty * ((op.nz + zc - 1) / zc) * nslab < 512) zc /= 2;
  const unsigned nb = (unsigned)((int64_t)ntx * nty * ((op.nz + zc - 1) / zc));
  hipLaunchKernelGGL((k_zmarch<T, MODE, VW, LPR, TX, TY, AT, SLAB, TI, TO>), dim3(nb, nslab), dim3(Z::NT), 0, s,
                     op, ntx, nty, zc, ld, omega, b, x, y);
}

// the z-march applies to 3-D FV7 operators with 2, 4 or 8 lanes of 16-byte
// vectors per row, when every byte offset within three planes fits 32 bits
template <typename T, int MODE>
inline bool try_zmarch(const OpDev& op, int R, T omega, const T* b, const T* x, T* y, hipStream_t s) {
  constexpr int VW = 16 / sizeof(T);
  if (op.kind != NLSP_OP_FV7 || op.nz < 2 || R % VW != 0) return false;
  const int lpr = R / VW;
  if (lpr != 2 && lpr != 4 && lpr != 8) return false;
  const int64_t sxy = (int64_t)op.nx * op.ny;
  if (sxy * R * (int64_t)sizeof(T) >= (int64_t(1) << 32) || 3 * sxy * 8 >= (int64_t(1) << 32)) return false;
  auto al = [](const void* p) { return reinterpret_cast<uintptr_t>(p) % 16 == 0; };
  if (!al(x) || !al(y) || (b && !al(b))) return false;
  switch (lpr) {
    case 2: launch_zmarch<T, MODE, VW, 2>(op, omega, b, x, y, s); break;
    case 4: launch_zmarch<T, MODE, VW, 4>(op, omega, b, x, y, s); break;
    default: launch_zmarch<T, MODE, VW, 8>(op, omega, b, x, y, s);
  }
  return true;
}

// The setup's multi-column passes over (n, ld) row-major blocks of a 3-D FV7
// operator as z-marches over column slabs of 8 lanes of 16-byte vectors (32
// float or 16 double columns, blockIdx.y the slab), arithmetic in the storage
// type (the mixed form's relaxation is a float32 smoother; float64 sums on
// float32 vectors made the sweep bound by the float64 units: 3-D setup 46.4
// -> 42.4 ms): mode 0 out = in - omega D^-1 A in, mode 1 out = A in.  False
// when the shape does not fit (the caller then takes its row-blocked pass).
template <typename T>
bool zmarch_cols(const OpDev& op, int mode, double omega, int ld, const T* in, T* out, hipStream_t s) {
  constexpr int VW = 16 / sizeof(T), LPR = 8, W = VW * LPR;
  if (op.kind != NLSP_OP_FV7 || op.nz < 2 || ld % W != 0 || in == out) return false;
  const int64_t sxy = (int64_t)op.nx * op.ny;
  if (sxy * ld * (int64_t)sizeof(T) >= (int64_t(1) << 32) || 3 * sxy * 8 >= (int64_t(1) << 32)) return false;
  if (reinterpret_cast<uintptr_t>(in) % 16 != 0 || reinterpret_cast<uintptr_t>(out) % 16 != 0) return false;
  if (mode == 0)
    launch_zmarch<T, 2, VW, LPR, T, true>(op, T(omega), nullptr, in, out, s, ld, ld / W);
  else
    launch_zmarch<T, 0, VW, LPR, T, true>(op, T(0), nullptr, in, out, s, ld, ld / W);
  return true;
}
template bool zmarch_cols<float>(const OpDev&, int, double, int, const float*, float*, hipStream_t);
template bool zmarch_cols<double>(const OpDev&, int, double, int, const double*, double*, hipStream_t);

// The float32 relaxation sweep (mode 0 above) reading float64 rows: the
// setup's first sweep takes the float64 S0 directly, each value rounded to
// float32 as it is loaded (the same values as a rounded copy, one pass less).
bool zmarch_cols_relax_f64in(const OpDev& op, double omega, int ld, const double* in, float* out, hipStream_t s) {
  constexpr int VW = 4, LPR = 8, W = VW * LPR;
  if (op.kind != NLSP_OP_FV7 || op.nz < 2 || ld % W != 0) return false;
  const int64_t sxy = (int64_t)op.nx * op.ny;
  if (sxy * ld * (int64_t)sizeof(double) >= (int64_t(1) << 32) || 3 * sxy * 8 >= (int64_t(1) << 32)) return false;
  if (reinterpret_cast<uintptr_t>(in) % 16 != 0 || reinterpret_cast<uintptr_t>(out) % 16 != 0) return false;
  launch_zmarch<float, 2, VW, LPR, float, true, double>(op, float(omega), nullptr, in, out, s, ld, ld / W);
  return true;
}

// The float64 relaxation sweep (mode 0 above) storing its result as float32
// (the rounded values, as a float64 pass and a rounding copy would give).
bool zmarch_cols_relax_f32out(const OpDev& op, double omega, int ld, const double* in, float* out, hipStream_t s) {
  constexpr int VW = 2, LPR = 8, W = VW * LPR;
  if (op.kind != NLSP_OP_FV7 || op.nz < 2 || ld % W != 0) return false;
  const int64_t sxy = (int64_t)op.nx * op.ny;
  if (sxy * ld * (int64_t)sizeof(double) >= (int64_t(1) << 32) || 3 * sxy * 8 >= (int64_t(1) << 32)) return false;
  if (reinterpret_cast<uintptr_t>(in) % 16 != 0 || reinterpret_cast<uintptr_t>(out) % 8 != 0) return false;
  launch_zmarch<double, 2, VW, LPR, double, true, double, float>(op, omega, nullptr, in, out, s, ld, ld / W);
  return true;
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

// A plain copy: one 16-byte vector per thread, non-temporal stores (the
// fastest of the simple forms measured: 6.35 TB/s on a 1 GiB copy, against
// 6.17 TB/s with ordinary stores and 5.8 TB/s with four vectors per thread).
__global__ __launch_bounds__(256) void k_stream_copy(const VecOf<double, 2>::type* __restrict__ a,
                                                     VecOf<double, 2>::type* __restrict__ b, int64_t n) {
  typedef double EV __attribute__((ext_vector_type(2)));
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const EV v = *reinterpret_cast<const EV*>(a + i);
  __builtin_nontemporal_store(v, reinterpret_cast<EV*>(b + i));
}

// Compressed-row operators: one thread per (row, right-hand side), the
// row's entries in stored order, arithmetic in T (float64 values rounded to T
// for the float32 sweep).  MODE as k_rows.
template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_csr_rows(OpDev op, int R, T omega, const T* __restrict__ b,
                                                  const T* __restrict__ x, T* __restrict__ y) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= op.n * R) return;
  const int64_t i = g / R;
  const int c = (int)(g - i * R);
  const int e0 = op.rp[i], e1 = op.rp[i + 1];
  T s = T(0), d = T(0);
  for (int e = e0; e < e1; ++e) {
    const int j = op.ci[e];
    const T a = T(op.coef[e]);
    s += a * x[(int64_t)j * R + c];
    if (j == (int)i) d = a;
  }
  y[g] = (MODE == 0) ? s : x[g] + omega * (b[g] - s) / d;
}

// launches k_rows for the operator kind with the widest vector the right-hand
// side count and the pointers allow
template <typename T, int MODE>
inline void launch_rows(const OpDev& op, int R, T omega, const T* b, const T* x, T* y, hipStream_t s) {
  if (op.kind == NLSP_OP_CSR) {
    hipLaunchKernelGGL((k_csr_rows<T, MODE>), dim3(ceil_div(op.n * R, 256)), dim3(256), 0, s, op, R, omega, b, x,
                       y);
    return;
  }
  if (try_zmarch<T, MODE>(op, R, omega, b, x, y, s)) return;
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

int stream_copy(const void* src, void* dst, int64_t bytes, void* stream) {
  if (!src || !dst || bytes < 0 || bytes % 16 != 0 || reinterpret_cast<uintptr_t>(src) % 16 != 0 ||
      reinterpret_cast<uintptr_t>(dst) % 16 != 0)
    return NLSP_E_INVALID;
  const int64_t n = bytes / 16;
  if (n == 0) return NLSP_OK;
  if (n > int64_t(0x7fffffff) * 256) return NLSP_E_INVALID;   // grid of at most 2^31 - 1 blocks
  hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, as_stream(stream),
                     static_cast<const VecOf<double, 2>::type*>(src), static_cast<VecOf<double, 2>::type*>(dst), n);
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
