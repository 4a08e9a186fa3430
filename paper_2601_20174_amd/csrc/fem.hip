// Linear (P1) finite elements on a triangulation, assembled into a
// compressed-row operator (the paper's own discretisation, FEM dataset
// appendix): per triangle T with vertices p_0, p_1, p_2 (counter-clockwise)
// and tensor K_T,
//   2|T| = (x1 - x0)(y2 - y0) - (x2 - x0)(y1 - y0),
//   g_a = (y_{a+1} - y_{a+2}, x_{a+2} - x_{a+1}) / (2|T|)   (indices mod 3),
//   stiffness |T| g_a^T K_T g_b,  mass |T|/12 (2 if a = b else 1),
// A = sK K + sM M, and a Dirichlet vertex keeps only a unit diagonal (its row
// and column zeroed).
//
// The pattern and, per stored entry, the list of element contributions are
// built on the host (a sort of the 9 nt element pairs); the values on the
// device, one thread per row summing its contributions in increasing
// triangle order, so the result does not depend on scheduling.  The local
// entry is evaluated in a form symmetric in (a, b): the assembled matrix is
// exactly symmetric.
#include <algorithm>
#include <vector>

#include "device_common.hpp"
#include "host_common.hpp"

namespace nlsp {
namespace fem {

// entry (a, b) of sK K_T + sM M_T for triangle t
NLSP_DEV double local_entry(const double* __restrict__ pts, const int* __restrict__ tris,
                            const double* __restrict__ kt, double sK, double sM, int t, int a, int b) {
  // no fused multiply-adds here: fma(ax, by, ay * bx) rounds differently from
  // fma(bx, ay, by * ax), which would break the exact symmetry below
#pragma clang fp contract(off)
  const int v0 = tris[3 * t], v1 = tris[3 * t + 1], v2 = tris[3 * t + 2];
  const double x[3] = {pts[2 * v0], pts[2 * v1], pts[2 * v2]};
  const double y[3] = {pts[2 * v0 + 1], pts[2 * v1 + 1], pts[2 * v2 + 1]};
  const double a2 = (x[1] - x[0]) * (y[2] - y[0]) - (x[2] - x[0]) * (y[1] - y[0]);
  const double area = 0.5 * a2;
  auto grad = [&](int q, double& gx, double& gy) {
    const int u = (q + 1) % 3, w = (q + 2) % 3;
    gx = (y[u] - y[w]) / a2;
    gy = (x[w] - x[u]) / a2;
  };
  double ax, ay, bx, by;
  grad(a, ax, ay);
  grad(b, bx, by);
  const double kxx = kt[3 * t], kxy = kt[3 * t + 1], kyy = kt[3 * t + 2];
  // symmetric in (a, b): each product is commutative and the middle sum has
  // two addends, so swapping a and b gives the same bits
  const double stiff = area * (kxx * (ax * bx) + kxy * (ax * by + ay * bx) + kyy * (ay * by));
  const double mass = area / 12.0 * (a == b ? 2.0 : 1.0);
  return sK * stiff + sM * mass;
}

__global__ __launch_bounds__(256) void k_p1_assemble(int np, const double* __restrict__ pts,
                                                     const int* __restrict__ tris, const double* __restrict__ kt,
                                                     double sK, double sM, const unsigned char* __restrict__ bnd,
                                                     const int* __restrict__ rp, const int* __restrict__ cptr,
                                                     const int* __restrict__ clist, double* __restrict__ vals) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const int e0 = rp[i], e1 = rp[i + 1];
  if (bnd[i]) {
    for (int e = e0; e < e1; ++e) vals[e] = 1.0;   // the diagonal only
    return;
  }
  for (int e = e0; e < e1; ++e) {
    double acc = 0.0;
    for (int c = cptr[e]; c < cptr[e + 1]; ++c) {
      const int code = clist[c];
      const int t = code / 9, ab = code - 9 * t;
      acc += local_entry(pts, tris, kt, sK, sM, t, ab / 3, ab % 3);
    }
    vals[e] = acc;
  }
}

struct Contrib {
  int64_t key;   // row * np + column
  int code;      // 9 t + 3 a + b
};

}  // namespace fem
}  // namespace nlsp

using namespace nlsp;
using namespace nlsp::fem;

extern "C" {

int p1_pattern(int np, int nt, const int* tris, const unsigned char* boundary, int64_t* nnz, int64_t* ncontrib,
               int* row_ptr, int* col_idx, int* cptr, int* clist) {
  if (np < 1 || nt < 0 || (nt > 0 && !tris) || !boundary || !nnz || !ncontrib) return NLSP_E_INVALID;
  const bool fill = row_ptr || col_idx || cptr || clist;
  if (fill && !(row_ptr && col_idx && cptr && clist)) return NLSP_E_INVALID;
  if ((int64_t)nt * 9 >= (int64_t(1) << 31)) return NLSP_E_INVALID;
  std::vector<Contrib> cs;
  cs.reserve((size_t)nt * 9);
  for (int t = 0; t < nt; ++t) {
    const int* v = tris + 3 * (int64_t)t;
    for (int a = 0; a < 3; ++a)
      if (v[a] < 0 || v[a] >= np) return NLSP_E_INVALID;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        if (!boundary[v[a]] && !boundary[v[b]])
          cs.push_back(Contrib{(int64_t)v[a] * np + v[b], 9 * t + 3 * a + b});
  }
  // a boundary vertex: one diagonal entry with no contribution
  for (int i = 0; i < np; ++i)
    if (boundary[i]) cs.push_back(Contrib{(int64_t)i * np + i, -1});
  // by (row, column), contributions in increasing triangle order
  std::sort(cs.begin(), cs.end(), [](const Contrib& p, const Contrib& q) {
    return p.key != q.key ? p.key < q.key : p.code < q.code;
  });
  int64_t n_e = 0, n_c = 0;
  for (size_t u = 0; u < cs.size(); ++u) {
    if (u == 0 || cs[u].key != cs[u - 1].key) ++n_e;
    if (cs[u].code >= 0) ++n_c;
  }
  if (n_e >= (int64_t(1) << 31)) return NLSP_E_INVALID;
  *nnz = n_e;
  *ncontrib = n_c;
  if (!fill) return NLSP_OK;
  for (int i = 0; i <= np; ++i) row_ptr[i] = 0;
  int64_t e = -1, c = 0;
  for (size_t u = 0; u < cs.size(); ++u) {
    if (u == 0 || cs[u].key != cs[u - 1].key) {
      ++e;
      const int row = (int)(cs[u].key / np);
      col_idx[e] = (int)(cs[u].key - (int64_t)row * np);
      cptr[e] = (int)c;
      ++row_ptr[row + 1];
    }
    if (cs[u].code >= 0) clist[c++] = cs[u].code;
  }
  cptr[n_e] = (int)c;
  for (int i = 0; i < np; ++i) row_ptr[i + 1] += row_ptr[i];
  return NLSP_OK;
}

int p1_assemble(int np, int nt, const double* points, const int* tris, const double* ktensor, double sK, double sM,
                const unsigned char* boundary, const int* row_ptr, const int* col_idx, const int* cptr,
                const int* clist, double* vals, void* stream) {
  if (np < 1 || nt < 0 || !points || (nt > 0 && (!tris || !ktensor)) || !boundary || !row_ptr || !col_idx ||
      !cptr || !clist || !vals)
    return NLSP_E_INVALID;
  hipLaunchKernelGGL(k_p1_assemble, dim3(ceil_div(np, 256)), dim3(256), 0, as_stream(stream), np, points, tris,
                     ktensor, sK, sM, boundary, row_ptr, cptr, clist, vals);
  NLSP_HIP(hipGetLastError());
  return NLSP_OK;
}

}  // extern "C"
