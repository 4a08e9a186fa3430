// Matrix-free operator entry points: Q1 anisotropic stencil build, float64
// operator application and the float32 weighted-Jacobi sweep.
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

__global__ void k_apply_f64(OpDev op, const double* __restrict__ x, double* __restrict__ y, int R) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= op.n * R) return;
  const int64_t i = (uint32_t)g / (uint32_t)R;
  const int c = (int)(g - i * R);
  int px, py, pz;
  decompose(op, i, px, py, pz);
  y[g] = op_row<double>(op, i, px, py, pz, [&](int64_t j) { return x[j * R + c]; });
}

__global__ void k_jacobi_f32(OpDev op, float omega, const float* __restrict__ b,
                             const float* __restrict__ x, float* __restrict__ y, int R) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= op.n * R) return;
  const int64_t i = (uint32_t)g / (uint32_t)R;
  const int c = (int)(g - i * R);
  int px, py, pz;
  decompose(op, i, px, py, pz);
  const float ax = op_row<float>(op, i, px, py, pz, [&](int64_t j) { return x[j * R + c]; });
  const float d = op_diag<float>(op, i, px, py, pz);
  y[g] = x[g] + omega * (b[g] - ax) / d;
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
  hipLaunchKernelGGL(k_apply_f64, dim3(ceil_div(n * R, 256)), dim3(256), 0, as_stream(stream), op, x,
                     y, R);
  NLSP_HIP(hipGetLastError());
  return NLSP_OK;
}

int jacobi_sweep_f32(const nlsp_operator* A, double omega, const float* b, const float* x,
                     float* y, int R, void* stream) {
  const int64_t n = op_size(A);
  if (n < 1 || !b || !x || !y || R < 1 || x == y || !(omega > 0) || n * R >= (int64_t(1) << 31))
    return NLSP_E_INVALID;
  const OpDev op = make_op(*A);
  hipLaunchKernelGGL(k_jacobi_f32, dim3(ceil_div(n * R, 256)), dim3(256), 0, as_stream(stream), op,
                     (float)omega, b, x, y, R);
  NLSP_HIP(hipGetLastError());
  return NLSP_OK;
}

}  // extern "C"
