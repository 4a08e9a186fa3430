// Host-side helpers: argument validation, HIP error mapping, workspace carving
// and launch-shape helpers (XCD-aware block order).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "nlsp.h"

#define NLSP_HIP(call)                                  \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return NLSP_E_HIP;            \
  } while (0)

namespace nlsp {

constexpr size_t WS_ALIGN = 256;

inline size_t align_up(size_t v, size_t a = WS_ALIGN) { return (v + a - 1) / a * a; }

// Sequential carving of a caller-provided workspace.  With base == nullptr it
// only measures (used by the *_workspace_bytes queries).
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <typename T>
  T* take(size_t count) {
    off = align_up(off);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
  size_t bytes() const { return align_up(off); }
};

// Number of unknowns, -1 if the descriptor is invalid.  Device index math
// is 32-bit: n must stay below 2^31.
inline int64_t op_size_raw(const nlsp_operator* A) {
  if (!A) return -1;
  if (A->nx < 1 || A->ny < 1) return -1;
  switch (A->kind) {
    case NLSP_OP_POISSON5:
      return (int64_t)A->nx * A->ny;
    case NLSP_OP_FV5:
    case NLSP_OP_STENCIL9:
      if (!A->coef) return -1;
      return (int64_t)A->nx * A->ny;
    case NLSP_OP_FV7:
      if (!A->coef || A->nz < 1) return -1;
      return (int64_t)A->nx * A->ny * A->nz;
    case NLSP_OP_CSR:
      if (!A->coef || !A->row_ptr || !A->col_idx || A->ny != 1 || A->nz != 1) return -1;
      return (int64_t)A->nx;
    default:
      return -1;
  }
}

inline int64_t op_size(const nlsp_operator* A) {
  const int64_t n = op_size_raw(A);
  return (n >= (int64_t(1) << 31)) ? -1 : n;
}

inline int padded_rank(int k) {
  if (k < 1 || k > 256) return -1;
  int kp = 16;
  while (kp < k) kp *= 2;
  return kp;
}

inline bool ws_ok(void* ws, size_t have, size_t need) {
  if (need == 0) return true;
  if (!ws) return false;
  if (reinterpret_cast<uintptr_t>(ws) % WS_ALIGN) return false;
  return have >= need;
}

inline unsigned ceil_div(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace nlsp
