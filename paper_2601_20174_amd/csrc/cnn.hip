// P-predictor: a small convolutional network mapping a coefficient field to
// an unconstrained basis, P_hat = Phi_k + CNN([log a standardised, Phi_k]),
// whose thin Q factor is the learned prolongation (Sec. 4, neural
// parameterisation followed by a thin QR; the paper's network is an MLP on
// the relaxed vectors, here a local CNN on the field with the k smoothest
// sine modes of the unit square as extra input channels and as a residual).
//
// Four 3x3 convolutions ('same', zero padding), hidden width CH, erf-GELU
// after the first three.  Activations are NHWC bfloat16 with channel counts
// padded to multiples of 16; products are v_mfma_f32_16x16x32_bf16 (two
// 16-deep slices of the contraction per instruction; v_mfma_f32_16x16x16_bf16
// for an odd last slice) with float32 accumulation.  Layer l stores its pre-activation z_l; the next
// layer applies GELU while staging its input, and the backward multiplies by
// GELU'(z_l) in the epilogue of the data gradient, so no activation is
// stored twice.  Master parameters, gradients and the optimiser are float32.
#include <algorithm>
#include <cmath>
#include <vector>

#include "device_common.hpp"
#include "host_common.hpp"

namespace nlsp {
namespace cnn {

constexpr int NT = 256;
constexpr int TILE = 16;            // 16 x 16 output pixels per workgroup
constexpr int HALO = TILE + 2;

typedef short s4 __attribute__((ext_vector_type(4)));
typedef short s8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

NLSP_DEV f4 mfma_bf16(s4 a, s4 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0); }
// Two 16-deep products in one instruction.  Lane l of the 32-deep form holds
// contraction slots 8 (l / 16) .. 8 (l / 16) + 7 of its row (A) or column
// (B); filling the low half of both operands from one 16-deep slice and the
// high half from another puts the same contraction index in the same slot of
// A and B, so the result is the sum of the two 16-deep products.
NLSP_DEV s8 cat(s4 lo, s4 hi) { return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7); }
NLSP_DEV f4 mfma_bf16x2(s4 a0, s4 a1, s4 b0, s4 b1, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, cat(a0, a1)), __builtin_bit_cast(bf8, cat(b0, b1)),
                                                 c, 0, 0, 0);
}

// float <-> bfloat16 (round to nearest even; inputs are finite)
NLSP_DEV unsigned short to_bf16(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
NLSP_DEV float from_bf16(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// erf-based GELU and its derivative
NLSP_DEV float gelu(float x) { return 0.5f * x * (1.f + erff(x * 0.70710678118654752f)); }
NLSP_DEV float gelu_grad(float x) {
  return 0.5f * (1.f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

// ------------------------------------------------------------- inputs
// per field: mean and standard deviation of log a (float64); log a itself is
// kept for the input kernel
__global__ __launch_bounds__(NT) void k_field_stats(const double* __restrict__ coef, int n,
                                                    double* __restrict__ stats, double* __restrict__ loga) {
  __shared__ double sh[NT / 64];
  const int b = blockIdx.x;
  const double* a = coef + (int64_t)b * n;
  double* la = loga + (int64_t)b * n;
  double s = 0.0, s2 = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) {
    const double l = log(a[i]);
    la[i] = l;
    s += l;
    s2 += l * l;
  }
  s = block_sum(s, sh);
  s2 = block_sum(s2, sh);
  if (threadIdx.x == 0) {
    const double mean = s / n;
    const double var = std::max(s2 / n - mean * mean, 0.0);
    stats[2 * b] = mean;
    stats[2 * b + 1] = var > 0.0 ? sqrt(var) : 1.0;
  }
}

// Phi (n x k, float32): the k sine modes sin(i pi x) sin(j pi y) of the unit
// square with the smallest i^2 + j^2 (ties by i), at the cell centres
// ((c + 1/2)/N), scaled to unit 2-norm on the grid.  modes: (k x 2) int pairs,
// passed by value (k <= 64).
struct ModeTable {
  int ij[128];
};
__global__ __launch_bounds__(NT) void k_sine_modes(int N, int k, const ModeTable modes, float* __restrict__ phi) {
  const int64_t g = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (g >= (int64_t)N * N * k) return;
  const int j = (int)(g % k);
  const int64_t p = g / k;
  const int x = (int)(p % N), y = (int)(p / N);
  const double h = 1.0 / N;
  const double v = sin(modes.ij[2 * j] * M_PI * (x + 0.5) * h) * sin(modes.ij[2 * j + 1] * M_PI * (y + 0.5) * h);
  phi[g] = (float)(v * 2.0 * h);   // sum over the grid of sin^2 sin^2 = N^2 / 4
}

// x0[b][pixel][c]: c = 0 standardised log a, c = 1..k Phi, zero up to C0p;
// one thread per 4 channels of one pixel, so a wave's 8-byte stores (and its
// Phi loads) are contiguous
__global__ __launch_bounds__(NT) void k_cnn_input(const double* __restrict__ loga, const double* __restrict__ stats,
                                                  const float* __restrict__ phi, int n, int k, int C0p,
                                                  unsigned short* __restrict__ x0) {
  const int b = blockIdx.y;
  const uint32_t q4 = (uint32_t)C0p / 4;
  const uint32_t g = blockIdx.x * NT + threadIdx.x;   // n * q4 < 2^31 (shape check)
  if (g >= (uint32_t)n * q4) return;
  const int p = (int)(g / q4);
  const int c0 = 4 * (int)(g - (uint32_t)p * q4);
  const float a0 = c0 == 0 ? (float)((loga[(int64_t)b * n + p] - stats[2 * b]) / stats[2 * b + 1]) : 0.f;
  const float* ph = phi + (int64_t)p * k;
  unsigned short h[4];
  for (int u = 0; u < 4; ++u) {
    const int c = c0 + u;
    h[u] = to_bf16(c == 0 ? a0 : (c <= k ? ph[c - 1] : 0.f));
  }
  *reinterpret_cast<uint2*>(x0 + ((int64_t)b * n + p) * C0p + c0) =
      make_uint2((unsigned)h[0] | ((unsigned)h[1] << 16), (unsigned)h[2] | ((unsigned)h[3] << 16));
}

// --------------------------------------------------------- weight layouts
// Master layout of layer l: W (Cout, Cin, 3, 3) then b (Cout), float32.
// Forward kernel weights:  Wf[tap][oc][icp]  = W[oc][ic][tap]
// Data-gradient weights:   Wb[tap][ocp][ic]  = W[oc][ic][8 - tap] (as a
// convolution from the Cout channels of dz to the Cin channels of dx)
// Channel counts are padded to Cinp, Coutp (multiples of 16) with zeros.
__global__ __launch_bounds__(NT) void k_prep_weights(const float* __restrict__ W, int Cin, int Cout, int Cinp,
                                                     int Coutp, unsigned short* __restrict__ Wf,
                                                     unsigned short* __restrict__ Wb) {
  const int g = blockIdx.x * NT + threadIdx.x;
  if (g >= 9 * Coutp * Cinp) return;
  const int tap = g / (Coutp * Cinp);
  const int rem = g % (Coutp * Cinp);
  {
    const int oc = rem / Cinp, ic = rem % Cinp;
    const float w = (oc < Cout && ic < Cin) ? W[((int64_t)oc * Cin + ic) * 9 + tap] : 0.f;
    Wf[g] = to_bf16(w);
  }
  {
    const int ic = rem / Coutp, oc = rem % Coutp;   // Wb[tap][ic][oc]: out channel ic, in channel oc
    const float w = (oc < Cout && ic < Cin) ? W[((int64_t)oc * Cin + ic) * 9 + (8 - tap)] : 0.f;
    Wb[g] = to_bf16(w);
  }
}

// ------------------------------------------------------------- convolution
// One 16 x 16 pixel tile of one field per workgroup, all OC output channels
// (OCT = OC / 16 tiles).  D (16 oc x 16 pixels) = sum over taps and input
// channels of Wk[tap][oc][ic] X[pixel + tap][ic]: A = weights (lane: oc =
// l % 16, 4 consecutive ic of each of two 16-channel slices), B = input
// (lane: pixel = l % 16, the same ic), so each lane holds 4 consecutive
// output channels of one pixel.
// Wave w owns output rows 4 w .. 4 w + 3 of the tile.
//   IN_GELU   input value = GELU(stored value)
//   MODE 0    out bf16 z = D + bias                           (hidden layers)
//   MODE 1    out float32 P_hat = Phi + D + bias, oc < k       (last layer)
//   MODE 2    out bf16 dz_prev = D * GELU'(zprev)              (data gradient)
template <int OCT, bool IN_GELU, int MODE>
__global__ __launch_bounds__(NT) void k_conv(int N, int ICp, int k, const unsigned short* __restrict__ X,
                                             const unsigned short* __restrict__ Wk, const float* __restrict__ bias,
                                             const float* __restrict__ phi, const unsigned short* __restrict__ zprev,
                                             void* __restrict__ out) {
  constexpr int OC = OCT * 16;
  extern __shared__ unsigned short lds[];
  const int xs = ICp + 4;                      // bf16 per staged pixel (padding against bank conflicts)
  unsigned short* Xs = lds;                    // HALO x HALO x xs
  unsigned short* Ws = lds + HALO * HALO * xs; // 9 x OC x xs
  const int b = blockIdx.z;
  const int ty0 = blockIdx.y * TILE, tx0 = blockIdx.x * TILE;
  const int64_t n = (int64_t)N * N;
  const unsigned short* Xb = X + (int64_t)b * n * ICp;
  // stage the halo tile and the weights, 4 channels (8 bytes) per load: a
  // thread keeps one channel group and steps over pixels (rows of weights)
  const int q4 = ICp / 4;
  const int per = NT / q4;                     // pixels per pass
  const int c4 = threadIdx.x % q4, p0 = threadIdx.x / q4;
  if (p0 < per) {
    for (int pix = p0; pix < HALO * HALO; pix += per) {
      const int hy = pix / HALO, hx = pix - hy * HALO;
      const int y = ty0 + hy - 1, x = tx0 + hx - 1;
      uint2 v = make_uint2(0u, 0u);
      if (y >= 0 && y < N && x >= 0 && x < N) {
        v = *reinterpret_cast<const uint2*>(Xb + ((int64_t)y * N + x) * ICp + 4 * c4);
        if (IN_GELU) {
          unsigned short h[4] = {(unsigned short)(v.x & 0xffff), (unsigned short)(v.x >> 16),
                                 (unsigned short)(v.y & 0xffff), (unsigned short)(v.y >> 16)};
          for (int u = 0; u < 4; ++u) h[u] = to_bf16(gelu(from_bf16(h[u])));
          v.x = (unsigned)h[0] | ((unsigned)h[1] << 16);
          v.y = (unsigned)h[2] | ((unsigned)h[3] << 16);
        }
      }
      *reinterpret_cast<uint2*>(Xs + pix * xs + 4 * c4) = v;
    }
    for (int row = p0; row < 9 * OC; row += per)   // row = tap * OC + oc
      *reinterpret_cast<uint2*>(Ws + row * xs + 4 * c4) =
          *reinterpret_cast<const uint2*>(Wk + (int64_t)row * ICp + 4 * c4);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lp = lane & 15, lg = lane >> 4;
  f4 acc[4][OCT];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int t = 0; t < OCT; ++t) acc[r][t] = f4{0.f, 0.f, 0.f, 0.f};
  // for one column offset dx the three row offsets dy read rows 4 w + r + dy
  // of the staged tile: the six rows are loaded once and serve all three
  for (int dx = 0; dx < 3; ++dx) {
    const unsigned short* xcol = Xs + (4 * w * HALO + lp + dx) * xs + 4 * lg;
    const unsigned short* wcol = Ws + (dx * OC + lp) * xs + 4 * lg;   // tap 3 dy + dx: + 3 dy OC rows
    int ic0 = 0;
    for (; ic0 + 32 <= ICp; ic0 += 32) {
      s4 bv[2][6];
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int q = 0; q < 6; ++q) bv[h][q] = *reinterpret_cast<const s4*>(xcol + q * HALO * xs + ic0 + 16 * h);
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) {
        s4 a[2][OCT];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int t = 0; t < OCT; ++t)
            a[h][t] = *reinterpret_cast<const s4*>(wcol + (3 * dy * OC + 16 * t) * xs + ic0 + 16 * h);
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int t = 0; t < OCT; ++t)
            acc[r][t] = mfma_bf16x2(a[0][t], a[1][t], bv[0][r + dy], bv[1][r + dy], acc[r][t]);
      }
    }
    if (ic0 < ICp) {   // ICp = 32 j + 16: the last 16 channels
      s4 bv[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) bv[q] = *reinterpret_cast<const s4*>(xcol + q * HALO * xs + ic0);
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) {
        s4 a[OCT];
#pragma unroll
        for (int t = 0; t < OCT; ++t) a[t] = *reinterpret_cast<const s4*>(wcol + (3 * dy * OC + 16 * t) * xs + ic0);
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int t = 0; t < OCT; ++t) acc[r][t] = mfma_bf16(a[t], bv[r + dy], acc[r][t]);
      }
    }
  }
  // epilogue: lane holds oc = 16 t + 4 lg + v of pixel (row 4 w + r, column lp)
  const bool vec4 = MODE == 1 && (k & 3) == 0 && ((reinterpret_cast<uintptr_t>(out) | reinterpret_cast<uintptr_t>(phi)) & 15) == 0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int y = ty0 + 4 * w + r, x = tx0 + lp;
    if (y >= N || x >= N) continue;
    const int64_t pix = (int64_t)b * n + (int64_t)y * N + x;
#pragma unroll
    for (int t = 0; t < OCT; ++t) {
      const int oc0 = 16 * t + 4 * lg;
      if (MODE == 0) {
        unsigned short h[4];
        for (int v = 0; v < 4; ++v) h[v] = to_bf16(acc[r][t][v] + bias[oc0 + v]);
        *reinterpret_cast<uint2*>(static_cast<unsigned short*>(out) + pix * OC + oc0) =
            make_uint2((unsigned)h[0] | ((unsigned)h[1] << 16), (unsigned)h[2] | ((unsigned)h[3] << 16));
      } else if (MODE == 1) {
        float* P = static_cast<float*>(out);
        const int64_t pl = (int64_t)y * N + x;
        if (vec4) {   // the lane's 4 channels as one 16-byte load of Phi and one store of P
          if (oc0 < k) {
            const float4 ph = *reinterpret_cast<const float4*>(phi + pl * k + oc0);
            *reinterpret_cast<float4*>(P + pix * k + oc0) =
                make_float4(ph.x + acc[r][t][0] + bias[oc0], ph.y + acc[r][t][1] + bias[oc0 + 1],
                            ph.z + acc[r][t][2] + bias[oc0 + 2], ph.w + acc[r][t][3] + bias[oc0 + 3]);
          }
        } else {
          for (int v = 0; v < 4; ++v)
            if (oc0 + v < k) P[pix * k + oc0 + v] = phi[pl * k + oc0 + v] + acc[r][t][v] + bias[oc0 + v];
        }
      } else {
        const uint2 zz = *reinterpret_cast<const uint2*>(zprev + pix * OC + oc0);
        const unsigned short zh[4] = {(unsigned short)(zz.x & 0xffff), (unsigned short)(zz.x >> 16),
                                      (unsigned short)(zz.y & 0xffff), (unsigned short)(zz.y >> 16)};
        unsigned short h[4];
        for (int v = 0; v < 4; ++v) h[v] = to_bf16(acc[r][t][v] * gelu_grad(from_bf16(zh[v])));
        *reinterpret_cast<uint2*>(static_cast<unsigned short*>(out) + pix * OC + oc0) =
            make_uint2((unsigned)h[0] | ((unsigned)h[1] << 16), (unsigned)h[2] | ((unsigned)h[3] << 16));
      }
    }
  }
}

// ------------------------------------------------------------ weight gradient
// Partial dW[tap][oc][ic] = sum over the workgroup's pixel tiles of
// dZ[p][oc] X[p + tap][ic] and db[oc] = sum dZ[p][oc].  D (16 oc x 16 ic)
// per (tap, oc-tile, ic-tile); the contraction runs over 16 pixels of one
// image row per step: A = dZ^T (lane: oc = l % 16, 4 consecutive pixels),
// B = shifted X (lane: 4 consecutive pixels, ic = l % 16), two image rows per
// 32-deep instruction.  Both tiles are
// staged channel-major.  The 9 x OCT x ICT output tiles form 3 x OCT x ICT
// groups (dy, oc-tile, ic-tile) of the three taps dx = 0, 1, 2, which share
// their A operand and the staged words their B operands come from; groups are
// dealt to the 4 waves, and a wave holds at most MAXT (a multiple of 3)
// accumulators.
constexpr int WG_TILES = 8;          // pixel tiles per workgroup
template <int MAXT, bool IN_GELU>
__global__ __launch_bounds__(NT) void k_conv_wgrad(int N, int ICp, int OCp, int ntiles_total,
                                                   const unsigned short* __restrict__ X,
                                                   const unsigned short* __restrict__ dZ,
                                                   float* __restrict__ part) {
  extern __shared__ unsigned short lds[];
  constexpr int HS = HALO * HALO + 4;          // channel stride of the staged halo tile
  constexpr int DS = TILE * TILE + 4;          // channel stride of the staged dz tile
  unsigned short* Xt = lds;                    // ICp x HS
  unsigned short* Dt = lds + ICp * HS;         // OCp x DS
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lp = lane & 15, lg = lane >> 4;
  const int ICT = ICp / 16, OCT = OCp / 16;
  const int ngrp = 3 * OCT * ICT;
  f4 acc[MAXT];
#pragma unroll
  for (int s = 0; s < MAXT; ++s) acc[s] = f4{0.f, 0.f, 0.f, 0.f};
  // bias gradient: thread t < nsl * OCp sums pixels slot, slot + nsl, ... of
  // channel oc = t % OCp (slot = t / OCp); slots are added in order at the end
  const int nsl = NT / OCp;
  const int boc = threadIdx.x % OCp, bsl = threadIdx.x / OCp;
  float dbias = 0.f;
  const int tiles_x = (N + TILE - 1) / TILE;
  const int per_field = tiles_x * tiles_x;
  const int64_t n = (int64_t)N * N;
  for (int ti = 0; ti < WG_TILES; ++ti) {
    const int tile = blockIdx.x * WG_TILES + ti;
    if (tile >= ntiles_total) break;
    const int b = tile / per_field, tt = tile % per_field;
    const int ty0 = (tt / tiles_x) * TILE, tx0 = (tt % tiles_x) * TILE;
    __syncthreads();
    {
      // halo tile channel-major, 4 channels per 8-byte load; one channel
      // group per thread, stepping over pixels
      const int q4 = ICp / 4, per = NT / q4;
      const int c4 = threadIdx.x % q4, p0 = threadIdx.x / q4;
      if (p0 < per)
        for (int pix = p0; pix < HALO * HALO; pix += per) {
          const int hy = pix / HALO, hx = pix - hy * HALO;
          const int y = ty0 + hy - 1, x = tx0 + hx - 1;
          uint2 v = make_uint2(0u, 0u);
          if (y >= 0 && y < N && x >= 0 && x < N)
            v = *reinterpret_cast<const uint2*>(X + ((int64_t)b * n + (int64_t)y * N + x) * ICp + 4 * c4);
          unsigned short h[4] = {(unsigned short)(v.x & 0xffff), (unsigned short)(v.x >> 16),
                                 (unsigned short)(v.y & 0xffff), (unsigned short)(v.y >> 16)};
          for (int u = 0; u < 4; ++u) Xt[(4 * c4 + u) * HS + pix] = IN_GELU ? to_bf16(gelu(from_bf16(h[u]))) : h[u];
        }
      const int o4 = OCp / 4, pero = NT / o4;
      const int d4 = threadIdx.x % o4, q0 = threadIdx.x / o4;
      if (q0 < pero)
        for (int pix = q0; pix < TILE * TILE; pix += pero) {
          const int y = ty0 + pix / TILE, x = tx0 + pix % TILE;
          uint2 v = make_uint2(0u, 0u);
          if (y < N && x < N) v = *reinterpret_cast<const uint2*>(dZ + ((int64_t)b * n + (int64_t)y * N + x) * OCp + 4 * d4);
          Dt[(4 * d4 + 0) * DS + pix] = (unsigned short)(v.x & 0xffff);
          Dt[(4 * d4 + 1) * DS + pix] = (unsigned short)(v.x >> 16);
          Dt[(4 * d4 + 2) * DS + pix] = (unsigned short)(v.y & 0xffff);
          Dt[(4 * d4 + 3) * DS + pix] = (unsigned short)(v.y >> 16);
        }
    }
    __syncthreads();
    if (bsl < nsl)
      for (int p = bsl; p < TILE * TILE; p += nsl) dbias += from_bf16(Dt[boc * DS + p]);
#pragma unroll
    for (int s = 0; s < MAXT / 3; ++s) {
      const int g = w + 4 * s;
      if (g >= ngrp) break;
      const int dy = g / (OCT * ICT), rem = g % (OCT * ICT);
      const int ot = rem / ICT, it = rem % ICT;
      const unsigned short* dr = Dt + (16 * ot + lp) * DS + 4 * lg;
      // the lane's 4 pixels of tap dx start at element dx of an even-aligned
      // group of 6: three aligned dwords serve all three taps (realigned by 2
      // bytes for dx = 1)
      const uint32_t* xb = reinterpret_cast<const uint32_t*>(Xt + (16 * it + lp) * HS + dy * HALO + 4 * lg);
      for (int row0 = 0; row0 < TILE; row0 += 4) {
        // pixels 4 lg .. 4 lg + 3 of output rows row0 .. row0 + 3: all operand
        // reads first, then the products
        s4 a[4], bv[3][4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int row = row0 + u;
          a[u] = *reinterpret_cast<const s4*>(dr + row * TILE);
          const uint32_t* xr = xb + row * (HALO / 2);
          const uint32_t w0 = xr[0], w1 = xr[1], w2 = xr[2];
          bv[0][u] = __builtin_bit_cast(s4, make_uint2(w0, w1));
          bv[1][u] = __builtin_bit_cast(s4, make_uint2(__builtin_amdgcn_alignbyte(w1, w0, 2),
                                                       __builtin_amdgcn_alignbyte(w2, w1, 2)));
          bv[2][u] = __builtin_bit_cast(s4, make_uint2(w1, w2));
        }
#pragma unroll
        for (int dx = 0; dx < 3; ++dx)
          acc[3 * s + dx] = mfma_bf16x2(a[0], a[1], bv[dx][0], bv[dx][1], acc[3 * s + dx]);
#pragma unroll
        for (int dx = 0; dx < 3; ++dx)
          acc[3 * s + dx] = mfma_bf16x2(a[2], a[3], bv[dx][2], bv[dx][3], acc[3 * s + dx]);
      }
    }
  }
  // partial record of this workgroup: [9][OCp][ICp] then [OCp]
  float* rec = part + (int64_t)blockIdx.x * (9 * OCp * ICp + OCp);
#pragma unroll
  for (int s = 0; s < MAXT / 3; ++s) {
    const int g = w + 4 * s;
    if (g >= ngrp) break;
    const int dy = g / (OCT * ICT), rem = g % (OCT * ICT);
    const int ot = rem / ICT, it = rem % ICT;
#pragma unroll
    for (int dx = 0; dx < 3; ++dx)
      for (int v = 0; v < 4; ++v)
        rec[((int64_t)(3 * dy + dx) * OCp + 16 * ot + 4 * lg + v) * ICp + 16 * it + lp] = acc[3 * s + dx][v];
  }
  __syncthreads();
  float* sb = reinterpret_cast<float*>(lds);   // staging area is free now
  if (bsl < nsl) sb[bsl * OCp + boc] = dbias;
  __syncthreads();
  if (threadIdx.x < OCp) {
    float tot = 0.f;
    for (int q = 0; q < nsl; ++q) tot += sb[q * OCp + threadIdx.x];
    rec[9 * OCp * ICp + threadIdx.x] = tot;
  }
}

// Weight-gradient records are added in two fixed-order levels: slices of
// RSL consecutive records first (many workgroups in flight), then the slices.
constexpr int RSL = 32;

__global__ __launch_bounds__(NT) void k_wgrad_slices(int nrec, int64_t stride, const float* __restrict__ part,
                                                     float* __restrict__ slices) {
  const int64_t g = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (g >= stride) return;
  const int sl = blockIdx.y;
  const int r0 = sl * RSL, r1 = min(nrec, r0 + RSL);
  float v[8];
  float s = 0.f;
  for (int r = r0; r < r1; r += 8) {
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = (r + j < r1) ? part[(int64_t)(r + j) * stride + g] : 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += v[j];
  }
  slices[(int64_t)sl * stride + g] = s;
}

// dW (master layout (Cout, Cin, 3, 3)) and db from the slices, in order
__global__ __launch_bounds__(NT) void k_wgrad_reduce(int nsl, int ICp, int OCp, int Cin, int Cout,
                                                     const float* __restrict__ slices, float* __restrict__ gW,
                                                     float* __restrict__ gb) {
  const int g = blockIdx.x * NT + threadIdx.x;
  const int nW = Cout * Cin * 9;
  if (g >= nW + Cout) return;
  int64_t src;
  if (g < nW) {
    const int oc = g / (Cin * 9), ic = (g / 9) % Cin, tap = g % 9;
    src = ((int64_t)tap * OCp + oc) * ICp + ic;
  } else {
    src = (int64_t)9 * OCp * ICp + (g - nW);
  }
  const int64_t stride = 9 * OCp * ICp + OCp;
  double s = 0.0;
  for (int q = 0; q < nsl; ++q) s += (double)slices[q * stride + src];
  if (g < nW)
    gW[g] = (float)s;
  else
    gb[g - nW] = (float)s;
}

// float32 -> bfloat16 with channel padding: (rows, C) -> (rows, Cp); one
// thread per 4 output channels of one row (one 8-byte store), with one
// 16-byte load where C = Cp and src is 16-byte aligned (vec)
__global__ __launch_bounds__(NT) void k_pad_bf16(int64_t rows, int C, int Cp, int vec, const float* __restrict__ src,
                                                 unsigned short* __restrict__ dst) {
  const uint32_t q4 = (uint32_t)Cp / 4;
  const uint32_t g = blockIdx.x * NT + threadIdx.x;   // rows * q4 < 2^31 (shape check)
  if (g >= (uint32_t)rows * q4) return;
  const uint32_t r = g / q4;
  const int c0 = 4 * (int)(g - r * q4);
  float v[4];
  if (vec) {
    const float4 f = *reinterpret_cast<const float4*>(src + (int64_t)r * C + c0);
    v[0] = f.x, v[1] = f.y, v[2] = f.z, v[3] = f.w;
  } else {
    for (int u = 0; u < 4; ++u) v[u] = c0 + u < C ? src[(int64_t)r * C + c0 + u] : 0.f;
  }
  *reinterpret_cast<uint2*>(dst + (int64_t)r * Cp + c0) =
      make_uint2((unsigned)to_bf16(v[0]) | ((unsigned)to_bf16(v[1]) << 16),
                 (unsigned)to_bf16(v[2]) | ((unsigned)to_bf16(v[3]) << 16));
}

// Adam (bias-corrected) on float32 parameters
__global__ __launch_bounds__(NT) void k_adam(int64_t count, float* __restrict__ p, const float* __restrict__ g,
                                             float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                                             float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------- host side
struct Net {
  int batch, N, k, ch;
  int64_t n;
  int cin[4], cout[4], cinp[4], coutp[4];
  int64_t woff[4], boff[4];   // offsets of W_l and b_l in the parameter vector
  int64_t nparams;
};

inline int r16(int v) { return (v + 15) / 16 * 16; }

inline bool make_net(const nlsp_cnn_shape* s, Net& t) {
  if (!s || s->batch < 1 || s->N < TILE || s->k < 1 || s->k > 64 || s->hidden < 1 || s->hidden > 64) return false;
  if (s->k % 16 || s->hidden % 16) return false;
  // the weight gradient holds at most 16 (oc-tile, ic-tile) pairs per layer
  if ((r16(1 + s->k) / 16) * (s->hidden / 16) > 16) return false;
  if ((int64_t)s->batch * s->N * s->N * 64 >= (int64_t(1) << 31)) return false;
  t.batch = s->batch;
  t.N = s->N;
  t.k = s->k;
  t.ch = s->hidden;
  t.n = (int64_t)s->N * s->N;
  const int cin[4] = {1 + s->k, s->hidden, s->hidden, s->hidden};
  const int cout[4] = {s->hidden, s->hidden, s->hidden, s->k};
  int64_t off = 0;
  for (int l = 0; l < 4; ++l) {
    t.cin[l] = cin[l];
    t.cout[l] = cout[l];
    t.cinp[l] = r16(cin[l]);
    t.coutp[l] = r16(cout[l]);
    t.woff[l] = off;
    off += (int64_t)cout[l] * cin[l] * 9;
    t.boff[l] = off;
    off += cout[l];
  }
  t.nparams = off;
  return true;
}

struct NetLayout {
  double* stats;                 // (batch, 2)
  double* loga;                  // (batch n) log of the cell coefficients
  float* phi;                    // (n, k)
  unsigned short* x0;            // (batch n, cinp[0])
  unsigned short* z[3];          // (batch n, ch) pre-activations of layers 1..3
  unsigned short* wf[4];         // forward weights per layer
  unsigned short* wb[4];         // data-gradient weights per layer
  unsigned short* dz[4];         // (batch n, coutp[l]) gradients of the pre-activations
  float* part;                   // weight-gradient partial records
  size_t bytes;
};

inline int wgrad_groups(const Net& t) {
  const int tx = (t.N + TILE - 1) / TILE;
  const int tiles = t.batch * tx * tx;
  return (tiles + WG_TILES - 1) / WG_TILES;
}

inline NetLayout carve_net(void* ws, const Net& t) {
  Carver c(ws);
  NetLayout L;
  L.stats = c.take<double>(2 * t.batch);
  L.loga = c.take<double>(t.batch * t.n);
  L.phi = c.take<float>(t.n * t.k);
  const int64_t bn = t.batch * t.n;
  L.x0 = c.take<unsigned short>(bn * t.cinp[0]);
  for (int l = 0; l < 3; ++l) L.z[l] = c.take<unsigned short>(bn * t.coutp[l]);
  int64_t maxrec = 0;
  for (int l = 0; l < 4; ++l) {
    L.wf[l] = c.take<unsigned short>((size_t)9 * t.coutp[l] * t.cinp[l]);
    L.wb[l] = c.take<unsigned short>((size_t)9 * t.coutp[l] * t.cinp[l]);
    L.dz[l] = c.take<unsigned short>(bn * t.coutp[l]);
    maxrec = std::max<int64_t>(maxrec, 9 * t.coutp[l] * t.cinp[l] + t.coutp[l]);
  }
  const int groups = wgrad_groups(t);
  L.part = c.take<float>((size_t)(groups + (groups + RSL - 1) / RSL) * maxrec);   // records, then slices
  L.bytes = c.bytes();
  return L;
}

inline size_t conv_lds(int ICp, int OC) { return ((size_t)HALO * HALO * (ICp + 4) + (size_t)9 * OC * (ICp + 4)) * 2; }
inline size_t wgrad_lds(int ICp, int OCp) {
  return ((size_t)ICp * (HALO * HALO + 4) + (size_t)OCp * (TILE * TILE + 4)) * 2;
}

template <typename K>
inline hipError_t allow(K kern, size_t bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

// k smoothest sine modes (i, j >= 1) by i^2 + j^2, ties by i
inline std::vector<int> smooth_modes(int k) {
  std::vector<std::pair<int, std::pair<int, int>>> all;
  for (int i = 1; i <= 64; ++i)
    for (int j = 1; j <= 64; ++j) all.push_back({i * i + j * j, {i, j}});
  std::sort(all.begin(), all.end());
  std::vector<int> m;
  for (int q = 0; q < k; ++q) {
    m.push_back(all[q].second.first);
    m.push_back(all[q].second.second);
  }
  return m;
}

// launch one convolution: input X (ICp channels), weights Wk (OC x ICp per tap)
template <bool IN_GELU, int MODE>
inline int conv(const Net& t, int ICp, int OC, const unsigned short* X, const unsigned short* Wk, const float* bias,
                const float* phi, const unsigned short* zprev, void* out, hipStream_t s) {
  const int tx = (t.N + TILE - 1) / TILE;
  const dim3 grid(tx, tx, t.batch);
  const size_t lds = conv_lds(ICp, OC);
  auto go = [&](auto kern) -> int {
    if (allow(kern, lds) != hipSuccess) return NLSP_E_HIP;
    hipLaunchKernelGGL(kern, grid, dim3(NT), lds, s, t.N, ICp, t.k, X, Wk, bias, phi, zprev, out);
    return NLSP_OK;
  };
  switch (OC / 16) {
    case 1: return go(k_conv<1, IN_GELU, MODE>);
    case 2: return go(k_conv<2, IN_GELU, MODE>);
    case 3: return go(k_conv<3, IN_GELU, MODE>);
    default: return go(k_conv<4, IN_GELU, MODE>);
  }
}

template <bool IN_GELU>
inline int wgrad(const Net& t, int l, const unsigned short* X, const unsigned short* dZ, float* part, float* gW,
                 float* gb, hipStream_t s) {
  const int ICp = t.cinp[l], OCp = t.coutp[l];
  const int groups = wgrad_groups(t);
  const int tx = (t.N + TILE - 1) / TILE;
  const int tiles = t.batch * tx * tx;
  const size_t lds = wgrad_lds(ICp, OCp);
  // accumulators per wave: three per (dy, oc-tile, ic-tile) group, groups dealt to 4 waves
  const int need = 3 * ((3 * (OCp / 16) * (ICp / 16) + 3) / 4);
  if (need > 36) return NLSP_E_INVALID;
  auto go = [&](auto kern) -> int {
    if (allow(kern, lds) != hipSuccess) return NLSP_E_HIP;
    hipLaunchKernelGGL(kern, dim3(groups), dim3(NT), lds, s, t.N, ICp, OCp, tiles, X, dZ, part);
    return NLSP_OK;
  };
  int rc;
  if (need <= 9)
    rc = go(k_conv_wgrad<9, IN_GELU>);
  else if (need <= 18)
    rc = go(k_conv_wgrad<18, IN_GELU>);
  else
    rc = go(k_conv_wgrad<36, IN_GELU>);
  if (rc != NLSP_OK) return rc;
  const int nout = t.cout[l] * t.cin[l] * 9 + t.cout[l];
  const int64_t stride = 9 * OCp * ICp + OCp;
  const int nsl = (groups + RSL - 1) / RSL;
  float* slices = part + (int64_t)groups * stride;
  hipLaunchKernelGGL(k_wgrad_slices, dim3(ceil_div(stride, NT), nsl), dim3(NT), 0, s, groups, stride, part, slices);
  hipLaunchKernelGGL(k_wgrad_reduce, dim3(ceil_div(nout, NT)), dim3(NT), 0, s, nsl, ICp, OCp, t.cin[l], t.cout[l],
                     slices, gW, gb);
  return NLSP_OK;
}

}  // namespace cnn
}  // namespace nlsp

using namespace nlsp;
using namespace nlsp::cnn;

extern "C" {

int64_t cnn_param_count(const nlsp_cnn_shape* shape) {
  Net t;
  return make_net(shape, t) ? t.nparams : -1;
}

size_t cnn_workspace_bytes(const nlsp_cnn_shape* shape) {
  Net t;
  if (!make_net(shape, t)) return 0;
  const size_t need = std::max({conv_lds(t.cinp[0], t.coutp[0]), conv_lds(t.ch, t.ch), wgrad_lds(t.cinp[0], t.ch),
                                wgrad_lds(t.ch, t.ch), wgrad_lds(t.ch, t.k)});
  if (need > 160 * 1024) return 0;
  return carve_net(nullptr, t).bytes;
}

int cnn_fwd(const nlsp_cnn_shape* shape, const float* params, const double* coef, float* Phat, void* ws,
            size_t ws_bytes, void* stream) {
  Net t;
  if (!make_net(shape, t) || !params || !coef || !Phat) return NLSP_E_INVALID;
  const size_t need = cnn_workspace_bytes(shape);
  if (need == 0) return NLSP_E_INVALID;
  if (!ws_ok(ws, ws_bytes, need)) return NLSP_E_WORKSPACE;
  const NetLayout L = carve_net(ws, t);
  hipStream_t s = as_stream(stream);
  const std::vector<int> modes = smooth_modes(t.k);
  ModeTable tab{};
  std::copy(modes.begin(), modes.end(), tab.ij);
  hipLaunchKernelGGL(k_sine_modes, dim3(ceil_div(t.n * t.k, NT)), dim3(NT), 0, s, t.N, t.k, tab, L.phi);
  hipLaunchKernelGGL(k_field_stats, dim3(t.batch), dim3(NT), 0, s, coef, (int)t.n, L.stats, L.loga);
  hipLaunchKernelGGL(k_cnn_input, dim3(ceil_div(t.n * (t.cinp[0] / 4), NT), t.batch), dim3(NT), 0, s, L.loga,
                     L.stats, L.phi, (int)t.n, t.k, t.cinp[0], L.x0);
  for (int l = 0; l < 4; ++l)
    hipLaunchKernelGGL(k_prep_weights, dim3(ceil_div(9 * t.coutp[l] * t.cinp[l], NT)), dim3(NT), 0, s,
                       params + t.woff[l], t.cin[l], t.cout[l], t.cinp[l], t.coutp[l], L.wf[l], L.wb[l]);
  int rc = conv<false, 0>(t, t.cinp[0], t.ch, L.x0, L.wf[0], params + t.boff[0], nullptr, nullptr, L.z[0], s);
  if (rc == NLSP_OK) rc = conv<true, 0>(t, t.ch, t.ch, L.z[0], L.wf[1], params + t.boff[1], nullptr, nullptr, L.z[1], s);
  if (rc == NLSP_OK) rc = conv<true, 0>(t, t.ch, t.ch, L.z[1], L.wf[2], params + t.boff[2], nullptr, nullptr, L.z[2], s);
  if (rc == NLSP_OK) rc = conv<true, 1>(t, t.ch, t.k, L.z[2], L.wf[3], params + t.boff[3], L.phi, nullptr, Phat, s);
  if (rc != NLSP_OK) return rc;
  NLSP_HIP(hipGetLastError());
  return NLSP_OK;
}

int cnn_bwd(const nlsp_cnn_shape* shape, const float* params, const float* gPhat, float* gparams, void* ws,
            size_t ws_bytes, void* stream) {
  Net t;
  if (!make_net(shape, t) || !params || !gPhat || !gparams) return NLSP_E_INVALID;
  const size_t need = cnn_workspace_bytes(shape);
  if (need == 0) return NLSP_E_INVALID;
  if (!ws_ok(ws, ws_bytes, need)) return NLSP_E_WORKSPACE;
  const NetLayout L = carve_net(ws, t);
  hipStream_t s = as_stream(stream);
  const int64_t bn = t.batch * t.n;
  // dz4 = dP_hat (the residual Phi and the bias add pass gradients through)
  const int vec = t.k == t.coutp[3] && (reinterpret_cast<uintptr_t>(gPhat) & 15) == 0;
  hipLaunchKernelGGL(k_pad_bf16, dim3(ceil_div(bn * (t.coutp[3] / 4), NT)), dim3(NT), 0, s, bn, t.k, t.coutp[3], vec,
                     gPhat, L.dz[3]);
  int rc = wgrad<true>(t, 3, L.z[2], L.dz[3], L.part, gparams + t.woff[3], gparams + t.boff[3], s);
  // dz3 = (W4^T * dz4) GELU'(z3), and so on down to layer 1
  for (int l = 3; l >= 1 && rc == NLSP_OK; --l) {
    rc = conv<false, 2>(t, t.coutp[l], t.cinp[l], L.dz[l], L.wb[l], nullptr, nullptr, L.z[l - 1], L.dz[l - 1], s);
    if (rc != NLSP_OK) break;
    if (l - 1 >= 1)
      rc = wgrad<true>(t, l - 1, L.z[l - 2], L.dz[l - 1], L.part, gparams + t.woff[l - 1], gparams + t.boff[l - 1], s);
    else
      rc = wgrad<false>(t, 0, L.x0, L.dz[0], L.part, gparams + t.woff[0], gparams + t.boff[0], s);
  }
  if (rc != NLSP_OK) return rc;
  NLSP_HIP(hipGetLastError());
  return NLSP_OK;
}

int adam_step(int64_t count, float* params, const float* grads, float* m, float* v, float lr, float beta1,
              float beta2, float eps, int step, void* stream) {
  if (count < 1 || !params || !grads || !m || !v || step < 1 || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) ||
      !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return NLSP_E_INVALID;
  const float c1 = 1.f - std::pow(beta1, (float)step), c2 = 1.f - std::pow(beta2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(ceil_div(count, NT)), dim3(NT), 0, as_stream(stream), count, params, grads, m, v,
                     lr, beta1, beta2, eps, c1, c2);
  NLSP_HIP(hipGetLastError());
  return NLSP_OK;
}

}  // extern "C"
